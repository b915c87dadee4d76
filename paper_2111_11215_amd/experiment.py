"""Training and evaluation loops used by the benchmark and the tests:
plain fine-stage training, the proposal form, held-out PSNR.

Inputs (ray batches, targets, held-out views) are prepared by the caller as
device tensors; every step runs through ``train``/``api`` into the library.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import torch

from . import api, train


@dataclass
class Batch:
    o: torch.Tensor
    d: torch.Tensor
    j: torch.Tensor
    target: torch.Tensor
    n_uniform: int = 0          # uniform in-box samples of the batch (the metric's numerator)


@dataclass
class View:
    o: torch.Tensor
    d: torch.Tensor
    target: torch.Tensor
    center: tuple = (0.0, 0.0, 4.0)     # camera centre (looking at the origin, up +z)
    c2w: tuple = ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))
    H: int = 800
    W: int = 800
    focal: float = 1000.0


@dataclass
class RunStats:
    iters: int = 0
    seconds: float = 0.0
    uniform_samples: int = 0
    losses: list = field(default_factory=list)
    prop_losses: list = field(default_factory=list)
    fallback_rate: list = field(default_factory=list)

    @property
    def samples_per_s(self) -> float:
        return self.uniform_samples / self.seconds if self.seconds > 0 else 0.0


def count_uniform_with(sample, batches) -> None:
    """Fill each batch's count of uniform in-box samples (the metric's
    numerator) from ``sample(o, d, j)``'s n_uniform."""
    for b in batches:
        b.n_uniform = int(sample(b.o, b.d, b.j).n_uniform.sum().item())


def count_uniform(model: train.FineModel, batches) -> None:
    """Fill each batch's uniform-sample count (clip and count, no list)."""
    for b in batches:
        s = api.sample_rays(b.o, b.d, b.j, model.grid.box_min, model.grid.box_max, model.cfg.step,
                            model.cfg.max_samples, clip_only=True)
        b.n_uniform = int(s.n_uniform.sum().item())


def run(model: train.FineModel, batches, iters: int, prop: train.ProposalModel | None = None,
        learn_prop: bool = True, record_every: int = 50, start: int = 0) -> RunStats:
    """Train for `iters` steps over the batch list (cycled).  Synchronises
    only at the start, at the end and at the recording points."""
    st = RunStats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        b = batches[(start + it) % len(batches)]
        if prop is None:
            res = model.train_step(b.o, b.d, b.target, b.j)
        else:
            res = train.proposal_train_step(model, prop, b.o, b.d, b.target, b.j, learn=learn_prop)
        st.uniform_samples += b.n_uniform
        if record_every and (it % record_every == 0 or it == iters - 1):
            st.losses.append((it, float(res["loss"].item())))
            if prop is not None:
                st.fallback_rate.append((it, float((res["mask"] == -1).float().mean().item())))
                if "prop_loss" in res:
                    st.prop_losses.append((it, float(res["prop_loss"].item())))
    torch.cuda.synchronize()
    st.seconds = time.perf_counter() - t0
    st.iters = iters
    return st


def evaluated_per_step(model: train.FineModel, batches, prop: train.ProposalModel | None = None, n: int = 4):
    """Average number of samples the fine pass evaluates per batch, plain or
    with the proposal's masks."""
    tot = 0
    for b in batches[:n]:
        if prop is None:
            s = model.sample(b.o, b.d, b.j)
        else:
            _, _, mask = prop.masks_rays(b.o, b.d)
            s = model.sample(b.o, b.d, b.j, seg_mask=mask)
        tot += int(s.n_kept.item())
    return tot / n


def psnr_views(model: train.FineModel, views) -> float:
    """Mean over views of -10 log10(MSE) of the plain-sampled render."""
    vals = []
    for v in views:
        rgb = train.render_rays(model, v.o, v.d)
        mse = float(((rgb - v.target) ** 2).mean().item())
        vals.append(-10.0 * math.log10(max(mse, 1e-12)))
    return sum(vals) / len(vals)


def render_view(model: train.FineModel, view, chunk: int = 1 << 16) -> dict:
    """One held-out view through dvgo_render_image (rays cast on the GPU,
    plain sampler without jitter, forward in chunks)."""
    c = model.cfg
    fine = (model.grid.density, model.fine_thr) if model.fine_thr is not None else None
    return api.render_image(model.grid, model.mlp, view.c2w, view.center, view.H, view.W, view.focal, c.step,
                            c.max_samples, coarse=model.coarse, bg=c.bg, precision=c.precision,
                            use_shadow=c.bf16_feat, chunk=chunk, fine=fine)


def frame_ms(model: train.FineModel, view, reps: int = 3) -> float:
    """Wall time of rendering one held-out view at test time
    (dvgo_render_image), in ms per frame, averaged over `reps` renders after
    one untimed one."""
    render_view(model, view)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        render_view(model, view)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def proposal_render_psnr(model: train.FineModel, prop: train.ProposalModel, views) -> float:
    """PSNR of the proposal-sampled render against the plain-sampled render
    of the same model (how much of the image the proposal keeps)."""
    vals = []
    for v in views:
        ref = train.render_rays(model, v.o, v.d)
        out = torch.empty_like(ref)
        for a in range(0, v.o.shape[0], 1 << 16):
            b = min(a + (1 << 16), v.o.shape[0])
            o, d = v.o[a:b].contiguous(), v.d[a:b].contiguous()
            _, _, mask = prop.masks_rays(o, d)
            s = model.sample(o, d, None, seg_mask=mask, morton=False)
            out[a:b] = model.render(s, want_depth_acc=False)["rgb"]
        mse = float(((out - ref) ** 2).mean().item())
        vals.append(-10.0 * math.log10(max(mse, 1e-12)))
    return sum(vals) / len(vals)


def fit_toy2d(target: torch.Tensor, stride: float, mode: int, iters: int = 2000, lr: float = 0.1,
              delta: float = 1.0) -> dict:
    """The image-fitting toy of Sec. 3: a grid of (H/stride) x (W/stride)
    vertices, zero-initialised (alpha 1/2 everywhere at delta 1), fitted to
    the binary ``target`` [H, W] by Adam on the mean squared error.  Returns
    the final loss, PSNR and the step time."""
    H, W = target.shape
    gh, gw = max(2, int(H / stride)), max(2, int(W / stride))
    V = torch.zeros((gh, gw), dtype=torch.float32, device=target.device)
    st = train.AdamState.of(V)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(1, iters + 1):
        api.toy2d_loss_grad(st.p, target, mode, delta, grad=st.g)
        api.adam_step(st.p, st.g, st.m, st.v, lr, it)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    img = api.toy2d_forward(st.p, H, W, mode, delta)
    mse = float(((img - target) ** 2).mean().item())
    return {"grid": (gh, gw), "mse": mse, "psnr": -10.0 * math.log10(max(mse, 1e-30)), "ms_per_step": 1e3 * sec / iters,
            "V": st.p}
