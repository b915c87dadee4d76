"""Training-step driver of the fine stage: sample, render, loss, adjoint,
Adam - every step a call into ``libdvgo.so`` on the current stream.

Hyperparameters follow the paper's implementation details: Adam with batch
8192, learning rates 0.1 for the grids and 1e-3 for the MLP, decayed
exponentially to 0.1x at 20k iterations.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import torch

from . import api
from ._lib import DVGO_BF16, DVGO_F32


@dataclass
class AdamState:
    p: torch.Tensor
    g: torch.Tensor
    m: torch.Tensor
    v: torch.Tensor
    shadow: Optional[torch.Tensor] = None

    @staticmethod
    def of(p: torch.Tensor, shadow: bool = False) -> "AdamState":
        st = AdamState(p, torch.zeros_like(p), torch.zeros_like(p), torch.zeros_like(p))
        if shadow:
            st.shadow = torch.empty(p.shape, dtype=torch.int16, device=p.device)
            # the first forward reads the shadow: a zero-rate Adam step with
            # zero moments leaves p, m, v unchanged and writes bf16(p)
            api.adam_step(st.p, st.g, st.m, st.v, 0.0, 1, shadow=st.shadow)
        return st


@dataclass
class FineConfig:
    step: float
    max_samples: int
    bg: tuple = (1.0, 1.0, 1.0)
    lr_grid: float = 0.1
    lr_mlp: float = 1e-3
    decay_steps: int = 20000
    betas: tuple = (0.9, 0.999)
    eps: float = 1e-8
    precision: int = DVGO_F32        # matrix-core arithmetic of the MLP
    bf16_feat: bool = False          # gather features from a bfloat16 shadow
    morton: bool = False
    capacity: Optional[int] = None
    fused_grid_adam: bool = True     # the whole step in one call (dvgo_train_step): no grid gradient in
                                     # memory, the adjoint reuses the forward's gathers and colours
    skip_idle: bool = True           # the fused grid Adam skips vertices with zero moments that no sample
                                     # touches (their step changes no bit), tracked by an activity mask
    fine_tau: Optional[float] = None  # second free-space rule: skip samples whose fine alpha is below this
    pg_ckpt: tuple = ()              # progressive scaling: iterations at which the grids double their voxels
    pg_final_n: int = 0              # vertices per axis after the last checkpoint (with pg_ckpt)
    w_pt_rgb: float = 0.0            # auxiliary losses of the fine objective (the paper: 1e-2 and 1e-3)
    w_bg_entropy: float = 0.0


class FineModel:
    """Fine-stage parameters (density grid, feature grid, colour MLP) with
    their Adam state, plus the frozen coarse keep-mask."""

    def __init__(self, density, feat, mlp_flat, box_min, box_max, act_shift, cfg: FineConfig, coarse=None):
        self.cfg = cfg
        self.mlp = mlp_flat
        self.coarse = coarse
        self.st_mlp = AdamState.of(mlp_flat)
        self.t = 0          # iterations (the network's Adam step count and the learning-rate schedule)
        self._set_grids(density, feat, box_min, box_max, act_shift)

    def _set_grids(self, density, feat, box_min, box_max, act_shift) -> None:
        """New grid tensors with fresh Adam state (zero moments, own step
        count) and a clear activity mask."""
        cfg = self.cfg
        self.grid = api.Grid(density, feat, tuple(box_min), tuple(box_max), float(act_shift))
        self.st_density = AdamState.of(density)
        self.st_feat = AdamState.of(feat, shadow=cfg.bf16_feat)
        self.grid.feat_shadow = self.st_feat.shadow
        self.t_grid = 0     # the grids' Adam step count (restarts when the grids are resized)
        # one bit per vertex: its moments may be non-zero (all clear with the zero moments above)
        self.active = None
        if cfg.fused_grid_adam and cfg.skip_idle:
            self.active = torch.zeros(api.grid_active_words(density.numel()), dtype=torch.int32,
                                      device=density.device)
        self.fine_thr = None
        if cfg.fine_tau is not None:
            self.fine_thr = api.coarse_raw_threshold(cfg.fine_tau, cfg.step, act_shift)

    def rescale(self, n_new: int) -> None:
        """Progressive scaling (Sec. 4.2): resize both grids to n_new vertices
        per axis by trilinear interpolation; the sample step follows the
        voxel size (half a voxel), the shift b stays, and the grids' Adam
        state restarts (the network's does not)."""
        g = self.grid
        dens = api.grid_resample(g.density, (n_new,) * 3, g.box_min, g.box_max)
        feat = api.grid_resample(g.feat, (n_new,) * 3, g.box_min, g.box_max)
        span = max(hi - lo for lo, hi in zip(g.box_min, g.box_max))
        self.cfg.step = 0.5 * span / (n_new - 1)
        self.cfg.max_samples = int(math.ceil(math.sqrt(3.0) * span / self.cfg.step)) + 1
        self._set_grids(dens, feat, g.box_min, g.box_max, g.act_shift)

    def lr(self, base: float) -> float:
        return api.lr_at(base, self.t, self.cfg.decay_steps)

    def sample(self, rays_o, rays_d, jitter, seg_mask=None, capacity=None, morton=None) -> api.Samples:
        c = self.cfg
        fine = (self.grid.density, self.fine_thr) if self.fine_thr is not None else None
        return api.sample_rays(rays_o, rays_d, jitter, self.grid.box_min, self.grid.box_max, c.step, c.max_samples,
                               coarse=self.coarse, seg_mask=seg_mask, morton=c.morton if morton is None else morton,
                               capacity=c.capacity if capacity is None else capacity, fine=fine)

    def render(self, s: api.Samples, **kw) -> dict:
        c = self.cfg
        return api.render_fwd(self.grid, self.mlp, s, c.bg, precision=c.precision, use_shadow=c.bf16_feat, **kw)

    def backward(self, s: api.Samples, out: dict, grad_rgb: torch.Tensor) -> None:
        c = self.cfg
        api.render_bwd(self.grid, self.mlp, s, out["log_t_end"], grad_rgb, self.st_density.g, self.st_feat.g,
                       self.st_mlp.g, c.bg, precision=c.precision, use_shadow=c.bf16_feat)

    def adam(self) -> None:
        c = self.cfg
        self.t += 1
        self.t_grid += 1
        lg, lm = self.lr(c.lr_grid), self.lr(c.lr_mlp)
        for st, lr, t in ((self.st_density, lg, self.t_grid), (self.st_feat, lg, self.t_grid),
                          (self.st_mlp, lm, self.t)):
            api.adam_step(st.p, st.g, st.m, st.v, lr, t, c.betas, c.eps, shadow=st.shadow)
        if self.active is not None:   # dense steps moved moments the mask does not know of
            d, f = self.st_density, self.st_feat
            api.grid_active_init(d.m, d.v, f.m, f.v, self.active)

    def backward_adam(self, s: api.Samples, out: dict, grad_rgb: torch.Tensor) -> None:
        """Adjoint with the grids' Adam step fused in, then the network's
        Adam step (same result as ``backward`` followed by ``adam``)."""
        c = self.cfg
        self.t += 1
        self.t_grid += 1
        lg, lm = self.lr(c.lr_grid), self.lr(c.lr_mlp)
        d, f = self.st_density, self.st_feat
        api.render_bwd_adam(self.grid, self.mlp, s, out["log_t_end"], grad_rgb, d.m, d.v, f.m, f.v, self.st_mlp.g,
                            lg, self.t_grid, c.betas, c.eps, c.bg, precision=c.precision, use_shadow=c.bf16_feat,
                            active=self.active)
        m = self.st_mlp
        api.adam_step(m.p, m.g, m.m, m.v, lm, self.t, c.betas, c.eps)

    def train_step(self, rays_o, rays_d, target, jitter=None, seg_mask=None) -> dict:
        """One full iteration: sample, render, photometric loss, adjoint,
        Adam.  Returns the loss (device tensor) and the sample list.  With
        progressive scaling the grids are resized when the iteration count
        reaches a checkpoint."""
        c = self.cfg
        if c.pg_ckpt and self.t in c.pg_ckpt:
            k = list(c.pg_ckpt).index(self.t) + 1
            self.rescale(api.pg_resolution(c.pg_final_n, len(c.pg_ckpt), k))
        s = self.sample(rays_o, rays_d, jitter, seg_mask)
        if self.cfg.fused_grid_adam:
            self.t += 1
            self.t_grid += 1
            lg, lm = self.lr(c.lr_grid), self.lr(c.lr_mlp)
            d, f, m = self.st_density, self.st_feat, self.st_mlp
            loss, rgb = api.train_step(self.grid, self.mlp, s, target, d.m, d.v, f.m, f.v, m.g, lg, self.t_grid,
                                       c.betas, c.eps, c.bg, precision=c.precision, use_shadow=c.bf16_feat,
                                       active=self.active, mlp_adam=(m.m, m.v, lm, self.t),
                                       aux=(c.w_pt_rgb, c.w_bg_entropy) if (c.w_pt_rgb or c.w_bg_entropy) else None)
            return {"loss": loss, "samples": s, "rgb": rgb}
        out = self.render(s, want_depth_acc=False)
        loss, grad = api.photo_loss(out["rgb"], target)
        if self.cfg.fused_grid_adam:
            self.backward_adam(s, out, grad)
        else:
            self.backward(s, out, grad)
            self.adam()
        return {"loss": loss, "samples": s, "rgb": out["rgb"]}


class ProposalModel:
    """Learned segment proposal (not in the paper): network weights with
    their Adam state and the selection thresholds.  Each training step it
    predicts a segment mask for every ray of the batch; every learn_every-th
    step it learns from a density-only pass of the fine model on the first
    1/sub_fraction of the batch (KL to the segment weight sums and the final
    transmittance).  The defaults (every 4th step, half a batch, lr 3e-3)
    see the same rays per step as learning every step on 1/8 with lr 1e-3,
    with the same selectivity at 1000 iterations, in a quarter of the
    launches."""

    def __init__(self, flat: torch.Tensor, box_min, box_max, lr: float = 3e-3, cum_frac: float = 0.99,
                 min_mass: float = 0.9, sub_fraction: int = 2, learn_every: int = 4):
        self.st = AdamState.of(flat)
        self.box_min, self.box_max = tuple(box_min), tuple(box_max)
        self.lr, self.cum_frac, self.min_mass, self.sub = lr, cum_frac, min_mass, sub_fraction
        self.learn_every = learn_every
        self.t = 0        # proposal updates taken
        self.calls = 0    # training iterations seen

    @property
    def flat(self) -> torch.Tensor:
        return self.st.p

    def masks(self, s: api.Samples):
        return api.proposal_fwd(s, self.box_min, self.box_max, self.flat, self.cum_frac, self.min_mass)

    def masks_rays(self, rays_o, rays_d):
        """Segment masks of bare rays (the call clips them itself)."""
        return api.proposal_fwd_rays(rays_o, rays_d, self.box_min, self.box_max, self.flat, self.cum_frac,
                                     self.min_mass)

    def learn(self, model: "FineModel", rays_o, rays_d, jitter) -> torch.Tensor:
        """One proposal update from a density-only pass on the given rays."""
        s = model.sample(rays_o, rays_d, jitter)
        tgt = api.render_fwd(model.grid, None, s, model.cfg.bg, want_seg_w=True, want_depth_acc=False)
        self.t += 1
        return api.proposal_bwd_adam(s, self.box_min, self.box_max, self.flat, tgt["seg_w"], tgt["log_t_end"],
                                     self.st.g, self.st.m, self.st.v, self.lr, self.t)


def proposal_train_step(model: FineModel, prop: ProposalModel, rays_o, rays_d, target, jitter=None,
                        learn: bool = True) -> dict:
    """One iteration of the proposal form: predict segment masks (the
    proposal call clips the rays itself), sample only the selected segments
    (all of them where the proposal falls back), render / adjoint / Adam,
    then (every learn_every-th iteration) update the proposal on the first
    1/sub of the batch."""
    _, mass, mask = prop.masks_rays(rays_o, rays_d)
    res = model.train_step(rays_o, rays_d, target, jitter, seg_mask=mask)
    prop.calls += 1
    if learn and (prop.calls - 1) % prop.learn_every == 0:
        k = max(rays_o.shape[0] // prop.sub, 1)
        res["prop_loss"] = prop.learn(model, rays_o[:k], rays_d[:k], jitter[:k] if jitter is not None else None)
    res["mask"] = mask
    res["mass"] = mass
    return res


@torch.no_grad()
def render_rays(model: FineModel, rays_o, rays_d, chunk: int = 1 << 16) -> torch.Tensor:
    """Colour of every ray with the plain sampler (no jitter), in chunks."""
    out = torch.empty((rays_o.shape[0], 3), dtype=torch.float32, device=rays_o.device)
    for a in range(0, rays_o.shape[0], chunk):
        b = min(a + chunk, rays_o.shape[0])
        s = model.sample(rays_o[a:b].contiguous(), rays_d[a:b].contiguous(), None, morton=False)
        out[a:b] = model.render(s, want_depth_acc=False)["rgb"]
    return out


class CoarseModel:
    """Coarse stage (Sec. 4.1): a density grid with the low-density
    initialisation (Prior 1: zero grid, shift from alpha_init at the coarse
    voxel size) and a view-invariant colour grid, trained with the
    photometric, per-point rgb and background entropy losses; the density's
    Adam step takes the view-count learning-rate factor (Prior 2).  The
    trained density gives the fine stage its free-space mask."""

    def __init__(self, n: int, box_min, box_max, cams: torch.Tensor, H: int, W: int, focal: float,
                 alpha_init: float = 1e-6, lr: float = 0.1, w_pt: float = 0.1, w_bg: float = 0.01,
                 decay_steps: int = 20000, bg=(1.0, 1.0, 1.0), view_count_lr: bool = True):
        dev = cams.device
        self.box_min, self.box_max = tuple(box_min), tuple(box_max)
        self.n = n
        span = max(hi - lo for lo, hi in zip(self.box_min, self.box_max))
        self.voxel = span / (n - 1)
        self.step = 0.5 * self.voxel
        self.max_samples = int(math.ceil(math.sqrt(3.0) * span / self.step)) + 1
        self.act_shift = api.low_density_bias(alpha_init, self.voxel)
        self.st_density = AdamState.of(torch.zeros((n, n, n), device=dev))
        self.st_rgb = AdamState.of(torch.zeros((n, n, n, 3), device=dev))
        self.counts, self.lr_scale = api.view_counts((n, n, n), self.box_min, self.box_max, cams, H, W, focal)
        if not view_count_lr:
            self.lr_scale = torch.ones_like(self.lr_scale)
        self.lr, self.w_pt, self.w_bg, self.decay_steps, self.bg = lr, w_pt, w_bg, decay_steps, bg
        self.t = 0

    @property
    def density(self) -> torch.Tensor:
        return self.st_density.p

    def sample(self, rays_o, rays_d, jitter) -> api.Samples:
        return api.sample_rays(rays_o, rays_d, jitter, self.box_min, self.box_max, self.step, self.max_samples)

    def train_step(self, rays_o, rays_d, target, jitter=None) -> dict:
        s = self.sample(rays_o, rays_d, jitter)
        d, c = self.st_density, self.st_rgb
        loss, _ = api.coarse_step(d.p, c.p, self.box_min, self.box_max, self.act_shift, s, target, d.g, c.g,
                                  self.max_samples, self.w_pt, self.w_bg, self.bg)
        self.t += 1
        lr = api.lr_at(self.lr, self.t, self.decay_steps)
        api.adam_step_scaled(d.p, d.g, d.m, d.v, self.lr_scale, lr, self.t)
        api.adam_step(c.p, c.g, c.m, c.v, lr, self.t)
        return {"loss": loss, "samples": s}

    def free_space_mask(self, tau: float, fine_step: float) -> torch.Tensor:
        """Known free space for the fine stage (Sec. 4.2): the per-cell keep
        bits of the trained density at threshold tau, with alpha taken over
        the fine sample spacing."""
        thr = api.coarse_raw_threshold(tau, fine_step, self.act_shift)
        return api.coarse_mask_build(self.density, self.box_min, self.box_max, thr)


def cams_table(c2ws, centers, device) -> torch.Tensor:
    """[ncam, 12] float32 for dvgo_view_counts: each camera's row-major
    camera-to-world rotation (columns right, up, back) and its centre."""
    rows = [[float(x) for row in R for x in row] + [float(x) for x in c] for R, c in zip(c2ws, centers)]
    return torch.tensor(rows, dtype=torch.float32, device=device)
