"""Benchmark of the fine-stage per-ray training step on one MI355X.

Workload: the full configuration - synthetic scene of 64 soft spheres,
160^3 float32 density and 12-channel feature grids initialised as in the
paper's fine stage (zero grids, low-density shift with alpha_init 1e-2),
frozen 100^3 coarse density rasterised from the scene with the alpha-mask
threshold 1e-4, 8192 rays per iteration drawn with replacement from 100
cameras of 800x800 pixels, step half a voxel, the 39-128-128-3 colour
network.  One step = the whole hot path over one batch, inputs resident in
HBM: in the default form (bfloat16 features and network plus the learned
proposal) proposal forward with its own clip and the segment masks,
sampling of the selected segments, forward, loss, adjoint with the grids'
Adam step, the network's Adam step, and, every 4th step, the proposal's own
update from a density-only pass on half of the batch.  Forms: proposal
(default), bf16, plain (float32, no proposal).

Before timing, the comparison trains, for --compare-iters iterations each
from identical states on identical batches, the plain float32, the bfloat16
and the bfloat16 + proposal forms, and beside them the paper's further
parts: the fine-alpha skip with progressive scaling, the auxiliary losses,
the network with the encoded position plus those losses (float32 and
bfloat16), and the mask learned by the coarse stage (throughput and
held-out PSNR of each); the timed steps continue training the selected
form from its trained state.  The coarse stage runs first (its learned mask
feeds one of the forms); the precision (16384 rays) and stress (256^3,
32768 rays) configurations and the image-fitting toy are timed after the
timed steps, and the oracle on the host last.

Metric: ray-samples/s = (sum over the timed iterations of the uniform
in-box samples of each batch, before coarse or proposal skipping) / wall
time of the timed iterations (HIP-synchronised on both sides).

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work per evaluated sample of the kernels the roofline can name.
FLOP_MLP_FWD = 2 * (12 * 128 + 128 * 128 + 3 * 128)
FLOP_MLP_BWD = FLOP_MLP_FWD + 2 * (3 * 128 + 128 * 128 + 12 * 128) + 2 * (3 * 128 + 128 * 128 + 128 * 40)
BYTES_SCATTER = 8 * (1 + 12) * 4 * 2 + (4 + 48) + 8
BYTES_GATHER_F32 = 8 * 4 + 8 * 48 + (4 + 48) + 8
BYTES_GATHER_BF16 = 8 * 4 + 8 * 24 + (4 + 48) + 8
# fused grid Adam per vertex: density and 12 features, each p, m, v read and
# written (24 B); bfloat16 copy 2 B per feature; binned sample records 64 B
BYTES_GRID_ADAM_VERTEX = 24 * 13
BYTES_REC = 64
# launched with the grid Adam: the network's gradient reduction, per
# parameter one float per partial row read, the flat gradient read and
# cleared, p, m, v read and written
BYTES_REDUCE_PARAM_FIXED = 4 + 4 + 24
# launched with the fine pass's gather: the preparation, per ray the
# direction read and the first layer's view part (128 floats) and encoding
# (32 floats) written; the cleared cell counts; the packed operands
BYTES_PREP_RAY = 12 + 128 * 4 + 32 * 4
BYTES_PREP_PACK = 2 * 16384 * 4 + 2 * 16384 * 2 + 4 * 2 * 64 * 4 + 4 * 64 * 8 * 2
PEAK = {"hbm": 8000.0, "f32": 157.3, "bf16": 2500.0}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--form", choices=["proposal", "bf16", "plain"], default="proposal")
    ap.add_argument("--morton", type=int, default=0, help="1: Morton-ordered ray slots in every form")
    ap.add_argument("--pretrain", type=int, default=0,
                    help="with --compare-iters 0: training iterations of the timed form before timing")
    ap.add_argument("--rays", type=int, default=8192)
    ap.add_argument("--profile-kernel", default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=0, help="oracle sample: rays of the first batch (0: all)")
    ap.add_argument("--cpu-reps", type=int, default=4, help="oracle steps timed (their mean is reported)")
    ap.add_argument("--profile-steps", type=int, default=10,
                    help="steps per kernel of the event-timed pass (0: skip it)")
    ap.add_argument("--compare-iters", type=int, default=1000,
                    help="iterations of the plain-fp32 / bf16 / bf16+proposal training comparison (0: skip);"
                         " the timed form continues from its trained state")
    ap.add_argument("--extra-configs", type=int, default=1, help="1: also time the precision and stress shapes")
    ap.add_argument("--toy", type=int, default=1, help="1: also run the image-fitting toy")
    ap.add_argument("--coarse-iters", type=int, default=5000,
                    help="train the coarse stage this long first and add a fine form on its learned mask")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def setup(args):
    import torch

    import synth
    from paper_2111_11215_amd import api

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sp, cams, held, raw = synth.full_scene(0)
    n = synth.FULL_N
    voxel = 2.0 / (n - 1)
    step = 0.5 * voxel
    max_samples = int(math.ceil(2.0 * math.sqrt(3.0) / step)) + 1
    b = api.low_density_bias(synth.FULL_ALPHA_INIT, voxel)
    bmin, bmax = tuple(synth.BOX_MIN), tuple(synth.BOX_MAX)
    thr = api.coarse_raw_threshold(synth.FULL_TAU, step)
    raw_t = torch.as_tensor(raw).to(dev)
    bits = api.coarse_mask_build(raw_t, bmin, bmax, thr)
    coarse = (bits, bmin, bmax, raw.shape)
    spheres = torch.as_tensor(sp.as_f32_table()).to(dev)
    return dict(step=step, max_samples=max_samples, b=b, raw=raw, bits=bits, coarse=coarse, spheres=sp,
                spheres_t=spheres, bmin=bmin, bmax=bmax, n=n, cams=cams, held=held, morton=bool(args.morton))


def make_batches(ctx, n_iter, rays, seed0=1000):
    """Per-iteration batches (pixels with replacement, then jitter, from
    default_rng(seed0 + t)) with targets rendered by the scene generator."""
    import numpy as np
    import torch

    import synth
    from paper_2111_11215_amd import api, experiment
    cams = ctx["cams"]
    flats, jits = [], []
    for t in range(n_iter):
        rng = np.random.default_rng(seed0 + t)
        flats.append(rng.integers(0, len(cams) * 800 * 800, size=rays))
        jits.append(rng.random(rays).astype(np.float32))
    o, d, *_ = synth.scenes._rays_for_flat_pixels(cams, 800, 800, 1000.0, np.concatenate(flats))
    dev = torch.device("cuda:0")
    ot, dt = torch.as_tensor(o).to(dev), torch.as_tensor(d).to(dev)
    jt = torch.as_tensor(np.concatenate(jits)).to(dev)
    tgt = api.scene_render(ot, dt, ctx["spheres_t"], ctx["bmin"], ctx["bmax"], ctx["step"] / 4)
    return [experiment.Batch(ot[t * rays:(t + 1) * rays], dt[t * rays:(t + 1) * rays],
                             jt[t * rays:(t + 1) * rays], tgt[t * rays:(t + 1) * rays]) for t in range(n_iter)]


def make_views(ctx):
    """The 10 held-out 800x800 views and their scene renders."""
    import numpy as np
    import torch

    import synth
    from paper_2111_11215_amd import api, experiment
    dev = torch.device("cuda:0")
    views = []
    for c in ctx["held"]:
        o, d = synth.scenes.image_rays(c, 800, 800, 1000.0)
        ot = torch.as_tensor(np.ascontiguousarray(o)).to(dev).contiguous()
        dt = torch.as_tensor(np.ascontiguousarray(d)).to(dev).contiguous()
        c2w = tuple(tuple(float(x) for x in row) for row in synth.look_at_c2w(c))
        views.append(experiment.View(ot, dt, api.scene_render(ot, dt, ctx["spheres_t"], ctx["bmin"], ctx["bmax"],
                                                              ctx["step"] / 4),
                                     center=tuple(float(x) for x in c), c2w=c2w))
    return views


def coarse_stage(ctx, iters, alpha_init, rays=8192, pool=64):
    """The coarse stage of Sec. 4.1 (100^3 grids, view-count learning rate,
    loss weights 0.1 and 0.01, lr 0.1) from ``alpha_init``, on the sphere
    scene, for ``iters`` iterations over a pool of batches; then its
    free-space mask (tau^(c) = 1e-3 over the fine step) against the mask
    rasterised from the analytic scene."""
    import numpy as np
    import torch

    import synth
    from paper_2111_11215_amd import api, experiment, train
    cams = ctx["cams"]
    R = [synth.look_at_c2w(c) for c in cams]
    model = train.CoarseModel(100, ctx["bmin"], ctx["bmax"], train.cams_table(R, cams, "cuda:0"), 800, 800, 1000.0,
                              alpha_init=alpha_init)
    batches = make_batches(ctx, pool, rays, seed0=90000)
    experiment.count_uniform_with(model.sample, batches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    for it in range(iters):
        b = batches[it % pool]
        res = model.train_step(b.o, b.d, b.target, b.j)
        if it % 500 == 0 or it == iters - 1:
            losses.append((it, float(res["loss"].item())))
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    n_uni = sum(batches[it % pool].n_uniform for it in range(iters))
    mask = model.free_space_mask(1e-3, ctx["step"])
    thr = api.coarse_raw_threshold(1e-3, ctx["step"])
    rast = api.coarse_mask_build(torch.as_tensor(ctx["raw"]).to("cuda:0"), ctx["bmin"], ctx["bmax"], thr)
    bits = lambda w: np.unpackbits(w.cpu().numpy().view(np.uint8), bitorder="little").astype(bool)
    lb, rb = bits(mask), bits(rast)
    rep = {"iters": iters, "rays_per_iter": rays, "alpha_init": alpha_init, "ms_per_step": 1e3 * sec / iters,
           "ray_samples_per_s": n_uni / sec, "loss_first_last": [losses[0][1], losses[-1][1]],
           "loss_curve": losses, "mask_cells_kept": {"learned": int(lb.sum()), "rasterised": int(rb.sum())},
           "mask_recall_of_rasterised": float((lb & rb).sum() / max(rb.sum(), 1))}
    return rep, (mask, ctx["bmin"], ctx["bmax"], (100, 100, 100))


def new_model(ctx, bf16, skip_pg=False, coarse=None, aux=False, pe_x=0):
    import numpy as np
    import torch

    import synth
    from paper_2111_11215_amd import api, train
    from paper_2111_11215_amd._lib import DVGO_BF16, DVGO_F32
    dev = torch.device("cuda:0")
    n = ctx["n"]
    # pe_x = 5: the paper's network that also takes the encoded position (72 inputs)
    Ws, bs = synth.xavier_uniform_mlp(np.random.default_rng(7), (72 if pe_x else 39, 128, 128, 3))
    flat = api.flat_from([Ws[0], bs[0], Ws[1], bs[1], Ws[2], bs[2]], api.mlp_shapes(pe_x), dev)
    cfg = train.FineConfig(step=ctx["step"], max_samples=ctx["max_samples"],
                           precision=DVGO_BF16 if bf16 else DVGO_F32, bf16_feat=bf16, morton=ctx["morton"])
    if aux:
        # the paper's fine objective: photometric + 1e-2 per-point rgb + 1e-3 background entropy
        cfg.w_pt_rgb, cfg.w_bg_entropy = 1e-2, 1e-3
    if skip_pg:
        # the paper's second free-space rule (tau^(f) = 1e-4) and progressive
        # scaling, its checkpoints at 1k, 2k, 3k of 20k iterations scaled to
        # this run's length
        it = ctx.get("compare_iters", 1000)
        cfg.fine_tau = 1e-4
        cfg.pg_ckpt = tuple(max(1, it * k // 20) for k in (1, 2, 3))
        cfg.pg_final_n = n
        n = api.pg_resolution(n, 3, 0)
        cfg.step = 0.5 * 2.0 / (n - 1)
        cfg.max_samples = int(math.ceil(2.0 * math.sqrt(3.0) / cfg.step)) + 1
    return train.FineModel(torch.zeros((n, n, n), device=dev), torch.zeros((n, n, n, 12), device=dev), flat,
                           ctx["bmin"], ctx["bmax"], ctx["b"], cfg,
                           coarse=ctx["coarse"] if coarse is None else coarse)


def new_proposal(ctx):
    import numpy as np

    import synth
    from paper_2111_11215_amd import api, train
    Ws, bs = synth.xavier_uniform_mlp(np.random.default_rng(11), (54, 64, 64, 32))
    flat = api.flat_from([Ws[0], bs[0], Ws[1], bs[1], Ws[2], bs[2]], api.PROP_SHAPES, "cuda:0")
    return train.ProposalModel(flat, ctx["bmin"], ctx["bmax"])


FORMS = {"plain": ("plain_fp32", False, False), "bf16": ("bf16", True, False),
         "proposal": ("bf16_proposal", True, True)}
# forms trained in the comparison only: bf16 with the fine-density skip and progressive scaling
EXTRA_FORMS = {"skip_pg": ("bf16_fine_skip_progressive", True, False),
               "aux": ("bf16_auxiliary_losses", True, False),
               "paper": ("fp32_paper_network_and_objective", False, False),
               "paper_bf16": ("bf16_paper_network_and_objective", True, False),
               "learned_coarse": ("bf16_learned_coarse_mask", True, False)}


def compare_forms(ctx, iters, rays, keep):
    """Train the plain fp32 form, the bf16 form and the bf16 + learned
    proposal form from identical initial states on identical batches;
    report throughput (uniform-equivalent ray-samples/s of the whole
    iteration, proposal work included) and mean PSNR on the 10 held-out
    views, the time of one 800x800 inference frame, plus what the trained
    proposal gains over an untrained one and over none.  Returns (report,
    (model, proposal) of the form ``keep``)."""
    from paper_2111_11215_amd import experiment
    log(f"bench: comparison, {iters} iterations per form")
    batches = make_batches(ctx, iters, rays)
    views = make_views(ctx)
    res = {"iters": iters, "rays_per_iter": rays, "views": len(views)}
    kept = None
    ctx = dict(ctx, compare_iters=iters)
    forms = ("plain", "bf16", "proposal", "skip_pg", "aux", "paper", "paper_bf16") + \
        (("learned_coarse",) if "coarse_learned" in ctx else ())

    def build(form):
        name, bf16, use_prop = FORMS.get(form) or EXTRA_FORMS[form]
        model = new_model(ctx, bf16, skip_pg=form == "skip_pg", aux=form in ("aux", "paper", "paper_bf16"),
                          coarse=ctx["coarse_learned"] if form == "learned_coarse" else None,
                          pe_x=5 if form in ("paper", "paper_bf16") else 0)
        return name, model, new_proposal(ctx) if use_prop else None

    # every form's code path on a throwaway state first, so that no timed run
    # pays for first use (code loading, allocator growth) on another's behalf
    for form in forms:
        _, model, prop = build(form)
        experiment.run(model, batches, min(50, iters), prop=prop, record_every=0)
        del model, prop
    for form in forms:
        name, model, prop = build(form)
        if form == "plain":
            experiment.count_uniform(model, batches)
        st = experiment.run(model, batches, iters, prop=prop, record_every=100)
        entry = {"seconds": st.seconds, "ms_per_step": 1e3 * st.seconds / iters,
                 "ray_samples_per_s": st.samples_per_s, "psnr_db": experiment.psnr_views(model, views),
                 "loss_first_last": [st.losses[0][1], st.losses[-1][1]],
                 "evaluated_per_step_end": experiment.evaluated_per_step(model, batches[-4:], prop),
                 "render_frame_ms": experiment.frame_ms(model, views[0])}
        if prop is not None:
            entry["all_segments_rate_end"] = st.fallback_rate[-1][1]
            entry["prop_loss_first_last"] = [st.prop_losses[0][1], st.prop_losses[-1][1]]
            fresh = new_proposal(ctx)
            entry["gain"] = {
                "evaluated_per_step": {"no_proposal": experiment.evaluated_per_step(model, batches[-4:]),
                                       "untrained": experiment.evaluated_per_step(model, batches[-4:], fresh),
                                       "trained": entry["evaluated_per_step_end"]},
                "render_psnr_vs_plain_sampling_db": {
                    "untrained": experiment.proposal_render_psnr(model, fresh, views[:2]),
                    "trained": experiment.proposal_render_psnr(model, prop, views[:2])}}
        res[name] = entry
        log(f"bench: {name}: {entry['ms_per_step']:.3f} ms/step, psnr {entry['psnr_db']:.3f} dB, "
            f"800x800 frame {entry['render_frame_ms']:.1f} ms")
        if form == keep:
            kept = (model, prop)
        else:
            del model, prop
    res["delta_psnr_db"] = res["bf16_proposal"]["psnr_db"] - res["plain_fp32"]["psnr_db"]
    res["speedup_vs_plain_fp32"] = res["bf16_proposal"]["ray_samples_per_s"] / res["plain_fp32"]["ray_samples_per_s"]
    res["gate_pass"] = bool(res["delta_psnr_db"] >= -0.1 and res["speedup_vs_plain_fp32"] > 1.0)
    sp, b16 = res["bf16_fine_skip_progressive"], res["bf16"]
    res["fine_skip_progressive_vs_bf16"] = {"speedup": sp["ray_samples_per_s"] / b16["ray_samples_per_s"],
                                            "delta_psnr_db": sp["psnr_db"] - b16["psnr_db"]}
    pp, f32 = res["fp32_paper_network_and_objective"], res["plain_fp32"]
    res["paper_network_and_objective_vs_plain_fp32"] = {"ms_per_step_ratio": pp["ms_per_step"] / f32["ms_per_step"],
                                                         "delta_psnr_db": pp["psnr_db"] - f32["psnr_db"]}
    pb = res["bf16_paper_network_and_objective"]
    res["paper_network_and_objective_vs_bf16"] = {"ms_per_step_ratio": pb["ms_per_step"] / res["bf16"]["ms_per_step"],
                                                  "delta_psnr_db": pb["psnr_db"] - res["bf16"]["psnr_db"]}
    ax = res["bf16_auxiliary_losses"]
    res["auxiliary_losses_vs_bf16"] = {"ms_per_step_ratio": ax["ms_per_step"] / b16["ms_per_step"],
                                       "delta_psnr_db": ax["psnr_db"] - b16["psnr_db"]}
    if "bf16_learned_coarse_mask" in res:
        lc = res["bf16_learned_coarse_mask"]
        res["learned_vs_rasterised_coarse_mask"] = {"delta_psnr_db": lc["psnr_db"] - b16["psnr_db"],
                                                    "evaluated_ratio": lc["evaluated_per_step_end"] /
                                                    b16["evaluated_per_step_end"]}
    return res, kept


def host_cpu_model():
    """The host CPU's model name, as the kernel reports it."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ctx, rays, B, reps=1):
    """The oracle as it stands, one thread, on a bounded sample: the plain
    float64 step (sample, forward, loss, adjoint) for ``rays`` rays drawn as
    the first batch is drawn, scaled to the B-ray batch, plus one oracle Adam
    step over every parameter of the configuration; the mean over ``reps``
    such steps."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as O
    import synth

    rng = np.random.default_rng(1000)
    flat = rng.integers(0, len(ctx["cams"]) * 800 * 800, size=B)[:rays]
    o, d, *_ = synth.scenes._rays_for_flat_pixels(ctx["cams"], 800, 800, 1000.0, flat)
    j = rng.random(B).astype(np.float32)[:rays]
    n = ctx["n"]
    tgt = np.zeros((rays, 3))
    Ws, bs = synth.xavier_uniform_mlp(np.random.default_rng(7), (39, 128, 128, 3))
    thr = O.coarse_raw_threshold(synth.FULL_TAU, ctx["step"])
    bits = O.coarse_cell_bits(ctx["raw"], thr)
    dens = np.zeros((n, n, n), np.float32)
    feat = np.zeros((n, n, n, 12), np.float32)
    t_rays = t_adam = 0.0
    with threadpool_limits(limits=1):
        for _ in range(reps):
            t0 = time.perf_counter()
            samp = O.sample_rays(o, d, j, ctx["bmin"], ctx["bmax"], ctx["step"], ctx["max_samples"],
                                 coarse=(bits, ctx["bmin"], ctx["bmax"], ctx["raw"].shape))
            prm = O.Params(dens, feat, Ws, bs, ctx["bmin"], ctx["bmax"], ctx["b"])
            fwd = O.render_forward(prm, o, d, j, samp, ctx["step"], (1.0, 1.0, 1.0))
            _, g = O.photo_loss(fwd["rgb"], tgt)
            gr = O.render_backward(prm, o, d, j, samp, ctx["step"], (1.0, 1.0, 1.0), fwd, g)
            t_rays += (time.perf_counter() - t0) / reps
            t0 = time.perf_counter()
            for p_, g_ in ((dens, gr["density"]), (feat, gr["feat"])):
                O.adam_step(p_, g_, np.zeros(p_.shape), np.zeros(p_.shape), 0.1, 0.9, 0.999, 1e-8, 1)
            for w_, gw in zip(Ws + bs, gr["Ws"] + gr["bs"]):
                O.adam_step(w_, gw, np.zeros(w_.shape), np.zeros(w_.shape), 1e-3, 0.9, 0.999, 1e-8, 1)
            t_adam += (time.perf_counter() - t0) / reps
    scale = B / rays
    per_iter = t_rays * scale + t_adam
    n_uni = float(np.sum(samp["n_uniform"])) * scale
    return {"value": n_uni / per_iter, "unit": "ray-samples/s", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu_model(), "host_cpus_available": len(os.sched_getaffinity(0)),
            "sample": (f"plain float64 step of the first {rays} of the {B} rays of the first batch (sample, "
                       f"forward, loss, adjoint: {t_rays:.2f} s" + (f", scaled x{scale:.0f}" if rays < B else "")
                       + f") + one Adam step over all {dens.size + feat.size + 22019} parameters "
                       f"({t_adam:.2f} s); mean of {reps} steps, {reps * (t_rays + t_adam):.1f} s in all; 1 thread")}


def unique_footprint(ctx, B, gather_ms):
    """The unique-footprint lower bound of the fine pass's gather, counted
    by the oracle (part of the CPU-baseline leg): the distinct grid vertices
    that the samples of the first B-ray batch touch (trilinear corners, plain
    coarse-mask sampler, no proposal), times the bytes a vertex holds for the
    gather (float32 density + 12 bfloat16 features), over the measured
    average gather launch; and the distinct 128-byte lines those vertices
    occupy, the least that a cache can fetch for them."""
    import numpy as np

    import oracle as O
    import synth

    rng = np.random.default_rng(1000)
    flat = rng.integers(0, len(ctx["cams"]) * 800 * 800, size=B)
    o, d, *_ = synth.scenes._rays_for_flat_pixels(ctx["cams"], 800, 800, 1000.0, flat)
    j = rng.random(B).astype(np.float32)
    n = ctx["n"]
    thr = O.coarse_raw_threshold(synth.FULL_TAU, ctx["step"])
    bits = O.coarse_cell_bits(ctx["raw"], thr)
    t0 = time.perf_counter()
    samp = O.sample_rays(o, d, j, ctx["bmin"], ctx["bmax"], ctx["step"], ctx["max_samples"],
                         coarse=(bits, ctx["bmin"], ctx["bmax"], ctx["raw"].shape))
    r = samp["sample_ray"].astype(np.int64)
    x = O.sample_x(o[r], d[r], O.sample_t(samp["t_near"][r], j[r], samp["sample_k"].astype(np.int64), ctx["step"]))
    i0, _, offs = O.trilinear_corners(x, ctx["bmin"], ctx["bmax"], (n, n, n))
    ids = np.concatenate([((i0[:, 0] + dx) * n + (i0[:, 1] + dy)) * n + (i0[:, 2] + dz) for dx, dy, dz in offs])
    uniq = np.unique(ids)
    verts = int(uniq.size)
    # the same vertices at the 128-byte line granularity of the caches: the
    # density array (4 B per vertex) and the bfloat16 feature copy (24 B)
    lines = int(np.unique(uniq * 4 // 128).size + np.unique(uniq * 24 // 128).size)
    secs = time.perf_counter() - t0
    per_vertex = 4 + 12 * 2
    out = {"distinct_vertices": verts, "samples": int(samp["sample_k"].size), "bytes_per_vertex": per_vertex,
           "bytes": verts * per_vertex, "distinct_128B_lines": lines, "line_bytes": lines * 128,
           "sample": (f"first {B}-ray batch, plain coarse-mask sampler (no proposal), trilinear corners "
                      f"counted by the oracle ({secs:.1f} s)")}
    if gather_ms:
        out["gather_GBps_lower_bound"] = verts * per_vertex / (gather_ms * 1e-3) / 1e9
        out["gather_launch_ms"] = gather_ms
    return out


def calibrate_copy(mib):
    """A plain device-to-device copy of known size, to scale the HBM
    traffic counters (FETCH_SIZE, WRITE_SIZE) of a profiled run; also
    prints the copy's own bandwidth (read + write bytes / time)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    print(json.dumps({"copy_mib": mib, "launches": 13, "ms_per_copy": ms,
                      "copy_gb_per_s": 2 * mib * (1 << 20) / (ms * 1e-3) / 1e9}))


TRAFFIC_SOURCES = {"grid_adam": ("paper_2111_11215_amd/csrc/render.hip", "paper_2111_11215_amd/csrc/adam.hpp",
                                 "paper_2111_11215_amd/csrc/common.hpp"),
                   # the fine pass's launch (density and features); the
                   # proposal's density-only pass has no gather launch
                   "gather": ("paper_2111_11215_amd/csrc/render.hip", "paper_2111_11215_amd/csrc/adam.hpp",
                              "paper_2111_11215_amd/csrc/common.hpp"),
                   "mlp_bwd": ("paper_2111_11215_amd/csrc/render.hip", "paper_2111_11215_amd/csrc/mlp_mfma.hpp",
                               "paper_2111_11215_amd/csrc/common.hpp")}


def sources_digest(kname):
    """sha256 over the sources that define the kernel (None if unknown)."""
    import hashlib
    if kname not in TRAFFIC_SOURCES:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[kname]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kname):
    """HBM bytes per launch of the kernel from the committed rocprofv3 --pmc
    summary (FETCH_SIZE scaled by the copy calibration, plus WRITE_SIZE), or
    None when there is none or the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(kname)
    if not rec or rec.get("sources_sha256") != sources_digest(kname):
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


def partial_rows():
    """Per-workgroup rows of the network adjoint's gradient partials: one
    workgroup per compute unit, at most 256."""
    import torch
    return min(torch.cuda.get_device_properties(0).multi_processor_count, 256)


def roofline(per_kernel, kname, n_prof, kept, nv, n_mlp, bf16, n_step=None, rays=0, rows=256):
    """Achieved rate of the named kernel: algorithmic work per launch over
    its event-timed average launch duration.  ``kept`` = evaluated samples
    per step, ``nv`` = grid vertices, ``n_step`` = vertices that take the
    grid Adam step (those with non-zero moments or samples; the others'
    step changes nothing and moves no byte), all of them when None.  Where
    the library launches the network's gradient reduction with the grid
    Adam (no launch of its own) or the preparation with the gather, their
    bytes count with that launch (``rays`` rays per step, ``rows``
    per-workgroup partial rows)."""
    k = per_kernel[kname]
    lps = k["launches"] / n_prof            # launches per step
    if kname in ("mlp_bwd", "mlp_fwd"):
        work = (FLOP_MLP_BWD if kname == "mlp_bwd" else FLOP_MLP_FWD) * kept / lps
        achieved = work / (k["ms_avg"] * 1e-3) / 1e12
        peak = PEAK["bf16" if bf16 else "f32"]
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak}
    else:
        if kname == "grid_adam":
            ns = nv if n_step is None else n_step
            work = BYTES_GRID_ADAM_VERTEX * ns + (2 * 12 * ns if bf16 else 0) + BYTES_REC * kept
            if n_step is not None:
                work += 2 * ((nv + 31) // 32) * 4      # activity mask read and written
            if "reduce" not in per_kernel or per_kernel["reduce"]["launches"] == 0:
                work += (4 * rows + BYTES_REDUCE_PARAM_FIXED) * n_mlp + 4 * rays
        elif kname == "adam":
            work = 32 * n_mlp + ((32 * 13 * nv + (2 * 12 * nv if bf16 else 0)) if "grid_adam" not in per_kernel
                                 or per_kernel["grid_adam"]["launches"] == 0 else 0)
        elif kname == "gather":
            work = (BYTES_GATHER_BF16 if bf16 else BYTES_GATHER_F32) * kept
            if "ray_base" not in per_kernel or per_kernel["ray_base"]["launches"] == 0:
                n1 = round(nv ** (1.0 / 3.0)) - 1
                work += BYTES_PREP_RAY * rays + 4 * (n1 ** 3 + 1) + BYTES_PREP_PACK + 4 * n_mlp
        else:
            work = BYTES_SCATTER * kept
        work /= lps
        achieved = work / (k["ms_avg"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm"], "unit": "GB/s",
                "frac": achieved / PEAK["hbm"]}
    roof["traffic"] = measured_traffic(kname)
    roof["kernel"] = kname
    roof["launch_ms"] = k["ms_avg"]
    roof["launches_per_step"] = lps
    return roof


def active_vertices(model):
    """Vertices whose activity bit is set (they take the fused grid Adam
    step), or None without a mask."""
    import torch
    if getattr(model, "active", None) is None:
        return None
    b = model.active.view(torch.uint8).to(torch.int32)
    return int(sum(((b >> i) & 1).sum().item() for i in range(8)))


def measure_config(ctx, model, batches, warmup, steps, bf16, n_prof=2):
    """Throughput of ``model`` on its own batches (no proposal): uniform
    ray-samples/s, ms/step, evaluated samples, and the event-timed roofline
    of the gather, the network kernels and the fused grid Adam over n_prof
    further steps per kernel."""
    import ctypes

    from paper_2111_11215_amd import _lib, experiment
    lib = _lib.load()
    experiment.count_uniform(model, batches)
    experiment.run(model, batches, warmup, record_every=0)
    st = experiment.run(model, batches, steps, record_every=0, start=warmup)
    timed = batches[warmup:warmup + steps]
    kept = experiment.evaluated_per_step(model, timed, None, n=min(4, len(timed)))
    n_active = active_vertices(model)
    per_kernel = {}
    for kn in ("gather", "mlp_fwd", "mlp_bwd", "grid_adam"):
        _lib.check("dvgo_profile_enable", lib.dvgo_profile_enable(_lib.KERNEL_IDS[kn]))
        experiment.run(model, batches, n_prof, record_every=0, start=warmup)
        tot, cnt = ctypes.c_double(), ctypes.c_int64()
        _lib.check("dvgo_profile_read", lib.dvgo_profile_read(ctypes.byref(tot), ctypes.byref(cnt)))
        if cnt.value:
            per_kernel[kn] = {"ms_total": tot.value, "launches": cnt.value, "ms_avg": tot.value / cnt.value}
    lib.dvgo_profile_enable(-1)
    nv = model.grid.density.numel()
    return {"rays_per_iter": int(batches[0].o.shape[0]), "steps": steps, "warmup": warmup,
            "ms_per_step": 1e3 * st.seconds / steps, "ray_samples_per_s": st.samples_per_s,
            "evaluated_samples_per_step": kept, "grid_vertices_stepped": n_active, "grid_vertices": nv,
            "kernels_roofline": {k: {f: v for f, v in roofline(per_kernel, k, n_prof, kept, nv,
                                                                model.st_mlp.p.numel(), bf16, n_active,
                                                                int(batches[0].o.shape[0]), partial_rows()).items()
                                     if f in ("bound", "achieved", "peak", "unit", "frac", "launch_ms")}
                                 for k in per_kernel}}


def stress_model(ctx):
    """The differentiation-stress shapes as a trained-from-random model:
    256^3 density and bfloat16 feature grids uniform in [-1, 1] (synth's
    stress draw), the shift from alpha_init 1e-2 at that voxel size, step
    half a voxel, at most 800 samples per ray, no coarse mask."""
    import torch

    import synth
    from paper_2111_11215_amd import api, train
    from paper_2111_11215_amd._lib import DVGO_BF16
    P = synth.stress_config(0, n_rays=8)
    dev = torch.device("cuda:0")
    flat = api.flat_from([P.Ws[0], P.bs[0], P.Ws[1], P.bs[1], P.Ws[2], P.bs[2]], api.MLP_SHAPES, dev)
    cfg = train.FineConfig(step=P.step, max_samples=P.max_samples, precision=DVGO_BF16, bf16_feat=True)
    b = api.low_density_bias(P.extra["alpha_init"], P.extra["voxel"])
    return train.FineModel(torch.as_tensor(P.density).to(dev), torch.as_tensor(P.feat).to(dev), flat, ctx["bmin"],
                           ctx["bmax"], b, cfg, coarse=None), P.step


def toy2d_report(iters=2000):
    """The image-fitting toy of Sec. 3: the seeded 256 x 256 binary image
    fitted by Adam (lr 0.1, zero start) at grid strides 2, 4, 8 and 16 with
    each order of activation; PSNR and time per step (forward, loss,
    gradient, Adam)."""
    import torch

    import synth
    from paper_2111_11215_amd import experiment
    T = torch.as_tensor(synth.binary_image(0, 256, 256)).to("cuda:0")
    out = {"image": "256x256 binary (12 discs, 6 triangles, seed 0)", "iters": iters, "lr": 0.1}
    for stride in (2, 4, 8, 16):
        row = {}
        for name, mode in (("pre", 0), ("in", 1), ("post", 2)):
            r = experiment.fit_toy2d(T, stride, mode, iters=iters)
            row[name] = {"psnr_db": r["psnr"], "us_per_step": 1e3 * r["ms_per_step"], "grid": list(r["grid"])}
        out[f"stride_{stride}"] = row
    return out


PROFILED = ("ray_setup", "count_kept", "scan", "fill_kept", "prop_fwd", "prop_bwd", "prop_reduce", "pack",
            "ray_base", "gather", "mlp_fwd", "compose_fwd", "photo_loss", "compose_bwd", "mlp_bwd", "reduce",
            "bin_count", "cell_scan", "bin_place", "scatter", "grid_adam", "adam")
ROOFLINE_MODELS = ("mlp_bwd", "mlp_fwd", "gather", "grid_adam", "adam", "scatter")


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only: the training step is data-parallel over "
                                   "rays but no multi-GPU path is built; run with --gpus 1"}))
        sys.exit(2)
    import ctypes

    import torch

    from paper_2111_11215_amd import _lib, experiment
    lib = _lib.load()
    log("bench: setup")
    ctx = setup(args)
    name, bf16, use_prop = FORMS[args.form]
    out_cmp = None
    coarse_rep = None
    if args.coarse_iters > 0:
        # the paper's alpha_init 1e-6, and 1e-4, whose mask the fine form below trains on: on this scene of
        # low-density spheres 1e-6 leaves a quarter of the occupied cells out of the mask after 5-10k
        # iterations (recall 0.69 / 0.75), 1e-4 keeps 97 % of them
        log(f"bench: coarse stage, {args.coarse_iters} iterations, alpha_init 1e-6 and 1e-4")
        coarse_rep = {"alpha_init_1e-6": coarse_stage(ctx, args.coarse_iters, 1e-6)[0]}
        coarse_rep["alpha_init_1e-4"], ctx["coarse_learned"] = coarse_stage(ctx, args.coarse_iters, 1e-4)
    if args.compare_iters > 0:
        out_cmp, (model, prop) = compare_forms(ctx, args.compare_iters, args.rays, args.form)
        seed0 = 1000 + args.compare_iters
    else:
        model = new_model(ctx, bf16)
        prop = new_proposal(ctx) if use_prop else None
        seed0 = 1000
        if args.pretrain > 0:
            log(f"bench: pretrain {args.pretrain}")
            experiment.run(model, make_batches(ctx, args.pretrain, args.rays, seed0), args.pretrain, prop=prop,
                           record_every=0)
            seed0 += args.pretrain
    n_prof = args.profile_steps
    batches = make_batches(ctx, args.warmup + args.steps, args.rays, seed0)
    experiment.count_uniform(model, batches)
    log(f"bench: warmup {args.warmup}")
    experiment.run(model, batches, args.warmup, prop=prop, record_every=0)
    log(f"bench: timed {args.steps} ({name})")
    st = experiment.run(model, batches, args.steps, prop=prop, record_every=0, start=args.warmup)
    value = st.samples_per_s
    ms = 1e3 * st.seconds / args.steps
    timed = [batches[args.warmup + i] for i in range(args.steps)]
    kept = experiment.evaluated_per_step(model, timed, prop, n=min(8, len(timed)))
    n_active = active_vertices(model)
    log(f"bench: {value:.4e} ray-samples/s, {ms:.3f} ms/step, evaluated {kept:.0f}/step")

    # per-kernel timing: HIP events around each launch of one kernel at a
    # time, recorded on the launch's own stream, over n_prof more steps
    per_kernel = {}
    for kn in PROFILED if n_prof > 0 else ():
        _lib.check("dvgo_profile_enable", lib.dvgo_profile_enable(_lib.KERNEL_IDS[kn]))
        experiment.run(model, batches, n_prof, prop=prop, record_every=0, start=args.warmup)
        tot, cnt = ctypes.c_double(), ctypes.c_int64()
        _lib.check("dvgo_profile_read", lib.dvgo_profile_read(ctypes.byref(tot), ctypes.byref(cnt)))
        if cnt.value:
            per_kernel[kn] = {"ms_total": tot.value, "launches": cnt.value, "ms_avg": tot.value / cnt.value}
    lib.dvgo_profile_enable(-1)
    out = {
        "metric": "fwd+bwd ray-samples/s per train iter",
        "value": value,
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if bf16 else "f32",
        "data": "synthetic",
        "config": {"workload": ("full configuration: 64-sphere synthetic scene, 160^3 fp32 density + 12-ch "
                                "feature grids, 100^3 coarse alpha mask (tau 1e-4), 8192 rays/iter from 100 "
                                "cameras 800x800, step 0.5 voxel, 39-128-128-3 MLP, Adam; form: "
                                + {"plain": "plain float32",
                                   "bf16": "bfloat16 features + bfloat16 MLP",
                                   "proposal": "bfloat16 features + bfloat16 MLP + learned proposal "
                                               "(54-64-64-32, top-99% segments, fallback at mass < 0.9)"}[args.form]
                                + (f", timed after {args.compare_iters} training iterations"
                                   if args.compare_iters > 0 else f", timed after {args.pretrain} iterations")),
                   "form": name, "rays_per_iter": args.rays, "grid": ctx["n"], "coarse": 100,
                   "max_samples": ctx["max_samples"], "morton": bool(args.morton)},
        "evaluated_samples_per_step": kept,
        "grid_vertices_stepped": n_active,
        "grid_vertices": ctx["n"] ** 3,
        "uniform_samples_per_step": st.uniform_samples / args.steps,
        "rays_per_s": args.rays * args.steps / st.seconds,
    }
    if per_kernel:
        kname = args.profile_kernel
        if kname == "auto":
            kname = max((k for k in ROOFLINE_MODELS if k in per_kernel), key=lambda k: per_kernel[k]["ms_total"])
        nv = ctx["n"] ** 3
        out["roofline"] = roofline(per_kernel, kname, n_prof, kept, nv, model.st_mlp.p.numel(), bf16, n_active,
                                   args.rays, partial_rows())
        out["kernels_roofline"] = {
            k: {f: v for f, v in roofline(per_kernel, k, n_prof, kept, nv, model.st_mlp.p.numel(), bf16,
                                          n_active, args.rays, partial_rows()).items()
                if f in ("bound", "achieved", "unit", "frac", "launch_ms", "launches_per_step", "traffic")}
            for k in ROOFLINE_MODELS if k in per_kernel and k != "adam"}
        out["kernels_ms_per_step"] = {k: v["ms_total"] / n_prof for k, v in per_kernel.items()}
    if out_cmp is not None:
        out["proposal_comparison"] = out_cmp
    if coarse_rep is not None:
        out["coarse_stage"] = coarse_rep
    if args.extra_configs:
        # the precision configuration's batch (16384 rays, bfloat16 form, no
        # proposal) on the trained model, and the stress shapes (256^3,
        # 32768 rays, <= 800 samples, no coarse mask)
        log("bench: precision configuration, 16384 rays")
        b16 = make_batches(ctx, 3 + 10, 16384, seed0 + 50000)
        extra = {"precision_16384_rays": measure_config(ctx, model, b16, 3, 10, True)}
        del b16
        log("bench: stress configuration, 256^3, 32768 rays")
        smodel, sstep = stress_model(ctx)
        sctx = dict(ctx, step=sstep)
        b32 = make_batches(sctx, 3 + 10, 32768, seed0 + 60000)
        extra["stress_256_32768_rays"] = measure_config(ctx, smodel, b32, 3, 10, True)
        del smodel, b32
        torch.cuda.empty_cache()
        out["configs"] = extra
    if args.toy:
        log("bench: image-fitting toy")
        out["toy2d"] = toy2d_report()
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(ctx, args.cpu_rays or args.rays, args.rays, args.cpu_reps)
        g = out.get("kernels_roofline", {}).get("gather", {})
        out["unique_footprint"] = unique_footprint(ctx, args.rays, g.get("launch_ms"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
