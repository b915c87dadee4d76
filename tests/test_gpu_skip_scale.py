"""GPU parity of the second free-space rule (the fine-density alpha skip in
the sampler: sample lists bit-exact against the oracle's float32 recipe)
and of progressive scaling (grid resize by trilinear interpolation against
the oracle), plus a training run that scales at its checkpoints.

The resize bound: the destination positions are float32 (min + j*step),
so a fraction moves by up to 4 u n (u = 2^-24, n vertices per axis) and a
value by that times its source cell's spread; the arithmetic adds 8
products: |err| <= 16 u max|V| + 4 u n spread."""

import numpy as np
import pytest

import oracle as O
import synth
from tests.helpers import np_of, to_dev
from tests.test_gpu_sampler import _check_samples

pytestmark = pytest.mark.gpu
F32 = np.float32


@pytest.mark.parametrize("morton,coarse,seg", [(False, False, False), (True, False, False), (False, True, True)])
def test_fine_skip_sample_lists_bit_exact(gpu_lib, morton, coarse, seg):
    from paper_2111_11215_amd import api
    P = synth.tiny_config(3, jitter=True, n_rays=2048)
    rng = np.random.default_rng(1)
    P.density = (rng.normal(size=P.density.shape) * 3 - 1).astype(F32)
    thr = api.coarse_raw_threshold(1e-2, P.step, 0.3)
    assert thr == float(O.coarse_raw_threshold(1e-2, P.step, 0.3))
    cg, cr = None, None
    if coarse:
        raw = rng.normal(-2, 3, (9, 9, 9)).astype(F32)
        cthr = O.coarse_raw_threshold(1e-3, P.step)
        cg = (api.coarse_mask_build(to_dev(raw), P.box_min, P.box_max, float(cthr)), P.box_min, P.box_max, raw.shape)
        cr = (O.coarse_cell_bits(raw, cthr), P.box_min, P.box_max, raw.shape)
    sm = rng.integers(0, 2 ** 32, 2048, dtype=np.uint64).astype(np.uint32) if seg else None
    s = api.sample_rays(to_dev(P.rays.o), to_dev(P.rays.d), to_dev(P.rays.jitter), P.box_min, P.box_max, P.step,
                        P.max_samples, coarse=cg, seg_mask=to_dev(sm.view(np.int32)) if seg else None, morton=morton,
                        fine=(to_dev(P.density), thr))
    ref = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples, coarse=cr,
                        seg_mask=sm, morton=morton, fine=(P.density, np.float32(thr)))
    plain = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples, coarse=cr,
                          seg_mask=sm, morton=morton)
    print(f"  kept {int(ref['ray_offset'][-1])} of {int(plain['ray_offset'][-1])}", flush=True)
    _check_samples(s, ref, 2048)


@pytest.mark.timeout(300)
def test_fine_skip_full_configuration(gpu_lib):
    """The full configuration's 8192-ray batch with the coarse mask and the
    fine rule on a 160^3 density rasterised from the scene (tau 1e-4)."""
    from paper_2111_11215_amd import api
    P = synth.full_config(0)
    P.density = synth.coarse_raw_from_spheres(P.extra["spheres"], P.density.shape[0]) - 4.0
    P.density = P.density.astype(F32)
    raw = P.coarse_raw
    cthr = api.coarse_raw_threshold(synth.FULL_TAU, P.step)
    bits = api.coarse_mask_build(to_dev(raw), P.box_min, P.box_max, cthr)
    thr = api.coarse_raw_threshold(1e-4, P.step, 0.2)
    s = api.sample_rays(to_dev(P.rays.o), to_dev(P.rays.d), to_dev(P.rays.jitter), P.box_min, P.box_max, P.step,
                        P.max_samples, coarse=(bits, P.box_min, P.box_max, raw.shape), fine=(to_dev(P.density), thr))
    cr = (O.coarse_cell_bits(raw, O.coarse_raw_threshold(synth.FULL_TAU, P.step)), P.box_min, P.box_max, raw.shape)
    ref = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples, coarse=cr,
                        fine=(P.density, np.float32(thr)))
    _check_samples(s, ref, 8192)


@pytest.mark.parametrize("n_src,n_dst,C", [((80, 80, 80), (101, 101, 101), 1), ((9, 7, 12), (17, 5, 23), 12),
                                           ((100, 100, 100), (126, 126, 126), 12), ((33, 33, 33), (16, 16, 16), 1)])
def test_grid_resample_parity(gpu_lib, n_src, n_dst, C):
    from paper_2111_11215_amd import api
    rng = np.random.default_rng(sum(n_src) + C)
    shape = n_src if C == 1 else n_src + (C,)
    V = rng.uniform(-3, 3, shape).astype(F32)
    got = np_of(api.grid_resample(to_dev(V), n_dst, synth.BOX_MIN, synth.BOX_MAX))
    ref = O.grid_resample(V, n_dst, synth.BOX_MIN, synth.BOX_MAX)
    u = 2.0 ** -24
    err = np.abs(got - ref)
    bound = 16 * u * np.abs(V).max() + 4 * u * max(n_dst) * 6.0
    print(f"  max err {err.max():.2e} (bound {bound:.2e}), normwise "
          f"{np.linalg.norm(got - ref) / np.linalg.norm(ref):.2e}", flush=True)
    assert np.all(err <= bound)


@pytest.mark.timeout(300)
def test_training_with_skip_and_progressive_scaling(gpu_lib):
    """200 iterations of the full configuration (bf16 form) with the fine
    rule (tau 1e-4) and checkpoints at 40, 80 and 120: the grids grow
    80 -> 100 -> 126 -> 160 vertices per axis at those iterations and the
    loss falls.  With alpha_init 1e-2 above tau^(f) the rule keeps every
    sample at first and sculpts free space only as the density falls there;
    at the end it keeps no more than the coarse mask does, and a stricter
    threshold (1e-2) on the trained grid skips samples."""
    import torch
    from paper_2111_11215_amd import api, train
    from paper_2111_11215_amd._lib import DVGO_BF16
    P = synth.full_config(0, n_rays=8)
    sp = P.extra["spheres"]
    dev = torch.device("cuda:0")
    n0 = api.pg_resolution(160, 3, 0)
    step0 = 0.5 * 2.0 / (n0 - 1)
    cams = P.extra["cams"]
    raw = P.coarse_raw
    bits = api.coarse_mask_build(to_dev(raw), P.box_min, P.box_max, api.coarse_raw_threshold(synth.FULL_TAU, P.step))
    Ws, bs = synth.xavier_uniform_mlp(np.random.default_rng(7), (39, 128, 128, 3))
    flat = api.flat_from([Ws[0], bs[0], Ws[1], bs[1], Ws[2], bs[2]], api.MLP_SHAPES, dev)
    cfg = train.FineConfig(step=step0, max_samples=int(np.ceil(2 * np.sqrt(3) / step0)) + 1, precision=DVGO_BF16,
                           bf16_feat=True, fine_tau=1e-4, pg_ckpt=(40, 80, 120), pg_final_n=160)
    b = api.low_density_bias(synth.FULL_ALPHA_INIT, 2.0 / 159)
    model = train.FineModel(torch.zeros((n0,) * 3, device=dev), torch.zeros((n0,) * 3 + (12,), device=dev), flat,
                            P.box_min, P.box_max, b, cfg, coarse=(bits, P.box_min, P.box_max, raw.shape))
    spheres = to_dev(sp.as_f32_table())
    sizes, losses, kept = [], [], []
    for it in range(200):
        rng = np.random.default_rng(5000 + it)
        o, d, *_ = synth.draw_pixels_with_replacement(rng, cams, 800, 800, 1000.0, 8192)
        j = rng.random(8192).astype(F32)
        ot, dt = to_dev(o), to_dev(d)
        tgt = api.scene_render(ot, dt, spheres, P.box_min, P.box_max, 0.5 * 2.0 / 159 / 4)
        res = model.train_step(ot, dt, tgt, to_dev(j))
        sizes.append(model.grid.density.shape[0])
        if it % 20 == 0 or it == 199:
            losses.append(float(res["loss"].item()))
            kept.append(int(res["samples"].n_kept.item()))
    assert sizes[39] == 80 and sizes[40] == 100 and sizes[80] == 126 and sizes[120] == 160 and sizes[-1] == 160
    print(f"  losses {losses[0]:.4f} -> {losses[-1]:.4f}, kept samples {kept[0]} -> {kept[-1]}", flush=True)
    assert losses[-1] < 0.5 * losses[0]
    assert torch.isfinite(model.grid.density).all() and torch.isfinite(model.grid.feat).all()
    # the rule at the end of training: fewer samples than the coarse mask alone keeps
    s_fine = model.sample(ot, dt, to_dev(j))
    fine_thr, model.fine_thr = model.fine_thr, None
    s_plain = model.sample(ot, dt, to_dev(j))
    model.fine_thr = api.coarse_raw_threshold(1e-2, model.cfg.step, b)
    s_strict = model.sample(ot, dt, to_dev(j))
    model.fine_thr = fine_thr
    n_f, n_p, n_s = (int(x.n_kept.item()) for x in (s_fine, s_plain, s_strict))
    print(f"  last batch: {n_f} kept with the rule, {n_p} without, {n_s} at tau 1e-2", flush=True)
    assert n_f <= n_p and n_s < n_p
