"""Test-time rendering of whole images (dvgo_render_image: rays cast on the
GPU, the plain sampler without jitter, the forward) against the oracle on
the same rays: a small view in several chunks with a ragged last one, both
forms, and one 800 x 800 view in the benchmark's chunking checked on 512
sampled pixels.  The cast rays match the input generator's (float64
geometry rounded to float32) to a few units in the last place.

Bounds as tests/test_gpu_render.py: float32 1e-5 normwise and the long-ray
bound max_samples x 2^-24 for the max metric; bfloat16 against the oracle's
bfloat16 form 5e-4 normwise and 4e-3 max."""

import numpy as np
import pytest

import oracle as O
import synth
from tests.helpers import assert_close, mlp_flat_np, np_of, to_dev

pytestmark = pytest.mark.gpu
F32 = np.float32


def _model(bf16):
    import torch
    from paper_2111_11215_amd import api
    P = synth.full_config(0, n_rays=16)
    rng = np.random.default_rng(5)
    P.density = synth.coarse_raw_from_spheres(P.extra["spheres"], P.density.shape[0])
    P.feat = rng.uniform(-1, 1, P.feat.shape).astype(F32)
    P.bs = [(rng.normal(size=b.shape) * 0.1).astype(F32) for b in P.bs]
    raw = P.coarse_raw
    thr = api.coarse_raw_threshold(synth.FULL_TAU, P.step)
    bits = api.coarse_mask_build(to_dev(raw), P.box_min, P.box_max, thr)
    grid = api.Grid(to_dev(P.density), to_dev(P.feat), tuple(P.box_min), tuple(P.box_max), 0.0)
    if bf16:
        grid.feat_shadow = grid.feat.to(torch.bfloat16).view(torch.int16).contiguous()
    bits_ref = O.coarse_cell_bits(raw, O.coarse_raw_threshold(synth.FULL_TAU, P.step))
    return P, grid, to_dev(mlp_flat_np(P.Ws, P.bs)), (bits, P.box_min, P.box_max, raw.shape), \
        (bits_ref, P.box_min, P.box_max, raw.shape)


def _check(P, out, ref_rows, o, d, coarse_ref, bf16):
    samp = O.sample_rays(o, d, None, P.box_min, P.box_max, P.step, P.max_samples, coarse=coarse_ref)
    feat = O.bf16_round(P.feat) if bf16 else P.feat
    prm = O.Params(P.density, feat, P.Ws, P.bs, P.box_min, P.box_max, 0.0, mlp_bf16=bf16)
    ref = O.render_forward(prm, o, d, None, samp, P.step, P.bg)
    tol = 5e-4 if bf16 else 1e-5
    tol_max = 4e-3 if bf16 else max(1e-5, P.max_samples * 2.0 ** -24)
    for k in ("rgb", "depth", "acc"):
        assert_close(k, np_of(out[k])[ref_rows], ref[k], tol, tol_max)


def _cam(P, idx):
    c = P.extra["held"][idx]
    return synth.look_at_c2w(c), c


@pytest.mark.parametrize("bf16", [False, True])
def test_render_image_small_view_in_chunks(gpu_lib, bf16):
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_BF16, DVGO_F32
    P, grid, flat, coarse, coarse_ref = _model(bf16)
    R, c = _cam(P, 3)
    H, W, focal = 96, 128, 1000.0 * 128 / 800
    out = api.render_image(grid, flat, R, c, H, W, focal, P.step, P.max_samples, coarse=coarse, bg=P.bg,
                           precision=DVGO_BF16 if bf16 else DVGO_F32, use_shadow=bf16, chunk=5000, want_rays=True)
    o_syn, d_syn = synth.image_rays(c, H, W, focal)
    o, d = np_of(out["rays_o"]), np_of(out["rays_d"])
    assert np.array_equal(o, o_syn)
    ulp = np.spacing(np.abs(d_syn)).max(axis=1, keepdims=True)
    assert np.all(np.abs(d - d_syn) <= 4 * ulp), "cast rays"
    print(f"  {H}x{W} in chunks of 5000, rays within {np.max(np.abs(d - d_syn) / ulp):.1f} ulp", flush=True)
    _check(P, out, np.arange(H * W), o, d, coarse_ref, bf16)


@pytest.mark.timeout(300)
def test_render_image_full_view_sampled_pixels(gpu_lib):
    """One 800 x 800 held-out view in chunks of 65536 (the benchmark's frame
    timing), 512 sampled pixels against the oracle on the cast rays."""
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_BF16
    P, grid, flat, coarse, coarse_ref = _model(True)
    R, c = _cam(P, 0)
    out = api.render_image(grid, flat, R, c, 800, 800, 1000.0, P.step, P.max_samples, coarse=coarse, bg=P.bg,
                           precision=DVGO_BF16, use_shadow=True, chunk=1 << 16, want_rays=True)
    sel = np.random.default_rng(0).choice(800 * 800, 512, replace=False)
    o, d = np_of(out["rays_o"])[sel], np_of(out["rays_d"])[sel]
    assert np.all(np.isfinite(np_of(out["rgb"])))
    _check(P, out, sel, o, d, coarse_ref, True)
