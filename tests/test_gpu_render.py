"""GPU parity of forward rendering and its adjoint against the FP64 oracle.

Every output tensor is held to both metrics of R23: the normwise relative
error ||gpu - ref||_2 / ||ref||_2 and max|gpu - ref| / max|ref|.

float32 form: both <= 1e-5 for rgb, depth, acc, log T, segment and sample
weights and the density gradient; where rays reach max_samples terms the
max metric takes the rounding bound of such sums, max_samples x 2^-24
(3.3e-5 at the full configuration's 552).  The feature and network
gradients pass through ReLU derivatives: a hidden unit whose pre-activation
lies within the float32 error bound of zero (|z| <= 1e-4 x the sum of the
absolute terms of its dot product) may take either branch, so entries and
tensors reached by such samples are checked against a proven error budget
(tests/helpers.kink_budget) and every other entry at the bounds above.

bfloat16 form, against the oracle's bfloat16 form (the fixed contract:
the same operands rounded to bfloat16, exact arithmetic otherwise).  The
library rounds float32 values that carry float32 accumulation error, at
most K x 2^-24 relative for K = 128 terms; an operand rounds to the
neighbouring bfloat16 value only when that error straddles a rounding
boundary, which happens to a fraction p <= K 2^-24 / 2^-8 = 2e-3 of the
operands, and moves its term by one bfloat16 step, 2^-8.  Such events are
independent, so the normwise error is about 2^-8 sqrt(p) = 1.7e-4; the bound
is three times that, 5e-4.  The max metric takes the single-event bound,
ZETA_BF16 = 4e-3 (2^-8 rounded up), which is also the kink budget's margin.
The form's own approximation error against the exact network is reported
and held to 2e-3 for rgb, depth and opacity.  Actual errors are printed."""

import numpy as np
import pytest

import oracle as O
import synth
from tests.helpers import (assert_close, check_grid_grad, check_weight_grads, kink_budget, mlp_flat_np, np_of,
                           report, to_dev)

pytestmark = pytest.mark.gpu
F32 = np.float32
TOL32 = 1e-5
TOLBF = 5e-4       # 3 x 2^-8 sqrt(128 2^-24 / 2^-8): bf16 operands near a rounding boundary (docstring)
ZETA = 1e-4        # float32: |z| within 1e-4 of its term sum may flip a ReLU
ZETA_BF16 = 4e-3   # bfloat16: one operand may round to the neighbouring bf16 value (2^-8 of a term)


def _problem(seed=0, jitter=True, n_rays=4096, bias=0.0):
    P = synth.tiny_config(seed, jitter=jitter, n_rays=n_rays)
    P.act_shift = bias
    rng = np.random.default_rng(seed + 100)
    P.bs = [(rng.normal(size=b.shape) * 0.1).astype(F32) for b in P.bs]
    return P


def _gpu(P, coarse=None, morton=True, bf16=False):
    import torch
    from paper_2111_11215_amd import api
    grid = api.Grid(to_dev(P.density), to_dev(P.feat), tuple(P.box_min), tuple(P.box_max), P.act_shift)
    if bf16:
        grid.feat_shadow = grid.feat.to(torch.bfloat16).view(torch.int16).contiguous()
    flat = to_dev(mlp_flat_np(P.Ws, P.bs))
    s = api.sample_rays(to_dev(P.rays.o), to_dev(P.rays.d),
                        to_dev(P.rays.jitter) if P.rays.jitter is not None else None, P.box_min, P.box_max,
                        P.step, P.max_samples, coarse=coarse, morton=morton)
    return grid, flat, s


def _oracle(P, morton=True, coarse=None, bf16=False, rays=None):
    """Oracle forward on the problem's rays (or the subset ``rays``); the
    network's input width (39 or 72) selects the encoded-position variant."""
    o, d, j = P.rays.o, P.rays.d, P.rays.jitter
    if rays is not None:
        o, d, j = o[rays], d[rays], (j[rays] if j is not None else None)
    samp = O.sample_rays(o, d, j, P.box_min, P.box_max, P.step, P.max_samples, coarse=coarse, morton=morton)
    feat = O.bf16_round(P.feat) if bf16 else P.feat
    prm = O.Params(P.density, feat, P.Ws, P.bs, P.box_min, P.box_max, P.act_shift, mlp_bf16=bf16,
                   pe_x=5 if P.Ws[0].shape[1] == 72 else 0)
    ref = O.render_forward(prm, o, d, j, samp, P.step, P.bg)
    return samp, prm, ref, (o, d, j)


def _with_position_encoding(P, seed):
    """The paper's colour network that also takes PE_5 of the query position:
    72 inputs [features, PE_5(u), PE_4(d)], Xavier weights from the seed."""
    Ws, _ = synth.xavier_uniform_mlp(np.random.default_rng(seed), (72, 128, 128, 3))
    P.Ws = [w.astype(F32) for w in Ws]
    return P


def _grads(api, grid, flat, s, out, g, P, bf16=False, gD=None, gA=None):
    import torch
    from paper_2111_11215_amd._lib import DVGO_BF16, DVGO_F32
    gd = torch.zeros_like(grid.density)
    gf = torch.zeros_like(grid.feat)
    gm = torch.zeros_like(flat)
    api.render_bwd(grid, flat, s, out["log_t_end"], to_dev(np.asarray(g, F32)), gd, gf, gm, P.bg,
                   precision=DVGO_BF16 if bf16 else DVGO_F32, use_shadow=bf16,
                   grad_depth=None if gD is None else to_dev(np.asarray(gD, F32)),
                   grad_acc=None if gA is None else to_dev(np.asarray(gA, F32)))
    return np_of(gd), np_of(gf), np_of(gm)


def _check_backward(P, prm, ref, ro, gd, gf, gm, g_oracle, tol, gD=None, gA=None, tol_max=None):
    o, d, j = ro
    tol_max = _tol_max(prm.mlp_bf16, tol) if tol_max is None else tol_max
    gr = O.render_backward(prm, o, d, j, ref["_samp"], P.step, P.bg, ref, g_oracle, gD, gA)
    assert_close("grad_density", gd, gr["density"], tol, tol_max)
    zeta = ZETA_BF16 if prm.mlp_bf16 else ZETA
    budget, wb, frac = kink_budget(prm, ref, g_oracle, zeta, P.feat.shape, P.box_min, P.box_max)
    print(f"  samples with an ambiguous ReLU unit: {frac:.2e}", flush=True)
    check_grid_grad("grad_feat", gf, gr["feat"], budget, tol, tol_max)
    check_weight_grads(gm, gr["Ws"], gr["bs"], wb, tol, tol_max)


def _tol_max(bf16, tol):
    """R23's second metric, max|gpu - ref| / max|ref|: the float32 bound
    itself; for the bfloat16 form ZETA_BF16, since one operand that rounds
    to the neighbouring bfloat16 value moves its product term by 2^-8 of
    itself (the normwise bound averages such events, the max does not)."""
    return ZETA_BF16 if bf16 else tol


def _fwd_keys(out, ref, keys, tol, sel=None, tol_max=None):
    for key in keys:
        got = np_of(out[key]) if sel is None else np_of(out[key])[sel]
        assert_close(key, got, ref[key], tol, tol if tol_max is None else tol_max)


@pytest.mark.parametrize("jitter", [True, False])
@pytest.mark.parametrize("bf16", [False, True])
def test_render_forward_parity_tiny(gpu_lib, bf16, jitter):
    """Forward of the tiny configuration; jitter False is the test-time
    path (p = 0, the sampler and the forward read no jitter at all)."""
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_BF16, DVGO_F32
    P = _problem(0, jitter=jitter, bias=0.4)
    grid, flat, s = _gpu(P, bf16=bf16)
    out = api.render_fwd(grid, flat, s, P.bg, precision=DVGO_BF16 if bf16 else DVGO_F32, use_shadow=bf16,
                         want_seg_w=True, want_sample_w=True)
    samp, prm, ref, _ = _oracle(P, bf16=bf16)
    n = int(samp["ray_offset"][-1])
    print(f"  rays {P.rays.o.shape[0]} samples {n}", flush=True)
    tol = TOLBF if bf16 else TOL32
    _fwd_keys(out, ref, ("rgb", "depth", "acc", "log_t_end", "seg_w"), tol, tol_max=_tol_max(bf16, tol))
    assert_close("sample_w", np_of(out["sample_w"])[:n], ref["sample_w"], tol, _tol_max(bf16, tol))
    if bf16:
        _, _, exact, _ = _oracle(P, bf16=False)
        print("  bf16 form vs exact network:", flush=True)
        _fwd_keys(out, exact, ("rgb", "depth", "acc"), 2e-3)


@pytest.mark.parametrize("jitter", [True, False])
@pytest.mark.parametrize("bf16", [False, True])
def test_render_backward_parity_tiny(gpu_lib, bf16, jitter):
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_BF16, DVGO_F32
    P = _problem(1, jitter=jitter, bias=-0.3)
    grid, flat, s = _gpu(P, bf16=bf16)
    out = api.render_fwd(grid, flat, s, P.bg, precision=DVGO_BF16 if bf16 else DVGO_F32, use_shadow=bf16)
    samp, prm, ref, ro = _oracle(P, bf16=bf16)
    ref["_samp"] = samp
    _, g = O.photo_loss(ref["rgb"], P.rays.target)
    gd, gf, gm = _grads(api, grid, flat, s, out, g, P, bf16)
    _check_backward(P, prm, ref, ro, gd, gf, gm, g, TOLBF if bf16 else TOL32)


@pytest.mark.parametrize("jitter", [True, False])
@pytest.mark.parametrize("bf16", [False, True])
def test_render_position_encoding_parity_tiny(gpu_lib, bf16, jitter):
    """The network with the encoded query position (Eq. fine_queries with
    k_x = 5): forward outputs and every gradient of the tiny configuration
    against the oracle at the bounds of each form (the bfloat16 form rounds
    the per-sample inputs [f, PE_5(u)] as it rounds f alone)."""
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_BF16, DVGO_F32
    P = _with_position_encoding(_problem(2, jitter=jitter, bias=0.2), 61)
    grid, flat, s = _gpu(P, bf16=bf16)
    assert flat.numel() == 26243
    out = api.render_fwd(grid, flat, s, P.bg, precision=DVGO_BF16 if bf16 else DVGO_F32, use_shadow=bf16,
                         want_seg_w=True, want_sample_w=True)
    samp, prm, ref, ro = _oracle(P, bf16=bf16)
    assert prm.pe_x == 5
    n = int(samp["ray_offset"][-1])
    tol = TOLBF if bf16 else TOL32
    _fwd_keys(out, ref, ("rgb", "depth", "acc", "log_t_end", "seg_w"), tol, tol_max=_tol_max(bf16, tol))
    assert_close("sample_w", np_of(out["sample_w"])[:n], ref["sample_w"], tol, _tol_max(bf16, tol))
    ref["_samp"] = samp
    _, g = O.photo_loss(ref["rgb"], P.rays.target)
    gd, gf, gm = _grads(api, grid, flat, s, out, g, P, bf16)
    _check_backward(P, prm, ref, ro, gd, gf, gm, g, tol)


def test_render_backward_depth_acc_channels(gpu_lib):
    from paper_2111_11215_amd import api
    P = _problem(2, n_rays=1024)
    grid, flat, s = _gpu(P, morton=False)
    out = api.render_fwd(grid, flat, s, P.bg)
    samp, prm, ref, ro = _oracle(P, morton=False)
    ref["_samp"] = samp
    rng = np.random.default_rng(3)
    gR, gD, gA = rng.normal(size=(1024, 3)), rng.normal(size=1024), rng.normal(size=1024)
    gd, gf, gm = _grads(api, grid, flat, s, out, gR, P, gD=gD, gA=gA)
    _check_backward(P, prm, ref, ro, gd, gf, gm, gR, TOL32, gD, gA)


def test_render_density_only_mode(gpu_lib):
    """No network: weights, depth, opacity, log T and segment sums only (the
    proposal's target pass)."""
    from paper_2111_11215_amd import api
    P = _problem(3, n_rays=2048)
    grid, flat, s = _gpu(P)
    out = api.render_fwd(grid, None, s, P.bg, want_seg_w=True)
    samp = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples,
                         morton=True)
    prm = O.Params(P.density, P.feat, P.Ws, P.bs, P.box_min, P.box_max, P.act_shift)
    ref = O.render_forward(prm, P.rays.o, P.rays.d, P.rays.jitter, samp, P.step, P.bg, with_color=False)
    _fwd_keys(out, ref, ("depth", "acc", "log_t_end", "seg_w"), TOL32)


def test_render_with_coarse_mask_and_large_values(gpu_lib):
    """Coarse skipping on, large raw densities (alpha near 1, tiny T) and a
    shift: forward and backward still at float32 tolerance."""
    from paper_2111_11215_amd import api
    P = _problem(4, n_rays=2048, bias=1.5)
    P.density = (P.density * 6).astype(F32)
    raw = np.random.default_rng(8).normal(-5, 3, (11, 11, 11)).astype(F32)
    thr = O.coarse_raw_threshold(1e-3, P.step)
    bits_ref = O.coarse_cell_bits(raw, thr)
    bits = api.coarse_mask_build(to_dev(raw), P.box_min, P.box_max, float(thr))
    grid, flat, s = _gpu(P, coarse=(bits, P.box_min, P.box_max, raw.shape))
    out = api.render_fwd(grid, flat, s, P.bg)
    samp, prm, ref, ro = _oracle(P, coarse=(bits_ref, P.box_min, P.box_max, raw.shape))
    ref["_samp"] = samp
    _fwd_keys(out, ref, ("rgb", "depth", "acc"), TOL32)
    _, g = O.photo_loss(ref["rgb"], P.rays.target)
    gd, gf, gm = _grads(api, grid, flat, s, out, g, P)
    _check_backward(P, prm, ref, ro, gd, gf, gm, g, TOL32)


def test_render_opaque_samples(gpu_lib):
    """Samples with sigma*delta from 100 to 150 (alpha = 1 in float32,
    T behind them below the float32 range): the adjoint forms each weight
    from the transmittance in front of the sample, so it stays finite, and
    forward and backward stay at float32 tolerance."""
    from paper_2111_11215_amd import api
    P = _problem(6, n_rays=2048, bias=0.0)
    rng = np.random.default_rng(9)
    hot = np.zeros(P.density.shape, bool)   # whole cells hot: every point inside reaches sd >= 100
    for i, j, k in rng.integers(0, P.density.shape[0] - 1, (40, 3)):
        hot[i:i + 2, j:j + 2, k:k + 2] = True
    sd_max = 150.0
    P.density = np.where(hot, rng.uniform(100.0, sd_max, P.density.shape) / P.step, P.density).astype(F32)
    # float32 interpolation of corners as large as sd_max/step moves a
    # sample's sigma*delta by up to about 10 u sd_max (u = 2^-24), and with it
    # the transmittance behind the sample by that much relative
    tol = max(TOL32, 10 * 2.0 ** -24 * sd_max)
    grid, flat, s = _gpu(P)
    out = api.render_fwd(grid, flat, s, P.bg)
    samp, prm, ref, ro = _oracle(P)
    ref["_samp"] = samp
    sd = O.softplus(ref["cache"]["raw"]) * P.step
    print(f"  samples with sigma*delta >= 100: {int((sd >= 100).sum())}", flush=True)
    assert (sd >= 100).sum() > 100
    _fwd_keys(out, ref, ("rgb", "depth", "acc"), tol)
    _, g = O.photo_loss(ref["rgb"], P.rays.target)
    gd, gf, gm = _grads(api, grid, flat, s, out, g, P)
    assert np.isfinite(gd).all() and np.isfinite(gf).all() and np.isfinite(gm).all()
    _check_backward(P, prm, ref, ro, gd, gf, gm, g, tol)


@pytest.mark.parametrize("bf16,pe_x", [(False, 0), (True, 0), (False, 5), (True, 5)])
def test_render_full_size_sampled_rays(gpu_lib, bf16, pe_x):
    """Full configuration (160^3 grids with random values, 8192 rays, coarse
    mask of the sphere scene, launch configuration of the benchmark): the
    outputs of 256 sampled rays against the oracle on those rays, and the
    gradients with the loss gradient restricted to those rays, which the
    oracle then computes exactly.  pe_x = 5: the network with the encoded
    query position."""
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_BF16, DVGO_F32
    P = synth.full_config(0)
    rng = np.random.default_rng(1)
    P.density = rng.uniform(-1, 1, P.density.shape).astype(F32)
    P.feat = rng.uniform(-1, 1, P.feat.shape).astype(F32)
    P.act_shift = O.low_density_bias(synth.FULL_ALPHA_INIT, 2.0 / 159)
    if pe_x:
        P = _with_position_encoding(P, 62)
    raw = P.coarse_raw
    thr = O.coarse_raw_threshold(synth.FULL_TAU, P.step)
    bits = api.coarse_mask_build(to_dev(raw), P.box_min, P.box_max, float(thr))
    bits_ref = O.coarse_cell_bits(raw, thr)
    grid, flat, s = _gpu(P, coarse=(bits, P.box_min, P.box_max, raw.shape), bf16=bf16)
    prec = DVGO_BF16 if bf16 else DVGO_F32
    out = api.render_fwd(grid, flat, s, P.bg, precision=prec, use_shadow=bf16)
    B = P.rays.o.shape[0]
    sel = rng.choice(B, 256, replace=False)
    samp, prm, ref, ro = _oracle(P, coarse=(bits_ref, P.box_min, P.box_max, raw.shape), bf16=bf16, rays=sel,
                                 morton=False)
    ref["_samp"] = samp
    tol = TOLBF if bf16 else TOL32
    # max metric of the float32 form: the rounding bound of sums along rays
    # of up to max_samples terms (n u), as for the stress shape
    tol_max = ZETA_BF16 if bf16 else max(TOL32, P.max_samples * 2.0 ** -24)
    _fwd_keys(out, ref, ("rgb", "depth", "acc", "log_t_end"), tol, sel=sel, tol_max=tol_max)
    g_sub = rng.normal(size=(256, 3)) * 1e-3
    g = np.zeros((B, 3))
    g[sel] = g_sub
    gd, gf, gm = _grads(api, grid, flat, s, out, g, P, bf16)
    _check_backward(P, prm, ref, ro, gd, gf, gm, g_sub, tol, tol_max=tol_max)


def test_photo_loss_parity(gpu_lib):
    from paper_2111_11215_amd import api
    rng = np.random.default_rng(0)
    c, t = rng.random((8192, 3)).astype(F32), rng.random((8192, 3)).astype(F32)
    loss, grad = api.photo_loss(to_dev(c), to_dev(t))
    L, g = O.photo_loss(c, t)
    assert abs(float(np_of(loss)[0]) - L) <= 1e-5 * L
    assert_close("grad", np_of(grad), g, 1e-6)
