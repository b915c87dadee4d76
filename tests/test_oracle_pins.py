"""Pins of the FP64 oracle against things other than itself: the paper's
printed worked examples, closed forms, library routines, autograd, finite
differences and brute force.  CPU only."""

import math
import os

import numpy as np
import pytest
import torch

import oracle as O
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
F32 = np.float32


def _rows(name):
    out = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append([float(v) for v in line.split()])
    return np.array(out)


# ---------------------------------------------------------------------------
# post-activation: worked numbers printed in the supplementary derivation
# ---------------------------------------------------------------------------
def _post_alpha_1d(a, b, x, delta):
    """Post-activated alpha along a 1D cell, through the oracle's own
    trilinear interpolation, softplus and alpha (no shift)."""
    grid = np.zeros((2, 2, 2))
    grid[0], grid[1] = a, b
    pts = np.stack([np.asarray(x, float) * 2 - 1, np.zeros_like(x), np.zeros_like(x)], axis=-1)
    raw = O.interp(grid, pts, [-1, -1, -1], [1, 1, 1])
    return O.post_activated_alpha(raw, 0.0, delta)


@pytest.mark.parametrize("fixture", ["post_activation_1d.txt", "post_activation_1d_extrapolation.txt"])
def test_cell_fit_1d_reproduces_printed_table(fixture):
    for c, a_p, b_p in _rows(fixture):
        a, b = O.cell_fit_1d(c, 0.5, 1e-4, 1e-2)
        assert abs(a - a_p) <= 0.05 + 1e-9 and abs(b - b_p) <= 0.05 + 1e-9, (c, a, b)


def test_cell_fit_2d_reproduces_printed_tables():
    for sl, off, D, tl, tr, bl, br in _rows("post_activation_2d.txt"):
        got = O.cell_fit_2d(off, off + sl, 0.5, 1e-4, D)
        assert np.allclose(got, [tl, tr, bl, br], atol=0.05 + 1e-9), (sl, off, D, got)


@pytest.mark.parametrize("c", [0.1, 0.5, 0.7])
def test_post_activation_fits_step_within_eps(c):
    """With the derived cell values, the oracle's interp->softplus->alpha
    meets the derivation's three conditions: S(c) = 1/2, 1 - S(c+D) = eps
    (the binding bound for delta < 1) and S(c-D) <= eps."""
    delta, eps, D = 0.5, 1e-4, 1e-2
    a, b = O.cell_fit_1d(c, delta, eps, D)
    s_c, s_hi, s_lo = _post_alpha_1d(a, b, np.array([c, c + D, c - D]), delta)
    assert abs(s_c - 0.5) < 1e-9
    assert abs((1 - s_hi) - eps) < 1e-9
    assert 0 <= s_lo <= eps
    # and the printed, rounded values still give a sharp step
    a_p, b_p = {0.1: (-172.1, 1560.1), 0.5: (-865.0, 867.2), 0.7: (-1211.4, 520.8)}[c]
    s_c, s_hi, s_lo = _post_alpha_1d(a_p, b_p, np.array([c, c + D, c - D]), delta)
    assert abs(s_c - 0.5) < 0.02 and (1 - s_hi) < 2e-4 and s_lo < 2e-4


def test_post_activation_2d_face_boundary():
    """On the 2D cell of c(t) = 0.5 t + 0.3, bilinear interpolation of the
    corner values followed by the activations gives S = 1/2 on the boundary
    at every scan line t (the point of the 2D derivation)."""
    delta = 0.5
    tl, tr, bl, br = O.cell_fit_2d(0.3, 0.8, delta, 1e-4, 0.2)
    grid = np.zeros((2, 2, 2))
    # axis 0 = horizontal x, axis 1 = vertical t
    grid[0, 0, :], grid[1, 0, :], grid[0, 1, :], grid[1, 1, :] = tl, tr, bl, br
    for t in np.linspace(0, 1, 11):
        x = 0.5 * t + 0.3
        pts = np.array([[2 * x - 1, 2 * t - 1, 0.0]])
        raw = O.interp(grid, pts, [-1, -1, -1], [1, 1, 1])
        assert abs(O.post_activated_alpha(raw, 0.0, delta)[0] - 0.5) < 1e-9


def test_post_activation_expansion():
    """alpha(softplus(v)) equals the expanded form 1 - (1 + e^v)^-delta."""
    v = np.linspace(-30, 30, 101)
    for delta in (0.01, 0.5, 2.0):
        assert np.allclose(O.post_activated_alpha(v, 0.0, delta), 1 - (1 + np.exp(v)) ** (-delta),
                           rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------
# low-density initialisation
# ---------------------------------------------------------------------------
def test_low_density_init_transmittance():
    """Zero grid and the shift of Eq. low_density_init: a ray crossing one
    voxel size s keeps transmittance 1 - alpha_init (supplementary derivation).
    Two samples at delta = s/2 on an axis-aligned ray through the box."""
    s = 2.0 / 159
    b = O.low_density_bias(1e-2, s)
    assert abs(b - 0.2015) < 5e-4
    prm = O.Params(np.zeros((8, 8, 8)), np.zeros((8, 8, 8, 12)),
                   *synth.xavier_uniform_mlp(np.random.default_rng(0), (39, 128, 128, 3)),
                   [-1, -1, -1], [1, 1, 1], b)
    step = s / 2
    o = np.array([[-1.0, 0.1, 0.2]], F32)
    d = np.array([[1.0, 0.0, 0.0]], F32)
    samp = O.sample_rays(o, d, None, prm.box_min, prm.box_max, step, 2)
    assert samp["n_uniform"][0] == 2
    out = O.render_forward(prm, o, d, None, samp, step, np.ones(3))
    assert abs(out["t_end"][0] - (1 - 1e-2)) < 1e-12


# ---------------------------------------------------------------------------
# compositing closed forms
# ---------------------------------------------------------------------------
def _const_params(raw, feat_val, b=0.0, n=6):
    Ws, bs = synth.xavier_uniform_mlp(np.random.default_rng(3), (39, 128, 128, 3))
    return O.Params(np.full((n, n, n), raw), np.full((n, n, n, 12), feat_val), Ws, bs,
                    [-1, -1, -1], [1, 1, 1], b)


def test_constant_slab_transmittance_exact():
    """Constant raw density r on an axis ray of length L = 2 with L/delta an
    integer and p = 0: T = exp(-softplus(r + b) L) and, with a constant
    colour c, C = (1 - T) c + T c_bg."""
    r, b = 0.3, -1.1
    prm = _const_params(r, 0.25, b)
    step = 2.0 / 32
    o = np.array([[-3.0, 0.1, 0.2]], F32)
    d = np.array([[1.0, 0.0, 0.0]], F32)
    samp = O.sample_rays(o, d, None, prm.box_min, prm.box_max, step, 1000)
    assert samp["n_uniform"][0] == 32
    bg = np.array([0.2, 0.5, 0.9])
    out = O.render_forward(prm, o, d, None, samp, step, bg)
    sig = math.log1p(math.exp(r + b))
    T = math.exp(-sig * 2.0)
    assert abs(out["t_end"][0] - T) < 1e-13
    assert abs(math.exp(out["log_t_end"][0]) - T) < 1e-13
    pe = O.positional_encoding(d.astype(float))
    c, _ = O.mlp_forward(prm.Ws, prm.bs, np.concatenate([np.full((1, 12), 0.25), pe], 1))
    assert np.allclose(out["rgb"][0], (1 - T) * c[0] + T * bg, atol=1e-13)
    assert abs(out["depth"][0] - sum((1 - math.exp(-sig * step)) * math.exp(-sig * step * k) *
                                     (2.0 + k * step) for k in range(32))) < 1e-12


def test_constant_slab_jittered_count():
    """With jitter p and any length: T = exp(-sigma N_r delta) exactly."""
    r = -0.7
    prm = _const_params(r, 0.0)
    rng = np.random.default_rng(5)
    o, d, *_ = synth.draw_pixels_without_replacement(rng, synth.cube_vertex_cameras(), 16, 16, 20.0, 64)
    p = rng.random(64).astype(F32)
    step = 0.037
    samp = O.sample_rays(o, d, p, prm.box_min, prm.box_max, step, 1000)
    out = O.render_forward(prm, o, d, p, samp, step, np.ones(3))
    sig = math.log1p(math.exp(r))
    assert np.allclose(out["t_end"], np.exp(-sig * step * samp["n_uniform"]), rtol=1e-12)


def test_weights_telescope_to_one():
    P = synth.tiny_config(1, n_rays=512)
    prm = O.Params(P.density, P.feat, P.Ws, P.bs, P.box_min, P.box_max, 0.5)
    samp = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples)
    out = O.render_forward(prm, P.rays.o, P.rays.d, None, samp, P.step, P.bg)
    assert np.allclose(out["acc"] + out["t_end"], 1.0, atol=1e-12)
    assert np.all(out["acc"] >= 0) and np.all(out["acc"] <= 1 + 1e-12)
    assert np.allclose(out["seg_w"].sum(1), out["acc"], atol=1e-12)


# ---------------------------------------------------------------------------
# interpolation and the network: library routines
# ---------------------------------------------------------------------------
def test_trilinear_matches_scipy():
    from scipy.interpolate import RegularGridInterpolator
    rng = np.random.default_rng(0)
    n = (5, 7, 6)
    g = rng.normal(size=n)
    bmin, bmax = np.array([-1.0, -0.5, 0.0]), np.array([1.0, 2.0, 0.7])
    x = rng.uniform(bmin, bmax, size=(500, 3))
    ref = RegularGridInterpolator([np.linspace(bmin[i], bmax[i], n[i]) for i in range(3)], g)(x)
    assert np.allclose(O.interp(g, x, bmin, bmax), ref, rtol=1e-12, atol=1e-12)


def test_trilinear_exact_for_affine_field():
    n = 9
    ax = np.linspace(-1, 1, n)
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    g = np.stack([0.3 + 2 * X - Y + 0.5 * Z, -X + 4 * Z], -1)
    x = np.random.default_rng(1).uniform(-1, 1, (300, 3))
    got = O.interp(g, x, [-1] * 3, [1] * 3)
    assert np.allclose(got[:, 0], 0.3 + 2 * x[:, 0] - x[:, 1] + 0.5 * x[:, 2], atol=1e-12)
    assert np.allclose(got[:, 1], -x[:, 0] + 4 * x[:, 2], atol=1e-12)


def test_trilinear_hand_corner_example():
    """Hand-worked 8-corner example in one unit cell: value at (0.25, 0.5,
    0.75) of corners v_ijk = i + 10 j + 100 k is 0.25 + 5 + 75."""
    g = np.zeros((2, 2, 2))
    for i in (0, 1):
        for j in (0, 1):
            for k in (0, 1):
                g[i, j, k] = i + 10 * j + 100 * k
    assert abs(O.interp(g, np.array([[0.25, 0.5, 0.75]]), [0, 0, 0], [1, 1, 1])[0] - 80.25) < 1e-12


def test_positional_encoding_values():
    d = np.array([[0.6, -0.8, 0.0]])
    pe = O.positional_encoding(d)
    assert pe.shape == (1, 27)
    assert np.allclose(pe[0, :3], d[0])
    assert np.allclose(pe[0, 3:6], np.sin(d[0]))
    assert np.allclose(pe[0, 6:9], np.cos(d[0]))
    assert np.allclose(pe[0, 21:24], np.sin(8 * d[0]))
    assert np.allclose(pe[0, 24:27], np.cos(8 * d[0]))
    assert abs(pe[0, 3] - 0.5646424733950354) < 1e-15


@pytest.mark.parametrize("channels", [0, 3])
def test_interp_scatter_is_the_transpose_of_interp(channels):
    """<interp(V, x), u> = <V, scatter(x, u)> for every V and u (the
    definition of the adjoint the grid gradients use), with points inside,
    on the faces of and outside the box (clamped cells)."""
    rng = np.random.default_rng(7)
    shape = (5, 4, 6) + ((channels,) if channels else ())
    bmin, bmax = np.array([-1.0, 0.0, 2.0]), np.array([1.0, 3.0, 4.5])
    x = bmin + (bmax - bmin) * rng.uniform(-0.2, 1.2, size=(200, 3))
    x[:4] = [bmin, bmax, [0.0, 1.5, 3.0], [bmin[0], bmax[1], 3.3]]
    V = rng.normal(size=shape)
    u = rng.normal(size=(200, channels) if channels else (200,))
    lhs = np.sum(O.interp(V, x, bmin, bmax) * u)
    rhs = np.sum(V * O.interp_scatter(shape, x, bmin, bmax, u))
    assert abs(lhs - rhs) < 1e-10 * (1.0 + abs(lhs))


def test_interp_scatter_hand_example():
    """One sample at the centre of the single cell of a 2x2x2 grid puts an
    eighth of its value on each vertex; one on a vertex puts all of it there."""
    out = O.interp_scatter((2, 2, 2), np.array([[0.5, 0.5, 0.5]]), [0, 0, 0], [1, 1, 1], np.array([8.0]))
    assert np.array_equal(out, np.ones((2, 2, 2)))
    out = O.interp_scatter((3, 3, 3), np.array([[1.0, 0.0, 0.5]]), [0, 0, 0], [1, 1, 1], np.array([2.0]))
    want = np.zeros((3, 3, 3))
    want[2, 0, 1] = 2.0
    assert np.allclose(out, want, atol=1e-15)


def test_lr_decay_reaches_a_tenth_at_20k():
    """The learning rate decays exponentially to 0.1x over 20k iterations
    (supplementary implementation details)."""
    assert O.lr_at(1e-3, 0) == 1e-3
    assert abs(O.lr_at(1e-3, 20000) - 1e-4) < 1e-18
    assert abs(O.lr_at(1e-3, 10000) - 1e-3 / math.sqrt(10.0)) < 1e-18
    lrs = [O.lr_at(0.1, it) for it in range(0, 20001, 1000)]
    assert all(a > b for a, b in zip(lrs, lrs[1:]))
    assert all(abs(b / a - 0.1 ** 0.05) < 1e-12 for a, b in zip(lrs, lrs[1:]))


def test_psnr_decibels():
    """PSNR of images in [0, 1] is -10 log10(MSE): 0 dB at MSE 1, 10 dB per
    decade."""
    assert O.psnr(1.0) == 0.0
    assert abs(O.psnr(1e-2) - 20.0) < 1e-12
    assert abs(O.psnr(1e-3) - 30.0) < 1e-12
    assert abs(O.psnr(0.5) - 3.010299956639812) < 1e-12


def test_proposal_encoding_entry_point_and_layout():
    """The proposal input is PE of the box-entry point in [-1, 1]^3 box
    coordinates followed by PE of the direction: rays entering at a face
    centre give known coordinates."""
    o = np.array([[-2.0, 0.0, 0.0], [1.0, 1.0, -1.0]])
    d = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    tn = np.array([1.0, 1.0])
    enc = O.proposal_encoding(o[:1], d[:1], tn[:1], [-1, -1, -1], [1, 1, 1])
    assert enc.shape == (1, 54)
    assert np.allclose(enc[0, :3], [-1.0, 0.0, 0.0])
    assert np.allclose(enc[0, 3:6], [math.sin(-1.0), 0.0, 0.0])
    assert np.allclose(enc[0, 6:9], [math.cos(-1.0), 1.0, 1.0])
    assert np.allclose(enc[0, 27:30], d[0])
    assert np.allclose(enc[0, 48:51], np.sin(8 * d[0]))
    # box [0,2]^3: entry point (1, 1, 0) is (0, 0, -1) in box coordinates
    enc = O.proposal_encoding(o[1:], d[1:], tn[1:], [0, 0, 0], [2, 2, 2])
    assert np.allclose(enc[0, :3], [0.0, 0.0, -1.0])
    assert np.allclose(enc[0, 27:30], [0.0, 0.0, 1.0])
    assert np.allclose(enc[0, 51:54], np.cos(8 * d[1]))


def test_mlp_matches_torch_functional():
    rng = np.random.default_rng(2)
    Ws, bs = synth.xavier_uniform_mlp(rng, (39, 128, 128, 3))
    bs = [rng.normal(size=b.shape) * 0.1 for b in bs]
    x = rng.normal(size=(50, 39))
    c, _ = O.mlp_forward(Ws, bs, x)
    F = torch.nn.functional
    t = lambda a: torch.tensor(np.asarray(a, np.float64))
    h = F.relu(F.linear(t(x), t(Ws[0]), t(bs[0])))
    h = F.relu(F.linear(h, t(Ws[1]), t(bs[1])))
    ref = torch.sigmoid(F.linear(h, t(Ws[2]), t(bs[2]))).numpy()
    assert np.allclose(c, ref, rtol=1e-13, atol=1e-14)


def test_softplus_sigmoid_textbook():
    x = np.linspace(-50, 50, 1001)
    assert np.allclose(O.softplus(x), np.logaddexp(0, x), rtol=1e-14, atol=1e-300)
    h = 1e-6
    assert np.allclose((O.softplus(x + h) - O.softplus(x - h)) / (2 * h), O.sigmoid(x), atol=1e-8)
    assert np.allclose(O.sigmoid(x), 1 / (1 + np.exp(-x)), rtol=1e-13)


# ---------------------------------------------------------------------------
# the hand adjoint: torch autograd of an independent forward, and FD
# ---------------------------------------------------------------------------
def _torch_forward(dens, feat, Ws, bs, b, o, d, jit, samp, step, bg, pe_x=0):
    """Independent float64 torch forward of the same quadrature (written with
    torch ops, product form of the transmittance, per-ray loop).  With
    pe_x > 0 the network input is [features, encoded position (box [-1,1]^3,
    so box coordinates are the position itself), encoded direction]."""
    t_near = samp["t_near"]
    outs = torch.zeros((o.shape[0], 3), dtype=torch.float64)
    n = np.array(dens.shape)
    ro = samp["ray_offset"]
    for slot in range(o.shape[0]):
        r = int(samp["perm"][slot])
        ks = samp["sample_k"][ro[slot]:ro[slot + 1]]
        T = torch.tensor(1.0, dtype=torch.float64)
        C = torch.zeros(3, dtype=torch.float64)
        pe = [torch.tensor(d[r], dtype=torch.float64)]
        for fr in range(4):
            pe += [torch.sin(pe[0] * 2 ** fr), torch.cos(pe[0] * 2 ** fr)]
        pe = torch.cat(pe)
        for k in ks:
            tk = F32(t_near[r]) + F32(F32(F32(k) + F32(0 if jit is None else jit[r])) * F32(step))
            x = o[r].astype(np.float64) + float(tk) * d[r].astype(np.float64)
            u = (x + 1) / 2 * (n - 1)
            i0 = np.clip(np.floor(u), 0, n - 2).astype(int)
            fr_ = np.clip(u - i0, 0, 1)
            raw = 0
            fv = 0
            for c in range(8):
                ofs = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1])
                wgt = np.prod(np.where(ofs == 1, fr_, 1 - fr_))
                ii = i0 + ofs
                raw = raw + wgt * dens[ii[0], ii[1], ii[2]]
                fv = fv + wgt * feat[ii[0], ii[1], ii[2]]
            sig = torch.nn.functional.softplus(raw + b)
            a = 1 - torch.exp(-sig * step)
            if pe_x:
                xt = torch.tensor(x, dtype=torch.float64)
                pex = [xt]
                for fr in range(pe_x):
                    pex += [torch.sin(xt * 2 ** fr), torch.cos(xt * 2 ** fr)]
                inp = torch.cat([fv, torch.cat(pex), pe])
            else:
                inp = torch.cat([fv, pe])
            h = torch.relu(Ws[0] @ inp + bs[0])
            h = torch.relu(Ws[1] @ h + bs[1])
            col = torch.sigmoid(Ws[2] @ h + bs[2])
            C = C + T * a * col
            T = T * (1 - a)
        outs[r] = C + T * torch.tensor(bg, dtype=torch.float64)
    return outs


def _small_problem(seed, n=4, rays=24, jitter=True):
    rng = np.random.default_rng(seed)
    dens = rng.uniform(-1, 1, (n, n, n))
    feat = rng.uniform(-1, 1, (n, n, n, 12))
    Ws, bs = synth.xavier_uniform_mlp(rng, (39, 128, 128, 3))
    bs = [rng.normal(size=b.shape) * 0.2 for b in bs]
    o, d, *_ = synth.draw_pixels_without_replacement(rng, synth.cube_vertex_cameras(), 8, 8, 9.0, rays)
    jit = rng.random(rays).astype(F32) if jitter else None
    tgt = rng.random((rays, 3))
    step = 0.5 * 2 / (n - 1)
    return dens, feat, Ws, bs, o, d, jit, tgt, step


def test_adjoint_matches_torch_autograd():
    dens, feat, Ws, bs, o, d, jit, tgt, step = _small_problem(0, n=5, rays=20)
    b = 0.3
    bg = np.array([1.0, 0.9, 0.8])
    samp = O.sample_rays(o, d, jit, [-1] * 3, [1] * 3, step, 64, morton=True)
    prm = O.Params(dens, feat, Ws, bs, [-1] * 3, [1] * 3, b)
    fwd = O.render_forward(prm, o, d, jit, samp, step, bg)
    loss, g = O.photo_loss(fwd["rgb"], tgt)
    gr = O.render_backward(prm, o, d, jit, samp, step, bg, fwd, g)
    T = lambda a: torch.tensor(np.asarray(a, np.float64), requires_grad=True)
    td, tf = T(dens), T(feat)
    tW = [T(w) for w in Ws]
    tb = [T(x) for x in bs]
    rgb = _torch_forward(td, tf, tW, tb, b, o, d, jit, samp, step, bg)
    assert np.allclose(rgb.detach().numpy(), fwd["rgb"], rtol=1e-12, atol=1e-13)
    L = ((rgb - torch.tensor(tgt)) ** 2).sum() / rgb.shape[0]
    assert abs(L.item() - loss) < 1e-12
    L.backward()
    assert np.allclose(gr["density"], td.grad.numpy(), rtol=1e-9, atol=1e-13)
    assert np.allclose(gr["feat"], tf.grad.numpy(), rtol=1e-9, atol=1e-13)
    for a, t in zip(gr["Ws"] + gr["bs"], tW + tb):
        assert np.allclose(a, t.grad.numpy(), rtol=1e-9, atol=1e-13)


def test_adjoint_with_position_encoding_matches_torch_autograd():
    """The variant whose network also takes PE_5 of the query position
    (72 inputs): forward and every gradient by autograd of the independent
    torch forward."""
    dens, feat, _, bs, o, d, jit, tgt, step = _small_problem(3, n=5, rays=16)
    rng = np.random.default_rng(31)
    Ws, _ = synth.xavier_uniform_mlp(rng, (72, 128, 128, 3))
    b, bg = 0.3, np.array([1.0, 0.9, 0.8])
    samp = O.sample_rays(o, d, jit, [-1] * 3, [1] * 3, step, 64, morton=True)
    prm = O.Params(dens, feat, Ws, bs, [-1] * 3, [1] * 3, b, pe_x=5)
    fwd = O.render_forward(prm, o, d, jit, samp, step, bg)
    loss, g = O.photo_loss(fwd["rgb"], tgt)
    gr = O.render_backward(prm, o, d, jit, samp, step, bg, fwd, g)
    T = lambda a: torch.tensor(np.asarray(a, np.float64), requires_grad=True)
    td, tf = T(dens), T(feat)
    tW = [T(w) for w in Ws]
    tb = [T(x) for x in bs]
    rgb = _torch_forward(td, tf, tW, tb, b, o, d, jit, samp, step, bg, pe_x=5)
    assert np.allclose(rgb.detach().numpy(), fwd["rgb"], rtol=1e-12, atol=1e-13)
    L = ((rgb - torch.tensor(tgt)) ** 2).sum() / rgb.shape[0]
    L.backward()
    assert np.allclose(gr["density"], td.grad.numpy(), rtol=1e-9, atol=1e-13)
    assert np.allclose(gr["feat"], tf.grad.numpy(), rtol=1e-9, atol=1e-13)
    for a, t in zip(gr["Ws"] + gr["bs"], tW + tb):
        assert np.allclose(a, t.grad.numpy(), rtol=1e-9, atol=1e-13)


def test_position_encoding_columns_sit_between_features_and_direction():
    """With the 33 position columns of W1 zero, the 72-input network renders
    what the 39-input network [W1_feat | W1_dir] renders, and its position
    columns still receive a gradient; box coordinates put the box's centre
    at 0 and its faces at -1 and 1."""
    dens, feat, Ws39, bs, o, d, jit, tgt, step = _small_problem(4, n=5, rays=16)
    rng = np.random.default_rng(32)
    W1 = np.zeros((128, 72))
    W1[:, :12] = Ws39[0][:, :12]
    W1[:, 45:] = Ws39[0][:, 12:]
    Ws72 = [W1, Ws39[1], Ws39[2]]
    samp = O.sample_rays(o, d, jit, [-1] * 3, [1] * 3, step, 64)
    p39 = O.Params(dens, feat, Ws39, bs, [-1] * 3, [1] * 3, 0.2)
    p72 = O.Params(dens, feat, Ws72, bs, [-1] * 3, [1] * 3, 0.2, pe_x=5)
    f39 = O.render_forward(p39, o, d, jit, samp, step, np.ones(3))
    f72 = O.render_forward(p72, o, d, jit, samp, step, np.ones(3))
    assert np.allclose(f39["rgb"], f72["rgb"], rtol=0, atol=1e-14)
    _, g = O.photo_loss(f72["rgb"], tgt)
    gr = O.render_backward(p72, o, d, jit, samp, step, np.ones(3), f72, g)
    assert np.abs(gr["Ws"][0][:, 12:45]).max() > 0
    u = O.box_coordinates(np.array([[3.0, -1.0, 0.5]]), [2, -3, 0], [4, 1, 1])
    assert np.allclose(u, [[0.0, 0.0, 0.0]])
    u = O.box_coordinates(np.array([[4.0, -3.0, 0.75]]), [2, -3, 0], [4, 1, 1])
    assert np.allclose(u, [[1.0, -1.0, 0.5]])


def test_adjoint_depth_acc_terms_match_fd():
    """The depth and opacity channels of the adjoint, by central FD."""
    dens, feat, Ws, bs, o, d, jit, tgt, step = _small_problem(4, n=4, rays=16)
    prm = O.Params(dens.copy(), feat, Ws, bs, [-1] * 3, [1] * 3, 0.1)
    samp = O.sample_rays(o, d, jit, [-1] * 3, [1] * 3, step, 64)
    rng = np.random.default_rng(9)
    gd, ga = rng.normal(size=16), rng.normal(size=16)
    fwd = O.render_forward(prm, o, d, jit, samp, step, np.ones(3))
    gr = O.render_backward(prm, o, d, jit, samp, step, np.ones(3), fwd, np.zeros((16, 3)), gd, ga)

    def L(dd):
        prm.density = dd
        f = O.render_forward(prm, o, d, jit, samp, step, np.ones(3), with_color=False)
        return float(np.dot(f["depth"], gd) + np.dot(f["acc"], ga))
    for idx in [(1, 1, 1), (2, 1, 2), (0, 3, 1), (2, 2, 2)]:
        e = 1e-6
        dp, dm = dens.copy(), dens.copy()
        dp[idx] += e
        dm[idx] -= e
        fd = (L(dp) - L(dm)) / (2 * e)
        assert abs(fd - gr["density"][idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, gr["density"][idx])


def test_adjoint_matches_central_fd_on_4cube():
    dens, feat, Ws, bs, o, d, jit, tgt, step = _small_problem(7, n=4, rays=32)
    b = -0.2
    bg = np.ones(3)
    samp = O.sample_rays(o, d, jit, [-1] * 3, [1] * 3, step, 64)
    prm = O.Params(dens.copy(), feat.copy(), Ws, bs, [-1] * 3, [1] * 3, b)

    def loss_of(dd, ff):
        prm.density, prm.feat = dd, ff
        f = O.render_forward(prm, o, d, jit, samp, step, bg)
        return O.photo_loss(f["rgb"], tgt)[0]

    fwd = O.render_forward(prm, o, d, jit, samp, step, bg)
    _, g = O.photo_loss(fwd["rgb"], tgt)
    gr = O.render_backward(prm, o, d, jit, samp, step, bg, fwd, g)
    rng = np.random.default_rng(11)
    for _ in range(12):
        idx = tuple(rng.integers(0, 4, 3))
        for eps in (1e-5,):
            dp, dm = dens.copy(), dens.copy()
            dp[idx] += eps
            dm[idx] -= eps
            fd = (loss_of(dp, feat) - loss_of(dm, feat)) / (2 * eps)
            assert abs(fd - gr["density"][idx]) <= 1e-7 + 1e-5 * abs(fd), (idx, fd, gr["density"][idx])
        ch = int(rng.integers(0, 12))
        fp, fm = feat.copy(), feat.copy()
        fp[idx + (ch,)] += 1e-5
        fm[idx + (ch,)] -= 1e-5
        fd = (loss_of(dens, fp) - loss_of(dens, fm)) / 2e-5
        assert abs(fd - gr["feat"][idx + (ch,)]) <= 1e-7 + 1e-5 * abs(fd)


def test_photo_loss_gradient():
    rng = np.random.default_rng(0)
    c, t = rng.random((7, 3)), rng.random((7, 3))
    L, g = O.photo_loss(c, t)
    assert abs(L - np.mean(np.sum((c - t) ** 2, 1))) < 1e-15
    e = 1e-7
    c2 = c.copy()
    c2[3, 1] += e
    assert abs((O.photo_loss(c2, t)[0] - L) / e - g[3, 1]) < 1e-6


# ---------------------------------------------------------------------------
# Adam: torch.optim.Adam in float64
# ---------------------------------------------------------------------------
def test_adam_matches_torch():
    rng = np.random.default_rng(0)
    p0 = rng.normal(size=1000)
    grads = [rng.normal(size=1000) * 10 ** rng.uniform(-9, 1, 1000) for _ in range(5)]
    tp = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=0.1, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(1000), np.zeros(1000)
    for t, g in enumerate(grads, 1):
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = O.adam_step(p, g, m, v, 0.1, 0.9, 0.999, 1e-8, t)
    assert np.allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------------------
# proposal
# ---------------------------------------------------------------------------
def test_proposal_kl_gradient_closed_form_and_autograd():
    rng = np.random.default_rng(0)
    z = rng.normal(size=(6, 32)) * 3
    p = rng.random((6, 33))
    p /= p.sum(1, keepdims=True)
    L, g = O.proposal_loss_grad(z, p)
    tz = torch.tensor(z, requires_grad=True)
    zz = torch.cat([tz, torch.zeros(6, 1, dtype=torch.float64)], 1)
    logq = torch.log_softmax(zz, 1)
    tp = torch.tensor(p)
    Lt = (tp * (torch.log(tp) - logq)).sum() / 6
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-12
    assert np.allclose(tz.grad.numpy(), g, atol=1e-14)


def test_proposal_backward_matches_autograd():
    rng = np.random.default_rng(1)
    Ws, bs = synth.xavier_uniform_mlp(rng, (54, 64, 64, 32))
    bs = [rng.normal(size=b.shape) * 0.1 for b in bs]
    enc = rng.normal(size=(10, 54))
    z, cache = O.proposal_forward(Ws, bs, enc)
    dz = rng.normal(size=z.shape)
    dWs, dbs = O.proposal_backward(Ws, cache, dz)
    T = lambda a: torch.tensor(np.asarray(a, np.float64), requires_grad=True)
    tW, tb = [T(w) for w in Ws], [T(b) for b in bs]
    h = torch.relu(torch.tensor(enc) @ tW[0].T + tb[0])
    h = torch.relu(h @ tW[1].T + tb[1])
    (h @ tW[2].T + tb[2]).mul(torch.tensor(dz)).sum().backward()
    for a, t in zip(dWs + dbs, tW + tb):
        assert np.allclose(a, t.grad.numpy(), rtol=1e-12, atol=1e-13)


def test_proposal_selection_special_cases():
    z = np.full((4, 32), -30.0)
    z[0, 7] = 30.0                       # one dominant segment
    z[1] = 10.0                          # uniform over all 32 -> needs >= 99% -> 32
    z[2] = -10.0                         # mass ~ 0 -> fallback
    z[3, :4] = [20.0, 20.0, 20.0, 20.0]  # four equal segments
    m = O.proposal_select(z)
    assert m[0] == np.uint32(1 << 7)
    assert m[1] == np.uint32(0xFFFFFFFF)
    assert m[2] == np.uint32(0xFFFFFFFF)
    assert m[3] == np.uint32(0xF)


def test_proposal_selection_brute_force():
    """Smallest set by probability reaching 99% of the mass, compared with
    exhaustive search over subset sizes on random logits (float64 sums of
    the recipe's float32 probabilities; a ray whose float64 partial sum lies
    within float32 rounding of the target may take one segment more or
    less, and is counted, not compared)."""
    rng = np.random.default_rng(3)
    z = (rng.normal(size=(400, 32)) * 2 + 4).astype(F32)
    masks = O.proposal_select(z)
    q, mass = O.proposal_select_probs(z)
    q64, mass64 = O.proposal_probs(z)
    assert np.abs(q - q64[:, :32]).max() < 1e-6 and np.abs(mass - mass64).max() < 1e-6
    near = 0
    for r in range(400):
        if mass[r] < F32(0.9):
            assert masks[r] == np.uint32(0xFFFFFFFF)
            continue
        qs = np.sort(q[r].astype(np.float64))[::-1]
        target = float(F32(F32(0.99) * mass[r]))
        cs = np.cumsum(qs)
        need = int(np.argmax(cs >= target)) + 1
        got = bin(int(masks[r])).count("1")
        if np.min(np.abs(cs - target)) < 1e-6 * target:
            near += 1
            assert abs(got - need) <= 1
        else:
            assert got == need
        chosen = [s for s in range(32) if (int(masks[r]) >> s) & 1]
        assert min(q[r, chosen]) >= max(np.delete(q[r], chosen), default=-1)
    assert near < 10


def test_exp_f32_recipe_accuracy():
    """The float32 exponential recipe against float64 exp: within 1.5 units
    in the last place over [-87, 0] (a dropped Taylor term or a wrong
    reduction constant exceeds it), exact at 0, zero below -87."""
    rng = np.random.default_rng(7)
    x = np.concatenate([-rng.random(100000) * 87.0, -rng.random(50000) * 0.5,
                        [0.0, -0.0, -1e-30, -1e-7, -87.0, -0.3465736, -0.6931472]]).astype(F32)
    y = O.exp_f32(x)
    ref = np.exp(x.astype(np.float64))
    ulp = np.spacing(ref.astype(F32)).astype(np.float64)
    assert y.dtype == F32
    assert np.max(np.abs(y - ref) / ulp) <= 1.5
    assert O.exp_f32(np.array([0.0], F32))[0] == F32(1.0)
    assert np.all(O.exp_f32(np.array([-87.01, -100.0, -np.inf], F32)) == 0.0)


def test_proposal_targets_sum_to_one():
    P = synth.tiny_config(2, n_rays=256)
    prm = O.Params(P.density, P.feat, P.Ws, P.bs, P.box_min, P.box_max, 0.0)
    samp = O.sample_rays(P.rays.o, P.rays.d, None, P.box_min, P.box_max, P.step, P.max_samples)
    out = O.render_forward(prm, P.rays.o, P.rays.d, None, samp, P.step, P.bg, with_color=False)
    tg = O.proposal_targets(out["seg_w"], out["t_end"])
    assert np.allclose(tg.sum(1), 1.0, atol=1e-12)


# ---------------------------------------------------------------------------
# analytic-scene reference
# ---------------------------------------------------------------------------
def test_scene_render_single_sphere_closed_form():
    """One hard-edged, constant-density sphere on the ray through its
    centre: T = exp(-rho * 2r), colour (1-T) c + T bg, up to the midpoint
    quadrature of the soft edge."""
    c = np.array([[0.0, 0.0, 0.0]])
    r, rho = np.array([0.5]), np.array([3.0])
    col = np.array([[0.2, 0.4, 0.6]])
    o = np.array([[-3.0, 0.0, 0.0]], F32)
    d = np.array([[1.0, 0.0, 0.0]], F32)
    out = O.scene_render(o, d, c, r, rho, col, [-1] * 3, [1] * 3, 1e-4, np.ones(3), edge=1e-4)
    T = math.exp(-3.0 * 1.0)
    assert np.allclose(out[0], (1 - T) * col[0] + T, atol=2e-4)


# ---------------------------------------------------------------------------
# bfloat16 form of the network
# ---------------------------------------------------------------------------
def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=10000) * 10 ** rng.uniform(-30, 30, 10000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, -0.0, 3e38])]).astype(F32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.bf16_round(x), ref)


def test_bf16_mlp_equals_exact_on_representable_inputs():
    """With weights and inputs already bfloat16 values (and ReLU outputs
    that stay representable because every hidden weight is a power of two
    times a small integer), the bfloat16 form is the exact network."""
    rng = np.random.default_rng(1)
    Ws = [O.bf16_round(rng.normal(size=(128, 39)) * 0.1), O.bf16_round(np.eye(128) * 0.5),
          O.bf16_round(rng.normal(size=(3, 128)) * 0.1)]
    bs = [np.zeros(128), np.zeros(128), np.zeros(3)]
    x = np.concatenate([O.bf16_round(rng.normal(size=(20, 12))), rng.normal(size=(20, 27))], 1)
    # make layer-1 outputs representable: only one nonzero feature, power-of-two weights there
    Ws[0][:, 1:] = 0.0
    Ws[0][:, 0] = 2.0 ** rng.integers(-3, 3, 128)
    c1, _ = O.mlp_forward(Ws, bs, x, bf16=True)
    c0, _ = O.mlp_forward(Ws, bs, x, bf16=False)
    assert np.allclose(c1, c0, rtol=0, atol=1e-15)


def test_bf16_backward_close_to_exact():
    """With the same ReLU masks and activations, the bfloat16 form's
    gradients differ from the exact network's only by bfloat16 operand
    rounding (catches dropped terms and transposes)."""
    rng = np.random.default_rng(2)
    Ws, bs = synth.xavier_uniform_mlp(rng, (39, 128, 128, 3))
    x = rng.normal(size=(400, 39))
    dc = rng.normal(size=(400, 3))
    c1, m1 = O.mlp_forward(Ws, bs, x, bf16=True)
    c0, _ = O.mlp_forward(Ws, bs, x, bf16=False)
    assert np.abs(c1 - c0).max() < 1e-2
    exact_same_masks = dict(m1, bf16=False)
    d1, W1g, b1g = O.mlp_backward(Ws, m1, dc)
    d0, W0g, b0g = O.mlp_backward(Ws, exact_same_masks, dc)
    assert np.linalg.norm(d1[:, :12] - d0[:, :12]) / np.linalg.norm(d0[:, :12]) < 2e-2
    for a, b in zip(W1g + b1g, W0g + b0g):
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 2e-2


def test_proposal_bf16_backward_close_to_exact():
    """Proposal network: with the same ReLU masks and activations the
    bfloat16 form's gradients differ from the exact ones only by operand
    rounding; with bfloat16-exact gradients and weights it is exact."""
    rng = np.random.default_rng(5)
    Ws, bs = synth.xavier_uniform_mlp(rng, (54, 64, 64, 32))
    enc = rng.normal(size=(300, 54))
    dz = rng.normal(size=(300, 32))
    z1, c1 = O.proposal_forward(Ws, bs, enc, bf16=True)
    g1 = O.proposal_backward(Ws, c1, dz)
    g0 = O.proposal_backward(Ws, dict(c1, bf16=False), dz)
    for a, b in zip(g1[0] + g1[1], g0[0] + g0[1]):
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 2e-2
    # a single nonzero logit gradient of 1 per ray, one-hot W3 rows and W2 = I/2:
    # every propagated gradient is a power of two, so no rounding happens
    Wx = [O.bf16_round(Ws[0]), np.eye(64) * 0.5, np.zeros((32, 64))]
    Wx[2][np.arange(32), np.arange(32)] = 1.0
    dz1 = np.zeros((300, 32))
    dz1[np.arange(300), rng.integers(0, 32, 300)] = 1.0
    _, cx = O.proposal_forward(Wx, bs, enc, bf16=True)
    ga = O.proposal_backward(Wx, cx, dz1)
    gb = O.proposal_backward(Wx, dict(cx, bf16=False), dz1)
    for a, b in zip(ga[0] + ga[1], gb[0] + gb[1]):
        assert np.array_equal(a, b)
