"""The fused adjoint + grid Adam call against the separate calls it
replaces (dvgo_render_bwd into zeroed gradients, then dvgo_adam_step on
both grids): same network gradient bit for bit, same parameter updates and
moments up to the summation order of the grid gradients (1e-5 normwise on
the update), the bfloat16 copy equal to the rounded new parameters; with no
sample in the batch every vertex takes the zero-gradient step."""

import numpy as np
import pytest

from tests.helpers import assert_close, np_of, to_dev
from tests.test_gpu_render import _gpu, _problem

pytestmark = pytest.mark.gpu
F32 = np.float32


def _state(rng, shape):
    return to_dev((rng.normal(size=shape) * 1e-3).astype(F32)), to_dev((rng.random(shape) * 1e-5).astype(F32))


def _clone_grid(api, grid):
    g = api.Grid(grid.density.clone(), grid.feat.clone(), grid.box_min, grid.box_max, grid.act_shift)
    g.feat_shadow = None if grid.feat_shadow is None else grid.feat_shadow.clone()
    return g


def _bf16_bits(x):
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


@pytest.mark.parametrize("bf16", [False, True])
def test_fused_backward_adam_equals_separate(gpu_lib, bf16):
    import torch
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_BF16, DVGO_F32
    prec = DVGO_BF16 if bf16 else DVGO_F32
    P = _problem(7, n_rays=2048, bias=0.3)
    grid, flat, s = _gpu(P, bf16=bf16)
    rng = np.random.default_rng(3)
    mD, vD = _state(rng, P.density.shape)
    mF, vF = _state(rng, P.feat.shape)
    out = api.render_fwd(grid, flat, s, P.bg, precision=prec, use_shadow=bf16)
    g = to_dev((rng.normal(size=(P.rays.o.shape[0], 3)) * 1e-3).astype(F32))
    lr, t = 0.1, 4

    ga = _clone_grid(api, grid)
    gd, gf, gm = torch.zeros_like(grid.density), torch.zeros_like(grid.feat), torch.zeros_like(flat)
    api.render_bwd(ga, flat, s, out["log_t_end"], g, gd, gf, gm, P.bg, precision=prec, use_shadow=bf16)
    mDa, vDa, mFa, vFa = mD.clone(), vD.clone(), mF.clone(), vF.clone()
    api.adam_step(ga.density, gd, mDa, vDa, lr, t)
    api.adam_step(ga.feat, gf, mFa, vFa, lr, t, shadow=ga.feat_shadow)

    gb = _clone_grid(api, grid)
    gmb = torch.zeros_like(flat)
    mDb, vDb, mFb, vFb = mD.clone(), vD.clone(), mF.clone(), vF.clone()
    api.render_bwd_adam(gb, flat, s, out["log_t_end"], g, mDb, vDb, mFb, vFb, gmb, lr, t, bg=P.bg, precision=prec,
                        use_shadow=bf16)

    assert torch.equal(gm, gmb)
    for name, p0, pa, pb in (("density", grid.density, ga.density, gb.density), ("feat", grid.feat, ga.feat,
                                                                                   gb.feat)):
        assert_close(f"{name} update", np_of(pb - p0), np_of(pa - p0), 1e-5)
    for name, a, b in (("m density", mDa, mDb), ("v density", vDa, vDb), ("m feat", mFa, mFb), ("v feat", vFa, vFb)):
        assert_close(name, np_of(b), np_of(a), 1e-5)
    if bf16:
        assert np.array_equal(np_of(gb.feat_shadow).view(np.uint16), _bf16_bits(np_of(gb.feat)))


def test_fused_backward_adam_without_samples(gpu_lib):
    """Every ray misses the box: the call is the zero-gradient Adam step of
    every vertex (compared with dvgo_adam_step on zero gradients)."""
    import torch
    from paper_2111_11215_amd import api
    P = _problem(8, n_rays=256)
    P.rays.o = (P.rays.o + np.float32(10.0)).astype(F32)        # all rays start beyond the box ...
    P.rays.d = np.abs(P.rays.d).astype(F32)                      # ... and point away from it
    grid, flat, s = _gpu(P)
    assert int(s.n_kept.item()) == 0
    rng = np.random.default_rng(5)
    mD, vD = _state(rng, P.density.shape)
    mF, vF = _state(rng, P.feat.shape)
    out = api.render_fwd(grid, flat, s, P.bg)
    g = torch.ones((256, 3), device="cuda")
    ga = _clone_grid(api, grid)
    mDa, vDa, mFa, vFa = mD.clone(), vD.clone(), mF.clone(), vF.clone()
    api.adam_step(ga.density, torch.zeros_like(ga.density), mDa, vDa, 0.1, 2)
    api.adam_step(ga.feat, torch.zeros_like(ga.feat), mFa, vFa, 0.1, 2)
    gb = _clone_grid(api, grid)
    gm = torch.zeros_like(flat)
    api.render_bwd_adam(gb, flat, s, out["log_t_end"], g, mD, vD, mF, vF, gm, 0.1, 2, bg=P.bg)
    for a, b in ((ga.density, gb.density), (ga.feat, gb.feat), (mDa, mD), (vDa, vD), (mFa, mF), (vFa, vF)):
        assert torch.allclose(a, b, rtol=1e-6, atol=0)
    assert float(gm.abs().max()) == 0.0


@pytest.mark.parametrize("bf16", [False, True])
def test_train_step_equals_separate_calls(gpu_lib, bf16):
    """dvgo_train_step (the adjoint reusing the forward's gathers, colours and
    prep inside one call) against dvgo_render_fwd + dvgo_photo_loss +
    dvgo_render_bwd_adam: identical colour, loss gradient and network
    gradient; the loss to float32 rounding (its sum runs in another order);
    the same grid update up to the summation order of the grid gradients."""
    import torch
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_BF16, DVGO_F32
    prec = DVGO_BF16 if bf16 else DVGO_F32
    P = _problem(9, n_rays=2048, bias=0.3)
    grid, flat, s = _gpu(P, bf16=bf16)
    rng = np.random.default_rng(11)
    mD, vD = _state(rng, P.density.shape)
    mF, vF = _state(rng, P.feat.shape)
    target = to_dev(P.rays.target.astype(F32))
    lr, t = 0.1, 3

    ga = _clone_grid(api, grid)
    out = api.render_fwd(ga, flat, s, P.bg, precision=prec, use_shadow=bf16, want_depth_acc=False)
    loss_a, g = api.photo_loss(out["rgb"], target)
    gma = torch.zeros_like(flat)
    mDa, vDa, mFa, vFa = mD.clone(), vD.clone(), mF.clone(), vF.clone()
    api.render_bwd_adam(ga, flat, s, out["log_t_end"], g, mDa, vDa, mFa, vFa, gma, lr, t, bg=P.bg, precision=prec,
                        use_shadow=bf16)

    gb = _clone_grid(api, grid)
    gmb = torch.zeros_like(flat)
    mDb, vDb, mFb, vFb = mD.clone(), vD.clone(), mF.clone(), vF.clone()
    loss_b, rgb_b = api.train_step(gb, flat, s, target, mDb, vDb, mFb, vFb, gmb, lr, t, bg=P.bg, precision=prec,
                                   use_shadow=bf16)
    assert torch.equal(out["rgb"], rgb_b)
    assert abs(float(loss_a[0]) - float(loss_b[0])) <= 1e-6 * float(loss_a[0])
    assert torch.equal(gma, gmb)
    for name, p0, pa, pb in (("density", grid.density, ga.density, gb.density),
                             ("feat", grid.feat, ga.feat, gb.feat)):
        assert_close(f"{name} update", np_of(pb - p0), np_of(pa - p0), 1e-5)
    for name, a, b in (("m density", mDa, mDb), ("v density", vDa, vDb), ("m feat", mFa, mFb), ("v feat", vFa, vFb)):
        assert_close(name, np_of(b), np_of(a), 1e-5)
    if bf16:
        assert np.array_equal(np_of(gb.feat_shadow).view(np.uint16), _bf16_bits(np_of(gb.feat)))


def _mask_np(mD, vD, mF, vF):
    """Activity bits written out from their definition: any non-zero moment."""
    nz = (mD.reshape(-1) != 0) | (vD.reshape(-1) != 0)
    nz |= (mF.reshape(nz.size, -1) != 0).any(1) | (vF.reshape(nz.size, -1) != 0).any(1)
    words = np.zeros((nz.size + 31) // 32, np.uint32)
    idx = np.nonzero(nz)[0]
    np.bitwise_or.at(words, idx // 32, (np.uint32(1) << (idx % 32).astype(np.uint32)))
    return words


@pytest.mark.parametrize("bf16", [False, True])
def test_activity_mask_skips_idle_vertices_exactly(gpu_lib, bf16):
    """The fused grid Adam with an activity mask against the same call
    without one (every vertex steps) over two consecutive steps, from
    moments that are non-zero on a random 30 % of the vertices only: vertices
    with zero moments that no sample touches keep their parameters, moments
    and bf16 copy bit for bit in both; every other value agrees to the
    summation order of the grid gradients (1e-6 normwise); the mask from
    dvgo_grid_active_init equals its definition, and after each step every
    vertex with a non-zero moment has its bit set."""
    import torch
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_BF16, DVGO_F32
    prec = DVGO_BF16 if bf16 else DVGO_F32
    P = _problem(12, n_rays=512, bias=0.3)
    grid, flat, s = _gpu(P, bf16=bf16)
    rng = np.random.default_rng(21)
    nv = P.density.size
    keep = rng.random(nv) < 0.3
    mD, vD = _state(rng, P.density.shape)
    mF, vF = _state(rng, P.feat.shape)
    kd = to_dev(keep.reshape(P.density.shape).astype(F32))
    mD, vD, mF, vF = mD * kd, vD * kd, mF * kd[..., None], vF * kd[..., None]
    active = torch.zeros(api.grid_active_words(nv), dtype=torch.int32, device="cuda")
    api.grid_active_init(mD, vD, mF, vF, active)
    assert np.array_equal(np_of(active).view(np.uint32), _mask_np(np_of(mD), np_of(vD), np_of(mF), np_of(vF)))
    out = api.render_fwd(grid, flat, s, P.bg, precision=prec, use_shadow=bf16)
    g = to_dev((rng.normal(size=(P.rays.o.shape[0], 3)) * 1e-3).astype(F32))

    ga, gb = _clone_grid(api, grid), _clone_grid(api, grid)
    sa = [x.clone() for x in (mD, vD, mF, vF)]
    sb = [x.clone() for x in (mD, vD, mF, vF)]
    for t in (5, 6):
        api.render_bwd_adam(ga, flat, s, out["log_t_end"], g, *sa, torch.zeros_like(flat), 0.1, t, bg=P.bg,
                            precision=prec, use_shadow=bf16)
        api.render_bwd_adam(gb, flat, s, out["log_t_end"], g, *sb, torch.zeros_like(flat), 0.1, t, bg=P.bg,
                            precision=prec, use_shadow=bf16, active=active)
        bits = np_of(active).view(np.uint32)
        need = _mask_np(*(np_of(x) for x in sb))
        assert np.array_equal(need & ~bits, np.zeros_like(need)), "a vertex with non-zero moments lost its bit"
    idle = np.ones(nv, bool)
    for x in sa:
        idle &= (np_of(x).reshape(nv, -1) == 0).all(1)
    print(f"  idle vertices after two steps: {idle.mean():.3f}", flush=True)
    assert 0.2 < idle.mean() < 0.95
    pairs = [("density", grid.density, ga.density, gb.density), ("feat", grid.feat, ga.feat, gb.feat)]
    for name, p0, pa, pb in pairs:
        a, b, z = np_of(pa).reshape(nv, -1), np_of(pb).reshape(nv, -1), np_of(p0).reshape(nv, -1)
        assert np.array_equal(a[idle], z[idle]) and np.array_equal(b[idle], z[idle]), name
        assert_close(f"{name} update", (b - z), (a - z), 1e-6)
    for name, a, b in zip(("m density", "v density", "m feat", "v feat"), sa, sb):
        assert_close(name, np_of(b), np_of(a), 1e-6)
        assert np.all(np_of(b).reshape(nv, -1)[idle] == 0), name
    if bf16:
        assert np.array_equal(np_of(gb.feat_shadow).view(np.uint16), _bf16_bits(np_of(gb.feat)))
        if not np.array_equal(np_of(gb.feat_shadow).view(np.uint16), np_of(ga.feat_shadow).view(np.uint16)):
            assert_close("shadow", np_of(gb.feat), np_of(ga.feat), 1e-6)


@pytest.mark.parametrize("bf16", [False, True])
def test_train_step_network_adam_equals_separate(gpu_lib, bf16):
    """dvgo_train_step taking the network's Adam step inside the call (fused
    into the partial reduction) against the same call followed by
    dvgo_adam_step on the accumulated gradient: network weights and moments
    bit for bit, the gradient left zero; the grids as the same call."""
    import torch
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_BF16, DVGO_F32
    prec = DVGO_BF16 if bf16 else DVGO_F32
    P = _problem(13, n_rays=1024, bias=0.3)
    grid, flat, s = _gpu(P, bf16=bf16)
    rng = np.random.default_rng(17)
    mD, vD = _state(rng, P.density.shape)
    mF, vF = _state(rng, P.feat.shape)
    mW = to_dev((rng.normal(size=flat.shape) * 1e-3).astype(F32))
    vW = to_dev((rng.random(flat.shape) * 1e-5).astype(F32))
    target = to_dev(P.rays.target.astype(F32))
    lr, lrw, t = 0.1, 1e-3, 7
    gw0 = to_dev((rng.normal(size=flat.shape) * 1e-4).astype(F32))   # gradient already accumulated

    ga, fa = _clone_grid(api, grid), flat.clone()
    gma, mWa, vWa = gw0.clone(), mW.clone(), vW.clone()
    sa = [x.clone() for x in (mD, vD, mF, vF)]
    la, _ = api.train_step(ga, fa, s, target, *sa, gma, lr, t, bg=P.bg, precision=prec, use_shadow=bf16)
    api.adam_step(fa, gma, mWa, vWa, lrw, t)

    gb, fb = _clone_grid(api, grid), flat.clone()
    gmb, mWb, vWb = gw0.clone(), mW.clone(), vW.clone()
    sb = [x.clone() for x in (mD, vD, mF, vF)]
    lb, _ = api.train_step(gb, fb, s, target, *sb, gmb, lr, t, bg=P.bg, precision=prec, use_shadow=bf16,
                           mlp_adam=(mWb, vWb, lrw))
    assert torch.equal(fa, fb) and torch.equal(mWa, mWb) and torch.equal(vWa, vWb)
    assert float(gmb.abs().max()) == 0.0 and float(gma.abs().max()) == 0.0
    assert not torch.equal(fa, flat)
    assert abs(float(la[0]) - float(lb[0])) <= 1e-6 * float(la[0])
    for name, p0, pa, pb in (("density", grid.density, ga.density, gb.density), ("feat", grid.feat, ga.feat,
                                                                                   gb.feat)):
        assert_close(f"{name} update", np_of(pb - p0), np_of(pa - p0), 1e-5)


def test_activity_mask_without_samples(gpu_lib):
    """No sample in the batch: with the activity mask only the vertices whose
    bit is set step (their zero-gradient step equals the dense call's), the
    others keep p, m, v bit for bit."""
    import torch
    from paper_2111_11215_amd import api
    P = _problem(14, n_rays=128)
    P.rays.o = (P.rays.o + np.float32(10.0)).astype(F32)
    P.rays.d = np.abs(P.rays.d).astype(F32)
    grid, flat, s = _gpu(P)
    assert int(s.n_kept.item()) == 0
    rng = np.random.default_rng(23)
    nv = P.density.size
    keep = to_dev((rng.random(nv) < 0.3).reshape(P.density.shape).astype(F32))
    mD, vD = _state(rng, P.density.shape)
    mF, vF = _state(rng, P.feat.shape)
    mD, vD, mF, vF = mD * keep, vD * keep, mF * keep[..., None], vF * keep[..., None]
    active = torch.zeros(api.grid_active_words(nv), dtype=torch.int32, device="cuda")
    api.grid_active_init(mD, vD, mF, vF, active)
    out = api.render_fwd(grid, flat, s, P.bg)
    g = torch.ones((128, 3), device="cuda")
    ga, gb = _clone_grid(api, grid), _clone_grid(api, grid)
    sa = [x.clone() for x in (mD, vD, mF, vF)]
    sb = [x.clone() for x in (mD, vD, mF, vF)]
    api.render_bwd_adam(ga, flat, s, out["log_t_end"], g, *sa, torch.zeros_like(flat), 0.1, 2, bg=P.bg)
    api.render_bwd_adam(gb, flat, s, out["log_t_end"], g, *sb, torch.zeros_like(flat), 0.1, 2, bg=P.bg,
                        active=active)
    for a, b in zip((ga.density, ga.feat, *sa), (gb.density, gb.feat, *sb)):
        assert torch.equal(a, b)
    idle = np_of(keep).reshape(-1) == 0
    assert np.array_equal(np_of(gb.density).reshape(-1)[idle], P.density.reshape(-1)[idle])


def test_train_step_full_size_matches_separate(gpu_lib):
    """The benchmark's configuration (160^3 grids, bfloat16 copy and
    network, 8192 rays of the scene, 100^3 coarse mask): one
    dvgo_train_step with the activity mask and the fused network Adam step
    against the separate calls (render forward, loss, backward into zeroed
    gradients, dense dvgo_adam_step on both grids and on the network), from
    moments that are non-zero on a random 40 % of the vertices.  Same loss
    and colour; network weights and moments bit for bit; grid updates and
    moments to the summation order of the grid gradients (1e-5)."""
    import math

    import torch

    import synth
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_BF16
    sp, cams, held, raw = synth.full_scene(0)
    n = synth.FULL_N
    voxel = 2.0 / (n - 1)
    step = 0.5 * voxel
    max_samples = int(math.ceil(2.0 * math.sqrt(3.0) / step)) + 1
    bmin, bmax = tuple(synth.BOX_MIN), tuple(synth.BOX_MAX)
    bits = api.coarse_mask_build(torch.as_tensor(raw).cuda(), bmin, bmax, api.coarse_raw_threshold(synth.FULL_TAU,
                                                                                                   step))
    coarse = (bits, bmin, bmax, raw.shape)
    rng = np.random.default_rng(1000)
    o, d, *_ = synth.draw_pixels_with_replacement(rng, cams, 800, 800, 1000.0, 8192)
    jit = torch.as_tensor(rng.random(8192).astype(F32)).cuda()
    ot, dt = torch.as_tensor(o).cuda(), torch.as_tensor(d).cuda()
    spheres = torch.as_tensor(sp.as_f32_table()).cuda()
    target = api.scene_render(ot, dt, spheres, bmin, bmax, step / 4)
    s = api.sample_rays(ot, dt, jit, bmin, bmax, step, max_samples, coarse=coarse)
    g0 = torch.Generator(device="cpu").manual_seed(5)
    dens = (torch.rand((n, n, n), generator=g0) * 4 - 3).cuda()
    feat = (torch.rand((n, n, n, 12), generator=g0) * 2 - 1).cuda()
    grid = api.Grid(dens, feat, bmin, bmax, api.low_density_bias(synth.FULL_ALPHA_INIT, voxel))
    grid.feat_shadow = feat.to(torch.bfloat16).view(torch.int16).contiguous()
    Ws, bs = synth.xavier_uniform_mlp(np.random.default_rng(7), (39, 128, 128, 3))
    flat = api.flat_from([Ws[0], bs[0], Ws[1], bs[1], Ws[2], bs[2]], api.MLP_SHAPES, "cuda:0")
    keep = (torch.rand((n, n, n), generator=g0) < 0.4).float().cuda()
    mD = torch.randn((n, n, n), generator=g0).cuda() * 1e-3 * keep
    vD = torch.rand((n, n, n), generator=g0).cuda() * 1e-5 * keep
    mF = torch.randn((n, n, n, 12), generator=g0).cuda() * 1e-3 * keep[..., None]
    vF = torch.rand((n, n, n, 12), generator=g0).cuda() * 1e-5 * keep[..., None]
    mW = torch.randn(flat.shape, generator=g0).cuda() * 1e-3
    vW = torch.rand(flat.shape, generator=g0).cuda() * 1e-5
    lr, lrw, t = 0.1, 1e-3, 9

    ga, fa = _clone_grid(api, grid), flat.clone()
    out = api.render_fwd(ga, fa, s, precision=DVGO_BF16, use_shadow=True, want_depth_acc=False)
    loss_a, grad = api.photo_loss(out["rgb"], target)
    gd, gf, gm = torch.zeros_like(dens), torch.zeros_like(feat), torch.zeros_like(flat)
    api.render_bwd(ga, fa, s, out["log_t_end"], grad, gd, gf, gm, precision=DVGO_BF16, use_shadow=True)
    sa = [x.clone() for x in (mD, vD, mF, vF, mW, vW)]
    api.adam_step(ga.density, gd, sa[0], sa[1], lr, t)
    api.adam_step(ga.feat, gf, sa[2], sa[3], lr, t, shadow=ga.feat_shadow)
    api.adam_step(fa, gm, sa[4], sa[5], lrw, t)

    gb, fb = _clone_grid(api, grid), flat.clone()
    sb = [x.clone() for x in (mD, vD, mF, vF, mW, vW)]
    active = torch.zeros(api.grid_active_words(n ** 3), dtype=torch.int32, device="cuda")
    api.grid_active_init(*sb[:4], active)
    gmb = torch.zeros_like(flat)
    loss_b, rgb_b = api.train_step(gb, fb, s, target, *sb[:4], gmb, lr, t, precision=DVGO_BF16, use_shadow=True,
                                   active=active, mlp_adam=(sb[4], sb[5], lrw))
    print(f"  {int(s.n_kept.item())} samples; loss {float(loss_a[0]):.6f}", flush=True)
    assert torch.equal(out["rgb"], rgb_b)
    assert abs(float(loss_a[0]) - float(loss_b[0])) <= 1e-6 * float(loss_a[0])
    assert torch.equal(fa, fb) and torch.equal(sa[4], sb[4]) and torch.equal(sa[5], sb[5])
    for name, p0, pa, pb in (("density", dens, ga.density, gb.density), ("feat", feat, ga.feat, gb.feat)):
        assert_close(f"{name} update", np_of(pb - p0), np_of(pa - p0), 1e-5)
    for name, a, b in zip(("m density", "v density", "m feat", "v feat"), sa[:4], sb[:4]):
        assert_close(name, np_of(b), np_of(a), 1e-5)
    assert np.array_equal(np_of(gb.feat_shadow).view(np.uint16), _bf16_bits(np_of(gb.feat)))
