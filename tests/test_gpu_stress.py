"""Differentiation stress at 256^3 with a 12-channel bfloat16 feature grid,
32768 rays per batch and up to 800 samples per ray (no coarse mask, so every
in-box sample is evaluated; the float32 network).

1. FP64 central finite differences (eps 1e-4) of the oracle's loss on 256
   random grid entries (128 density, 128 feature) touched by the checked rays
   and 16 network parameters, against the oracle's hand-written adjoint:
   relative 1e-6 (an entry whose +eps and -eps evaluations take different
   ReLU branches somewhere is a kink of the function and is skipped, counted).
2. The GPU adjoint of the full launch (grad_rgb non-zero on 64 random rays,
   the rest zero, so the oracle can compute the exact result on those rays)
   against the oracle's adjoint on the whole of both grid gradients and the
   network gradient with the ReLU-kink budget, at 3e-5: the adjoint's
   transmittance and suffix sums run over up to 800 float32 terms per ray,
   whose rounding bound n*u is 800 * 6e-8 = 4.8e-5 (measured 1.2e-5 for the
   density gradient; the 1e-5 of the other tests covers rays of <= 551).
3. Peak device memory of the step (recompute adjoint) against the estimate
   for a variant that stores every sample's intermediate state (printed).
"""

import numpy as np
import pytest

import oracle as O
import synth
from tests.helpers import (assert_close, check_grid_grad, check_weight_grads, kink_budget, mlp_flat_np, np_of, report,
                           to_dev)

pytestmark = pytest.mark.gpu
F32 = np.float32
EPS = 1e-4
TOL32 = 1e-5
TOL_LONG = 3e-5    # float32 sums over up to 800 terms per ray
ZETA = 1e-4
# bytes per evaluated sample a store-everything backward keeps: 8 corner
# indices and weights (64), raw/sigma/alpha/T (16), features (48), network
# input (156), two hidden layers (1024), colour pre- and post-sigmoid (24)
STORE_ALL_BYTES_PER_SAMPLE = 64 + 16 + 48 + 156 + 1024 + 24


def _loss(prm, o, d, j, rays, g, P):
    samp = O.sample_rays(o[rays], d[rays], j[rays], P.box_min, P.box_max, P.step, P.max_samples, morton=False)
    ref = O.render_forward(prm, o[rays], d[rays], j[rays], samp, P.step, P.bg)
    mc = ref["cache"].get("mcache")
    masks = (mc["z1"] > 0, mc["z2"] > 0) if mc is not None else None
    return float(np.sum(g[rays] * ref["rgb"])), masks


def _central(prm, arr, idx, o, d, j, rays, g, P):
    v0 = arr[idx]
    arr[idx] = v0 + EPS
    lp, mp = _loss(prm, o, d, j, rays, g, P)
    arr[idx] = v0 - EPS
    lm, mm = _loss(prm, o, d, j, rays, g, P)
    arr[idx] = v0
    kink = not (np.array_equal(mp[0], mm[0]) and np.array_equal(mp[1], mm[1]))
    return (lp - lm) / (2 * EPS), kink


def oracle_fd_check(P, sel, g_sub, rng, rgb_sel=None, n_entries=256, n_params=16):
    """Oracle forward/adjoint on the rays ``sel`` with float64 grids holding
    the stored values (features rounded to bfloat16), then central finite
    differences against the adjoint.  Returns (params, forward, adjoint)."""
    n = P.density.shape[0]
    dens64 = P.density.astype(np.float64)
    feat64 = O.bf16_round(P.feat)
    Ws64 = [w.astype(np.float64) for w in P.Ws]
    bs64 = [b.astype(np.float64) for b in P.bs]
    prm = O.Params(dens64, feat64, Ws64, bs64, P.box_min, P.box_max, P.act_shift)
    o, d, j = P.rays.o[sel], P.rays.d[sel], P.rays.jitter[sel]
    samp = O.sample_rays(o, d, j, P.box_min, P.box_max, P.step, P.max_samples, morton=False)
    ref = O.render_forward(prm, o, d, j, samp, P.step, P.bg)
    ref["_samp"] = samp
    if rgb_sel is not None:
        assert_close("rgb (checked rays)", rgb_sel, ref["rgb"], TOL32, TOL_LONG)
    gr = O.render_backward(prm, o, d, j, samp, P.step, P.bg, ref, g_sub)

    # ---- 1. finite differences of the oracle against its adjoint
    x = ref["cache"]["x"]
    ray_of = np.asarray(ref["_sample_ray"])
    i0, wts, offs = O.trilinear_corners(x, P.box_min, P.box_max, (n, n, n))
    pick = rng.choice(x.shape[0], n_entries, replace=False)
    corner = rng.integers(0, 8, n_entries)
    verts = i0[pick] + offs[corner]
    verts_all = i0[:, None, :] + offs[None, :, :]              # [S, 8, 3]
    rays_local = np.arange(len(sel))
    fd, adj, kinks = [], [], 0
    for e in range(n_entries):
        v = verts[e]
        hit = np.any(np.all(verts_all == v, axis=2) & (wts > 0), axis=1)
        rays = np.unique(ray_of[hit])
        if e < n_entries // 2:
            idx, arr, a = tuple(v), dens64, gr["density"][tuple(v)]
        else:
            ch = int(rng.integers(0, 12))
            idx, arr, a = (v[0], v[1], v[2], ch), feat64, gr["feat"][v[0], v[1], v[2], ch]
        f, kink = _central(prm, arr, idx, o, d, j, rays, g_sub, P)
        if kink:
            kinks += 1
            continue
        fd.append(f)
        adj.append(a)
    flat64 = mlp_flat_np(P.Ws, P.bs).astype(np.float64)
    shapes = [w.shape for w in P.Ws]
    offsets = np.cumsum([0] + [int(np.prod(s_)) + s_[0] for s_ in shapes])
    grad_flat = np.concatenate([gr["Ws"][0].ravel(), gr["bs"][0], gr["Ws"][1].ravel(), gr["bs"][1],
                                gr["Ws"][2].ravel(), gr["bs"][2]])
    for q in rng.choice(flat64.size, n_params, replace=False):
        layer = int(np.searchsorted(offsets, q, side="right") - 1)
        r = q - offsets[layer]
        nW = int(np.prod(shapes[layer]))
        arr, idx = (Ws64[layer], np.unravel_index(r, shapes[layer])) if r < nW else (bs64[layer], (r - nW,))
        f, kink = _central(prm, arr, idx, o, d, j, rays_local, g_sub, P)
        if kink:
            kinks += 1
            continue
        fd.append(f)
        adj.append(grad_flat[q])
    fd, adj = np.array(fd), np.array(adj)
    rel = np.abs(fd - adj) / np.maximum(np.abs(adj), 1e-3 * np.max(np.abs(adj)))
    print(f"  finite differences: {fd.size} checked, {kinks} kinks skipped, max rel err {rel.max():.3e}, "
          f"normwise {np.linalg.norm(fd - adj) / np.linalg.norm(adj):.3e}", flush=True)
    assert fd.size >= 0.8 * (n_entries + n_params)
    assert rel.max() <= 1e-6
    return prm, ref, gr


@pytest.mark.timeout(600)
def test_stress_finite_differences_and_adjoint(gpu_lib):
    import torch
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_F32
    P = synth.stress_config(0)
    P.act_shift = O.low_density_bias(P.extra["alpha_init"], P.extra["voxel"])
    B, n = P.rays.o.shape[0], P.density.shape[0]
    rng = np.random.default_rng(9)
    sel = np.sort(rng.choice(B, 64, replace=False))
    g_sub = rng.normal(size=(64, 3)).astype(F32).astype(np.float64)

    print(f"  GPU step: {n}^3 grids, bf16 features, {B} rays, <= {P.max_samples} samples/ray", flush=True)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    grid = api.Grid(to_dev(P.density), to_dev(P.feat), tuple(P.box_min), tuple(P.box_max), P.act_shift)
    grid.feat_shadow = grid.feat.to(torch.bfloat16).view(torch.int16).contiguous()
    flat = to_dev(mlp_flat_np(P.Ws, P.bs))
    s = api.sample_rays(to_dev(P.rays.o), to_dev(P.rays.d), to_dev(P.rays.jitter), P.box_min, P.box_max, P.step,
                        P.max_samples)
    out = api.render_fwd(grid, flat, s, P.bg, precision=DVGO_F32, use_shadow=True, want_depth_acc=False)
    g = np.zeros((B, 3), F32)
    g[sel] = g_sub
    gd, gf, gm = torch.zeros_like(grid.density), torch.zeros_like(grid.feat), torch.zeros_like(flat)
    api.render_bwd(grid, flat, s, out["log_t_end"], to_dev(g), gd, gf, gm, P.bg, precision=DVGO_F32,
                   use_shadow=True)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - base
    n_kept = int(s.n_kept.item())
    fixed = 4 * n ** 3 * (1 + 12) * 2 + 2 * n ** 3 * 12       # grids, their gradients, bf16 shadow
    store_all = fixed + n_kept * STORE_ALL_BYTES_PER_SAMPLE
    print(f"  evaluated samples {n_kept}; peak device memory {peak / 2**30:.2f} GiB "
          f"(grids+grads+shadow {fixed / 2**30:.2f} GiB); store-all estimate {store_all / 2**30:.2f} GiB "
          f"({STORE_ALL_BYTES_PER_SAMPLE} B/sample)", flush=True)
    assert peak < store_all
    rgb_sel = np_of(out["rgb"])[sel]
    gd, gf, gm = np_of(gd), np_of(gf), np_of(gm)
    del grid, s, out
    torch.cuda.empty_cache()

    prm, ref, gr = oracle_fd_check(P, sel, g_sub, rng, rgb_sel)

    # ---- 2. the GPU adjoint against the oracle's
    assert_close("grad_density", gd, gr["density"], TOL_LONG)
    budget, wb, frac = kink_budget(prm, ref, g_sub, ZETA, P.feat.shape, P.box_min, P.box_max)
    print(f"  samples with an ambiguous ReLU unit: {frac:.2e}", flush=True)
    check_grid_grad("grad_feat", gf, gr["feat"], budget, TOL_LONG)
    check_weight_grads(gm, gr["Ws"], gr["bs"], wb, TOL_LONG)


# Perturbations of the stored values: large enough that the float32
# forward's rounding, divided by the step, stays below the gradient; the
# truncation error this leaves is measured on the float64 oracle, and
# evaluations that cross a ReLU kink are skipped.
FD_H_DENSITY = 2.0 ** -4
FD_H_FEAT = 2.0 ** -4


def _perturbed(v, h, bf16):
    """The stored values nearest v + h and v - h as the grid holds them
    (float32, or bfloat16 for the feature shadow); both sides of the check
    evaluate at exactly these values and divide by their difference."""
    import torch
    dt = torch.bfloat16 if bf16 else torch.float32
    vp = float(torch.tensor(v + h, dtype=torch.float64).to(dt).double())
    vm = float(torch.tensor(v - h, dtype=torch.float64).to(dt).double())
    return vp, vm


def _set_stored(grid, idx, val, bf16):
    import torch
    if bf16:
        grid.feat_shadow[idx] = torch.tensor([val], dtype=torch.float32).to(torch.bfloat16).view(torch.int16)[0].item()
    else:
        grid.density[idx] = float(np.float32(val))


@pytest.mark.timeout(600)
def test_stress_fd_through_gpu_forwards(gpu_lib):
    """Central differences of the GPU's own float32 forward (bfloat16 feature
    storage, 256^3 grids) with the per-ray loss terms reduced in float64 on
    the GPU (dvgo_fd_reduce_f64), against the GPU adjoint, on density and
    feature entries touched by 64 rays of up to 800 samples.  The stored
    value moves to the nearest stored values to v +- 2^-4; a feature entry
    takes the vertex's channel with the largest gradient.  Per entry the
    allowed gap is the sum of: the central
    difference's own truncation at that step (the float64 oracle's
    difference minus its adjoint), the float32 forward's rounding (the
    measured per-ray colour errors of both GPU forwards against the float64
    oracle, weighted by |g| and divided by the step), and the adjoint's
    asserted accuracy (3e-5 of the gradient's maximum).  Entries whose two
    evaluations take different ReLU branches in the oracle are kinks and
    skipped (density entries never meet a ReLU): 24 density entries, and
    feature entries until 24 are free of kinks (at least 12 required).  The float64 reduction is
    also checked against the host's float64 sum of the same values."""
    import torch
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd._lib import DVGO_F32
    P = synth.stress_config(0)
    P.act_shift = O.low_density_bias(P.extra["alpha_init"], P.extra["voxel"])
    n = P.density.shape[0]
    rng = np.random.default_rng(19)
    sel = np.sort(rng.choice(P.rays.o.shape[0], 64, replace=False))
    o, d, j = P.rays.o[sel], P.rays.d[sel], P.rays.jitter[sel]
    g = rng.normal(size=(64, 3)).astype(F32)

    grid = api.Grid(to_dev(P.density), to_dev(P.feat), tuple(P.box_min), tuple(P.box_max), P.act_shift)
    grid.feat_shadow = grid.feat.to(torch.bfloat16).view(torch.int16).contiguous()
    flat = to_dev(mlp_flat_np(P.Ws, P.bs))
    s = api.sample_rays(to_dev(o), to_dev(d), to_dev(j), P.box_min, P.box_max, P.step, P.max_samples)
    g_dev = to_dev(g)

    def fwd():
        return api.render_fwd(grid, flat, s, P.bg, precision=DVGO_F32, use_shadow=True, want_depth_acc=False)

    out = fwd()
    gd, gf, gm = torch.zeros_like(grid.density), torch.zeros_like(grid.feat), torch.zeros_like(flat)
    api.render_bwd(grid, flat, s, out["log_t_end"], g_dev, gd, gf, gm, P.bg, precision=DVGO_F32, use_shadow=True)
    gd, gf = np_of(gd), np_of(gf)

    # float64 reduction against the host's
    rgb0 = np_of(out["rgb"])
    rays_all = to_dev(np.arange(64, dtype=np.int32))
    red = float(np_of(api.fd_reduce_f64(out["rgb"], g_dev, rays_all))[0])
    terms = g.astype(np.float64) * rgb0.astype(np.float64)
    assert abs(red - terms.sum()) <= 1e-14 * np.abs(terms).sum()
    assert float(np_of(api.fd_reduce_f64(out["rgb"], g_dev))[0]) == red

    dens64 = P.density.astype(np.float64)
    feat64 = O.bf16_round(P.feat)
    prm = O.Params(dens64, feat64, [w.astype(np.float64) for w in P.Ws], [b.astype(np.float64) for b in P.bs],
                   P.box_min, P.box_max, P.act_shift)
    samp = O.sample_rays(o, d, j, P.box_min, P.box_max, P.step, P.max_samples, morton=False)
    ref = O.render_forward(prm, o, d, j, samp, P.step, P.bg)
    gr = O.render_backward(prm, o, d, j, samp, P.step, P.bg, ref, g.astype(np.float64))
    x = ref["cache"]["x"]
    ray_of = np.asarray(ref["_sample_ray"])
    i0, wts, offs = O.trilinear_corners(x, P.box_min, P.box_max, (n, n, n))
    verts_all = i0[:, None, :] + offs[None, :, :]

    def orc(rays):
        sp = O.sample_rays(o[rays], d[rays], j[rays], P.box_min, P.box_max, P.step, P.max_samples, morton=False)
        rf = O.render_forward(prm, o[rays], d[rays], j[rays], sp, P.step, P.bg)
        mc = rf["cache"]["mcache"]
        return rf["rgb"], (mc["z1"] > 0, mc["z2"] > 0)

    # 24 density entries, and feature entries until 24 without a kink (at
    # most 150 candidates: at this step most feature entries meet one)
    want, n_cand = 24, 150
    picks = rng.choice(x.shape[0], want + n_cand, replace=False)
    corners = rng.integers(0, 8, want + n_cand)
    checked, kinks, worst = 0, 0, 0.0
    rels = {False: [], True: []}
    parts = {False: [], True: []}
    max_gd, max_gf = np.abs(gr["density"]).max(), np.abs(gr["feat"]).max()
    for e in range(want + n_cand):
        is_feat = e >= want
        if is_feat and len(rels[True]) >= want:
            break
        v = i0[picks[e]] + offs[corners[e]]
        if is_feat:
            ch = int(np.argmax(np.abs(gr["feat"][v[0], v[1], v[2]])))
            idx = (int(v[0]), int(v[1]), int(v[2]), ch)
            arr, a_orc, a_gpu, amax = feat64, gr["feat"][idx], gf[idx], max_gf
        else:
            idx = tuple(int(t) for t in v)
            arr, a_orc, a_gpu, amax = dens64, gr["density"][idx], gd[idx], max_gd
        v0 = float(arr[idx])
        vp, vm = _perturbed(v0, FD_H_FEAT if is_feat else FD_H_DENSITY, is_feat)
        hit = np.any(np.all(verts_all == v, axis=2) & (wts > 0), axis=1)
        rays = np.unique(ray_of[hit])
        rays_dev = to_dev(rays.astype(np.int32))
        # GPU: two forwards, float64 reduction over the touching rays
        _set_stored(grid, idx, vp, is_feat)
        out_p = fwd()
        lp = api.fd_reduce_f64(out_p["rgb"], g_dev, rays_dev)
        rgb_p = np_of(out_p["rgb"])[rays]
        _set_stored(grid, idx, vm, is_feat)
        out_m = fwd()
        lm = api.fd_reduce_f64(out_m["rgb"], g_dev, rays_dev)
        rgb_m = np_of(out_m["rgb"])[rays]
        _set_stored(grid, idx, v0, is_feat)
        fd_gpu = (float(np_of(lp)[0]) - float(np_of(lm)[0])) / (vp - vm)
        # oracle at the same stored values
        arr[idx] = vp
        orc_p, mp = orc(rays)
        arr[idx] = vm
        orc_m, mm = orc(rays)
        arr[idx] = v0
        if not (np.array_equal(mp[0], mm[0]) and np.array_equal(mp[1], mm[1])):
            kinks += 1
            continue
        gr_rays = np.abs(g[rays].astype(np.float64))
        fd_orc = float(np.sum(g[rays] * orc_p) - np.sum(g[rays] * orc_m)) / (vp - vm)
        noise = float(np.sum(gr_rays * (np.abs(rgb_p - orc_p) + np.abs(rgb_m - orc_m)))) / (vp - vm)
        trunc = abs(fd_orc - a_orc)
        allowed = trunc + noise + TOL_LONG * amax
        gap = abs(fd_gpu - a_gpu)
        worst = max(worst, gap / allowed)
        scale = max(abs(a_gpu), 1e-3 * amax)
        rels[is_feat].append(gap / scale)
        parts[is_feat].append((trunc / scale, noise / scale))
        assert gap <= allowed, (idx, fd_gpu, a_gpu, trunc, noise)
        checked += 1
    for is_feat, name in ((False, "density"), (True, "feature")):
        r, pt = np.array(rels[is_feat]), np.array(parts[is_feat])
        print(f"  {name}: {r.size} entries; |FD(GPU) - adjoint(GPU)| / |adjoint| median {np.median(r):.2e} "
              f"max {r.max():.2e}; of which truncation (median) {np.median(pt[:, 0]):.2e}, float32 forward "
              f"rounding (median) {np.median(pt[:, 1]):.2e}", flush=True)
    print(f"  {checked} entries checked, {kinks} kinks skipped; gap / allowed max {worst:.3f}", flush=True)
    assert len(rels[False]) == want and len(rels[True]) >= want // 2
