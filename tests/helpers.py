"""Shared helpers of the test-suite (comparison metrics, tensor plumbing)."""

import numpy as np


def to_dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def np_of(t):
    return t.detach().cpu().numpy()


def normwise(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((got - ref).ravel())
    return num / den if den > 0 else num


def maxrel(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.max(np.abs(ref))
    return np.max(np.abs(got - ref)) / den if den > 0 else np.max(np.abs(got - ref))


def report(name, got, ref):
    nw, mr = normwise(got, ref), maxrel(got, ref)
    print(f"  {name}: normwise {nw:.3e}  max/max {mr:.3e}", flush=True)
    return nw, mr


def mlp_flat_np(Ws, bs):
    return np.concatenate([Ws[0].ravel(), bs[0].ravel(), Ws[1].ravel(), bs[1].ravel(), Ws[2].ravel(),
                           bs[2].ravel()]).astype(np.float32)


def mlp_unflat(g, channels=12, hidden=128):
    """Split a flat network vector; its size gives the first layer's input
    width (39, or 72 with the encoded position)."""
    n_in = (np.asarray(g).size - (hidden + hidden * hidden + hidden + 3 * hidden + 3)) // hidden
    assert n_in in (channels + 27, channels + 33 + 27)
    i = 0
    out = []
    for shp in [(hidden, n_in), (hidden,), (hidden, hidden), (hidden,), (3, hidden), (3,)]:
        n = int(np.prod(shp))
        out.append(g[i:i + n].reshape(shp))
        i += n
    return out


def kink_budget(prm, ref, grad_rgb, zeta_rel, feat_shape, box_min, box_max, dc_extra=None):
    """Error budget from ReLU decisions that the arithmetic cannot resolve.

    A hidden unit whose oracle pre-activation z satisfies |z| <= zeta_rel *
    (sum of |terms| of its dot product + |bias|) may legitimately take the
    other branch in a float32 (or bfloat16) evaluation; only such units can
    flip.  With absolute adjoint magnitudes that hold for any masks,
    a2 = |dz3| |W3| (layer-2 units) and a1 = a2 |W2| (layer-1 units), any
    set of flips among a sample's ambiguous units changes
      dz2 by at most a2 on the ambiguous layer-2 units J (zero elsewhere),
      dz1 by at most D1 = (a2 . 1_J) |W2| + a1 . 1_I (I: ambiguous layer-1
        units; the first term is the change of dh1 that J's flips cause),
    hence that sample's contributions to dW1 and db1 by ||D1|| ||x|| and
    ||D1||, to dW2 and db2 by ||a2 . 1_J|| ||h1|| and ||a2 . 1_J||, and its
    feature gradient by D1 |W1f| per channel (the forward's change of a
    flipped unit's output is |z| <= zeta_rel of its terms, below the other
    bounds, and is not counted).  Budgets are twice these (either branch),
    summed over samples.  Returns (per-grid-entry feature budget, per-tensor
    weight budgets dict, fraction of samples with an ambiguous unit)."""
    import oracle as O
    cache = ref["cache"]
    mc = cache["mcache"]
    W1, W2, W3 = [np.asarray(w, np.float64) for w in prm.Ws]
    b1, b2, _ = [np.asarray(b, np.float64) for b in prm.bs]
    x, h1 = mc["x"], mc["h1"]
    s1 = np.abs(x) @ np.abs(W1).T + np.abs(b1)
    s2 = np.abs(h1) @ np.abs(W2).T + np.abs(b2)
    amb1 = np.abs(mc["z1"]) <= zeta_rel * s1
    amb2 = np.abs(mc["z2"]) <= zeta_rel * s2
    g = np.asarray(grad_rgb, np.float64)[np.asarray(ref_perm_slots(ref))]
    dc = cache["w"][:, None] * g
    if dc_extra is not None:     # direct colour gradients (the per-point rgb loss)
        dc = np.abs(dc) + np.abs(dc_extra)
    c = mc["c"]
    dz3 = np.abs(dc * c * (1 - c))
    a2 = dz3 @ np.abs(W3)
    a1 = a2 @ np.abs(W2)
    d2 = a2 * amb2
    d1 = d2 @ np.abs(W2) + a1 * amb1
    df = d1 @ np.abs(W1[:, :feat_shape[-1]])
    grid_budget = O.interp_scatter(feat_shape, cache["x"], box_min, box_max, 2.0 * df)
    n1, n2 = np.linalg.norm(d1, axis=1), np.linalg.norm(d2, axis=1)
    w_b = {
        "W1": 2.0 * np.sum(n1 * np.linalg.norm(x, axis=1)),
        "b1": 2.0 * np.sum(n1),
        "W2": 2.0 * np.sum(n2 * np.linalg.norm(h1, axis=1)),
        "b2": 2.0 * np.sum(n2),
        "W3": 0.0, "b3": 0.0,
    }
    return grid_budget, w_b, float((amb1.any(1) | amb2.any(1)).mean())


def ref_perm_slots(ref):
    """Ray id of every compact sample of an oracle forward (slot -> ray)."""
    return ref["_sample_ray"]


def check_grid_grad(name, got, ref, budget, tol, tol_max=None):
    """On entries no ambiguous sample touches: normwise <= tol and
    max|got - ref| <= tol_max * max|ref| (R23's two metrics; tol_max
    defaults to tol); elsewhere the difference must stay within the kink
    budget plus tol_max of the largest entry."""
    tol_max = tol if tol_max is None else tol_max
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    touched = budget > 0
    nw = normwise(got[~touched], ref[~touched])
    big = np.max(np.abs(ref))
    mr = float(np.max(np.abs(got - ref)[~touched]) / big) if (~touched).any() and big > 0 else 0.0
    slack = np.abs(got - ref)[touched] - budget[touched] - tol_max * big
    worst = float(slack.max()) if slack.size else -1.0
    print(f"  {name}: normwise(untouched) {nw:.3e}, max/max(untouched) {mr:.3e}, touched entries "
          f"{int(touched.sum())}, max excess over budget {worst:.3e}", flush=True)
    assert nw <= tol, name
    assert mr <= tol_max, name
    assert worst <= 0.0, name


def check_weight_grads(got_flat, ref_Ws, ref_bs, budgets, tol, tol_max=None):
    """Per network tensor: ||got - ref|| <= tol ||ref|| + budget and
    max|got - ref| <= tol_max max|ref| + budget (the kink budget bounds the
    2-norm of the kink part of the difference, so it bounds every entry)."""
    tol_max = tol if tol_max is None else tol_max
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    refs = [ref_Ws[0], ref_bs[0], ref_Ws[1], ref_bs[1], ref_Ws[2], ref_bs[2]]
    for name, a, b in zip(names, mlp_unflat(np.asarray(got_flat)), refs):
        d = np.asarray(a, np.float64) - b
        err = np.linalg.norm(d)
        allowed = tol * np.linalg.norm(b) + budgets[name]
        emax, allowed_max = np.max(np.abs(d)), tol_max * np.max(np.abs(b)) + budgets[name]
        print(f"  {name}: normwise {err / np.linalg.norm(b):.3e} (allowed {allowed / np.linalg.norm(b):.3e}), "
              f"max/max {emax / np.max(np.abs(b)):.3e} (allowed {allowed_max / np.max(np.abs(b)):.3e})", flush=True)
        assert err <= allowed, name
        assert emax <= allowed_max, name


def assert_close(name, got, ref, tol, tol_max=None):
    """R23's two metrics for one output tensor: normwise relative error and
    max|got - ref| / max|ref|, each held to its bound (tol_max defaults to
    tol)."""
    nw, mr = report(name, got, ref)
    assert nw <= tol, f"{name}: normwise {nw:.3e} > {tol:.1e}"
    lim = tol if tol_max is None else tol_max
    assert mr <= lim, f"{name}: max/max {mr:.3e} > {lim:.1e}"
    return nw, mr


def f32_hyper(lr, betas, eps):
    """The Adam hyperparameters as the library receives them (float32), as
    exact float64 inputs of the oracle."""
    f = lambda x: float(np.float32(x))
    return f(lr), f(betas[0]), f(betas[1]), f(eps)


def check_adam_entries(name, p1, m1, v1, p0, m0, v0, g_ref, err_g, lr, t, betas=(0.9, 0.999), eps=1e-8,
                       untouched=None):
    """One Adam step of the library (p1, m1, v1 from p0, m0, v0) against the
    oracle's step taken with the oracle's gradient g_ref, entry by entry.

    err_g bounds |g_gpu - g_ref| per entry (scalar or array).  Then, with
    u = 2^-24 the float32 unit roundoff,
      |m1 - m_ref| <= (1-b1)(err_g + 2u|g_ref|) + 2 ulp(m_ref),
      |v1 - v_ref| <= (1-b2)(2|g_ref| err_g + err_g^2 + 4u g_ref^2) + 2 ulp(v_ref),
      |p1 - p_ref| <= max over g in [g_ref - err_g, g_ref + err_g] of
                      |A(g) - A(g_ref)| (A the oracle's update, evaluated at
                      both ends and the centre) + 1e-6 |A(g_ref)| + ulp(p_ref),
    the learning-rate- and eps-aware bound of an update that is
    ill-conditioned where |g| is near eps.  Entries of ``untouched`` (no
    sample reaches them on either side) whose moments are zero must keep p,
    m and v bit for bit."""
    import oracle as O
    lr_, b1, b2, ep = f32_hyper(lr, betas, eps)
    p0d, m0d, v0d = (np.asarray(a, np.float64) for a in (p0, m0, v0))
    g = np.asarray(g_ref, np.float64)
    e = np.broadcast_to(np.asarray(err_g, np.float64), g.shape)
    p_ref, m_ref, v_ref = O.adam_step(p0d, g, m0d, v0d, lr_, b1, b2, ep, t)
    ulp = lambda a: np.spacing(np.abs(a).astype(np.float32)).astype(np.float64)
    p1, m1, v1 = (np.asarray(a, np.float64) for a in (p1, m1, v1))
    u = 2.0 ** -24
    dm = np.abs(m1 - m_ref) - ((1 - b1) * (e + 2 * u * np.abs(g)) + 2 * ulp(m_ref))
    dv = np.abs(v1 - v_ref) - ((1 - b2) * (2 * np.abs(g) * e + e * e + 4 * u * g * g) + 2 * ulp(v_ref))
    upd = p0d - p_ref
    spread = np.zeros_like(upd)
    for s in (-1.0, 1.0):
        ps, _, _ = O.adam_step(p0d, g + s * e, m0d, v0d, lr_, b1, b2, ep, t)
        spread = np.maximum(spread, np.abs((p0d - ps) - upd))
    dp = np.abs(p1 - p_ref) - (spread + 1e-6 * np.abs(upd) + ulp(p_ref))
    idle = np.zeros(g.shape, bool) if untouched is None else \
        (np.broadcast_to(np.asarray(untouched, bool), g.shape) & (m0d == 0) & (v0d == 0))
    assert not np.any(g[idle]), f"{name}: an untouched entry has a gradient"
    print(f"  {name}: {g.size} entries, idle {int(idle.sum())}; worst excess m {dm.max():.2e} "
          f"v {dv.max():.2e} p {dp.max():.2e}; normwise m {normwise(m1, m_ref):.2e} "
          f"v {normwise(v1, v_ref):.2e} update {normwise(p0d - p1, upd):.2e}", flush=True)
    assert dm.max() <= 0, f"{name}: m"
    assert dv.max() <= 0, f"{name}: v"
    assert dp.max() <= 0, f"{name}: p"
    assert np.array_equal(p1[idle], p0d[idle]), f"{name}: idle p"
    assert not np.any(m1[idle]) and not np.any(v1[idle]), f"{name}: idle moments"
    return p_ref, m_ref, v_ref


def untouched_vertices(x, box_min, box_max, shape):
    """Vertices that no sample can reach in either precision: outside the
    corners of every sample's cell widened by one cell on each side (a
    float32 cell index may differ from the float64 one by one at a cell
    face).  x: float64 sample points [S, 3]; returns bool [nx, ny, nz]."""
    import oracle as O
    n = np.asarray(shape[:3])
    i0, _, _ = O.trilinear_corners(x, box_min, box_max, n)
    hit = np.zeros(tuple(n), bool)
    for dx in range(-1, 3):
        for dy in range(-1, 3):
            for dz in range(-1, 3):
                ii = np.clip(i0 + np.array([dx, dy, dz]), 0, n - 1)
                hit[ii[:, 0], ii[:, 1], ii[:, 2]] = True
    return ~hit


def density_grad_condition(ref, grad_rgb, step, act_shift, bg):
    """Per-sample running-error scale of the density adjoint: the sum of the
    absolute values of the terms whose difference forms dL/draw_k,
      step * sigmoid(raw_k + b) * sum_ch |g_ch| (T_{k+1} |v_ch| + |S_ch,k+1|),
    with v = (c, t, 1) and S_{k+1} the suffix sum behind sample k (the
    oracle's forward cache; loss gradient on rgb only).  A float32
    evaluation of that difference and of the sums feeding it errs by at most
    about n u times this scale for n terms along the ray."""
    import oracle as O
    cache = ref["cache"]
    slot, col, kmax = cache["slot"], cache["col"], cache["kmax"]
    B = cache["T_excl"].shape[0]
    n = slot.size
    v = np.zeros((n, 4))
    v[:, :3] = np.abs(cache["c"])
    v[:, 3] = np.abs(cache["t"])
    Wv = np.zeros((B, kmax, 4))
    Wv[slot, col] = cache["w"][:, None] * v
    rev = np.cumsum(Wv[:, ::-1, :], axis=1)[:, ::-1, :]
    S_after = np.concatenate([rev[:, 1:, :], np.zeros((B, 1, 4))], axis=1)
    t_end = np.asarray(ref["t_end"], np.float64)[np.asarray(ref["_sample_ray"], np.int64)]
    S = S_after[slot, col]
    S[:, :3] += t_end[:, None] * np.abs(np.asarray(bg, np.float64))[None, :]
    T_next = cache["T_excl"][slot, col] * (1.0 - cache["alpha"])
    gs = np.abs(np.asarray(grad_rgb, np.float64))[np.asarray(ref["_sample_ray"], np.int64)]
    terms = np.sum(gs * (T_next[:, None] * v[:, :3] + S[:, :3]), axis=1)
    return step * O.sigmoid(cache["raw"] + act_shift) * terms


def feat_grad_condition(prm, ref, grad_rgb, dc_extra=None):
    """Per-sample, per-channel scale of the feature adjoint's terms: with
    dz3 = dc c (1 - c) and absolute values throughout,
      U = ((|dz3| |W3|) |W2|) |W1f|,
    which bounds the sum of the absolute values of every product term that
    forms the sample's dL/df (ReLU masks only remove terms).  A float32
    evaluation (contractions of K <= 128 terms, then the vertex's sum over
    its samples) errs by at most about (K_total + n) u times the vertex's
    share of U."""
    cache = ref["cache"]
    mc = cache["mcache"]
    W1, W2, W3 = [np.abs(np.asarray(w, np.float64)) for w in prm.Ws]
    g = np.asarray(grad_rgb, np.float64)[np.asarray(ref["_sample_ray"], np.int64)]
    c = mc["c"]
    dc = np.abs(cache["w"][:, None] * g)
    if dc_extra is not None:
        dc = dc + np.abs(dc_extra)
    dz3 = dc * c * (1 - c)
    return ((dz3 @ W3) @ W2) @ W1[:, :prm.feat.shape[-1]]


def samples_per_vertex(x, box_min, box_max, shape):
    """Number of samples whose cell has the vertex as a corner, [nx, ny, nz]."""
    import oracle as O
    n = np.asarray(shape[:3])
    i0, _, offs = O.trilinear_corners(x, box_min, box_max, n)
    cnt = np.zeros(tuple(n), np.int64)
    for c in range(8):
        ii = i0 + offs[c]
        np.add.at(cnt, (ii[:, 0], ii[:, 1], ii[:, 2]), 1)
    return cnt
