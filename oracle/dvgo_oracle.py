"""FP64 NumPy oracle for the fine-stage per-ray training step of DVGO.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.

Every function cites the part of the paper it follows.  Two kinds of
arithmetic appear:

* Discrete decisions (ray validity, per-ray sample counts, which samples the
  coarse mask keeps, Morton keys, the proposal's segment mask) are taken in
  an explicit float32 recipe - every operation rounded to float32 in the
  order written, no fused multiply-add - because those decisions must match
  a float32 GPU implementation bit for bit.
* Everything continuous (interpolation, activations, compositing, the MLP,
  the loss, the adjoint, Adam) is float64, evaluated from the float32 input
  values.

Parity status: every public function is pinned by tests in
``tests/test_oracle_*.py`` against closed forms, worked numbers printed in
the paper, library routines, autograd, finite differences or brute force.
"""

from __future__ import annotations

import math

import numpy as np

F32 = np.float32
NSEG = 32                     # proposal segments per ray
MORTON_BITS = 5               # Morton quantisation bits per axis
MORTON_INVALID = 1 << (3 * MORTON_BITS)


# ===========================================================================
# 1. Discrete sampler, float32 recipe
# ===========================================================================
def ray_box_clip(o, d, box_min, box_max):
    """Ray-box clipping of the fine-stage sampler (Sec. 4.2, "Fine-stage
    points sampling"): the near and far bounds become the two ends of the
    ray-box intersection, the near bound is not moved when the origin is
    already inside the box (t_near = max(t_enter, 0)), and rays that miss the
    box are dropped (valid = 0).

    Slab test in float32: per axis inv = 1/d, t0 = (min - o)*inv,
    t1 = (max - o)*inv; t_enter = max_i fmin(t0,t1), t_exit = min_i
    fmax(t0,t1).  An axis with d = 0 imposes no bound when min <= o <= max and
    misses otherwise.  valid iff t_near < t_far (strict).  Invalid rays get
    t_near = t_far = 0.
    """
    o = np.asarray(o, F32)
    d = np.asarray(d, F32)
    B = o.shape[0]
    t_enter = np.full(B, -np.inf, F32)
    t_exit = np.full(B, np.inf, F32)
    miss = np.zeros(B, bool)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        for i in range(3):
            di, oi = d[:, i], o[:, i]
            lo_b, hi_b = F32(box_min[i]), F32(box_max[i])
            zero = di == 0
            inv = F32(1.0) / np.where(zero, F32(1.0), di)
            t0 = (lo_b - oi) * inv
            t1 = (hi_b - oi) * inv
            lo = np.where(zero, F32(-np.inf), np.fmin(t0, t1))
            hi = np.where(zero, F32(np.inf), np.fmax(t0, t1))
            miss |= zero & ((oi < lo_b) | (oi > hi_b))
            t_enter = np.fmax(t_enter, lo)
            t_exit = np.fmin(t_exit, hi)
    t_near = np.fmax(t_enter, F32(0.0))
    t_far = t_exit
    valid = (~miss) & (t_near < t_far)
    t_near = np.where(valid, t_near, F32(0.0)).astype(F32)
    t_far = np.where(valid, t_far, F32(0.0)).astype(F32)
    return t_near, t_far, valid


def sample_t(t_near, jitter, k, step):
    """Distance of uniform sample k (Eq. coarse_sample with the training
    jitter of the supplementary implementation details): with a unit
    direction, t_k = t_near + (k + p) * delta, three float32 roundings in that
    order (k + p, then * delta, then t_near +)."""
    k = np.asarray(k)
    kp = k.astype(F32) + np.asarray(jitter, F32)
    return (np.asarray(t_near, F32) + (kp * F32(step)).astype(F32)).astype(F32)


def uniform_count(t_near, t_far, valid, jitter, step, max_samples):
    """Number of uniform samples per ray (Eq. coarse_sample, index range
    clipped to the box): N_r = #{k >= 0 : t_k < t_far, k < max_samples},
    counted by brute-force enumeration of every k.  Invalid rays have 0."""
    B = t_near.shape[0]
    p = np.zeros(B, F32) if jitter is None else np.asarray(jitter, F32)
    k = np.arange(max_samples, dtype=np.int64)[None, :]
    t = sample_t(t_near[:, None], p[:, None], k, step)
    inside = t < t_far[:, None]
    # t_k is non-decreasing in k, so the kept k form a prefix; count it
    n = inside.sum(axis=1).astype(np.int32)
    return np.where(valid, n, 0).astype(np.int32)


def sample_x(o, d, t):
    """Sample position x = o + t * d per component (multiply, then add),
    float32."""
    return (np.asarray(o, F32) + (np.asarray(t, F32)[..., None] * np.asarray(d, F32))
            .astype(F32)).astype(F32)


def coarse_raw_threshold(tau, step, act_shift=0.0):
    """Free-space test of Sec. 4.2 ("Known free space and unknown space"):
    a point is known-free when alpha(softplus(raw + b), delta) < tau.  Both
    activations increase with raw, so alpha >= tau  <=>  raw >= thr with
    thr = softplus^{-1}(-log(1 - tau)/delta) - b = log(expm1(-log1p(-tau)/delta)) - b.
    Returned as the largest float32 not above the float64 threshold, so the
    float32 comparison never drops a point the exact test keeps."""
    sig = -math.log1p(-tau) / step
    thr = math.log(math.expm1(sig)) - act_shift
    t32 = F32(thr)
    if float(t32) > thr:
        t32 = np.nextafter(t32, F32(-np.inf))
    return F32(t32)


def coarse_cell_bits(raw, raw_thr):
    """Per-cell keep bits of the frozen coarse density grid (Sec. 4.2,
    "Free space skipping", first rule).  A cell is kept when the largest of
    its 8 corner raw values reaches ``raw_thr``: trilinear interpolation is a
    convex combination of the corners and the activations are increasing, so
    every point whose own post-activated coarse alpha reaches tau lies in a
    kept cell.  Bit c of word c>>5 (c = (ix*(ny-1)+iy)*(nz-1)+iz) is cell c."""
    raw = np.asarray(raw, F32)
    m = raw[:-1, :-1, :-1]
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                m = np.maximum(m, raw[dx:raw.shape[0] - 1 + dx, dy:raw.shape[1] - 1 + dy,
                                      dz:raw.shape[2] - 1 + dz])
    keep = (m >= F32(raw_thr)).ravel()
    nwords = (keep.size + 31) // 32
    bits = np.zeros(nwords * 32, np.uint64)
    bits[:keep.size] = keep
    words = (bits.reshape(nwords, 32) << np.arange(32, dtype=np.uint64)).sum(axis=1)
    return words.astype(np.uint32)


def coarse_cell_index(x, cmin, cmax, cn):
    """Cell containing a float32 point: clamp(floor((x - min) * s), 0, n-2)
    per axis with s = (n-1)/(max-min) rounded once to float32."""
    x = np.asarray(x, F32)
    idx = []
    for i in range(3):
        s = F32(F32(cn[i] - 1) / F32(F32(cmax[i]) - F32(cmin[i])))
        u = ((x[..., i] - F32(cmin[i])).astype(F32) * s).astype(F32)
        fi = np.floor(u).astype(np.int64)
        idx.append(np.clip(fi, 0, cn[i] - 2))
    return idx


def coarse_keep(x, cmin, cmax, cn, bits):
    """Look up the coarse keep bit of the cell holding each point."""
    ix, iy, iz = coarse_cell_index(x, cmin, cmax, cn)
    c = (ix * (cn[1] - 1) + iy) * (cn[2] - 1) + iz
    return ((bits[c >> 5] >> (c & 31).astype(np.uint32)) & 1).astype(bool)


def trilinear_f32(grid, x, box_min, box_max):
    """Trilinear interpolation of a float32 vertex grid [nx,ny,nz] in an
    explicit float32 recipe (every operation rounded to float32 in the order
    written, no fused multiply-add), for discrete decisions taken on an
    interpolated value: per axis scale = (n-1)/(max-min) rounded once,
    u = (x - min) * scale, fl = clamp(floor(u), 0, n-2), f = clamp(u - fl,
    0, 1), g = (1 - f, f); corner c = (c>>2 &1, c>>1 &1, c &1) has weight
    (gx * gy) * gz; the value is w_0 V_0 + w_1 V_1 + ... + w_7 V_7, added
    one product at a time in corner order."""
    g = np.asarray(grid, F32)
    x = np.asarray(x, F32)
    n = g.shape
    i0, gw = [], []
    for i in range(3):
        s = F32(F32(n[i] - 1) / F32(F32(box_max[i]) - F32(box_min[i])))
        u = ((x[..., i] - F32(box_min[i])).astype(F32) * s).astype(F32)
        fl = np.clip(np.floor(u), F32(0.0), F32(n[i] - 2)).astype(F32)
        f = np.clip((u - fl).astype(F32), F32(0.0), F32(1.0)).astype(F32)
        i0.append(fl.astype(np.int64))
        gw.append(((F32(1.0) - f).astype(F32), f))
    val = None
    for c in range(8):
        bx, by, bz = (c >> 2) & 1, (c >> 1) & 1, c & 1
        w = ((gw[0][bx] * gw[1][by]).astype(F32) * gw[2][bz]).astype(F32)
        term = (w * g[i0[0] + bx, i0[1] + by, i0[2] + bz]).astype(F32)
        val = term if val is None else (val + term).astype(F32)
    return val


def fine_keep(x, density, box_min, box_max, raw_thr):
    """Second free-space rule of Sec. 4.2 ("Free space skipping"): a sample
    in unknown space is skipped when its post-activated alpha from the fine
    density grid is below tau^(f).  Both activations increase with the raw
    value, so the test is raw >= raw_thr (``coarse_raw_threshold`` of tau^(f),
    the fine step and the fine shift), with raw from ``trilinear_f32``."""
    return trilinear_f32(density, x, box_min, box_max) >= F32(raw_thr)


def segment_of(k, n_uniform):
    """Equal-count proposal segment of sample k on a ray with N_r uniform
    samples: floor(32 k / N_r), integer arithmetic."""
    return (NSEG * np.asarray(k, np.int64)) // np.maximum(np.asarray(n_uniform, np.int64), 1)


def morton_keys(o, d, t_near, t_far, valid, box_min, box_max):
    """Spatial sort key of a ray: the 5-bit-per-axis Morton code of its
    in-box segment midpoint.  float32 recipe: tm = (t_near + t_far) * 0.5,
    m = o + tm * d, q = clamp(floor((m - min) * (32/(max-min))), 0, 31);
    bits interleaved x (most significant), y, z.  Invalid rays get the key
    2^15, after every valid key."""
    tm = ((np.asarray(t_near, F32) + np.asarray(t_far, F32)).astype(F32) * F32(0.5)).astype(F32)
    m = sample_x(o, d, tm)
    q = []
    for i in range(3):
        s = F32(F32(1 << MORTON_BITS) / F32(F32(box_max[i]) - F32(box_min[i])))
        u = ((m[:, i] - F32(box_min[i])).astype(F32) * s).astype(F32)
        q.append(np.clip(np.floor(u).astype(np.int64), 0, (1 << MORTON_BITS) - 1))
    key = np.zeros(o.shape[0], np.int64)
    for b in range(MORTON_BITS):
        key |= ((q[0] >> b) & 1) << (3 * b + 2)
        key |= ((q[1] >> b) & 1) << (3 * b + 1)
        key |= ((q[2] >> b) & 1) << (3 * b)
    key = np.where(valid, key, MORTON_INVALID)
    return key.astype(np.uint32)


def sample_rays(o, d, jitter, box_min, box_max, step, max_samples, coarse=None,
                seg_mask=None, morton=False, fine=None):
    """The fine-stage sampler (Sec. 4.2 "Fine-stage points sampling" and
    "Free space skipping"; Eq. coarse_sample): clip, count the uniform
    samples, keep those whose coarse cell bit (and, when given, whose
    proposal segment bit) is set and, with ``fine``, that pass the second
    rule (``fine_keep``), and list them per ray in ascending k.

    ``coarse`` is (bits, cmin, cmax, cn) or None; ``fine`` is
    (density [nx,ny,nz] float32 on the sampling box, raw_thr) or None.  The ray order of the
    compact list is the identity, or ascending (Morton key, ray id) when
    ``morton``.  Returns a dict of numpy arrays.
    """
    o = np.asarray(o, F32)
    d = np.asarray(d, F32)
    B = o.shape[0]
    p = np.zeros(B, F32) if jitter is None else np.asarray(jitter, F32)
    t_near, t_far, valid = ray_box_clip(o, d, box_min, box_max)
    n_uni = uniform_count(t_near, t_far, valid, p, step, max_samples)
    if morton:
        keys = morton_keys(o, d, t_near, t_far, valid, box_min, box_max)
        perm = np.lexsort((np.arange(B), keys)).astype(np.int32)
    else:
        keys = None
        perm = np.arange(B, dtype=np.int32)
    counts = np.zeros(B, np.int64)
    ks_per_ray = []
    for slot in range(B):
        r = perm[slot]
        k = np.arange(n_uni[r], dtype=np.int64)
        keep = np.ones(k.size, bool)
        if k.size and coarse is not None:
            bits, cmin, cmax, cn = coarse
            x = sample_x(o[r][None, :], d[r][None, :], sample_t(t_near[r], p[r], k, step))
            keep &= coarse_keep(x, cmin, cmax, cn, bits)
        if k.size and seg_mask is not None:
            seg = segment_of(k, n_uni[r])
            keep &= ((np.uint64(seg_mask[r]) >> seg.astype(np.uint64)) & np.uint64(1)).astype(bool)
        if k.size and fine is not None:
            x = sample_x(o[r][None, :], d[r][None, :], sample_t(t_near[r], p[r], k, step))
            keep &= fine_keep(x, fine[0], box_min, box_max, fine[1])
        ks_per_ray.append(k[keep])
        counts[slot] = keep.sum()
    ray_offset = np.zeros(B + 1, np.int64)
    ray_offset[1:] = np.cumsum(counts)
    sample_k = np.concatenate(ks_per_ray) if B else np.zeros(0, np.int64)
    sample_ray = np.repeat(perm.astype(np.int64), counts)
    return dict(t_near=t_near, t_far=t_far, valid=valid, n_uniform=n_uni, perm=perm,
                keys=keys, ray_offset=ray_offset.astype(np.int32),
                sample_ray=sample_ray.astype(np.int32), sample_k=sample_k.astype(np.int32))


# ===========================================================================
# 2. Continuous part, float64
# ===========================================================================
def trilinear_corners(x, box_min, box_max, n):
    """Trilinear interpolation weights on a vertex grid of n[i] points per
    axis spanning the box (Eq. interp, trilinear by default).
    u = (x - min)/(max - min)*(n-1), i0 = clamp(floor(u), 0, n-2),
    f = clamp(u - i0, 0, 1).  Returns (i0 [S,3] int, weights [S,8],
    corner offsets [8,3]) with corner c = (c>>2 &1, c>>1 &1, c &1)."""
    x = np.asarray(x, np.float64)
    bmin = np.asarray(box_min, np.float64)
    bmax = np.asarray(box_max, np.float64)
    nn = np.asarray(n, np.float64)
    u = (x - bmin) / (bmax - bmin) * (nn - 1)
    i0 = np.clip(np.floor(u), 0, nn - 2).astype(np.int64)
    f = np.clip(u - i0, 0.0, 1.0)
    offs = np.array([[(c >> 2) & 1, (c >> 1) & 1, c & 1] for c in range(8)], np.int64)
    w = np.ones((x.shape[0], 8))
    for c in range(8):
        for a in range(3):
            w[:, c] *= f[:, a] if offs[c, a] else (1.0 - f[:, a])
    return i0, w, offs


def interp(grid, x, box_min, box_max):
    """interp(x, V) of Eq. interp for a channel-last grid [nx,ny,nz,C] (or
    [nx,ny,nz]); float64 result [S,C] (or [S])."""
    g = np.asarray(grid, np.float64)
    squeeze = g.ndim == 3
    if squeeze:
        g = g[..., None]
    i0, w, offs = trilinear_corners(x, box_min, box_max, g.shape[:3])
    out = np.zeros((w.shape[0], g.shape[3]))
    for c in range(8):
        ii = i0 + offs[c]
        out += w[:, c:c + 1] * g[ii[:, 0], ii[:, 1], ii[:, 2]]
    return out[:, 0] if squeeze else out


def interp_scatter(shape, x, box_min, box_max, g):
    """Adjoint of ``interp``: scatter-add g [S,C] (or [S]) into a zero grid
    of ``shape`` with the trilinear weights."""
    out = np.zeros(shape, np.float64)
    o3 = out if out.ndim == 4 else out[..., None]
    gg = np.asarray(g, np.float64)
    gg = gg if gg.ndim == 2 else gg[:, None]
    i0, w, offs = trilinear_corners(x, box_min, box_max, shape[:3])
    for c in range(8):
        ii = i0 + offs[c]
        np.add.at(o3, (ii[:, 0], ii[:, 1], ii[:, 2]), w[:, c:c + 1] * gg)
    return out


def softplus(x):
    """log(1 + exp(x)), evaluated stably (Eq. density_activation)."""
    x = np.asarray(x, np.float64)
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def sigmoid(x):
    x = np.asarray(x, np.float64)
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def density_to_alpha(sigma, delta):
    """alpha = 1 - exp(-sigma * delta) (Eq. density_2_alpha)."""
    return 1.0 - np.exp(-np.asarray(sigma, np.float64) * delta)


def post_activated_alpha(raw, act_shift, delta):
    """Post-activation (Eq. post_activation): alpha(softplus(interp + b))."""
    return density_to_alpha(softplus(np.asarray(raw, np.float64) + act_shift), delta)


def low_density_bias(alpha_init, voxel):
    """Shift b of the low-density initialisation (Eq. low_density_init):
    b = log((1 - alpha_init)^(-1/s) - 1)."""
    return math.log((1.0 - alpha_init) ** (-1.0 / voxel) - 1.0)


def positional_encoding(d, n_freq=4):
    """Positional embedding of the view direction (Sec. 3, NeRF's encoding;
    k_d = 4 in the supplementary details): [d, sin(2^0 d), cos(2^0 d), ...,
    sin(2^{k-1} d), cos(2^{k-1} d)], 3 + 6k values, no pi factor."""
    d = np.asarray(d, np.float64)
    parts = [d]
    for k in range(n_freq):
        parts.append(np.sin(d * (2.0 ** k)))
        parts.append(np.cos(d * (2.0 ** k)))
    return np.concatenate(parts, axis=-1)


def box_coordinates(x, box_min, box_max):
    """Position in the box's own coordinates, [-1, 1] on each axis:
    u = (x - centre) / half-extent (the input of the position encoding)."""
    lo = np.asarray(box_min, np.float64)
    hi = np.asarray(box_max, np.float64)
    return (np.asarray(x, np.float64) - 0.5 * (lo + hi)) / (0.5 * (hi - lo))


def bf16_round(x):
    """Round float32 values to bfloat16 (round to nearest, ties to even) and
    return them as float64: keep the top 16 bits of the float32 pattern after
    adding 0x7FFF plus the lowest kept bit."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(a), out, a.astype(np.float64))


def mlp_forward(Ws, bs, x, bf16=False, n_feat=12):
    """The shallow colour MLP of Eq. fine_queries: two ReLU hidden layers of
    128, sigmoid output (Sec. 3 output activation).  Ws[l] is [out][in].

    bf16=True evaluates the bfloat16 form: the inputs of every product
    (feature part of the first-layer input, hidden activations, weights) are
    rounded to bfloat16 and the products summed exactly; the view-encoding
    part of the first layer and the biases stay unrounded."""
    W1, W2, W3 = [np.asarray(w, np.float64) for w in Ws]
    b1, b2, b3 = [np.asarray(b, np.float64) for b in bs]
    if bf16:
        z1 = bf16_round(x[:, :n_feat]) @ bf16_round(W1[:, :n_feat]).T + (x[:, n_feat:] @ W1[:, n_feat:].T + b1)
    else:
        z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = (bf16_round(h1) @ bf16_round(W2).T if bf16 else h1 @ W2.T) + b2
    h2 = np.maximum(z2, 0.0)
    z3 = (bf16_round(h2) @ bf16_round(W3).T if bf16 else h2 @ W3.T) + b3
    c = sigmoid(z3)
    return c, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, c=c, bf16=bf16, n_feat=n_feat)


def mlp_backward(Ws, cache, dc):
    """Reverse-mode derivative of ``mlp_forward`` for output gradient dc.
    ReLU'(0) is taken as 0.  Returns (dx, [dW1,dW2,dW3], [db1,db2,db3]); dx
    holds only the feature part in the bfloat16 form.

    bfloat16 form: every backward product takes bfloat16-rounded weights
    and bfloat16-rounded propagated gradients (dz3 into W3^T, dz2 into W2^T,
    dz1 into W1^T, and both factors of every weight gradient); bias
    gradients sum the rounded dz (dz3 unrounded)."""
    W1, W2, W3 = [np.asarray(w, np.float64) for w in Ws]
    c = cache["c"]
    dz3 = dc * c * (1.0 - c)
    if not cache.get("bf16"):
        dW3 = dz3.T @ cache["h2"]
        db3 = dz3.sum(0)
        dz2 = (dz3 @ W3) * (cache["z2"] > 0)
        dW2 = dz2.T @ cache["h1"]
        db2 = dz2.sum(0)
        dz1 = (dz2 @ W2) * (cache["z1"] > 0)
        dW1 = dz1.T @ cache["x"]
        db1 = dz1.sum(0)
        dx = dz1 @ W1
        return dx, [dW1, dW2, dW3], [db1, db2, db3]
    nf = cache["n_feat"]
    bf = bf16_round
    dW3 = bf(dz3).T @ bf(cache["h2"])
    db3 = dz3.sum(0)
    dz2 = (bf(dz3) @ bf(W3)) * (cache["z2"] > 0)
    dW2 = bf(dz2).T @ bf(cache["h1"])
    db2 = bf(dz2).sum(0)
    dz1 = (bf(dz2) @ bf(W2)) * (cache["z1"] > 0)
    dW1 = bf(dz1).T @ bf(cache["x"])
    db1 = bf(dz1).sum(0)
    dx = bf(dz1) @ bf(W1[:, :nf])
    return dx, [dW1, dW2, dW3], [db1, db2, db3]


def _sample_geometry(o, d, jitter, t_near, sample_ray, sample_k, step):
    """float32 t and x of every listed sample, upcast to float64."""
    B = o.shape[0]
    p = np.zeros(B, F32) if jitter is None else np.asarray(jitter, F32)
    r = np.asarray(sample_ray, np.int64)
    t32 = sample_t(t_near[r], p[r], sample_k, step)
    x = np.asarray(o, F32)[r].astype(np.float64) + t32.astype(np.float64)[:, None] * \
        np.asarray(d, F32)[r].astype(np.float64)
    return t32.astype(np.float64), x


def _padded(ray_offset, n):
    """Row/column of each compact sample in a [B, Kmax] per-ray layout."""
    ro = np.asarray(ray_offset, np.int64)
    counts = np.diff(ro)
    kmax = int(counts.max()) if counts.size and counts.max() > 0 else 1
    slot = np.repeat(np.arange(counts.size), counts)
    col = np.arange(n) - np.repeat(ro[:-1], counts)
    return slot, col, kmax


class Params:
    """Scene representation: the fine stage's density grid, feature grid and
    MLP (Eq. fine_queries), or the coarse stage's density grid and
    view-invariant colour grid (Eq. coarse_queries: feat holds V^(rgb), Ws
    and bs are None, the colour is sigmoid(interp(x, V^(rgb))), the output
    activation of Sec. 3), with the softplus shift b and the AABB.  With
    pe_x = k_x > 0 the colour MLP also takes the encoded query position
    (Eq. fine_queries with k_x frequencies): its input is [interp(x, V_feat),
    PE_{k_x}(u), PE_4(d)], u the position in box coordinates."""

    def __init__(self, density, feat, Ws, bs, box_min, box_max, act_shift, mlp_bf16=False, pe_x=0):
        self.mlp_bf16 = bool(mlp_bf16)
        self.pe_x = int(pe_x)       # frequencies of the position encoding in the MLP input (0: none)
        self.density = np.asarray(density)
        self.feat = np.asarray(feat)
        self.grid_colour = Ws is None
        self.Ws = None if Ws is None else [np.asarray(w) for w in Ws]
        self.bs = None if bs is None else [np.asarray(b) for b in bs]
        self.box_min = np.asarray(box_min, F32)
        self.box_max = np.asarray(box_max, F32)
        self.act_shift = float(act_shift)


def render_forward(P: Params, o, d, jitter, samp, step, bg, with_color=True):
    """Forward volume rendering of every ray (Eq. volume_rendering with
    Eq. fine_queries and the post-activated density of Eq. post_activation).

    For each ray, over its kept samples in ascending k:
      raw_k = interp(x_k, V_density), sigma_k = softplus(raw_k + b),
      alpha_k = 1 - exp(-sigma_k delta),  T_k = prod_{j<k} (1 - alpha_j),
      c_k = MLP([interp(x_k, V_feat), PE(d)])  (with P.pe_x > 0:
            MLP([interp(x_k, V_feat), PE_{k_x}(u_k), PE(d)])),
      C = sum_k T_k alpha_k c_k + T_{K+1} c_bg.
    Also depth = sum w_k t_k, acc = sum w_k, log T_{K+1} = -delta sum sigma_k
    (equal to log prod (1 - alpha_k)), per-segment weight sums and the
    per-sample weights w_k = T_k alpha_k.  ``samp`` is a ``sample_rays`` dict.
    """
    o = np.asarray(o, F32)
    d = np.asarray(d, F32)
    B = o.shape[0]
    ro, sr, sk = samp["ray_offset"], samp["sample_ray"], samp["sample_k"]
    n = sr.size
    t, x = _sample_geometry(o, d, jitter, samp["t_near"], sr, sk, step)
    raw = interp(P.density, x, P.box_min, P.box_max)
    sigma = softplus(raw + P.act_shift)
    alpha = density_to_alpha(sigma, step)
    slot, col, kmax = _padded(ro, n)
    perm = np.asarray(samp["perm"], np.int64)
    A = np.zeros((B, kmax))
    A[slot, col] = alpha
    T_incl = np.cumprod(1.0 - A, axis=1)
    T_excl = np.concatenate([np.ones((B, 1)), T_incl[:, :-1]], axis=1)
    T_end_slot = T_incl[:, -1]
    w = T_excl[slot, col] * alpha
    cache = dict(t=t, x=x, raw=raw, sigma=sigma, alpha=alpha, w=w, slot=slot, col=col,
                 kmax=kmax, T_excl=T_excl)
    sig_sum = np.zeros(B)
    np.add.at(sig_sum, slot, sigma)
    out_slot = dict(acc=np.zeros(B), depth=np.zeros(B))
    np.add.at(out_slot["acc"], slot, w)
    np.add.at(out_slot["depth"], slot, w * t)
    seg = segment_of(sk, samp["n_uniform"][sr])
    seg_w = np.zeros((B, NSEG))
    np.add.at(seg_w, (slot, seg), w)
    res = {}
    if with_color and P.grid_colour:
        c = sigmoid(interp(P.feat, x, P.box_min, P.box_max))
        mcache = None
    elif with_color:
        f = interp(P.feat, x, P.box_min, P.box_max)
        pe = positional_encoding(d.astype(np.float64))[sr]
        if P.pe_x > 0:
            pex = positional_encoding(box_coordinates(x, P.box_min, P.box_max), P.pe_x)
            xin = np.concatenate([f, pex, pe], axis=1)
        else:
            xin = np.concatenate([f, pe], axis=1)
        c, mcache = mlp_forward(P.Ws, P.bs, xin, bf16=P.mlp_bf16, n_feat=xin.shape[1] - pe.shape[1])
    if with_color:
        rgb = np.zeros((B, 3))
        np.add.at(rgb, slot, w[:, None] * c)
        rgb += T_end_slot[:, None] * np.asarray(bg, np.float64)[None, :]
        cache.update(c=c, mcache=mcache)
        res["rgb"] = np.empty((B, 3))
        res["rgb"][perm] = rgb
    for key in ("acc", "depth"):
        res[key] = np.empty(B)
        res[key][perm] = out_slot[key]
    res["log_t_end"] = np.empty(B)
    res["log_t_end"][perm] = -step * sig_sum
    res["t_end"] = np.empty(B)
    res["t_end"][perm] = T_end_slot
    res["seg_w"] = np.empty((B, NSEG))
    res["seg_w"][perm] = seg_w
    res["sample_w"] = w
    res["cache"] = cache
    res["_sample_ray"] = np.asarray(sr, np.int64)
    return res


def render_backward(P: Params, o, d, jitter, samp, step, bg, fwd, grad_rgb,
                    grad_depth=None, grad_acc=None, grad_c=None, grad_t_end=None):
    """Hand-written adjoint of ``render_forward`` walked from each ray's end.

    With per-sample channel vectors v_k = (c_k, t_k, 1), background
    v_bg = (c_bg, 0, 0) and output gradient g = (dL/dC, dL/ddepth, dL/dacc):
      S_{K+1} = T_{K+1} v_bg,  S_k = S_{k+1} + w_k v_k   (suffix sums),
      dL/dsigma_k = delta * g . (T_{k+1} v_k - S_{k+1}),
      dL/draw_k   = dL/dsigma_k * sigmoid(raw_k + b),
      dL/dc_k     = w_k dL/dC, then back through the MLP to the features,
    followed by the transpose of the trilinear interpolation into both grids.
    Optional direct gradients: grad_c [n, 3] on every listed sample's colour
    (added to w_k dL/dC) and grad_t_end [B] on each ray's final
    transmittance, which reaches every sample of the ray through
    dT_end/dsigma_k = -delta T_end.  In the coarse stage's grid-colour form
    the colour gradient goes through the sigmoid into the colour grid.
    Returns dict(density, feat, Ws, bs) of float64 gradients (Ws, bs absent
    in the grid-colour form).
    """
    cache = fwd["cache"]
    B = np.asarray(o).shape[0]
    perm = np.asarray(samp["perm"], np.int64)
    slot, col, kmax = cache["slot"], cache["col"], cache["kmax"]
    n = slot.size
    bgv = np.asarray(bg, np.float64)
    g = np.zeros((B, 5))
    g[:, :3] = np.asarray(grad_rgb, np.float64)[perm]
    if grad_depth is not None:
        g[:, 3] = np.asarray(grad_depth, np.float64)[perm]
    if grad_acc is not None:
        g[:, 4] = np.asarray(grad_acc, np.float64)[perm]
    v = np.zeros((n, 5))
    v[:, :3] = cache["c"] if "c" in cache else 0.0
    v[:, 3] = cache["t"]
    v[:, 4] = 1.0
    Wv = np.zeros((B, kmax, 5))
    Wv[slot, col] = cache["w"][:, None] * v
    t_end = fwd["t_end"][perm]
    v_bg = np.zeros(5)
    v_bg[:3] = bgv
    # S_after[k] = sum_{m>k} w_m v_m + T_end v_bg
    rev = np.cumsum(Wv[:, ::-1, :], axis=1)[:, ::-1, :]
    S_after = np.concatenate([rev[:, 1:, :], np.zeros((B, 1, 5))], axis=1) + \
        t_end[:, None, None] * v_bg[None, None, :]
    T_next = cache["T_excl"][slot, col] * (1.0 - cache["alpha"])
    gs = g[slot]
    dsigma = step * np.sum(gs * (T_next[:, None] * v - S_after[slot, col]), axis=1)
    if grad_t_end is not None:
        dsigma = dsigma - step * t_end[slot] * np.asarray(grad_t_end, np.float64)[perm][slot]
    draw = dsigma * sigmoid(cache["raw"] + P.act_shift)
    grads = dict(density=interp_scatter(P.density.shape, cache["x"], P.box_min, P.box_max, draw))
    if "c" in cache:
        dc = cache["w"][:, None] * gs[:, :3]
        if grad_c is not None:
            dc = dc + np.asarray(grad_c, np.float64)
        if P.grid_colour:
            c = cache["c"]
            grads["feat"] = interp_scatter(P.feat.shape, cache["x"], P.box_min, P.box_max, dc * c * (1.0 - c))
        else:
            dx, dWs, dbs = mlp_backward(P.Ws, cache["mcache"], dc)
            df = dx[:, :P.feat.shape[-1]]
            grads["feat"] = interp_scatter(P.feat.shape, cache["x"], P.box_min, P.box_max, df)
            grads["Ws"], grads["bs"] = dWs, dbs
    grads["sample_draw"] = draw
    return grads


def grid_resample(grid, n_new, box_min, box_max):
    """Progressive scaling (Sec. 4.2): a vertex grid [nx,ny,nz(,C)] resized
    to n_new vertices per axis by trilinear interpolation (Eq. interp): new
    vertex j of axis i sits at min_i + j (max_i - min_i)/(n_new_i - 1), both
    grids spanning the box."""
    g = np.asarray(grid, np.float64)
    axes = [np.asarray(box_min[i], np.float64) + np.arange(n_new[i]) * (float(box_max[i]) - float(box_min[i])) /
            (n_new[i] - 1) for i in range(3)]
    X = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    out = interp(g, X, box_min, box_max)
    return out.reshape(tuple(n_new) + g.shape[3:])


def pg_resolutions(n_final, n_checkpoints):
    """Vertices per axis of the progressively scaled grid (Sec. 4.2
    "Progressive scaling"): the voxel count starts at 1/2^K of the final one
    (K checkpoints) and doubles at each checkpoint, so before checkpoint k
    (k = 0..K) the grid has floor((n_final^3 / 2^(K-k))^(1/3)) vertices per
    axis (a cube root within 1e-9 of an integer counts as that integer)."""
    out = []
    for k in range(n_checkpoints + 1):
        x = (float(n_final) ** 3 / 2.0 ** (n_checkpoints - k)) ** (1.0 / 3.0)
        out.append(int(math.floor(x + 1e-9)))
    return out


def photo_loss(rgb, target):
    """Photometric MSE of Eq. photo_loss: (1/|R|) sum_r ||C_r - C*_r||^2
    (sum over the three channels, mean over rays) and its gradient
    2 (C - C*) / |R|."""
    rgb = np.asarray(rgb, np.float64)
    tgt = np.asarray(target, np.float64)
    B = rgb.shape[0]
    diff = rgb - tgt
    return float(np.sum(diff * diff) / B), 2.0 * diff / B


def view_counts(n, box_min, box_max, centers, c2ws, H, W, focal):
    """Prior 2 of Sec. 4.1 (view-count-based learning rate): for each vertex
    j of an n[0] x n[1] x n[2] grid spanning the box, n_j = the number of
    training views it is visible to.  Reading: visible means inside the
    view's pinhole frustum: with p = R^T (x_j - centre) in camera
    coordinates (the camera looks down -z), p_z < 0 and the projection
    (focal p_x / (-p_z) + W/2, -focal p_y / (-p_z) + H/2) lies in
    [0, W) x [0, H) (no occlusion test).  Returns int64 counts [n]."""
    axes = [float(box_min[i]) + np.arange(n[i]) * (float(box_max[i]) - float(box_min[i])) / (n[i] - 1)
            for i in range(3)]
    X = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    cnt = np.zeros(X.shape[0], np.int64)
    for c, R in zip(np.asarray(centers, np.float64), np.asarray(c2ws, np.float64)):
        pc = (X - c) @ R            # rows: R^T (x - c)
        z = -pc[:, 2]
        with np.errstate(divide="ignore", invalid="ignore"):
            u = focal * pc[:, 0] / z + W / 2.0
            v = -focal * pc[:, 1] / z + H / 2.0
        vis = (z > 0) & (u >= 0) & (u < W) & (v >= 0) & (v < H)
        cnt += vis
    return cnt.reshape(tuple(n))


def view_count_lr_scale(counts):
    """Per-vertex learning-rate factor n_j / n_max (Prior 2)."""
    c = np.asarray(counts, np.float64)
    return c / max(float(c.max()), 1.0)


BG_CLAMP = 1e-6


def aux_losses(fwd, target):
    """The two auxiliary losses of the training objectives (Sec. 4.1 and 4.2
    "Training objective", supplementary table of the auxiliary losses),
    unweighted, with their gradients:
    per-point rgb: (1/|R|) sum_r sum_k w_k ||c_k - C(r)||^2, which supervises
      each sample's colour directly: the weights w_k are held fixed, so the
      gradient reaches the colours only, 2 w_k (c_k - C(r))/|R|;
    background entropy: (1/|R|) sum_r H(T_end(r)) with H(p) = -p log p -
      (1-p) log(1-p), the background probability clamped to [1e-6, 1-1e-6];
      dH/dT_end = log((1-p)/p), zero where the clamp is active.
    Returns dict(pt, bg, grad_c [n,3] in list order, grad_t_end [B] by ray)."""
    cache = fwd["cache"]
    sr = np.asarray(fwd["_sample_ray"], np.int64)
    tgt = np.asarray(target, np.float64)
    B = tgt.shape[0]
    diff = cache["c"] - tgt[sr]
    pt = float(np.sum(cache["w"] * np.sum(diff * diff, axis=1)) / B)
    grad_c = 2.0 * cache["w"][:, None] * diff / B
    te = np.asarray(fwd["t_end"], np.float64)
    p = np.clip(te, BG_CLAMP, 1.0 - BG_CLAMP)
    bg = float(np.sum(-p * np.log(p) - (1.0 - p) * np.log(1.0 - p)) / B)
    inside = (te > BG_CLAMP) & (te < 1.0 - BG_CLAMP)
    grad_t = np.where(inside, np.log((1.0 - p) / p), 0.0) / B
    return dict(pt=pt, bg=bg, grad_c=grad_c, grad_t_end=grad_t)


def adam_step(p, g, m, v, lr, beta1, beta2, eps, t):
    """One Adam update (the optimiser of Sec. 5.2, Kingma & Ba): m <- b1 m +
    (1-b1) g; v <- b2 v + (1-b2) g^2; p <- p - lr * mhat / (sqrt(vhat) + eps)
    with mhat = m/(1-b1^t), vhat = v/(1-b2^t).  float64, returns new arrays."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def lr_at(base_lr, it, decay_steps=20000, decay=0.1):
    """Exponential learning-rate decay reaching 0.1x at 20k iterations
    (supplementary implementation details)."""
    return base_lr * decay ** (it / decay_steps)


def psnr(mse):
    return -10.0 * math.log10(mse)


# ===========================================================================
# 3. Post-activation cell fits of the supplementary derivation
# ===========================================================================
def cell_fit_1d(c, delta, eps, Delta):
    """Grid values (a, b) at the two ends of a unit 1D cell whose
    post-activated alpha S(x) = 1 - (1 + exp(a(1-x) + bx))^-delta approximates
    a step at x = c within eps outside |x - c| < Delta, with S(c) = 1/2
    (supplementary Sec. "Derivation for a 1D grid cell": the upper bound on a
    for delta < 1 or delta >= 1, then b from the S(c) = 1/2 relation)."""
    L2 = math.log(2.0 ** (1.0 / delta) - 1.0)
    Le = math.log(1.0 / eps ** (1.0 / delta) - 1.0)
    L1 = math.log(1.0 / (1.0 - eps) ** (1.0 / delta) - 1.0)
    if delta < 1.0:
        a = L2 * (c + Delta) / Delta - Le * c / Delta
    else:
        a = L1 * c / Delta - L2 * (c - Delta) / Delta
    b = a * (c - 1.0) / c + L2 / c
    return a, b


def cell_fit_2d(c0, c1, delta, eps, Delta):
    """Corner values (V_tl, V_tr, V_bl, V_br) of a 2D cell whose boundary
    crosses the top edge at c0 and the bottom edge at c1 (supplementary
    Sec. "Derivation for a 2D grid cell"): each horizontal edge is a 1D fit."""
    a0, b0 = cell_fit_1d(c0, delta, eps, Delta)
    a1, b1 = cell_fit_1d(c1, delta, eps, Delta)
    return a0, b0, a1, b1


# ===========================================================================
# 4. Learned proposal (segment weights predicted per ray)
# ===========================================================================
def proposal_encoding(o, d, t_near, box_min, box_max, n_freq=4):
    """Proposal input: positional encoding of the box-entry point in box
    coordinates [-1,1]^3 followed by that of the direction (54 values)."""
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    x0 = o + np.asarray(t_near, np.float64)[:, None] * d
    bmin = np.asarray(box_min, np.float64)
    bmax = np.asarray(box_max, np.float64)
    u = (x0 - 0.5 * (bmin + bmax)) / (0.5 * (bmax - bmin))
    return np.concatenate([positional_encoding(u, n_freq), positional_encoding(d, n_freq)], axis=1)


def proposal_forward(Ws, bs, enc, bf16=False):
    """Proposal MLP enc -> 64 ReLU -> 64 ReLU -> 32 logits.  bf16=True rounds
    the input encoding, the hidden activations and the weights to bfloat16
    before each product (exact sums), as the bfloat16 form does."""
    W1, W2, W3 = [np.asarray(w, np.float64) for w in Ws]
    b1, b2, b3 = [np.asarray(b, np.float64) for b in bs]
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    z1 = r(enc) @ r(W1).T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = r(h1) @ r(W2).T + b2
    h2 = np.maximum(z2, 0.0)
    z = r(h2) @ r(W3).T + b3
    return z, dict(x=r(enc), z1=z1, h1=r(h1), z2=z2, h2=r(h2), bf16=bf16)


def proposal_probs(z):
    """33-way softmax of the 32 segment logits and an implicit transmitted
    logit fixed at 0, in float64 (the continuous part: the KL loss and its
    gradient); returns (q [B,33], predicted mass sum_{s<32} q_s)."""
    z = np.asarray(z, np.float64)
    zz = np.concatenate([z, np.zeros((z.shape[0], 1))], axis=1)
    m = np.max(zz, axis=1)
    e = np.exp(zz - m[:, None])
    q = e / e.sum(axis=1, keepdims=True)
    return q, q[:, :NSEG].sum(axis=1)


# float32 constants of the exponential recipe below (hexadecimal: exact)
_LOG2E = F32(float.fromhex("0x1.715476p+0"))      # log2(e) rounded to float32
_LN2_HI = F32(float.fromhex("0x1.62e4p-1"))       # ln 2 with its low mantissa bits cleared
_LN2_LO = F32(float.fromhex("0x1.7f7d1cp-20"))    # ln 2 - _LN2_HI rounded to float32
_EXP_TAYLOR = [F32(1.0 / math.factorial(j)) for j in range(7, -1, -1)]   # 1/7!, ..., 1/1!, 1/0!


def exp_f32(x):
    """exp(x) for float32 x <= 0 in an explicit float32 recipe (every
    operation rounded to float32 in the order written, no fused multiply-add),
    so that a float32 GPU implementation of the same steps gives the same
    bits.  Method: Cody-Waite range reduction x = k ln2 + r with ln 2 split in
    two parts (k ln2_hi is exact for |k| < 2^9), then the Taylor polynomial of
    e^r to degree 7 by Horner's rule (|r| <= ln2/2, truncation error below
    1e-8 relative), scaled by 2^k.  Arguments below -87 return 0 (the result
    would leave the normal float32 range)."""
    x = np.asarray(x, F32)
    with np.errstate(over="ignore", invalid="ignore"):
        k = np.rint((x * _LOG2E).astype(F32)).astype(F32)
        r = (x - (k * _LN2_HI).astype(F32)).astype(F32)
        r = (r - (k * _LN2_LO).astype(F32)).astype(F32)
        p = np.full(x.shape, _EXP_TAYLOR[0], F32)
        for c in _EXP_TAYLOR[1:]:
            p = ((p * r).astype(F32) + c).astype(F32)
        out = np.ldexp(p, np.where(np.isfinite(k), k, 0).astype(np.int32)).astype(F32)
    return np.where(x < F32(-87.0), F32(0.0), out).astype(F32)


def proposal_select_probs(z):
    """The selection's float32 softmax (reading of the benchmark spec's
    proposal: an implicit transmitted logit 0 beside the 32 segment logits).
    float32 recipe: m = max(0, z_s); e_s = exp_f32(z_s - m), e_T = exp_f32(-m);
    tot = the sum of e_0..e_31 then e_T, added one at a time in that order;
    q_s = e_s / tot (correctly rounded); mass = q_0 + ... + q_31 in index
    order.  Returns (q [B,32] float32, mass [B] float32)."""
    z = np.asarray(z, F32)
    B = z.shape[0]
    m = np.zeros(B, F32)
    for s in range(NSEG):
        m = np.maximum(m, z[:, s])
    e = exp_f32((z - m[:, None]).astype(F32))
    tot = np.zeros(B, F32)
    for s in range(NSEG):
        tot = (tot + e[:, s]).astype(F32)
    tot = (tot + exp_f32((F32(0.0) - m).astype(F32))).astype(F32)
    q = (e / tot[:, None]).astype(F32)
    mass = np.zeros(B, F32)
    for s in range(NSEG):
        mass = (mass + q[:, s]).astype(F32)
    return q, mass


def proposal_select(z, cum_frac=0.99, min_mass=0.9):
    """Segment mask per ray: the smallest set of segments, taken by
    descending probability (ties to the lower index), whose probability
    reaches cum_frac of the predicted mass; all 32 segments when the mass is
    below min_mass (uniform fallback).  float32 recipe from the float32
    logits: the probabilities of ``proposal_select_probs``, target =
    cum_frac * mass rounded to float32, the chosen probabilities added one
    at a time in the order chosen, stopping once the sum reaches the target.
    Returns uint32 masks."""
    q, mass = proposal_select_probs(z)
    cf, mm = F32(cum_frac), F32(min_mass)
    B = q.shape[0]
    out = np.zeros(B, np.uint32)
    for r in range(B):
        if not mass[r] >= mm:
            out[r] = np.uint32(0xFFFFFFFF)
            continue
        target = F32(cf * mass[r])
        order = sorted(range(NSEG), key=lambda s: (-float(q[r, s]), s))
        acc = F32(0.0)
        bits = 0
        for s in order:
            bits |= 1 << s
            acc = F32(acc + q[r, s])
            if acc >= target:
                break
        out[r] = np.uint32(bits)
    return out


def proposal_targets(seg_w, t_end):
    """KL target per ray: the 32 segment weight sums of the plain renderer
    and its final transmittance (they sum to one)."""
    return np.concatenate([np.asarray(seg_w, np.float64),
                           np.asarray(t_end, np.float64)[:, None]], axis=1)


def proposal_loss_grad(z, p):
    """Mean over rays of KL(p || q) with q the 33-way softmax; gradient with
    respect to the 32 logits is (q_s - p_s)/B."""
    q, _ = proposal_probs(z)
    B = q.shape[0]
    with np.errstate(divide="ignore", invalid="ignore"):
        kl = np.where(p > 0, p * (np.log(np.where(p > 0, p, 1.0)) - np.log(q)), 0.0)
    return float(kl.sum() / B), (q[:, :NSEG] - p[:, :NSEG]) / B


def proposal_backward(Ws, cache, dz):
    """Reverse-mode derivative of ``proposal_forward``.  In the bfloat16 form
    both operands of every product are bfloat16 values, as in the forward:
    the propagated gradient is rounded before it meets a bfloat16 weight
    matrix and before it multiplies the bfloat16 activations that give the
    weight gradients (bias gradients sum the rounded gradient)."""
    W1, W2, W3 = [np.asarray(w, np.float64) for w in Ws]
    r = bf16_round if cache.get("bf16") else (lambda a: np.asarray(a, np.float64))
    g3 = r(dz)
    dW3 = g3.T @ cache["h2"]
    db3 = g3.sum(0)
    g2 = r((g3 @ r(W3)) * (cache["z2"] > 0))
    dW2 = g2.T @ cache["h1"]
    db2 = g2.sum(0)
    g1 = r((g2 @ r(W2)) * (cache["z1"] > 0))
    dW1 = g1.T @ cache["x"]
    db1 = g1.sum(0)
    return [dW1, dW2, dW3], [db1, db2, db3]


# ===========================================================================
# 5. Ground-truth targets of the analytic scene
# ===========================================================================
def scene_render(o, d, centers, radii, rho, rgb, box_min, box_max, step, bg, edge=0.01):
    """Reference image of the analytic sphere scene by the same quadrature
    (Eq. volume_rendering) at midpoint samples t_k = t_near + (k + 1/2) step
    while t_k < t_far, density sum_i rho_i sigmoid((r_i - |x - c_i|)/edge),
    colour the density-weighted mean.  float64, one ray at a time (use on
    small spot-check sets)."""
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    t_near, t_far, valid = ray_box_clip(np.asarray(o, F32), np.asarray(d, F32), box_min, box_max)
    out = np.tile(np.asarray(bg, np.float64), (o.shape[0], 1))
    for r in range(o.shape[0]):
        if not valid[r]:
            continue
        nk = int(math.ceil((float(t_far[r]) - float(t_near[r])) / step - 0.5))
        nk = max(nk, 0)
        while nk > 0 and float(t_near[r]) + (nk - 0.5) * step >= float(t_far[r]):
            nk -= 1
        while float(t_near[r]) + (nk + 0.5) * step < float(t_far[r]):
            nk += 1
        t = float(t_near[r]) + (np.arange(nk) + 0.5) * step
        x = o[r][None, :] + t[:, None] * d[r][None, :]
        dist = np.linalg.norm(x[:, None, :] - np.asarray(centers)[None], axis=-1)
        si = np.asarray(rho)[None, :] * sigmoid((np.asarray(radii)[None, :] - dist) / edge)
        s = si.sum(1)
        col = np.where(s[:, None] > 0, (si @ np.asarray(rgb)) / np.maximum(s[:, None], 1e-300), 0)
        a = 1.0 - np.exp(-s * step)
        T = np.concatenate([[1.0], np.cumprod(1.0 - a)])
        out[r] = (T[:-1, None] * a[:, None] * col).sum(0) + T[-1] * np.asarray(bg, np.float64)
    return out


# ===========================================================================
# 6. Image-fitting toy of Sec. 3 ("Sharp decision boundary via
#    post-activation"): a low-resolution 2D grid fitted to a binary image
#    with pre-, in- or post-activation (Eq. pre_activation, in_activation,
#    post_activation, with bilinear interpolation and no shift b)
# ===========================================================================
TOY_MODES = ("pre", "in", "post")


def toy2d_weights(H, W, gh, gw):
    """Bilinear weights of every pixel centre on a vertex grid of gh x gw
    points spanning the image inclusively: pixel (i, j) sits at grid
    coordinates u = (i + 1/2)(gh - 1)/H, v = (j + 1/2)(gw - 1)/W; cell
    i0 = clamp(floor(u), 0, gh - 2) (likewise j0), fractions clamped to
    [0, 1].  Returns (i0 [H*W], j0 [H*W], weights [H*W, 4]) for the corners
    (i0, j0), (i0, j0+1), (i0+1, j0), (i0+1, j0+1)."""
    ii, jj = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    u = (ii.ravel() + 0.5) * (gh - 1) / H
    v = (jj.ravel() + 0.5) * (gw - 1) / W
    i0 = np.clip(np.floor(u), 0, gh - 2).astype(np.int64)
    j0 = np.clip(np.floor(v), 0, gw - 2).astype(np.int64)
    fu = np.clip(u - i0, 0.0, 1.0)
    fv = np.clip(v - j0, 0.0, 1.0)
    w = np.stack([(1 - fu) * (1 - fv), (1 - fu) * fv, fu * (1 - fv), fu * fv], axis=1)
    return i0, j0, w


def _toy_corners(V, i0, j0):
    V = np.asarray(V, np.float64)
    return np.stack([V[i0, j0], V[i0, j0 + 1], V[i0 + 1, j0], V[i0 + 1, j0 + 1]], axis=1)


def toy2d_forward(V, H, W, mode, delta=1.0):
    """Predicted alpha image [H, W] of the grid V [gh, gw]:
    pre:  interp(x, alpha(softplus(V)));   in: alpha(interp(x, softplus(V)));
    post: alpha(softplus(interp(x, V))),   alpha(s) = 1 - exp(-s delta)."""
    gh, gw = np.asarray(V).shape
    i0, j0, w = toy2d_weights(H, W, gh, gw)
    c = _toy_corners(V, i0, j0)
    if mode == "pre":
        a = np.sum(w * density_to_alpha(softplus(c), delta), axis=1)
    elif mode == "in":
        a = density_to_alpha(np.sum(w * softplus(c), axis=1), delta)
    elif mode == "post":
        a = density_to_alpha(softplus(np.sum(w * c, axis=1)), delta)
    else:
        raise ValueError(mode)
    return a.reshape(H, W)


def toy2d_loss_grad(V, target, mode, delta=1.0):
    """Mean squared error of the predicted alpha image against ``target``
    [H, W] and its gradient with respect to V, by the chain rule through the
    mode's activation order (softplus' = sigmoid, alpha'(s) = delta e^{-s delta})
    and the transpose of the bilinear interpolation."""
    V = np.asarray(V, np.float64)
    gh, gw = V.shape
    H, W = np.asarray(target).shape
    i0, j0, w = toy2d_weights(H, W, gh, gw)
    c = _toy_corners(V, i0, j0)
    a = toy2d_forward(V, H, W, mode, delta).ravel()
    r = a - np.asarray(target, np.float64).ravel()
    loss = float(np.mean(r * r))
    da = 2.0 * r / r.size
    if mode == "pre":
        dc = da[:, None] * w * delta * np.exp(-delta * softplus(c)) * sigmoid(c)
    elif mode == "in":
        sbar = np.sum(w * softplus(c), axis=1)
        dc = (da * delta * np.exp(-delta * sbar))[:, None] * w * sigmoid(c)
    else:
        vbar = np.sum(w * c, axis=1)
        dc = (da * delta * np.exp(-delta * softplus(vbar)) * sigmoid(vbar))[:, None] * w
    g = np.zeros_like(V)
    for k, (di, dj) in enumerate(((0, 0), (0, 1), (1, 0), (1, 1))):
        np.add.at(g, (i0 + di, j0 + dj), dc[:, k])
    return loss, g
