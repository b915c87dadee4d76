"""Pins of the oracle's discrete sampler: analytic clip bounds, brute-force
sample counts, the coarse-mask invariant and the Morton key definition."""

import math

import numpy as np

import oracle as O
import synth

F32 = np.float32
BMIN, BMAX = np.array([-1, -1, -1], F32), np.array([1, 1, 1], F32)


def test_clip_analytic_cases():
    o = np.array([[-3, 0.2, 0.3],    # axis ray, enters at 2, leaves at 4
                  [0, 0, 0],         # inside: near stays 0
                  [-3, 2, 0],        # d_y = 0 with o_y outside: miss
                  [-3, 1, 1],        # grazing edge: o_y = o_z = max, allowed
                  [3, 0, 0],         # pointing away: miss
                  [-3, -3, -3],      # diagonal through the corner region
                  [0.5, 0.5, 0.5]], F32)
    s3 = 1 / math.sqrt(3)
    d = np.array([[1, 0, 0], [1, 0, 0], [1, 0, 0], [1, 0, 0], [1, 0, 0],
                  [s3, s3, s3], [0, 0, -1]], F32)
    tn, tf, v = O.ray_box_clip(o, d, BMIN, BMAX)
    assert list(v) == [True, True, False, True, False, True, True]
    assert (tn[0], tf[0]) == (2, 4)
    assert (tn[1], tf[1]) == (0, 1)
    assert (tn[3], tf[3]) == (2, 4)
    assert abs(tn[5] - 2 * math.sqrt(3)) < 1e-5 and abs(tf[5] - 4 * math.sqrt(3)) < 1e-5
    assert (tn[6], tf[6]) == (0, 1.5)
    assert tn[2] == tf[2] == 0 and tn[4] == tf[4] == 0


def test_clip_matches_float64_geometry():
    rng = np.random.default_rng(0)
    o, d, *_ = synth.draw_pixels_without_replacement(rng, synth.cube_vertex_cameras(), 32, 32, 40.0, 2000)
    tn, tf, v = O.ray_box_clip(o, d, BMIN, BMAX)
    o64, d64 = o.astype(float), d.astype(float)
    t0 = (BMIN - o64) / d64
    t1 = (BMAX - o64) / d64
    en = np.max(np.minimum(t0, t1), 1)
    ex = np.min(np.maximum(t0, t1), 1)
    v64 = np.maximum(en, 0) < ex
    ok = np.abs(ex - np.maximum(en, 0)) > 1e-5   # away from grazing ties
    assert np.all(v[ok] == v64[ok])
    assert np.allclose(tn[v], np.maximum(en, 0)[v], atol=1e-5)
    assert np.allclose(tf[v], ex[v], atol=1e-5)


def _count_loop(tn, tf, p, step, cap):
    """Scalar float32 brute force, one k at a time."""
    n = 0
    while n < cap:
        t = F32(tn) + F32(F32(F32(n) + F32(p)) * F32(step))
        if not t < F32(tf):
            break
        n += 1
    return n


def test_uniform_count_brute_force_and_closed_form():
    rng = np.random.default_rng(1)
    o, d, *_ = synth.draw_pixels_without_replacement(rng, synth.cube_vertex_cameras(), 32, 32, 40.0, 500)
    p = rng.random(500).astype(F32)
    tn, tf, v = O.ray_box_clip(o, d, BMIN, BMAX)
    step = 2.0 / 31 * 0.5
    n = O.uniform_count(tn, tf, v, p, step, 128)
    for r in range(500):
        want = _count_loop(tn[r], tf[r], p[r], step, 128) if v[r] else 0
        assert n[r] == want
        if v[r]:
            # closed form N = ceil((t_far - t_near)/delta - p), up to rounding at ties
            cf = math.ceil((float(tf[r]) - float(tn[r])) / step - float(p[r]))
            assert abs(n[r] - min(cf, 128)) <= 1


def test_sample_t_monotone():
    tn = np.full(1000, F32(1.2345))
    p = np.full(1000, F32(0.7))
    t = O.sample_t(tn, p, np.arange(1000), 0.0123)
    assert np.all(np.diff(t) >= 0)


def test_count_cap_truncates_far_end():
    o = np.array([[-3, 0, 0]], F32)
    d = np.array([[1, 0, 0]], F32)
    samp = O.sample_rays(o, d, None, BMIN, BMAX, 0.01, 50)
    assert samp["n_uniform"][0] == 50
    assert list(samp["sample_k"]) == list(range(50))


def test_coarse_threshold_inverts_alpha():
    for tau, step, b in [(1e-4, 2 / 159 * 0.5, 0.0), (1e-3, 0.01, 0.7), (1e-2, 0.1, -2.0)]:
        thr = O.coarse_raw_threshold(tau, step, b)
        a_thr = O.post_activated_alpha(float(thr), b, step)
        a_next = O.post_activated_alpha(float(np.nextafter(thr, F32(np.inf))), b, step)
        assert a_thr <= tau * (1 + 1e-6)
        assert abs(a_thr - tau) < 1e-5 * tau
        assert a_next >= a_thr


def test_coarse_mask_is_conservative_brute_force():
    """Every point whose own post-activated coarse alpha reaches tau lies in a
    kept cell (brute force over random points)."""
    rng = np.random.default_rng(2)
    cn = (9, 7, 8)
    raw = rng.normal(-8, 2, cn).astype(F32)
    step, tau = 0.05, 1e-3
    thr = O.coarse_raw_threshold(tau, step)
    bits = O.coarse_cell_bits(raw, thr)
    x = rng.uniform(-1, 1, (200000, 3)).astype(F32)
    alpha = O.post_activated_alpha(O.interp(raw, x.astype(float), BMIN, BMAX), 0.0, step)
    keep = O.coarse_keep(x, BMIN, BMAX, cn, bits)
    assert np.all(keep[alpha >= tau])
    assert 0.0 < keep.mean() < 0.9


def test_coarse_cell_bits_layout():
    cn = (3, 4, 5)
    raw = np.full(cn, -100, F32)
    raw[2, 3, 4] = 100        # only the last cell (1,2,3) has it as a corner
    bits = O.coarse_cell_bits(raw, F32(0))
    c = (1 * 3 + 2) * 4 + 3
    assert bits[c >> 5] == np.uint32(1 << (c & 31))
    assert sum(bin(int(w)).count("1") for w in bits) == 1


def test_morton_interleave_definition():
    o = np.zeros((4, 3), F32)
    d = np.tile(np.array([[1, 0, 0]], F32), (4, 1))
    # midpoints placed in chosen voxels of the 32^3 quantisation
    vox = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [31, 31, 31]])
    mids = (-1 + (vox + 0.5) * (2 / 32)).astype(F32)
    o[:] = mids
    tn = np.zeros(4, F32)
    tf = np.zeros(4, F32)
    keys = O.morton_keys(o, d, tn, tf, np.ones(4, bool), BMIN, BMAX)
    assert list(keys) == [4, 2, 1, (1 << 15) - 1]
    brute = []
    for q in vox:
        k = 0
        for b in range(5):
            k |= ((int(q[0]) >> b) & 1) << (3 * b + 2)
            k |= ((int(q[1]) >> b) & 1) << (3 * b + 1)
            k |= ((int(q[2]) >> b) & 1) << (3 * b)
        brute.append(k)
    assert list(keys) == brute
    assert O.morton_keys(o, d, tn, tf, np.zeros(4, bool), BMIN, BMAX)[0] == 1 << 15


def test_morton_order_is_a_sorted_permutation():
    P = synth.tiny_config(0, n_rays=1024)
    s = O.sample_rays(P.rays.o, P.rays.d, None, P.box_min, P.box_max, P.step, P.max_samples, morton=True)
    perm = s["perm"]
    assert sorted(perm) == list(range(1024))
    k = s["keys"][perm]
    assert np.all((np.diff(k.astype(np.int64)) > 0) | ((np.diff(k.astype(np.int64)) == 0) & (np.diff(perm) > 0)))
    s0 = O.sample_rays(P.rays.o, P.rays.d, None, P.box_min, P.box_max, P.step, P.max_samples)
    for slot in range(0, 1024, 37):
        r = perm[slot]
        a = s["sample_k"][s["ray_offset"][slot]:s["ray_offset"][slot + 1]]
        b = s0["sample_k"][s0["ray_offset"][r]:s0["ray_offset"][r + 1]]
        assert list(a) == list(b)


def test_all_ones_segment_mask_equals_plain():
    P = synth.tiny_config(3, n_rays=512, jitter=True)
    raw = np.random.default_rng(4).normal(-3, 2, (9, 9, 9)).astype(F32)
    bits = O.coarse_cell_bits(raw, O.coarse_raw_threshold(1e-3, P.step))
    coarse = (bits, P.box_min, P.box_max, raw.shape)
    a = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples, coarse)
    b = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples, coarse,
                      seg_mask=np.full(512, 0xFFFFFFFF, np.uint32))
    for key in ("ray_offset", "sample_ray", "sample_k", "n_uniform"):
        assert np.array_equal(a[key], b[key])
    # a single segment keeps exactly the samples with 32k // N_r == s
    c = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples,
                      seg_mask=np.full(512, 1 << 5, np.uint32))
    nu = c["n_uniform"][c["sample_ray"]]
    assert np.all((32 * c["sample_k"]) // nu == 5)


def test_segments_equal_count():
    for n in (1, 5, 31, 32, 33, 100, 551):
        seg = O.segment_of(np.arange(n), n)
        counts = np.bincount(seg, minlength=32)
        assert seg.min() >= 0 and seg.max() <= 31 and np.all(np.diff(seg) >= 0)
        if n >= 32:
            assert counts.max() - counts.min() <= 1
