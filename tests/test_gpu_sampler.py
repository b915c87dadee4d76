"""GPU parity of the sampler and the coarse mask: bit-exact against the
oracle's float32 recipe (float outputs compared by value)."""

import numpy as np
import pytest

import oracle as O
import synth
from tests.helpers import np_of, to_dev

pytestmark = pytest.mark.gpu
F32 = np.float32


def _coarse(raw, cmin, cmax, tau, step):
    from paper_2111_11215_amd import api
    thr = O.coarse_raw_threshold(tau, step)
    assert abs(api.coarse_raw_threshold(tau, step) - float(thr)) == 0.0
    bits_ref = O.coarse_cell_bits(raw, thr)
    bits = api.coarse_mask_build(to_dev(raw), cmin, cmax, float(thr))
    return bits, bits_ref, thr


def _check_samples(s, ref, B):
    print(f"  B={B} kept={int(ref['ray_offset'][-1])}", flush=True)
    assert np.array_equal(np_of(s.valid).astype(bool), ref["valid"])
    assert np.array_equal(np_of(s.t_near), ref["t_near"])
    assert np.array_equal(np_of(s.t_far), ref["t_far"])
    assert np.array_equal(np_of(s.n_uniform), ref["n_uniform"])
    assert np.array_equal(np_of(s.perm), ref["perm"])
    assert np.array_equal(np_of(s.ray_offset), ref["ray_offset"])
    n = int(ref["ray_offset"][-1])
    assert int(np_of(s.n_kept)[0]) == n
    assert np.array_equal(np_of(s.sample_ray)[:n], ref["sample_ray"])
    assert np.array_equal(np_of(s.sample_k)[:n], ref["sample_k"])


@pytest.mark.parametrize("jitter,morton,coarse,seg", [
    (False, False, False, False), (True, False, False, False), (True, True, False, False),
    (True, False, True, False), (True, True, True, True)])
def test_sampler_bit_exact_tiny(gpu_lib, jitter, morton, coarse, seg):
    from paper_2111_11215_amd import api
    P = synth.tiny_config(0, jitter=jitter)
    B = P.rays.o.shape[0]
    cinfo = None
    crefinfo = None
    if coarse:
        raw = np.random.default_rng(5).normal(-6, 3, (17, 19, 15)).astype(F32)
        bits, bits_ref, _ = _coarse(raw, P.box_min, P.box_max, 1e-3, P.step)
        assert np.array_equal(np_of(bits).view(np.uint32), bits_ref)
        cinfo = (bits, P.box_min, P.box_max, raw.shape)
        crefinfo = (bits_ref, P.box_min, P.box_max, raw.shape)
    segm = np.random.default_rng(6).integers(0, 2 ** 32, B, dtype=np.uint64).astype(np.uint32) if seg else None
    s = api.sample_rays(to_dev(P.rays.o), to_dev(P.rays.d), to_dev(P.rays.jitter) if jitter else None,
                        P.box_min, P.box_max, P.step, P.max_samples, coarse=cinfo,
                        seg_mask=to_dev(segm.view(np.int32)) if seg else None, morton=morton)
    ref = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples,
                        coarse=crefinfo, seg_mask=segm, morton=morton)
    _check_samples(s, ref, B)


def test_sampler_edge_rays(gpu_lib):
    """Axis-aligned, grazing, inside-origin, missing, zero-component rays and
    a cap that truncates."""
    from paper_2111_11215_amd import api
    o = np.array([[-3, 0.2, 0.3], [0, 0, 0], [-3, 2, 0], [-3, 1, 1], [3, 0, 0], [0.5, 0.5, 0.5],
                  [-3, -1, 0.25], [0.99, -0.99, 0.0]], F32)
    d = np.array([[1, 0, 0], [1, 0, 0], [1, 0, 0], [1, 0, 0], [1, 0, 0], [0, 0, -1], [1, 0, 0],
                  [-0.6, 0.8, 0.0]], F32)
    bmin, bmax = np.array([-1, -1, -1], F32), np.array([1, 1, 1], F32)
    for cap in (7, 40, 1000):
        s = api.sample_rays(to_dev(o), to_dev(d), None, bmin, bmax, 0.05, cap)
        ref = O.sample_rays(o, d, None, bmin, bmax, 0.05, cap)
        _check_samples(s, ref, len(o))


def test_sampler_empty_batch_and_all_missing(gpu_lib):
    import torch
    from paper_2111_11215_amd import api
    bmin, bmax = np.array([-1, -1, -1], F32), np.array([1, 1, 1], F32)
    z = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    s = api.sample_rays(z, z, None, bmin, bmax, 0.05, 10)
    assert int(np_of(s.n_kept)[0]) == 0 and int(np_of(s.ray_offset)[0]) == 0
    o = np.tile(np.array([[5, 5, 5]], F32), (100, 1))
    d = np.tile(np.array([[1, 0, 0]], F32), (100, 1))
    s = api.sample_rays(to_dev(o), to_dev(d), None, bmin, bmax, 0.05, 10)
    assert int(np_of(s.n_kept)[0]) == 0 and not np_of(s.valid).any()


def test_sampler_clip_only(gpu_lib):
    """Clip only (no list): t_near, t_far, valid and n_uniform equal those of
    the full call and of the oracle; an empty batch is accepted."""
    import torch
    from paper_2111_11215_amd import api
    P = synth.tiny_config(2, jitter=True, n_rays=1024)
    args = (to_dev(P.rays.o), to_dev(P.rays.d), to_dev(P.rays.jitter), P.box_min, P.box_max, P.step,
            P.max_samples)
    c = api.sample_rays(*args, clip_only=True)
    f = api.sample_rays(*args)
    ref = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples)
    for k in ("t_near", "t_far", "valid", "n_uniform"):
        assert np.array_equal(np_of(getattr(c, k)), np_of(getattr(f, k))), k
    for k in ("t_near", "valid", "n_uniform"):
        assert np.array_equal(np_of(getattr(c, k)).astype(ref[k].dtype), ref[k]), k
    z = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    api.sample_rays(z, z, None, P.box_min, P.box_max, P.step, 10, clip_only=True)


def test_sampler_capacity_overflow_reported(gpu_lib):
    """A capacity below the kept count truncates the list and reports the
    true count, leaving memory past the capacity untouched."""
    import torch
    from paper_2111_11215_amd import api
    P = synth.tiny_config(0, n_rays=256)
    ref = O.sample_rays(P.rays.o, P.rays.d, None, P.box_min, P.box_max, P.step, P.max_samples)
    total = int(ref["ray_offset"][-1])
    cap = total // 2
    s = api.sample_rays(to_dev(P.rays.o), to_dev(P.rays.d), None, P.box_min, P.box_max, P.step, P.max_samples,
                        capacity=cap)
    torch.cuda.synchronize()
    assert int(np_of(s.n_kept)[0]) == total
    assert np.array_equal(np_of(s.sample_k)[:cap], ref["sample_k"][:cap])


def test_sampler_full_size_scene(gpu_lib):
    """The full configuration (8192 rays, 160^3 box step, 100^3 coarse mask
    of the sphere scene, tau 1e-4): every per-ray quantity bit-exact, the
    kept lists of 300 sampled rays bit-exact against the oracle."""
    from paper_2111_11215_amd import api
    P = synth.full_config(0)
    raw = P.coarse_raw
    bits, bits_ref, _ = _coarse(raw, P.box_min, P.box_max, synth.FULL_TAU, P.step)
    assert np.array_equal(np_of(bits).view(np.uint32), bits_ref)
    s = api.sample_rays(to_dev(P.rays.o), to_dev(P.rays.d), to_dev(P.rays.jitter), P.box_min, P.box_max, P.step,
                        P.max_samples, coarse=(bits, P.box_min, P.box_max, raw.shape), morton=True)
    tn, tf, v = O.ray_box_clip(P.rays.o, P.rays.d, P.box_min, P.box_max)
    nu = O.uniform_count(tn, tf, v, P.rays.jitter, P.step, P.max_samples)
    assert np.array_equal(np_of(s.t_near), tn) and np.array_equal(np_of(s.t_far), tf)
    assert np.array_equal(np_of(s.n_uniform), nu)
    keys = O.morton_keys(P.rays.o, P.rays.d, tn, tf, v, P.box_min, P.box_max)
    perm_ref = np.lexsort((np.arange(len(keys)), keys))
    perm = np_of(s.perm)
    assert np.array_equal(perm, perm_ref)
    ro = np_of(s.ray_offset)
    sk = np_of(s.sample_k)
    rng = np.random.default_rng(0)
    slots = rng.choice(len(perm), 300, replace=False)
    rays = perm[slots]
    sub = O.sample_rays(P.rays.o[rays], P.rays.d[rays], P.rays.jitter[rays], P.box_min, P.box_max, P.step,
                        P.max_samples, coarse=(bits_ref, P.box_min, P.box_max, raw.shape))
    for i, slot in enumerate(slots):
        got = sk[ro[slot]:ro[slot + 1]]
        want = sub["sample_k"][sub["ray_offset"][i]:sub["ray_offset"][i + 1]]
        assert np.array_equal(got, want), slot
    print(f"  kept {int(np_of(s.n_kept)[0])} of {int(nu.sum())} uniform samples", flush=True)


@pytest.mark.parametrize("n_rays", [1, 7, 8193, 20001])
def test_sampler_offsets_span_several_scan_passes(gpu_lib, n_rays):
    """Ray offsets over batches that take one, two and three passes of the
    single-workgroup scan (8192 rays each), ragged tails included.  Without a
    coarse or segment mask every uniform sample is kept, so the offsets are
    the exclusive cumulative sum of the oracle's uniform counts."""
    from paper_2111_11215_amd import api
    P = synth.tiny_config(3, jitter=True, n_rays=n_rays)
    s = api.sample_rays(to_dev(P.rays.o), to_dev(P.rays.d), to_dev(P.rays.jitter), P.box_min, P.box_max, P.step,
                        P.max_samples)
    tn, tf, v = O.ray_box_clip(P.rays.o, P.rays.d, P.box_min, P.box_max)
    nu = O.uniform_count(tn, tf, v, P.rays.jitter, P.step, P.max_samples).astype(np.int64)
    want = np.concatenate([[0], np.cumsum(nu)])
    print(f"  B={n_rays} kept={int(want[-1])}", flush=True)
    assert np.array_equal(np_of(s.n_uniform), nu)
    assert np.array_equal(np_of(s.ray_offset).astype(np.int64), want)
    assert int(np_of(s.n_kept)[0]) == int(want[-1])
    sr = np_of(s.sample_ray)[:int(want[-1])]
    assert np.array_equal(sr, np.repeat(np.arange(n_rays), nu))


@pytest.mark.parametrize("max_samples", [1024, 1100])
def test_sampler_long_rays_both_fill_paths(gpu_lib, max_samples):
    """Rays of up to 1024 uniform samples are filled from the counting pass's
    keep ballots, longer ones by evaluating the keep rule again: both
    bit-exact against the oracle, with a coarse and a segment mask, on rays
    that reach the sample cap, so every ballot word (lanes 31/32 included) is
    used."""
    from paper_2111_11215_amd import api
    P = synth.tiny_config(4, jitter=True, n_rays=300)
    step = 0.0025
    raw = np.random.default_rng(8).normal(-4, 3, (17, 19, 15)).astype(F32)
    bits, bits_ref, _ = _coarse(raw, P.box_min, P.box_max, 1e-3, step)
    segm = np.random.default_rng(9).integers(0, 2 ** 32, 300, dtype=np.uint64).astype(np.uint32)
    segm[:100] = 0xFFFFFFFF
    s = api.sample_rays(to_dev(P.rays.o), to_dev(P.rays.d), to_dev(P.rays.jitter), P.box_min, P.box_max, step,
                        max_samples, coarse=(bits, P.box_min, P.box_max, raw.shape),
                        seg_mask=to_dev(segm.view(np.int32)))
    ref = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, step, max_samples,
                        coarse=(bits_ref, P.box_min, P.box_max, raw.shape), seg_mask=segm)
    assert ref["n_uniform"].max() == max_samples
    _check_samples(s, ref, 300)
