"""dvgo_sample_rays_noalloc (the sampler with its scratch in the library's
static device array) against dvgo_sample_rays with a caller workspace: every
output bit for bit, over two calls in a row of which the second is smaller
(the static array keeps the first call's contents), with and without the
coarse mask, jitter and Morton order; and the size limit refused before
anything is enqueued."""

import ctypes

import numpy as np
import pytest

import oracle as O
import synth
from tests.helpers import np_of, to_dev

pytestmark = pytest.mark.gpu
F32 = np.float32


def _same(a, b, n):
    for k in ("t_near", "t_far", "valid", "n_uniform", "perm", "ray_offset", "n_kept"):
        assert np.array_equal(np_of(getattr(a, k)), np_of(getattr(b, k))), k
    m = int(np_of(a.n_kept)[0])
    assert m == n
    assert np.array_equal(np_of(a.sample_ray)[:m], np_of(b.sample_ray)[:m])
    assert np.array_equal(np_of(a.sample_k)[:m], np_of(b.sample_k)[:m])


@pytest.mark.parametrize("morton", [False, True])
def test_noalloc_sampler_equals_workspace_sampler(gpu_lib, morton):
    import torch
    from paper_2111_11215_amd import api
    P = synth.full_config(0, n_rays=20000)
    raw = P.coarse_raw
    thr = api.coarse_raw_threshold(synth.FULL_TAU, P.step)
    bits = api.coarse_mask_build(to_dev(raw), P.box_min, P.box_max, thr)
    coarse = (bits, P.box_min, P.box_max, raw.shape)
    for B, with_coarse in ((20000, True), (3000, False)):
        o, d, j = (to_dev(np.ascontiguousarray(a[:B])) for a in (P.rays.o, P.rays.d, P.rays.jitter))
        c = coarse if with_coarse else None
        print(f"  B={B} coarse={with_coarse} morton={morton}", flush=True)
        ref = api.sample_rays(o, d, j, P.box_min, P.box_max, P.step, P.max_samples, coarse=c, morton=morton)
        got = api.sample_rays(o, d, j, P.box_min, P.box_max, P.step, P.max_samples, coarse=c, morton=morton,
                              no_alloc=True)
        torch.cuda.synchronize()
        n = int(np_of(ref.n_kept)[0])
        _same(got, ref, n)
        if B <= 3000:   # the smaller call also against the oracle's sampler
            want = O.sample_rays(P.rays.o[:B], P.rays.d[:B], P.rays.jitter[:B], P.box_min, P.box_max, P.step,
                                 P.max_samples, morton=morton)
            assert np.array_equal(np_of(got.ray_offset), want["ray_offset"])
            assert np.array_equal(np_of(got.sample_k)[:n], want["sample_k"])


def test_noalloc_sampler_refuses_beyond_its_limit(gpu_lib):
    from paper_2111_11215_amd import _lib
    lib = _lib.load()
    box = _lib.make_box((-1, -1, -1), (1, 1, 1))
    fake = ctypes.c_void_p(16)
    st = lib.dvgo_sample_rays_noalloc(fake, fake, None, (1 << 18) + 1, ctypes.byref(box), 0.1, 10, None, None, None,
                                      None, 0, fake, fake, fake, fake, fake, fake, fake, fake, 1, fake, None)
    assert st == -6
    assert b"static scratch" in lib.dvgo_last_error()
