"""The C ABI library loads, exports every symbol the header declares, and
rejects bad arguments on the host before any launch (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dvgo.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dvgo_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2111_11215_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libdvgo.so not built: run __graft_entry__.build()")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_2111_11215_amd import _lib
    names = _declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, f"binding lacks a signature for {n}"


def test_status_strings(lib):
    assert lib.dvgo_status_string(0) == b"ok"
    for s in range(-6, 0):
        assert lib.dvgo_status_string(s) != b"unknown status"
    assert lib.dvgo_version() >= 1


def test_param_counts(lib):
    assert lib.dvgo_mlp_param_count(12, 128, 0) == 128 * 39 + 128 + 128 * 128 + 128 + 3 * 128 + 3 == 22019
    assert lib.dvgo_mlp_param_count(12, 128, 5) == 128 * 72 + 128 + 128 * 128 + 128 + 3 * 128 + 3 == 26243
    assert lib.dvgo_prop_param_count() == 64 * 54 + 64 + 64 * 64 + 64 + 32 * 64 + 32


def test_workspace_queries(lib):
    assert lib.dvgo_sample_workspace_bytes(8192) >= 8192 * 8
    from paper_2111_11215_amd import _lib
    g = _lib.make_box((-1, -1, -1), (1, 1, 1), (160, 160, 160))
    assert lib.dvgo_render_workspace_bytes(8192, 8192 * 552, 12, ctypes.byref(g)) >= 8192 * 552 * 128
    assert lib.dvgo_render_workspace_bytes(8192, 100, 11, ctypes.byref(g)) == 0
    assert lib.dvgo_render_workspace_bytes(8192, 100, 12, None) == 0
    assert lib.dvgo_proposal_workspace_bytes(1024) > 0


def test_host_validation_rejects_before_launch(lib):
    from paper_2111_11215_amd import _lib
    box = _lib.make_box((-1, -1, -1), (1, 1, 1), (2, 2, 2))
    bad_box = _lib.make_box((1, -1, -1), (-1, 1, 1), (2, 2, 2))
    nul = None
    # negative batch
    assert lib.dvgo_sample_rays(nul, nul, nul, -1, ctypes.byref(box), 0.1, 10, nul, nul, nul, nul, 0, nul, nul, nul,
                                nul, nul, nul, nul, nul, 0, nul, nul, 0, nul) == -1
    # inverted box
    assert lib.dvgo_sample_rays(nul, nul, nul, 0, ctypes.byref(bad_box), 0.1, 10, nul, nul, nul, nul, 0, nul, nul, nul,
                                nul, nul, nul, nul, nul, 0, nul, nul, 0, nul) == -1
    # zero step
    assert lib.dvgo_sample_rays(nul, nul, nul, 0, ctypes.byref(box), 0.0, 10, nul, nul, nul, nul, 0, nul, nul, nul,
                                nul, nul, nul, nul, nul, 0, nul, nul, 0, nul) == -1
    # Morton order beyond the packed-id limit
    fake = ctypes.c_void_p(16)
    assert lib.dvgo_sample_rays(fake, fake, nul, 40000, ctypes.byref(box), 0.1, 10, nul, nul, nul, nul, 1, fake, fake,
                                fake, fake, fake, fake, fake, fake, 1, fake, fake, 1 << 20, nul) == -6
    # workspace too small
    assert lib.dvgo_sample_rays(fake, fake, nul, 100, ctypes.byref(box), 0.1, 10, nul, nul, nul, nul, 0, fake, fake,
                                fake, fake, fake, fake, fake, fake, 1, fake, fake, 8, nul) == -4
    # fine filter without a density grid
    ff = _lib.FineFilter(None, _lib.make_box((-1, -1, -1), (1, 1, 1), (4, 4, 4)), 0.0)
    assert lib.dvgo_sample_rays(fake, fake, nul, 100, ctypes.byref(box), 0.1, 10, nul, nul, nul, ctypes.byref(ff), 0,
                                fake, fake, fake, fake, fake, fake, fake, fake, 1, fake, fake, 1 << 20, nul) == -1
    # adam: t = 0 and bad beta
    assert lib.dvgo_adam_step(fake, fake, fake, fake, nul, 10, 0.1, 0.9, 0.999, 1e-8, 0, nul) == -1
    assert lib.dvgo_adam_step(fake, fake, fake, fake, nul, 10, 0.1, 1.0, 0.999, 1e-8, 1, nul) == -1
    # render: wrong channel count / hidden width / precision code
    f = _lib.Field()
    f.density = 16
    f.feat = 16
    f.channels = 11
    f.box = _lib.make_box((-1, -1, -1), (1, 1, 1), (4, 4, 4))
    m = _lib.Mlp()
    for nm in ("w1", "b1", "w2", "b2", "w3", "b3"):
        setattr(m, nm, 16)
    m.hidden = 128
    bg = (ctypes.c_float * 3)(1, 1, 1)
    args = [fake] * 8 + [fake, fake, 10, 4, 0.1, bg, nul, nul, nul, fake, nul, nul, fake, 1 << 30, nul]
    assert lib.dvgo_render_fwd(ctypes.byref(f), ctypes.byref(m), fake, fake, nul, *args[3:]) == -2
    f.channels = 12
    m.hidden = 64
    assert lib.dvgo_render_fwd(ctypes.byref(f), ctypes.byref(m), fake, fake, nul, *args[3:]) == -2
    m.hidden = 128
    # a grid of 2^31 vertices or more is beyond the int32 vertex and cell indexing
    f.box = _lib.make_box((-1, -1, -1), (1, 1, 1), (2048, 2048, 512))
    assert lib.dvgo_render_fwd(ctypes.byref(f), ctypes.byref(m), fake, fake, nul, *args[3:]) == -6
    f.box = _lib.make_box((-1, -1, -1), (1, 1, 1), (4, 4, 4))
    m.precision = 7
    assert lib.dvgo_render_fwd(ctypes.byref(f), ctypes.byref(m), fake, fake, nul, *args[3:]) == -3
    # the encoded-position network: k_x other than 5
    m.precision = 0
    m.pe_x = 3
    assert lib.dvgo_render_fwd(ctypes.byref(f), ctypes.byref(m), fake, fake, nul, *args[3:]) == -6
    m.pe_x = 0
    # scene: too many spheres
    assert lib.dvgo_scene_render(fake, fake, 1, ctypes.byref(box), fake, 100000, 0.01, 0.01, bg, fake, nul) == -1
    # proposal: bad selection fraction
    assert lib.dvgo_proposal_fwd(fake, fake, fake, nul, 1, ctypes.byref(box), nul, 1.5, 0.9, fake, nul, nul,
                                 nul) == -1
    # proposal: a validity mask without the t_near it belongs to
    assert lib.dvgo_proposal_fwd(fake, fake, nul, fake, 1, ctypes.byref(box), nul, 0.99, 0.9, fake, nul, nul,
                                 nul) == -1
    # proposal backward with its Adam step: no optimiser state, then a bad beta
    pr = _lib.Prop(16, 16, 16, 16, 16, 16)
    pargs = [fake, fake, nul, nul, 1, ctypes.byref(box), ctypes.byref(pr), fake, fake, fake]
    assert lib.dvgo_proposal_bwd_adam(*pargs, None, fake, fake, 1 << 30, nul) == -1
    st = _lib.AdamState(16, 16, 16, 1e-3, 1.0, 0.999, 1e-8, 1)
    assert lib.dvgo_proposal_bwd_adam(*pargs, ctypes.byref(st), fake, fake, 1 << 30, nul) == -1
    # fused backward + grid Adam: missing optimiser state, bad beta, misaligned
    # feature pointer, then a shape error from the shared validation
    ga = _lib.GridAdam(16, 16, 16, 16, 16, 16, None, 0.1, 0.9, 0.999, 1e-8, 1)
    bargs = [fake, fake, nul, fake, fake, fake, fake, fake, fake, fake, 10, 4, 0.1, bg, fake, fake, nul, nul]
    f.channels = 12
    m.precision = 0
    assert lib.dvgo_render_bwd_adam(ctypes.byref(f), ctypes.byref(m), *bargs, None, fake, fake, 1 << 30, nul) == -1
    ga.beta1 = 1.0
    assert lib.dvgo_render_bwd_adam(ctypes.byref(f), ctypes.byref(m), *bargs, ctypes.byref(ga), fake, fake, 1 << 30,
                                    nul) == -1
    ga.beta1 = 0.9
    ga.feat = 20
    assert lib.dvgo_render_bwd_adam(ctypes.byref(f), ctypes.byref(m), *bargs, ctypes.byref(ga), fake, fake, 1 << 30,
                                    nul) == -1
    ga.feat = 16
    ga.active = 18   # activity mask not 4-byte aligned
    assert lib.dvgo_render_bwd_adam(ctypes.byref(f), ctypes.byref(m), *bargs, ctypes.byref(ga), fake, fake, 1 << 30,
                                    nul) == -1
    ga.active = None
    f.channels = 11
    assert lib.dvgo_render_bwd_adam(ctypes.byref(f), ctypes.byref(m), *bargs, ctypes.byref(ga), fake, fake, 1 << 30,
                                    nul) == -2
    # activity mask from moments: negative count, missing or misaligned
    # pointers; an empty grid is a no-op
    assert lib.dvgo_grid_active_init(fake, fake, fake, fake, -1, fake, nul) == -1
    assert lib.dvgo_grid_active_init(fake, fake, None, fake, 10, fake, nul) == -1
    assert lib.dvgo_grid_active_init(fake, fake, 20, fake, 10, fake, nul) == -1
    assert lib.dvgo_grid_active_init(fake, fake, fake, fake, 10, 18, nul) == -1
    assert lib.dvgo_grid_active_init(None, None, None, None, 0, None, nul) == 0
    # finite-difference reduction: no output, negative counts, more rays than
    # the batch without an index list, missing inputs
    assert lib.dvgo_fd_reduce_f64(fake, fake, nul, 4, 4, nul, nul) == -1
    assert lib.dvgo_fd_reduce_f64(fake, fake, nul, -1, 4, fake, nul) == -1
    assert lib.dvgo_fd_reduce_f64(fake, fake, nul, 5, 4, fake, nul) == -2
    assert lib.dvgo_fd_reduce_f64(nul, fake, fake, 5, 4, fake, nul) == -1


def test_host_scalars_match_the_oracle(lib):
    """The method's scalar hyperparameters computed by the library (no GPU):
    the low-density shift, the coarse free-space threshold and the learning
    rate schedule, against the oracle's definitions."""
    import math

    import numpy as np

    import oracle as O
    from paper_2111_11215_amd import api
    for a, s in [(1e-2, 2.0 / 159), (1e-6, 2.0 / 99), (0.5, 1.0), (1e-3, 2.0 / 255)]:
        b = api.low_density_bias(a, s)
        ref = O.low_density_bias(a, s)
        # the oracle evaluates the formula as written, (1-a)^(-1/s) - 1, which
        # cancels for small a (about 1e-11 relative at a = 1e-6)
        assert abs(b - ref) <= 1e-10 * abs(ref)
        # definition: one voxel at sigma = softplus(b) lets 1 - alpha_init through
        assert abs(math.exp(-math.log1p(math.exp(b)) * s) - (1 - a)) < 1e-12
    for tau, step, b in [(1e-4, 0.5 * 2 / 159, 0.0), (1e-3, 0.5 * 2 / 99, 0.2016), (1e-4, 0.5 * 2 / 255, -1.3)]:
        thr = api.coarse_raw_threshold(tau, step, b)
        assert thr == float(O.coarse_raw_threshold(tau, step, b))
        # largest float32 not above the exact threshold: alpha at thr is below tau
        # or at it, and at the next float32 above it reaches tau
        nxt = float(np.nextafter(np.float32(thr), np.float32(np.inf)))
        alpha = lambda raw: -math.expm1(-math.log1p(math.exp(raw + b)) * step)
        assert alpha(thr) <= tau * (1 + 1e-9) and alpha(nxt) >= tau
    for base, it in [(0.1, 0), (0.1, 20000), (1e-3, 777), (1e-3, 123456)]:
        assert abs(api.lr_at(base, it) - O.lr_at(base, it)) <= 1e-15 * base
    assert abs(api.lr_at(1e-3, 20000) - 1e-4) < 1e-18


def test_host_scalars_reject_bad_arguments(lib):
    import ctypes as C
    d, f = C.c_double(), C.c_float()
    assert lib.dvgo_low_density_bias(0.0, 0.1, C.byref(d)) == -1
    assert lib.dvgo_low_density_bias(1e-2, 0.0, C.byref(d)) == -1
    assert lib.dvgo_low_density_bias(1e-2, 0.1, None) == -1
    assert lib.dvgo_coarse_raw_threshold(1.0, 0.1, 0.0, C.byref(f)) == -1
    assert lib.dvgo_coarse_raw_threshold(1e-4, -0.1, 0.0, C.byref(f)) == -1
    assert lib.dvgo_coarse_raw_threshold(1e-4, 0.1, float("nan"), C.byref(f)) == -1
    assert lib.dvgo_lr_at(0.1, -1, 20000, 0.1, C.byref(d)) == -1
    assert lib.dvgo_lr_at(0.1, 1, 0, 0.1, C.byref(d)) == -1


def test_pg_resolution_matches_the_oracle(lib):
    import oracle as O
    from paper_2111_11215_amd import api
    for n, K in ((160, 3), (256, 3), (100, 2), (64, 0)):
        assert [api.pg_resolution(n, K, k) for k in range(K + 1)] == O.pg_resolutions(n, K)
