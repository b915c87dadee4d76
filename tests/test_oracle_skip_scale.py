"""Pins of the oracle's second free-space rule (the fine-density alpha skip)
and of progressive scaling (grid resize by trilinear interpolation and the
resolution schedule).  CPU only."""

import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle as O
import synth

F32 = np.float32


def test_trilinear_f32_recipe_close_to_float64():
    """The float32 recipe agrees with float64 trilinear interpolation to
    float32 rounding of 8 products and 7 sums (also on a constant grid), and
    is exact at vertices."""
    rng = np.random.default_rng(0)
    g = rng.uniform(-3, 3, (9, 7, 11)).astype(F32)
    x = rng.uniform(-1.2, 1.2, (5000, 3)).astype(F32)
    a = O.trilinear_f32(g, x, [-1] * 3, [1] * 3)
    b = O.interp(g, x.astype(np.float64), [-1] * 3, [1] * 3)
    assert a.dtype == F32
    assert np.max(np.abs(a - b)) <= 32 * 2.0 ** -24 * 3.0
    c = np.full((4, 4, 4), F32(1.75))
    assert np.max(np.abs(O.trilinear_f32(c, x, [-1] * 3, [1] * 3) - 1.75)) <= 16 * 2.0 ** -24 * 1.75
    v = np.array([[-1, -1, -1], [1, 1, 1], [-1, 1, -1]], F32)
    assert np.array_equal(O.trilinear_f32(g, v, [-1] * 3, [1] * 3), np.array([g[0, 0, 0], g[-1, -1, -1], g[0, -1, 0]]))


def test_fine_skip_keeps_every_point_above_tau():
    """Brute force over every sample of a batch: the kept samples are those
    whose float64 post-activated fine alpha reaches tau (up to float32
    rounding of the interpolated value), and with the rule off the list is
    the plain one."""
    P = synth.tiny_config(3, jitter=True, n_rays=256)
    rng = np.random.default_rng(1)
    P.density = (rng.normal(size=P.density.shape) * 3 - 1).astype(F32)
    b, tau = 0.3, 1e-2
    thr = O.coarse_raw_threshold(tau, P.step, b)
    plain = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples)
    skip = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples,
                         fine=(P.density, thr))
    r = plain["sample_ray"].astype(np.int64)
    t = O.sample_t(plain["t_near"][r], P.rays.jitter[r], plain["sample_k"], P.step)
    x = O.sample_x(P.rays.o[r], P.rays.d[r], t)
    raw64 = O.interp(P.density, x.astype(np.float64), P.box_min, P.box_max)
    alpha = O.post_activated_alpha(raw64, b, P.step)
    kept = set(zip(skip["sample_ray"].tolist(), skip["sample_k"].tolist()))
    keep = np.array([(a_, k_) in kept for a_, k_ in zip(plain["sample_ray"].tolist(), plain["sample_k"].tolist())])
    assert 0.1 < keep.mean() < 0.9
    margin = 1e-4   # relative: float32 rounding of the interpolated raw value moves alpha by far less
    assert np.all(alpha[keep] >= tau * (1 - margin))
    assert np.all(alpha[~keep] < tau * (1 + margin))
    off = O.sample_rays(P.rays.o, P.rays.d, P.rays.jitter, P.box_min, P.box_max, P.step, P.max_samples,
                        fine=(P.density, np.float32(-np.inf)))
    for k in ("ray_offset", "sample_ray", "sample_k"):
        assert np.array_equal(off[k], plain[k])


def test_grid_resample_identity_affine_and_scipy():
    rng = np.random.default_rng(2)
    g = rng.normal(size=(6, 5, 7, 3))
    same = O.grid_resample(g, (6, 5, 7), [-1] * 3, [1] * 3)
    assert np.allclose(same, g, rtol=0, atol=1e-13)
    # an affine field is reproduced exactly at any resolution
    ax = [np.linspace(-1, 1, n) for n in (6, 5, 7)]
    X = np.stack(np.meshgrid(*ax, indexing="ij"), -1)
    aff = (X @ np.array([0.3, -1.2, 2.0]) + 0.7)[..., None]
    up = O.grid_resample(aff, (11, 9, 4), [-1] * 3, [1] * 3)
    ax2 = [np.linspace(-1, 1, n) for n in (11, 9, 4)]
    X2 = np.stack(np.meshgrid(*ax2, indexing="ij"), -1)
    assert np.allclose(up[..., 0], X2 @ np.array([0.3, -1.2, 2.0]) + 0.7, atol=1e-12)
    # scipy's linear grid interpolator at the new vertices
    ref = RegularGridInterpolator(ax, g[..., 1])(X2.reshape(-1, 3)).reshape(11, 9, 4)
    assert np.allclose(O.grid_resample(g, (11, 9, 4), [-1] * 3, [1] * 3)[..., 1], ref, atol=1e-12)


def test_pg_resolutions_double_the_voxels():
    """160^3 with three checkpoints: 80, 100, 126, 160 vertices per axis; the
    vertex count roughly doubles at each checkpoint (floors aside) and the
    first grid has 1/8 of the final count."""
    r = O.pg_resolutions(160, 3)
    assert r == [80, 100, 126, 160]
    assert r[0] ** 3 * 8 == 160 ** 3
    for a, b in zip(r[:-1], r[1:]):
        assert 1.9 < b ** 3 / a ** 3 < 2.1
    assert O.pg_resolutions(64, 0) == [64]
