"""The torch.autograd face of the renderer: a torch loss over (rgb, depth,
acc) back-propagates through the library's hand-written adjoint, and the
grid and network gradients match the FP64 oracle's adjoint (same tolerances
and ReLU-kink budget as the direct parity tests); gradients of outputs the
loss does not use arrive as None and are skipped."""

import numpy as np
import pytest

from tests.helpers import assert_close, np_of, to_dev
from tests.test_gpu_render import TOL32, _check_backward, _gpu, _oracle, _problem

pytestmark = pytest.mark.gpu
F32 = np.float32


def _leaves(grid, flat):
    d = grid.density.clone().requires_grad_()
    f = grid.feat.clone().requires_grad_()
    m = flat.clone().requires_grad_()
    return d, f, m


def test_autograd_matches_oracle_adjoint(gpu_lib):
    from paper_2111_11215_amd import autograd as AG
    P = _problem(5, n_rays=2048, bias=0.2)
    grid, flat, s = _gpu(P)
    d, f, m = _leaves(grid, flat)
    rgb, depth, acc = AG.render(d, f, m, s, P.box_min, P.box_max, P.act_shift, P.bg)
    rng = np.random.default_rng(6)
    B = P.rays.o.shape[0]
    gR, gD, gA = rng.normal(size=(B, 3)), rng.normal(size=B), rng.normal(size=B)
    loss = (rgb * to_dev(gR.astype(F32))).sum() + (depth * to_dev(gD.astype(F32))).sum() + \
        (acc * to_dev(gA.astype(F32))).sum()
    loss.backward()
    samp, prm, ref, ro = _oracle(P)
    ref["_samp"] = samp
    for key, got in (("rgb", rgb), ("depth", depth), ("acc", acc)):
        assert_close(key, np_of(got.detach()), ref[key], TOL32)
    _check_backward(P, prm, ref, ro, np_of(d.grad), np_of(f.grad), np_of(m.grad), gR, TOL32, gD, gA)


def test_autograd_rgb_only_equals_direct_adjoint(gpu_lib):
    """Loss on rgb alone: depth and opacity gradients are None and the
    result equals one direct adjoint call with those channels left out:
    bit-identical outputs and network gradient (fixed reduction order), grid
    gradients to float32 rounding (samples reach their cell bins through
    atomics, so the summation order inside a cell may differ between calls)."""
    import torch
    from paper_2111_11215_amd import api
    from paper_2111_11215_amd import autograd as AG
    P = _problem(6, n_rays=1024)
    grid, flat, s = _gpu(P)
    d, f, m = _leaves(grid, flat)
    rgb, _, _ = AG.render(d, f, m, s, P.box_min, P.box_max, P.act_shift, P.bg)
    (rgb * 0.5).sum().backward()
    out = api.render_fwd(grid, flat, s, P.bg)
    gd, gf, gm = torch.zeros_like(grid.density), torch.zeros_like(grid.feat), torch.zeros_like(flat)
    api.render_bwd(grid, flat, s, out["log_t_end"], torch.full_like(out["rgb"], 0.5), gd, gf, gm, P.bg)
    assert torch.equal(rgb.detach(), out["rgb"])
    assert torch.equal(m.grad, gm)
    assert_close("grad_density", np_of(d.grad), np_of(gd), 1e-6)
    assert_close("grad_feat", np_of(f.grad), np_of(gf), 1e-6)
