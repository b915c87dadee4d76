"""Pins of the oracle's image-fitting toy (Sec. 3, pre-, in- and
post-activation on a 2D grid): bilinear interpolation against torch's
grid_sample, the gradient against torch autograd, and the supplementary
2D-cell derivation (a post-activated cell reproduces a sharp linear
boundary; the pre-activated one cannot).  CPU only."""

import numpy as np
import pytest
import torch

import oracle as O


def _torch_forward(V, H, W, mode, delta):
    """Independent torch form: grid_sample (bilinear, align_corners=True)
    at the pixel centres, the activations from torch."""
    gh, gw = V.shape
    ii, jj = torch.meshgrid(torch.arange(H, dtype=torch.float64), torch.arange(W, dtype=torch.float64),
                            indexing="ij")
    y = 2.0 * ((ii + 0.5) * (gh - 1) / H) / (gh - 1) - 1.0
    x = 2.0 * ((jj + 0.5) * (gw - 1) / W) / (gw - 1) - 1.0
    grid = torch.stack([x, y], dim=-1)[None]
    F = torch.nn.functional
    alpha = lambda s: 1.0 - torch.exp(-s * delta)
    samp = lambda t: F.grid_sample(t[None, None], grid, mode="bilinear", align_corners=True)[0, 0]
    if mode == "pre":
        return samp(alpha(F.softplus(V)))
    if mode == "in":
        return alpha(samp(F.softplus(V)))
    return alpha(F.softplus(samp(V)))


@pytest.mark.parametrize("mode", O.TOY_MODES)
def test_toy2d_forward_matches_grid_sample(mode):
    rng = np.random.default_rng(3)
    V = rng.normal(size=(9, 13)) * 3
    got = O.toy2d_forward(V, 40, 52, mode, delta=0.7)
    ref = _torch_forward(torch.tensor(V), 40, 52, mode, 0.7).numpy()
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("mode", O.TOY_MODES)
def test_toy2d_gradient_matches_autograd(mode):
    rng = np.random.default_rng(4)
    V = rng.normal(size=(7, 6)) * 2
    T = (rng.random((30, 24)) < 0.4).astype(np.float64)
    L, g = O.toy2d_loss_grad(V, T, mode, delta=1.0)
    tV = torch.tensor(V, requires_grad=True)
    Lt = ((_torch_forward(tV, 30, 24, mode, 1.0) - torch.tensor(T)) ** 2).mean()
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-13
    assert np.allclose(g, tV.grad.numpy(), rtol=1e-10, atol=1e-15)


def test_toy2d_cell_reproduces_the_2d_derivation():
    """One cell (2 x 2 vertices) with the corner values of the 2D derivation
    for c(t) = 0.5 t + 0.3 (eps 1e-4, Delta 0.2, delta 0.5): on every image
    row, post-activation is within eps of the step outside the Delta band
    around the boundary; pre-activation with the same values is not (it is
    a bilinear blend of the corner alphas)."""
    eps, D, delta = 1e-4, 0.2, 0.5
    tl, tr, bl, br = O.cell_fit_2d(0.3, 0.8, delta, eps, D)
    V = np.array([[tl, tr], [bl, br]])      # rows: t = 0 (top), t = 1; columns: x = 0, 1
    H = W = 400
    a = O.toy2d_forward(V, H, W, "post", delta)
    t = (np.arange(H) + 0.5) / H
    x = (np.arange(W) + 0.5) / W
    c = 0.5 * t + 0.3
    far_lo = x[None, :] < c[:, None] - D
    far_hi = x[None, :] > c[:, None] + D
    assert np.all(a[far_lo] <= eps * (1 + 1e-9))
    assert np.all(a[far_hi] >= 1 - eps * (1 + 1e-9))
    pre = O.toy2d_forward(V, H, W, "pre", delta)
    assert np.mean((pre[far_lo | far_hi] > 0.01) & (pre[far_lo | far_hi] < 0.99)) > 0.3
    # the pre-activated value at the cell centre is the mean of the corner alphas
    Vc = np.array([[tl, tr], [bl, br]])
    mid = O.toy2d_forward(Vc, 2, 2, "pre", delta)
    corner_alpha = O.density_to_alpha(O.softplus(Vc), delta)
    w = O.toy2d_weights(2, 2, 2, 2)[2]
    assert np.allclose(mid.ravel(), w @ np.array([corner_alpha[0, 0], corner_alpha[0, 1], corner_alpha[1, 0],
                                                   corner_alpha[1, 1]]), rtol=1e-13)
