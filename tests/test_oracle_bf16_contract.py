"""Pins of the oracle's bfloat16 network forms against an independent torch
emulation of the fixed bfloat16 contract, and of the proposal network's
float64 forward against torch.  CPU only.

The contract (the "bfloat16 form" of both networks) names exactly which
operands of which products are rounded.  bf(v) is v's float32 value rounded
to bfloat16, round to nearest, ties to even.  Products and sums are exact.

Colour network (input x = [f (12), PE(d) (27)], W1 = [W1f | W1d]; with the
encoded position, x = [f, PE_5(u) (33), PE(d)] and f below stands for the
45 per-sample inputs [f, PE_5(u)], W1f for their 45 columns):
  z1 = bf(f) bf(W1f)^T + (PE(d) W1d^T + b1)     h1 = relu(z1)
  z2 = bf(h1) bf(W2)^T + b2                     h2 = relu(z2)
  z3 = bf(h2) bf(W3)^T + b3                     c  = sigmoid(z3)
  dz3 = dc * c * (1 - c)
  dW3 = bf(dz3)^T bf(h2)       db3 = sum dz3
  dz2 = (bf(dz3) bf(W3)) * [z2 > 0]
  dW2 = bf(dz2)^T bf(h1)       db2 = sum bf(dz2)
  dz1 = (bf(dz2) bf(W2)) * [z1 > 0]
  dW1 = bf(dz1)^T bf(x)        db1 = sum bf(dz1)
  df  = bf(dz1) bf(W1f)
Proposal network (input e, 54 values):
  z1 = bf(e) bf(W1)^T + b1,  z2 = bf(h1) bf(W2)^T + b2,  z = bf(h2) bf(W3)^T + b3
  g3 = bf(dz)                             dW3 = g3^T bf(h2), db3 = sum g3
  g2 = bf((g3 bf(W3)) * [z2 > 0])         dW2 = g2^T bf(h1), db2 = sum g2
  g1 = bf((g2 bf(W2)) * [z1 > 0])         dW1 = g1^T bf(e),  db1 = sum g1

The emulation below is written with torch operations only (its own
rounding through torch's bfloat16 conversion, torch float64 matrix
products), so a misplaced or missing rounding point, a dropped bias or a
transposed operand in the oracle shows up as a difference far above 1e-12.
"""

import numpy as np
import pytest
import torch

import oracle as O
import synth

TOL = 1e-12


def _t(a):
    return torch.tensor(np.asarray(a, np.float64), dtype=torch.float64)


def bf(t: torch.Tensor) -> torch.Tensor:
    """float32 value rounded to bfloat16 (torch's round-to-nearest-even)."""
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    den = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / den)


def _colour_problem(seed, S=300, pe_x=False):
    rng = np.random.default_rng(seed)
    Ws, bs = synth.xavier_uniform_mlp(rng, (72 if pe_x else 39, 128, 128, 3))
    bs = [(rng.normal(size=b.shape) * 0.1).astype(np.float32) for b in bs]
    f = rng.uniform(-1, 1, (S, 12)).astype(np.float32)
    d = rng.normal(size=(S, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    parts = [f.astype(np.float64)]
    if pe_x:
        parts.append(O.positional_encoding(rng.uniform(-1, 1, (S, 3)), 5))
    x = np.concatenate(parts + [O.positional_encoding(d)], axis=1)
    dc = rng.normal(size=(S, 3)) * 1e-2
    return Ws, bs, x, dc


def _torch_colour_bf16(Ws, bs, x, dc, ns=12):
    """ns: the per-sample inputs (12, or 45 with the encoded position)."""
    W1, W2, W3 = [_t(w) for w in Ws]
    b1, b2, b3 = [_t(b) for b in bs]
    X = _t(x)
    f, pe = X[:, :ns], X[:, ns:]
    W1f, W1d = W1[:, :ns], W1[:, ns:]
    z1 = torch.matmul(bf(f), bf(W1f).T) + (torch.matmul(pe, W1d.T) + b1)
    h1 = torch.clamp(z1, min=0.0)
    z2 = torch.matmul(bf(h1), bf(W2).T) + b2
    h2 = torch.clamp(z2, min=0.0)
    z3 = torch.matmul(bf(h2), bf(W3).T) + b3
    c = torch.sigmoid(z3)
    dz3 = _t(dc) * c * (1.0 - c)
    dW3 = torch.matmul(bf(dz3).T, bf(h2))
    db3 = dz3.sum(0)
    dz2 = torch.matmul(bf(dz3), bf(W3)) * (z2 > 0).to(torch.float64)
    dW2 = torch.matmul(bf(dz2).T, bf(h1))
    db2 = bf(dz2).sum(0)
    dz1 = torch.matmul(bf(dz2), bf(W2)) * (z1 > 0).to(torch.float64)
    dW1 = torch.matmul(bf(dz1).T, bf(X))
    db1 = bf(dz1).sum(0)
    df = torch.matmul(bf(dz1), bf(W1f))
    return c, df, [dW1, dW2, dW3], [db1, db2, db3]


@pytest.mark.parametrize("seed,pe_x", [(0, False), (1, False), (2, True)])
def test_colour_bf16_form_matches_torch_emulation(seed, pe_x):
    Ws, bs, x, dc = _colour_problem(seed, pe_x=pe_x)
    ns = 45 if pe_x else 12
    c_ref, df_ref, dW_ref, db_ref = _torch_colour_bf16(Ws, bs, x, dc, ns)
    c, cache = O.mlp_forward(Ws, bs, x, bf16=True, n_feat=ns)
    dx, dWs, dbs = O.mlp_backward(Ws, cache, dc)
    assert _rel(c, c_ref.numpy()) < TOL
    assert _rel(dx[:, :ns], df_ref.numpy()) < TOL
    for name, a, b in zip(["dW1", "dW2", "dW3", "db1", "db2", "db3"], dWs + dbs, dW_ref + db_ref):
        assert _rel(a, b.numpy()) < TOL, name


def test_colour_bf16_emulation_detects_a_moved_rounding_point():
    """The comparison is sharp enough to see one rounding point moved: the
    oracle with the first layer's view part rounded too differs from the
    contract by far more than the tolerance."""
    Ws, bs, x, dc = _colour_problem(3)
    c_ref, *_ = _torch_colour_bf16(Ws, bs, x, dc)
    xr = np.concatenate([x[:, :12], O.bf16_round(x[:, 12:])], axis=1)
    Wr = [np.concatenate([Ws[0][:, :12], O.bf16_round(Ws[0][:, 12:])], axis=1), Ws[1], Ws[2]]
    c_moved, _ = O.mlp_forward(Wr, bs, xr, bf16=True)
    assert _rel(c_moved, c_ref.numpy()) > 1e3 * TOL


def _proposal_problem(seed, B=200):
    rng = np.random.default_rng(seed)
    Ws, bs = synth.xavier_uniform_mlp(rng, (54, 64, 64, 32))
    bs = [(rng.normal(size=b.shape) * 0.1).astype(np.float32) for b in bs]
    o = rng.normal(size=(B, 3)) * 3
    d = rng.normal(size=(B, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    enc = O.proposal_encoding(o, d, rng.random(B), [-1, -1, -1], [1, 1, 1])
    dz = rng.normal(size=(B, 32)) * 1e-2
    return Ws, bs, enc, dz


@pytest.mark.parametrize("seed", [0, 1])
def test_proposal_bf16_form_matches_torch_emulation(seed):
    Ws, bs, enc, dz = _proposal_problem(seed)
    W1, W2, W3 = [_t(w) for w in Ws]
    b1, b2, b3 = [_t(b) for b in bs]
    E = _t(enc)
    z1 = torch.matmul(bf(E), bf(W1).T) + b1
    h1 = torch.clamp(z1, min=0.0)
    z2 = torch.matmul(bf(h1), bf(W2).T) + b2
    h2 = torch.clamp(z2, min=0.0)
    z = torch.matmul(bf(h2), bf(W3).T) + b3
    g3 = bf(_t(dz))
    g2 = bf(torch.matmul(g3, bf(W3)) * (z2 > 0).to(torch.float64))
    g1 = bf(torch.matmul(g2, bf(W2)) * (z1 > 0).to(torch.float64))
    ref_W = [torch.matmul(g1.T, bf(E)), torch.matmul(g2.T, bf(h1)), torch.matmul(g3.T, bf(h2))]
    ref_b = [g1.sum(0), g2.sum(0), g3.sum(0)]

    zo, cache = O.proposal_forward(Ws, bs, enc, bf16=True)
    dWs, dbs = O.proposal_backward(Ws, cache, dz)
    assert _rel(zo, z.numpy()) < TOL
    for name, a, b in zip(["dW1", "dW2", "dW3", "db1", "db2", "db3"], dWs + dbs, ref_W + ref_b):
        assert _rel(a, b.numpy()) < TOL, name


@pytest.mark.parametrize("seed", [0, 1])
def test_proposal_forward_logits_match_torch(seed):
    """float64 proposal logits against torch.nn.functional; a dropped or
    doubled output bias would move them by about 0.1."""
    Ws, bs, enc, _ = _proposal_problem(seed)
    F = torch.nn.functional
    h = F.relu(F.linear(_t(enc), _t(Ws[0]), _t(bs[0])))
    h = F.relu(F.linear(h, _t(Ws[1]), _t(bs[1])))
    ref = F.linear(h, _t(Ws[2]), _t(bs[2])).numpy()
    z, _ = O.proposal_forward(Ws, bs, enc)
    assert _rel(z, ref) < TOL
