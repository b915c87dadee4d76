"""GPU parity of the learned proposal: the segment selection and the
predicted mass bit-exact from the same float32 logits (float32 recipe), the
bfloat16 network forward and backward against the oracle's bfloat16 form:
1e-3 normwise and 4e-3 of the largest entry per entry (R23's two metrics; the
float32 encoding may round to a neighbouring bfloat16 value, which moves one
product term by 2^-8 of itself; measured values printed)."""

import numpy as np
import pytest

import oracle as O
import synth
from tests.helpers import assert_close, np_of, to_dev

pytestmark = pytest.mark.gpu
F32 = np.float32


def _prop_weights(seed):
    rng = np.random.default_rng(seed)
    Ws, bs = synth.xavier_uniform_mlp(rng, (54, 64, 64, 32))
    Ws = [(w * 3).astype(F32) for w in Ws]
    bs = [(rng.normal(size=b.shape) * 0.5).astype(F32) for b in bs]
    flat = np.concatenate([Ws[0].ravel(), bs[0], Ws[1].ravel(), bs[1], Ws[2].ravel(), bs[2]]).astype(F32)
    return Ws, bs, flat


def _samples(P):
    from paper_2111_11215_amd import api
    return api.sample_rays(to_dev(P.rays.o), to_dev(P.rays.d), None, P.box_min, P.box_max, P.step, P.max_samples)


def test_selection_bit_exact_from_logits(gpu_lib):
    from paper_2111_11215_amd import api
    P = synth.tiny_config(0, n_rays=2048)
    s = _samples(P)
    rng = np.random.default_rng(4)
    z = (rng.normal(size=(2048, 32)) * rng.uniform(0.1, 6, (2048, 1)) + rng.normal(size=(2048, 1)) * 3).astype(F32)
    z[:64] = -20.0         # one dominant segment and ten tied ones: nine of the
    z[:64, 10] = 20.0      # ties are needed, so the lower indices must win
    z[:64, 0:10] = 15.4
    z[64:128] = -20.0      # tiny mass: fallback
    _, mass, mask = api.proposal_fwd(s, P.box_min, P.box_max, None, logits=to_dev(z))
    want = O.proposal_select(z)
    valid = np_of(s.valid).astype(bool)
    want = np.where(valid, want, np.uint32(0xFFFFFFFF))
    assert np.array_equal(np_of(mask).view(np.uint32), want)
    tie_rows = np.where(valid[:64])[0]
    assert np.all(want[tie_rows] == np.uint32((1 << 10) | 0x1FF))
    _, m_ref = O.proposal_select_probs(z)
    assert np.array_equal(np_of(mass), m_ref)


def test_proposal_forward_backward_bf16(gpu_lib):
    import torch
    from paper_2111_11215_amd import api
    P = synth.tiny_config(1, n_rays=1024)
    s = _samples(P)
    Ws, bs, flat = _prop_weights(2)
    ft = to_dev(flat)
    logits, mass, mask = api.proposal_fwd(s, P.box_min, P.box_max, ft)
    tn, tf, v = O.ray_box_clip(P.rays.o, P.rays.d, P.box_min, P.box_max)
    enc = O.proposal_encoding(P.rays.o, P.rays.d, tn, P.box_min, P.box_max)
    z, cache = O.proposal_forward(Ws, bs, enc, bf16=True)
    assert_close("logits", np_of(logits)[v], z[v], 1e-3, 4e-3)
    # targets from the oracle's density-only render of a random grid
    prm = O.Params(P.density, P.feat, P.Ws, P.bs, P.box_min, P.box_max, 0.0)
    samp = O.sample_rays(P.rays.o, P.rays.d, None, P.box_min, P.box_max, P.step, P.max_samples)
    ref = O.render_forward(prm, P.rays.o, P.rays.d, None, samp, P.step, P.bg, with_color=False)
    seg_w = ref["seg_w"].astype(F32)
    lte = ref["log_t_end"].astype(F32)
    grad = torch.zeros_like(ft)
    loss = api.proposal_bwd(s, P.box_min, P.box_max, ft, to_dev(seg_w), to_dev(lte), grad)
    p = O.proposal_targets(seg_w.astype(np.float64), np.exp(lte.astype(np.float64)))
    zc = z.copy()
    L, dz = O.proposal_loss_grad(zc[v], p[v])
    # the device averages over the whole batch (invalid rays contribute 0)
    L = L * v.sum() / len(v)
    dz_full = np.zeros_like(z)
    dz_full[v] = dz * v.sum() / len(v)
    cache_v = cache
    dWs, dbs = O.proposal_backward(Ws, cache_v, dz_full)
    assert abs(float(np_of(loss)[0]) - L) <= 1e-3 * abs(L) + 1e-6
    g = np_of(grad)
    off = 0
    for name, ref_t in zip(["W1", "b1", "W2", "b2", "W3", "b3"], [dWs[0], dbs[0], dWs[1], dbs[1], dWs[2], dbs[2]]):
        n = ref_t.size
        assert_close(name, g[off:off + n].reshape(ref_t.shape), ref_t, 1e-3, 4e-3)
        off += n


def test_proposal_clips_rays_itself_bit_identically(gpu_lib):
    """dvgo_proposal_fwd without t_near clips each ray itself: logits, mass
    and masks equal those of the call fed by the sampler's clip, bit for bit,
    on rays that miss the box, start inside it, graze it or run along an
    axis; the backward without t_near equals the backward with it."""
    import torch
    from paper_2111_11215_amd import api
    P = synth.tiny_config(2, n_rays=1000)
    o, d = P.rays.o.copy(), P.rays.d.copy()
    o[:8] = [[5, 5, 5], [0.2, 0.1, -0.3], [-3, 1.0, 0.2], [-3, 0.3, 0.2], [0.5, -3, 0.5], [0, 0, 3], [-3, 1, 1],
             [0.99, -0.99, 0.0]]
    d[:8] = [[1, 0, 0], [0, 0, 1], [1, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, -1], [1, 0, 0], [-0.6, 0.8, 0.0]]
    s = api.sample_rays(to_dev(o), to_dev(d), None, P.box_min, P.box_max, P.step, P.max_samples, clip_only=True)
    _, _, flat = _prop_weights(5)
    ft = to_dev(flat)
    z0, m0, k0 = api.proposal_fwd(s, P.box_min, P.box_max, ft, cum_frac=0.9, min_mass=0.2)
    z1, m1, k1 = api.proposal_fwd_rays(s.rays_o, s.rays_d, P.box_min, P.box_max, ft, cum_frac=0.9, min_mass=0.2)
    assert np.array_equal(np_of(z0), np_of(z1))
    assert np.array_equal(np_of(m0), np_of(m1))
    assert np.array_equal(np_of(k0), np_of(k1))
    assert (np_of(k0).view(np.uint32) != 0xFFFFFFFF).any()
    seg_w = to_dev(np.full((1000, 32), 1.0 / 64, F32))
    lte = to_dev(np.full(1000, np.log(0.5), F32))
    g0, g1 = torch.zeros_like(ft), torch.zeros_like(ft)
    l0 = api.proposal_bwd(s, P.box_min, P.box_max, ft, seg_w, lte, g0)
    s_bare = api.Samples(**{**s.__dict__, "t_near": None, "valid": None})
    l1 = api.proposal_bwd(s_bare, P.box_min, P.box_max, ft, seg_w, lte, g1)
    assert np.array_equal(np_of(g0), np_of(g1)) and np.array_equal(np_of(l0), np_of(l1))


def _first_rays(s, n):
    """The per-ray inputs the proposal calls read, cut to the first n rays."""
    from paper_2111_11215_amd import api
    cut = {k: getattr(s, k)[:n].contiguous() for k in ("rays_o", "rays_d", "t_near", "valid")}
    return api.Samples(**{**s.__dict__, **cut})


def test_proposal_bwd_adam_equals_separate_calls(gpu_lib):
    """dvgo_proposal_bwd_adam (the Adam step taken where the gradient is
    summed) equals dvgo_proposal_bwd then dvgo_adam_step bit for bit:
    parameters, both moments and the loss over three steps in a row (the
    first on a gradient that already holds a value, the last on fewer rays),
    the gradient left zero, and a call on no rays that still takes the step."""
    import torch
    from paper_2111_11215_amd import api
    P = synth.tiny_config(3, n_rays=1500)
    s_full = _samples(P)
    _, _, flat = _prop_weights(6)
    rng = np.random.default_rng(7)
    seg_w = rng.uniform(0, 1, (1500, 32)).astype(F32)
    seg_w /= seg_w.sum(1, keepdims=True) * 1.25
    lte = np.log(rng.uniform(0.05, 0.3, 1500)).astype(F32)
    pa, pb = to_dev(flat), to_dev(flat)
    ma, va = torch.zeros_like(pa), torch.zeros_like(pa)
    mb, vb = torch.zeros_like(pa), torch.zeros_like(pa)
    ga = to_dev(rng.normal(size=flat.shape).astype(F32) * 1e-3)
    gb = ga.clone()
    for t, n in ((1, 1500), (2, 1500), (3, 777)):
        s = _first_rays(s_full, n)
        sw, lt = to_dev(seg_w[:n]), to_dev(lte[:n])
        la = api.proposal_bwd(s, P.box_min, P.box_max, pa, sw, lt, ga)
        api.adam_step(pa, ga, ma, va, 3e-3, t)
        lb = api.proposal_bwd_adam(s, P.box_min, P.box_max, pb, sw, lt, gb, mb, vb, 3e-3, t)
        for x, y in ((pa, pb), (ma, mb), (va, vb), (la, lb), (ga, gb)):
            assert np.array_equal(np_of(x), np_of(y)), t
        assert not np_of(gb).any()
    s0 = _first_rays(s_full, 0)
    ga.copy_(to_dev(rng.normal(size=flat.shape).astype(F32) * 1e-3))
    gb.copy_(ga)
    api.adam_step(pa, ga, ma, va, 3e-3, 4)
    api.proposal_bwd_adam(s0, P.box_min, P.box_max, pb, to_dev(seg_w[:0]), to_dev(lte[:0]), gb, mb, vb, 3e-3, 4)
    for x, y in ((pa, pb), (ma, mb), (va, vb), (ga, gb)):
        assert np.array_equal(np_of(x), np_of(y))
