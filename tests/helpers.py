"""Shared helpers of the test-suite (comparison metrics, tensor plumbing)."""

import numpy as np


def to_dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def np_of(t):
    return t.detach().cpu().numpy()


def normwise(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((got - ref).ravel())
    return num / den if den > 0 else num


def maxrel(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.max(np.abs(ref))
    return np.max(np.abs(got - ref)) / den if den > 0 else np.max(np.abs(got - ref))


def report(name, got, ref):
    nw, mr = normwise(got, ref), maxrel(got, ref)
    print(f"  {name}: normwise {nw:.3e}  max/max {mr:.3e}", flush=True)
    return nw, mr


def mlp_flat_np(Ws, bs):
    return np.concatenate([Ws[0].ravel(), bs[0].ravel(), Ws[1].ravel(), bs[1].ravel(), Ws[2].ravel(),
                           bs[2].ravel()]).astype(np.float32)


def mlp_unflat(g, channels=12, hidden=128):
    i = 0
    out = []
    for shp in [(hidden, channels + 27), (hidden,), (hidden, hidden), (hidden,), (3, hidden), (3,)]:
        n = int(np.prod(shp))
        out.append(g[i:i + n].reshape(shp))
        i += n
    return out


def kink_budget(prm, ref, grad_rgb, zeta_rel, feat_shape, box_min, box_max):
    """Error budget from ReLU decisions that the arithmetic cannot resolve.

    A hidden unit whose oracle pre-activation z satisfies |z| <= zeta_rel *
    (sum of |terms| of its dot product + |bias|) may legitimately take the
    other branch in a float32 (or bfloat16) evaluation.  For every sample
    holding such a unit, any two choices of masks change that sample's
    feature gradient by at most 2*U, U = |dz3| |W3| |W2| |W1f| (absolute
    values bound every masked product), and its weight-gradient
    contributions by at most 2x the norms bounded the same way.  Returns
    (per-grid-entry feature budget, per-tensor weight budgets dict, fraction
    of ambiguous samples)."""
    import oracle as O
    cache = ref["cache"]
    mc = cache["mcache"]
    W1, W2, W3 = [np.asarray(w, np.float64) for w in prm.Ws]
    b1, b2, _ = [np.asarray(b, np.float64) for b in prm.bs]
    x, h1 = mc["x"], mc["h1"]
    s1 = np.abs(x) @ np.abs(W1).T + np.abs(b1)
    s2 = np.abs(h1) @ np.abs(W2).T + np.abs(b2)
    amb = (np.abs(mc["z1"]) <= zeta_rel * s1).any(1) | (np.abs(mc["z2"]) <= zeta_rel * s2).any(1)
    g = np.asarray(grad_rgb, np.float64)[np.asarray(ref_perm_slots(ref))]
    dc = cache["w"][:, None] * g
    c = mc["c"]
    dz3 = np.abs(dc * c * (1 - c))
    dh2 = dz3 @ np.abs(W3)
    dh1 = dh2 @ np.abs(W2)
    U = dh1 @ np.abs(W1[:, :feat_shape[-1]])
    Ua = np.where(amb[:, None], 2.0 * U, 0.0)
    grid_budget = O.interp_scatter(feat_shape, cache["x"], box_min, box_max, Ua)
    nx = np.linalg.norm(x, axis=1)
    nh1 = np.linalg.norm(h1, axis=1)
    w_b = {
        "W1": 2.0 * np.sum(np.linalg.norm(dh1, axis=1)[amb] * nx[amb]),
        "b1": 2.0 * np.sum(np.linalg.norm(dh1, axis=1)[amb]),
        "W2": 2.0 * np.sum(np.linalg.norm(dh2, axis=1)[amb] * nh1[amb]),
        "b2": 2.0 * np.sum(np.linalg.norm(dh2, axis=1)[amb]),
        "W3": 0.0, "b3": 0.0,
    }
    return grid_budget, w_b, float(amb.mean())


def ref_perm_slots(ref):
    """Ray id of every compact sample of an oracle forward (slot -> ray)."""
    return ref["_sample_ray"]


def check_grid_grad(name, got, ref, budget, tol):
    """Normwise tol on entries no ambiguous sample touches; elsewhere the
    difference must stay within the kink budget (plus tol of the max)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    touched = budget > 0
    nw = normwise(got[~touched], ref[~touched])
    slack = np.abs(got - ref)[touched] - budget[touched] - tol * np.max(np.abs(ref))
    worst = float(slack.max()) if slack.size else -1.0
    print(f"  {name}: normwise(untouched) {nw:.3e}, touched entries {int(touched.sum())}, "
          f"max excess over budget {worst:.3e}", flush=True)
    assert nw <= tol, name
    assert worst <= 0.0, name


def check_weight_grads(got_flat, ref_Ws, ref_bs, budgets, tol):
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    refs = [ref_Ws[0], ref_bs[0], ref_Ws[1], ref_bs[1], ref_Ws[2], ref_bs[2]]
    for name, a, b in zip(names, mlp_unflat(np.asarray(got_flat)), refs):
        err = np.linalg.norm(np.asarray(a, np.float64) - b)
        allowed = tol * np.linalg.norm(b) + budgets[name]
        print(f"  {name}: normwise {err / np.linalg.norm(b):.3e} (allowed {allowed / np.linalg.norm(b):.3e})",
              flush=True)
        assert err <= allowed, name
