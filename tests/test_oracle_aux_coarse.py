"""Pins of the oracle's auxiliary losses (per-point rgb, background entropy)
and of the coarse stage's grid-colour form, by torch autograd of an
independently written per-ray torch forward, and by closed forms.  CPU
only."""

import math

import numpy as np
import torch

import oracle as O
import synth

F32 = np.float32


def _torch_render(dens, feat, Ws, bs, b, o, d, jit, samp, step, bg, grid_colour):
    """Per ray: rgb, T_end and the list of (w_k, c_k), with torch ops (product
    form of the transmittance); the colour is the network's, or
    sigmoid(interp(V_rgb)) in the grid-colour form."""
    t_near = samp["t_near"]
    n = np.array(dens.shape)
    ro = samp["ray_offset"]
    rgbs, tends, per = [], [], []
    for slot in range(o.shape[0]):
        r = int(samp["perm"][slot])
        ks = samp["sample_k"][ro[slot]:ro[slot + 1]]
        T = torch.tensor(1.0, dtype=torch.float64)
        C = torch.zeros(3, dtype=torch.float64)
        pe = [torch.tensor(d[r], dtype=torch.float64)]
        for fr in range(4):
            pe += [torch.sin(pe[0] * 2 ** fr), torch.cos(pe[0] * 2 ** fr)]
        pe = torch.cat(pe)
        wc = []
        for k in ks:
            tk = F32(t_near[r]) + F32(F32(F32(k) + F32(0 if jit is None else jit[r])) * F32(step))
            x = o[r].astype(np.float64) + float(tk) * d[r].astype(np.float64)
            u = (x + 1) / 2 * (n - 1)
            i0 = np.clip(np.floor(u), 0, n - 2).astype(int)
            f = np.clip(u - i0, 0, 1)
            raw, fv = 0, 0
            for c in range(8):
                ofs = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1])
                wgt = float(np.prod(np.where(ofs == 1, f, 1 - f)))
                ii = i0 + ofs
                raw = raw + wgt * dens[ii[0], ii[1], ii[2]]
                fv = fv + wgt * feat[ii[0], ii[1], ii[2]]
            a = 1 - torch.exp(-torch.nn.functional.softplus(raw + b) * step)
            if grid_colour:
                col = torch.sigmoid(fv)
            else:
                h = torch.relu(Ws[0] @ torch.cat([fv, pe]) + bs[0])
                h = torch.relu(Ws[1] @ h + bs[1])
                col = torch.sigmoid(Ws[2] @ h + bs[2])
            wc.append((T * a, col))
            C = C + T * a * col
            T = T * (1 - a)
        rgbs.append(C + T * torch.tensor(bg, dtype=torch.float64))
        tends.append(T)
        per.append(wc)
    return rgbs, tends, per


def _problem(seed, grid_colour, n=4, rays=16):
    rng = np.random.default_rng(seed)
    dens = rng.uniform(-1, 1, (n, n, n)) * 2
    feat = rng.uniform(-1, 1, (n, n, n, 3 if grid_colour else 12))
    Ws, bs = synth.xavier_uniform_mlp(rng, (39, 128, 128, 3))
    bs = [rng.normal(size=b.shape) * 0.2 for b in bs]
    o, d, *_ = synth.draw_pixels_without_replacement(rng, synth.cube_vertex_cameras(), 8, 8, 9.0, rays)
    jit = rng.random(rays).astype(F32)
    tgt = rng.random((rays, 3))
    return dens, feat, (None if grid_colour else Ws), (None if grid_colour else bs), o, d, jit, tgt, 0.5 * 2 / (n - 1)


def _check(grid_colour, w_pt, w_bg, seed):
    dens, feat, Ws, bs, o, d, jit, tgt, step = _problem(seed, grid_colour)
    b, bg = 0.2, np.array([1.0, 0.9, 0.8])
    samp = O.sample_rays(o, d, jit, [-1] * 3, [1] * 3, step, 64)
    prm = O.Params(dens, feat, Ws, bs, [-1] * 3, [1] * 3, b)
    fwd = O.render_forward(prm, o, d, jit, samp, step, bg)
    L_photo, g = O.photo_loss(fwd["rgb"], tgt)
    aux = O.aux_losses(fwd, tgt)
    gr = O.render_backward(prm, o, d, jit, samp, step, bg, fwd, g, grad_c=w_pt * aux["grad_c"],
                           grad_t_end=w_bg * aux["grad_t_end"])
    T = lambda a: torch.tensor(np.asarray(a, np.float64), requires_grad=True)
    td, tf = T(dens), T(feat)
    tW = None if Ws is None else [T(w) for w in Ws]
    tb = None if bs is None else [T(x) for x in bs]
    rgbs, tends, per = _torch_render(td, tf, tW, tb, b, o, d, jit, samp, step, bg, grid_colour)
    B = len(rgbs)
    tt = torch.tensor(tgt)
    photo = sum(((rgbs[r] - tt[r]) ** 2).sum() for r in range(B)) / B
    pt = sum(sum(w.detach() * ((c - tt[r]) ** 2).sum() for w, c in per[r]) for r in range(B) if per[r]) / B
    eps = O.BG_CLAMP
    ent = 0
    for te in tends:
        p = torch.clamp(te, eps, 1 - eps)
        ent = ent + (-p * torch.log(p) - (1 - p) * torch.log(1 - p))
    ent = ent / B
    assert abs(photo.item() - L_photo) < 1e-12
    assert abs(pt.item() - aux["pt"]) < 1e-12
    assert abs(ent.item() - aux["bg"]) < 1e-12
    (photo + w_pt * pt + w_bg * ent).backward()
    assert np.allclose(gr["density"], td.grad.numpy(), rtol=1e-9, atol=1e-13)
    assert np.allclose(gr["feat"], tf.grad.numpy(), rtol=1e-9, atol=1e-13)
    if tW is not None:
        for a, t in zip(gr["Ws"] + gr["bs"], tW + tb):
            assert np.allclose(a, t.grad.numpy(), rtol=1e-9, atol=1e-13)


def test_aux_losses_fine_form_match_autograd():
    _check(False, 1e-2, 1e-3, 0)
    _check(False, 0.7, 0.3, 1)     # weights large enough that a dropped term shows


def test_coarse_grid_colour_form_matches_autograd():
    _check(True, 1e-1, 1e-2, 2)
    _check(True, 0.0, 0.0, 3)


def test_background_entropy_closed_form():
    """H(1/2) = log 2 is the maximum; H is 0 at the clamp ends (up to the
    clamp's own value) and its gradient vanishes at T = 1/2."""
    fwd = {"cache": {"c": np.zeros((0, 3)), "w": np.zeros(0)}, "_sample_ray": np.zeros(0, np.int64),
           "t_end": np.array([0.5, 1.0, 0.0, 0.25])}
    aux = O.aux_losses(fwd, np.zeros((4, 3)))
    h = lambda p: -p * math.log(p) - (1 - p) * math.log(1 - p)
    e = O.BG_CLAMP
    assert abs(aux["bg"] - (math.log(2) + 2 * h(e) + h(0.25)) / 4) < 1e-15
    assert aux["grad_t_end"][0] == 0.0 and aux["grad_t_end"][1] == 0.0 and aux["grad_t_end"][2] == 0.0
    assert abs(aux["grad_t_end"][3] - math.log(3) / 4) < 1e-15


def test_view_counts_frustum_cases():
    """Cameras on the cube vertices looking at the origin: the centre vertex
    is seen by all 8; a vertex behind every camera's image plane direction
    is not seen by the camera it lies behind; the count field has the
    cameras' symmetry; a hand-placed camera with a narrow field of view
    sees only the vertices near its axis."""
    cams = synth.cube_vertex_cameras(4.0)
    R = [synth.look_at_c2w(c) for c in cams]
    n = (9, 9, 9)
    cnt = O.view_counts(n, [-1] * 3, [1] * 3, cams, R, 64, 64, 80.0)
    assert cnt[4, 4, 4] == 8
    assert cnt.max() == 8 and cnt.min() >= 0
    assert np.array_equal(cnt, cnt[::-1, ::-1, ::-1])        # the camera set is symmetric under x -> -x
    # one camera on +z looking down with a field of view of about 2 x 3 degrees
    c = np.array([[0.0, 0.0, 4.0]])
    Rz = [synth.look_at_c2w(c[0])]
    one = O.view_counts(n, [-1] * 3, [1] * 3, c, Rz, 10, 10, 100.0)
    # visible iff -0.05 (4 - z) <= x < 0.05 (4 - z) and -0.05 (4 - z) < y <= 0.05 (4 - z)
    # (image edges at u = 0 and v = 0 included): the axis column x = y = 0, and at
    # z = -1 (half-width 0.25, one vertex spacing) also x = -0.25 and y = 0.25
    assert np.all(one[4, 4, :] == 1) and one.sum() == 12
    assert one[3, 4, 0] == one[4, 5, 0] == one[3, 5, 0] == 1 and one[5, 4, 0] == one[4, 3, 0] == 0
    s = O.view_count_lr_scale(cnt)
    assert s.max() == 1.0 and s[4, 4, 4] == 1.0
