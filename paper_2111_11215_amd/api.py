"""Thin torch-facing wrappers of the C ABI (argument marshalling only).

Every function takes and returns device tensors, allocates its outputs with
torch (device memory is torch's), passes raw pointers and the current HIP
stream to ``libdvgo.so`` and raises ``DvgoError`` on a non-zero status.  No
arithmetic of the method happens here.
"""

from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib
from ._lib import DVGO_BF16, DVGO_F32, AdamState, Box, Field, GridAdam, Mlp, Prop, check, load, make_box

NSEG = 32
HIDDEN = 128
CHANNELS = 12


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return ctypes.c_void_p(t.data_ptr())


def _stream(device=None) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


_WS: dict = {}


def workspace(nbytes: int, device) -> torch.Tensor:
    """A cached uint8 device buffer of at least ``nbytes`` per (device,
    stream); calls on one stream are ordered, so reuse is safe."""
    key = (torch.device(device).index, torch.cuda.current_stream(device).cuda_stream)
    buf = _WS.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        _WS[key] = buf
    return buf


# ---------------------------------------------------------------------------
# host-side scalar hyperparameters
# ---------------------------------------------------------------------------
def low_density_bias(alpha_init: float, voxel: float) -> float:
    """``dvgo_low_density_bias``: the softplus shift b of the low-density
    initialisation for voxel size ``voxel``."""
    out = ctypes.c_double()
    check("dvgo_low_density_bias", load().dvgo_low_density_bias(float(alpha_init), float(voxel), ctypes.byref(out)))
    return out.value


def coarse_raw_threshold(tau: float, step: float, act_shift: float = 0.0) -> float:
    """``dvgo_coarse_raw_threshold``: the float32 raw-density threshold of
    the coarse free-space test at sample spacing ``step``."""
    out = ctypes.c_float()
    check("dvgo_coarse_raw_threshold", load().dvgo_coarse_raw_threshold(float(tau), float(step), float(act_shift),
                                                                        ctypes.byref(out)))
    return out.value


def lr_at(base_lr: float, it: int, decay_steps: int = 20000, decay: float = 0.1) -> float:
    """``dvgo_lr_at``: the learning rate at iteration ``it`` of the
    exponential schedule."""
    out = ctypes.c_double()
    check("dvgo_lr_at", load().dvgo_lr_at(float(base_lr), int(it), int(decay_steps), float(decay), ctypes.byref(out)))
    return out.value


def pg_resolution(n_final: int, n_checkpoints: int, k: int) -> int:
    """``dvgo_pg_resolution``: vertices per axis before checkpoint k of a
    progressively scaled grid."""
    out = ctypes.c_int32()
    check("dvgo_pg_resolution", load().dvgo_pg_resolution(int(n_final), int(n_checkpoints), int(k),
                                                          ctypes.byref(out)))
    return out.value


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------
@dataclass
class Grid:
    """Fine scene grids on the device: density [n,n,n] and channel-last
    features [n,n,n,12] float32, an optional bfloat16 feature shadow, the box
    and the softplus shift."""
    density: torch.Tensor
    feat: torch.Tensor
    box_min: tuple
    box_max: tuple
    act_shift: float
    feat_shadow: Optional[torch.Tensor] = None   # int16 storage of bf16 values

    @property
    def n(self):
        return tuple(self.density.shape)

    def field(self, use_shadow: bool = False) -> Field:
        f = Field()
        f.density = self.density.data_ptr()
        if use_shadow:
            assert self.feat_shadow is not None
            f.feat = self.feat_shadow.data_ptr()
            f.feat_dtype = DVGO_BF16
        else:
            f.feat = self.feat.data_ptr()
            f.feat_dtype = DVGO_F32
        f.channels = self.feat.shape[-1]
        f.box = make_box(self.box_min, self.box_max, self.n)
        f.act_shift = float(self.act_shift)
        return f


def mlp_shapes(pe_x: int = 0):
    """Flat layout of the colour network; pe_x = 5 adds the encoded query
    position (33 inputs) between the features and the view encoding."""
    n_in = CHANNELS + (3 + 6 * pe_x if pe_x else 0) + 27
    return [("w1", (HIDDEN, n_in)), ("b1", (HIDDEN,)), ("w2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
            ("w3", (3, HIDDEN)), ("b3", (3,))]


MLP_SHAPES = mlp_shapes(0)
MLP_SHAPES_PE_X = mlp_shapes(5)
PROP_SHAPES = [("w1", (64, 54)), ("b1", (64,)), ("w2", (64, 64)), ("b2", (64,)), ("w3", (NSEG, 64)),
               ("b3", (NSEG,))]


def split_flat(flat: torch.Tensor, shapes):
    out, off = {}, 0
    for name, shp in shapes:
        n = math.prod(shp)
        out[name] = flat[off:off + n].view(shp)
        off += n
    assert off == flat.numel()
    return out


def flat_from(arrays, shapes, device) -> torch.Tensor:
    parts = [torch.as_tensor(a, dtype=torch.float32).reshape(-1) for a in arrays]
    flat = torch.cat(parts).to(device)
    assert flat.numel() == sum(math.prod(s) for _, s in shapes)
    return flat


def mlp_struct(flat: torch.Tensor, precision: int = DVGO_F32) -> Mlp:
    """dvgo_mlp over a flat parameter tensor; its size tells the 39-input
    network from the one with the encoded position (72 inputs)."""
    pe_x = 5 if flat.numel() == sum(math.prod(s) for _, s in MLP_SHAPES_PE_X) else 0
    v = split_flat(flat, mlp_shapes(pe_x))
    m = Mlp()
    for name in ("w1", "b1", "w2", "b2", "w3", "b3"):
        setattr(m, name, v[name].data_ptr())
    m.hidden = HIDDEN
    m.precision = precision
    m.pe_x = pe_x
    return m


def prop_struct(flat: torch.Tensor) -> Prop:
    v = split_flat(flat, PROP_SHAPES)
    p = Prop()
    for name in ("w1", "b1", "w2", "b2", "w3", "b3"):
        setattr(p, name, v[name].data_ptr())
    return p


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------
@dataclass
class Samples:
    """Output of ``sample_rays`` plus the per-ray inputs later calls need."""
    rays_o: torch.Tensor
    rays_d: torch.Tensor
    jitter: Optional[torch.Tensor]
    step: float
    t_near: torch.Tensor
    t_far: torch.Tensor
    valid: torch.Tensor
    n_uniform: torch.Tensor
    perm: torch.Tensor
    ray_offset: torch.Tensor
    sample_ray: torch.Tensor
    sample_k: torch.Tensor
    n_kept: torch.Tensor
    capacity: int

    @property
    def B(self) -> int:
        return self.rays_o.shape[0]


def coarse_mask_build(raw: torch.Tensor, cmin, cmax, raw_threshold: float) -> torch.Tensor:
    lib = load()
    n = tuple(raw.shape)
    ncell = (n[0] - 1) * (n[1] - 1) * (n[2] - 1)
    bits = torch.empty((ncell + 31) // 32, dtype=torch.int32, device=raw.device)
    box = make_box(cmin, cmax, n)
    check("dvgo_coarse_mask_build",
          lib.dvgo_coarse_mask_build(_ptr(raw), ctypes.byref(box), raw_threshold, _ptr(bits), _stream(raw.device)))
    return bits


def sample_rays(rays_o, rays_d, jitter, box_min, box_max, step, max_samples, coarse=None, seg_mask=None,
                morton=False, capacity=None, clip_only=False, no_alloc=False, fine=None) -> Samples:
    """``coarse`` = (bits, cmin, cmax, cn) or None; seg_mask int32 [B] or None;
    ``fine`` = (fine density [n0,n1,n2], raw threshold) on the sampling box,
    the second free-space rule, or None.
    ``clip_only``: t_near, t_far, valid, n_uniform and perm only (no list).
    ``no_alloc``: call dvgo_sample_rays_noalloc (the library's static scratch
    instead of a workspace)."""
    lib = load()
    dev = rays_o.device
    B = rays_o.shape[0]
    if clip_only:
        capacity = 0
    if capacity is None:
        capacity = B * int(max_samples)
    t_near = torch.empty(B, dtype=torch.float32, device=dev)
    t_far = torch.empty_like(t_near)
    valid = torch.empty(B, dtype=torch.uint8, device=dev)
    n_uniform = torch.empty(B, dtype=torch.int32, device=dev)
    perm = torch.empty(B, dtype=torch.int32, device=dev)
    if clip_only:
        ray_offset = sample_ray = sample_k = n_kept = None
    else:
        ray_offset = torch.empty(B + 1, dtype=torch.int32, device=dev)
        sample_ray = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        sample_k = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        n_kept = torch.empty(1, dtype=torch.int64, device=dev)
    box = make_box(box_min, box_max)
    cbits, cbox = None, None
    if coarse is not None:
        cbits = coarse[0]
        cbox = make_box(coarse[1], coarse[2], coarse[3])
    ff = None
    if fine is not None:
        assert fine[0].is_cuda and fine[0].is_contiguous()
        ff = _lib.FineFilter(fine[0].data_ptr(), make_box(box_min, box_max, tuple(fine[0].shape)), float(fine[1]))
    fptr = ctypes.byref(ff) if ff is not None else None
    if no_alloc:
        check("dvgo_sample_rays_noalloc", lib.dvgo_sample_rays_noalloc(
            _ptr(rays_o), _ptr(rays_d), _ptr(jitter), B, ctypes.byref(box), float(step), int(max_samples),
            _ptr(cbits), ctypes.byref(cbox) if cbox is not None else None, _ptr(seg_mask), fptr, int(bool(morton)),
            _ptr(t_near), _ptr(t_far), _ptr(valid), _ptr(n_uniform), _ptr(perm), _ptr(ray_offset), _ptr(sample_ray),
            _ptr(sample_k), int(capacity), _ptr(n_kept), _stream(dev)))
        return Samples(rays_o, rays_d, jitter, float(step), t_near, t_far, valid, n_uniform, perm, ray_offset,
                       sample_ray, sample_k, n_kept, int(capacity))
    nws = lib.dvgo_sample_workspace_bytes(B)
    ws = workspace(nws, dev)
    check("dvgo_sample_rays", lib.dvgo_sample_rays(
        _ptr(rays_o), _ptr(rays_d), _ptr(jitter), B, ctypes.byref(box), float(step), int(max_samples),
        _ptr(cbits), ctypes.byref(cbox) if cbox is not None else None, _ptr(seg_mask), fptr, int(bool(morton)),
        _ptr(t_near), _ptr(t_far), _ptr(valid), _ptr(n_uniform), _ptr(perm), _ptr(ray_offset), _ptr(sample_ray),
        _ptr(sample_k), int(capacity), _ptr(n_kept), _ptr(ws), nws, _stream(dev)))
    return Samples(rays_o, rays_d, jitter, float(step), t_near, t_far, valid, n_uniform, perm, ray_offset,
                   sample_ray, sample_k, n_kept, int(capacity))


def _bg(bg):
    arr = (ctypes.c_float * 3)(*[float(x) for x in bg])
    return arr


def render_fwd(grid: Grid, mlp_flat: Optional[torch.Tensor], s: Samples, bg=(1.0, 1.0, 1.0),
               precision: int = DVGO_F32, use_shadow: bool = False, want_seg_w: bool = False,
               want_sample_w: bool = False, want_depth_acc: bool = True) -> dict:
    lib = load()
    dev = s.rays_o.device
    B = s.B
    field = grid.field(use_shadow)
    mlp = mlp_struct(mlp_flat, precision) if mlp_flat is not None else None
    out = {
        "rgb": torch.empty((B, 3), dtype=torch.float32, device=dev) if mlp is not None else None,
        "depth": torch.empty(B, dtype=torch.float32, device=dev) if want_depth_acc else None,
        "acc": torch.empty(B, dtype=torch.float32, device=dev) if want_depth_acc else None,
        "log_t_end": torch.empty(B, dtype=torch.float32, device=dev),
        "seg_w": torch.empty((B, NSEG), dtype=torch.float32, device=dev) if want_seg_w else None,
        "sample_w": torch.empty(max(s.capacity, 1), dtype=torch.float32, device=dev) if want_sample_w else None,
    }
    nws = lib.dvgo_render_workspace_bytes(B, s.capacity, CHANNELS, ctypes.byref(field.box))
    ws = workspace(nws, dev)
    check("dvgo_render_fwd", lib.dvgo_render_fwd(
        ctypes.byref(field), ctypes.byref(mlp) if mlp is not None else None, _ptr(s.rays_o), _ptr(s.rays_d),
        _ptr(s.jitter), _ptr(s.t_near), _ptr(s.n_uniform), _ptr(s.perm), _ptr(s.ray_offset), _ptr(s.sample_ray),
        _ptr(s.sample_k), _ptr(s.n_kept), s.capacity, B, s.step, _bg(bg), _ptr(out["rgb"]), _ptr(out["depth"]),
        _ptr(out["acc"]), _ptr(out["log_t_end"]), _ptr(out["seg_w"]), _ptr(out["sample_w"]), _ptr(ws), nws,
        _stream(dev)))
    return out


def render_bwd(grid: Grid, mlp_flat: Optional[torch.Tensor], s: Samples, log_t_end: torch.Tensor,
               grad_rgb: Optional[torch.Tensor], grad_density: torch.Tensor, grad_feat: Optional[torch.Tensor],
               grad_mlp: Optional[torch.Tensor], bg=(1.0, 1.0, 1.0), precision: int = DVGO_F32,
               use_shadow: bool = False, grad_depth=None, grad_acc=None) -> None:
    """Accumulates (+=) into grad_density, grad_feat and grad_mlp."""
    lib = load()
    dev = s.rays_o.device
    field = grid.field(use_shadow)
    mlp = mlp_struct(mlp_flat, precision) if mlp_flat is not None else None
    nws = lib.dvgo_render_workspace_bytes(s.B, s.capacity, CHANNELS, ctypes.byref(field.box))
    ws = workspace(nws, dev)
    check("dvgo_render_bwd", lib.dvgo_render_bwd(
        ctypes.byref(field), ctypes.byref(mlp) if mlp is not None else None, _ptr(s.rays_o), _ptr(s.rays_d),
        _ptr(s.jitter), _ptr(s.t_near), _ptr(s.n_uniform), _ptr(s.perm), _ptr(s.ray_offset), _ptr(s.sample_ray),
        _ptr(s.sample_k), _ptr(s.n_kept), s.capacity, s.B, s.step, _bg(bg), _ptr(log_t_end), _ptr(grad_rgb),
        _ptr(grad_depth), _ptr(grad_acc), _ptr(grad_density), _ptr(grad_feat), _ptr(grad_mlp), _ptr(ws), nws,
        _stream(dev)))


def grid_active_words(n_vertices: int) -> int:
    return (n_vertices + 31) // 32


def grid_active_init(density_m: torch.Tensor, density_v: torch.Tensor, feat_m: torch.Tensor,
                     feat_v: torch.Tensor, active: torch.Tensor) -> None:
    """Rewrite the activity mask (int32 words, one bit per vertex) from the
    given moments: bit set iff any of the vertex's moments is non-zero."""
    lib = load()
    nv = density_m.numel()
    assert active.dtype == torch.int32 and active.numel() >= grid_active_words(nv)
    check("dvgo_grid_active_init", lib.dvgo_grid_active_init(_ptr(density_m), _ptr(density_v), _ptr(feat_m),
                                                             _ptr(feat_v), nv, _ptr(active), _stream(active.device)))


def _grid_adam(grid: Grid, density_m, density_v, feat_m, feat_v, lr, t, betas, eps, active) -> GridAdam:
    return GridAdam(_ptr(grid.density), _ptr(density_m), _ptr(density_v), _ptr(grid.feat), _ptr(feat_m),
                    _ptr(feat_v), _ptr(grid.feat_shadow), float(lr), float(betas[0]), float(betas[1]), float(eps),
                    int(t), _ptr(active))


def render_bwd_adam(grid: Grid, mlp_flat: torch.Tensor, s: Samples, log_t_end: torch.Tensor,
                    grad_rgb: torch.Tensor, density_m: torch.Tensor, density_v: torch.Tensor,
                    feat_m: torch.Tensor, feat_v: torch.Tensor, grad_mlp: torch.Tensor, lr: float, t: int,
                    betas=(0.9, 0.999), eps=1e-8, bg=(1.0, 1.0, 1.0), precision: int = DVGO_F32,
                    use_shadow: bool = False, grad_depth=None, grad_acc=None, active=None) -> None:
    """Adjoint plus the Adam step of both grids (parameters and moments
    updated in place, the bfloat16 feature copy rewritten when the grid has
    one); accumulates (+=) the network gradient into grad_mlp.  ``active``:
    the optional per-vertex activity mask (int32 words) that lets the step
    skip vertices with zero moments and no samples."""
    lib = load()
    dev = s.rays_o.device
    field = grid.field(use_shadow)
    mlp = mlp_struct(mlp_flat, precision)
    opt = _grid_adam(grid, density_m, density_v, feat_m, feat_v, lr, t, betas, eps, active)
    nws = lib.dvgo_render_workspace_bytes(s.B, s.capacity, CHANNELS, ctypes.byref(field.box))
    ws = workspace(nws, dev)
    check("dvgo_render_bwd_adam", lib.dvgo_render_bwd_adam(
        ctypes.byref(field), ctypes.byref(mlp), _ptr(s.rays_o), _ptr(s.rays_d), _ptr(s.jitter), _ptr(s.t_near),
        _ptr(s.n_uniform), _ptr(s.perm), _ptr(s.ray_offset), _ptr(s.sample_ray), _ptr(s.sample_k), _ptr(s.n_kept),
        s.capacity, s.B, s.step, _bg(bg), _ptr(log_t_end), _ptr(grad_rgb), _ptr(grad_depth), _ptr(grad_acc),
        ctypes.byref(opt), _ptr(grad_mlp), _ptr(ws), nws, _stream(dev)))


def train_step(grid: Grid, mlp_flat: torch.Tensor, s: Samples, target: torch.Tensor, density_m: torch.Tensor,
               density_v: torch.Tensor, feat_m: torch.Tensor, feat_v: torch.Tensor, grad_mlp: torch.Tensor,
               lr: float, t: int, betas=(0.9, 0.999), eps=1e-8, bg=(1.0, 1.0, 1.0), precision: int = DVGO_F32,
               use_shadow: bool = False, want_rgb: bool = True, active=None, mlp_adam=None, aux=None):
    """Forward, photometric loss, adjoint and the grids' Adam step in one
    library call; accumulates (+=) the network gradient into grad_mlp.
    ``active`` as in render_bwd_adam.  ``mlp_adam`` = (m, v, lr) or
    (m, v, lr, t_net): the network (``mlp_flat``) also takes its Adam step in
    the call, with the same betas and eps and step count t (or t_net), and
    grad_mlp is left zero.  ``aux`` = (w_pt_rgb, w_bg_entropy): the
    auxiliary losses' weights.  Returns (loss [1], rgb [B,3] or None)."""
    lib = load()
    dev = s.rays_o.device
    field = grid.field(use_shadow)
    mlp = mlp_struct(mlp_flat, precision)
    opt = _grid_adam(grid, density_m, density_v, feat_m, feat_v, lr, t, betas, eps, active)
    net = None
    if mlp_adam is not None:
        m_, v_, lr_ = mlp_adam[:3]
        t_net = mlp_adam[3] if len(mlp_adam) > 3 else t
        net = AdamState(_ptr(mlp_flat), _ptr(m_), _ptr(v_), float(lr_), float(betas[0]), float(betas[1]), float(eps),
                        int(t_net))
    rgb = torch.empty((s.B, 3), dtype=torch.float32, device=dev) if want_rgb else None
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    nws = lib.dvgo_render_workspace_bytes(s.B, s.capacity, CHANNELS, ctypes.byref(field.box))
    ws = workspace(nws, dev)
    check("dvgo_train_step", lib.dvgo_train_step(
        ctypes.byref(field), ctypes.byref(mlp), _ptr(s.rays_o), _ptr(s.rays_d), _ptr(s.jitter), _ptr(s.t_near),
        _ptr(s.n_uniform), _ptr(s.perm), _ptr(s.ray_offset), _ptr(s.sample_ray), _ptr(s.sample_k), _ptr(s.n_kept),
        s.capacity, s.B, s.step, _bg(bg), _ptr(target), _ptr(rgb), _ptr(loss), ctypes.byref(opt), _ptr(grad_mlp),
        ctypes.byref(net) if net is not None else None,
        ctypes.byref(_lib.AuxLoss(float(aux[0]), float(aux[1]))) if aux is not None else None, _ptr(ws), nws,
        _stream(dev)))
    return loss, rgb


def photo_loss(rgb: torch.Tensor, target: torch.Tensor):
    lib = load()
    grad = torch.empty_like(rgb)
    loss = torch.empty(1, dtype=torch.float32, device=rgb.device)
    check("dvgo_photo_loss", lib.dvgo_photo_loss(_ptr(rgb), _ptr(target), rgb.shape[0], _ptr(grad), _ptr(loss),
                                                 _stream(rgb.device)))
    return loss, grad


def fd_reduce_f64(rgb: torch.Tensor, weight: torch.Tensor, rays: Optional[torch.Tensor] = None) -> torch.Tensor:
    """sum over the listed rays (all when None) of weight . rgb, in float64
    on the device (a one-element double tensor)."""
    lib = load()
    out = torch.empty(1, dtype=torch.float64, device=rgb.device)
    n = rays.numel() if rays is not None else rgb.shape[0]
    check("dvgo_fd_reduce_f64", lib.dvgo_fd_reduce_f64(_ptr(rgb), _ptr(weight), _ptr(rays), n, rgb.shape[0],
                                                       _ptr(out), _stream(rgb.device)))
    return out


def adam_step(p, g, m, v, lr, t, betas=(0.9, 0.999), eps=1e-8, shadow=None) -> None:
    lib = load()
    check("dvgo_adam_step", lib.dvgo_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), _ptr(shadow), p.numel(),
                                               float(lr), float(betas[0]), float(betas[1]), float(eps), int(t),
                                               _stream(p.device)))


def proposal_fwd(s: Samples, box_min, box_max, prop_flat: Optional[torch.Tensor], cum_frac=0.99, min_mass=0.9,
                 logits: Optional[torch.Tensor] = None):
    """With prop_flat None, ``logits`` is an input and only the selection runs."""
    lib = load()
    dev = s.rays_o.device
    B = s.B
    if logits is None:
        logits = torch.empty((B, NSEG), dtype=torch.float32, device=dev)
    mass = torch.empty(B, dtype=torch.float32, device=dev)
    mask = torch.empty(B, dtype=torch.int32, device=dev)
    box = make_box(box_min, box_max)
    prop = prop_struct(prop_flat) if prop_flat is not None else None
    check("dvgo_proposal_fwd", lib.dvgo_proposal_fwd(
        _ptr(s.rays_o), _ptr(s.rays_d), _ptr(s.t_near), _ptr(s.valid), B, ctypes.byref(box),
        ctypes.byref(prop) if prop is not None else None, float(cum_frac), float(min_mass), _ptr(logits),
        _ptr(mass), _ptr(mask), _stream(dev)))
    return logits, mass, mask


def proposal_fwd_rays(rays_o: torch.Tensor, rays_d: torch.Tensor, box_min, box_max, prop_flat: torch.Tensor,
                      cum_frac=0.99, min_mass=0.9):
    """proposal_fwd on bare rays: the call clips them against the box itself
    (the sampler's recipe), so no clip pass runs before it."""
    lib = load()
    dev = rays_o.device
    B = rays_o.shape[0]
    logits = torch.empty((B, NSEG), dtype=torch.float32, device=dev)
    mass = torch.empty(B, dtype=torch.float32, device=dev)
    mask = torch.empty(B, dtype=torch.int32, device=dev)
    box = make_box(box_min, box_max)
    prop = prop_struct(prop_flat)
    check("dvgo_proposal_fwd", lib.dvgo_proposal_fwd(
        _ptr(rays_o), _ptr(rays_d), None, None, B, ctypes.byref(box), ctypes.byref(prop), float(cum_frac),
        float(min_mass), _ptr(logits), _ptr(mass), _ptr(mask), _stream(dev)))
    return logits, mass, mask


def proposal_bwd(s: Samples, box_min, box_max, prop_flat: torch.Tensor, seg_w: torch.Tensor,
                 log_t_end: torch.Tensor, grad_prop: torch.Tensor):
    lib = load()
    dev = s.rays_o.device
    box = make_box(box_min, box_max)
    prop = prop_struct(prop_flat)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    nws = lib.dvgo_proposal_workspace_bytes(s.B)
    ws = torch.empty(max(nws, 256), dtype=torch.uint8, device=dev)
    check("dvgo_proposal_bwd", lib.dvgo_proposal_bwd(
        _ptr(s.rays_o), _ptr(s.rays_d), _ptr(s.t_near), _ptr(s.valid), s.B, ctypes.byref(box), ctypes.byref(prop),
        _ptr(seg_w), _ptr(log_t_end), _ptr(grad_prop), _ptr(loss), _ptr(ws), nws, _stream(dev)))
    return loss


def proposal_bwd_adam(s: Samples, box_min, box_max, prop_flat: torch.Tensor, seg_w: torch.Tensor,
                      log_t_end: torch.Tensor, grad_prop: torch.Tensor, m: torch.Tensor, v: torch.Tensor, lr, t,
                      betas=(0.9, 0.999), eps=1e-8):
    """proposal_bwd then the Adam step of prop_flat, in one call (the step is
    taken where the gradient is summed; grad_prop is left zero)."""
    lib = load()
    dev = s.rays_o.device
    box = make_box(box_min, box_max)
    prop = prop_struct(prop_flat)
    opt = AdamState(_ptr(prop_flat), _ptr(m), _ptr(v), float(lr), float(betas[0]), float(betas[1]), float(eps),
                    int(t))
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    nws = lib.dvgo_proposal_workspace_bytes(s.B)
    ws = torch.empty(max(nws, 256), dtype=torch.uint8, device=dev)
    check("dvgo_proposal_bwd_adam", lib.dvgo_proposal_bwd_adam(
        _ptr(s.rays_o), _ptr(s.rays_d), _ptr(s.t_near), _ptr(s.valid), s.B, ctypes.byref(box), ctypes.byref(prop),
        _ptr(seg_w), _ptr(log_t_end), _ptr(grad_prop), ctypes.byref(opt), _ptr(loss), _ptr(ws), nws, _stream(dev)))
    return loss


def scene_render(rays_o, rays_d, spheres_f32: torch.Tensor, box_min, box_max, step, bg=(1.0, 1.0, 1.0),
                 edge=0.01) -> torch.Tensor:
    lib = load()
    dev = rays_o.device
    B = rays_o.shape[0]
    rgb = torch.empty((B, 3), dtype=torch.float32, device=dev)
    box = make_box(box_min, box_max)
    check("dvgo_scene_render", lib.dvgo_scene_render(_ptr(rays_o), _ptr(rays_d), B, ctypes.byref(box),
                                                     _ptr(spheres_f32), spheres_f32.shape[0], float(edge),
                                                     float(step), _bg(bg), _ptr(rgb), _stream(dev)))
    return rgb


def toy2d_forward(V: torch.Tensor, H: int, W: int, mode: int, delta: float = 1.0) -> torch.Tensor:
    """``dvgo_toy2d_forward``: the predicted alpha image [H, W] of grid V."""
    lib = load()
    img = torch.empty((H, W), dtype=torch.float32, device=V.device)
    check("dvgo_toy2d_forward", lib.dvgo_toy2d_forward(_ptr(V), V.shape[0], V.shape[1], H, W, int(mode),
                                                       float(delta), _ptr(img), _stream(V.device)))
    return img


def toy2d_loss_grad(V: torch.Tensor, target: torch.Tensor, mode: int, delta: float = 1.0, grad=None):
    """``dvgo_toy2d_loss_grad``: (loss [1], dloss/dV [gh, gw])."""
    lib = load()
    H, W = target.shape
    grad = torch.empty_like(V) if grad is None else grad
    loss = torch.empty(1, dtype=torch.float32, device=V.device)
    nws = lib.dvgo_toy2d_workspace_bytes(H, W)
    ws = workspace(nws, V.device)
    check("dvgo_toy2d_loss_grad", lib.dvgo_toy2d_loss_grad(_ptr(V), V.shape[0], V.shape[1], _ptr(target), H, W,
                                                           int(mode), float(delta), _ptr(grad), _ptr(loss), _ptr(ws),
                                                           nws, _stream(V.device)))
    return loss, grad


def render_image(grid: Grid, mlp_flat: torch.Tensor, c2w, origin, H: int, W: int, focal: float, step: float,
                 max_samples: int, coarse=None, bg=(1.0, 1.0, 1.0), precision: int = DVGO_F32,
                 use_shadow: bool = False, chunk: int = 1 << 16, want_rays: bool = False, fine=None) -> dict:
    """``dvgo_render_image``: rgb [H*W, 3], depth and acc [H*W] of one
    pinhole view (c2w: 3x3 camera-to-world rotation); with ``want_rays``
    also the cast rays."""
    lib = load()
    dev = grid.density.device
    field = grid.field(use_shadow)
    mlp = mlp_struct(mlp_flat, precision)
    cam = _lib.Camera()
    for k, v in enumerate([float(x) for row in c2w for x in row]):
        cam.c2w[k] = v
    for k in range(3):
        cam.origin[k] = float(origin[k])
    cam.H, cam.W, cam.focal = int(H), int(W), float(focal)
    n = H * W
    out = {"rgb": torch.empty((n, 3), dtype=torch.float32, device=dev),
           "depth": torch.empty(n, dtype=torch.float32, device=dev),
           "acc": torch.empty(n, dtype=torch.float32, device=dev)}
    if want_rays:
        out["rays_o"] = torch.empty((n, 3), dtype=torch.float32, device=dev)
        out["rays_d"] = torch.empty((n, 3), dtype=torch.float32, device=dev)
    cbits, cbox = None, None
    if coarse is not None:
        cbits = coarse[0]
        cbox = make_box(coarse[1], coarse[2], coarse[3])
    ff = None
    if fine is not None:
        ff = _lib.FineFilter(fine[0].data_ptr(), make_box(grid.box_min, grid.box_max, tuple(fine[0].shape)),
                             float(fine[1]))
    nws = lib.dvgo_render_image_workspace_bytes(int(chunk), int(max_samples), ctypes.byref(field.box))
    ws = workspace(nws, dev)
    check("dvgo_render_image", lib.dvgo_render_image(
        ctypes.byref(field), ctypes.byref(mlp), ctypes.byref(cam), float(step), int(max_samples), _ptr(cbits),
        ctypes.byref(cbox) if cbox is not None else None, ctypes.byref(ff) if ff is not None else None, _bg(bg),
        int(chunk), _ptr(out["rgb"]), _ptr(out["depth"]),
        _ptr(out["acc"]), _ptr(out.get("rays_o")), _ptr(out.get("rays_d")), _ptr(ws), nws, _stream(dev)))
    return out


def grid_resample(src: torch.Tensor, n_new, box_min, box_max) -> torch.Tensor:
    """``dvgo_grid_resample``: src [n0,n1,n2(,C)] resized to n_new vertices per
    axis over the same box."""
    lib = load()
    C = 1 if src.dim() == 3 else src.shape[3]
    out_shape = tuple(n_new) + (() if src.dim() == 3 else (C,))
    dst = torch.empty(out_shape, dtype=torch.float32, device=src.device)
    sb = make_box(box_min, box_max, tuple(src.shape[:3]))
    db = make_box(box_min, box_max, tuple(n_new))
    check("dvgo_grid_resample", lib.dvgo_grid_resample(_ptr(src), ctypes.byref(sb), int(C), _ptr(dst),
                                                       ctypes.byref(db), _stream(src.device)))
    return dst


def coarse_step(density: torch.Tensor, rgb_grid: torch.Tensor, box_min, box_max, act_shift: float, s: Samples,
                target: torch.Tensor, grad_density: torch.Tensor, grad_rgb: torch.Tensor, max_samples: int,
                w_pt: float = 0.1, w_bg: float = 0.01, bg=(1.0, 1.0, 1.0), want_rgb: bool = False):
    """``dvgo_coarse_step``: forward, the coarse objective and its gradient
    accumulated (+=) into grad_density and grad_rgb.  Returns (loss [1],
    rgb [B,3] or None)."""
    lib = load()
    dev = density.device
    f = _lib.CoarseField(density.data_ptr(), rgb_grid.data_ptr(), make_box(box_min, box_max, tuple(density.shape)),
                         float(act_shift))
    rgb = torch.empty((s.B, 3), dtype=torch.float32, device=dev) if want_rgb else None
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    nws = lib.dvgo_coarse_workspace_bytes(s.B)
    ws = workspace(nws, dev)
    check("dvgo_coarse_step", lib.dvgo_coarse_step(
        ctypes.byref(f), _ptr(s.rays_o), _ptr(s.rays_d), _ptr(s.jitter), _ptr(s.t_near), _ptr(s.perm),
        _ptr(s.ray_offset), _ptr(s.sample_k), _ptr(s.n_kept), s.capacity, s.B, int(max_samples), s.step, _bg(bg),
        _ptr(target), float(w_pt), float(w_bg), _ptr(rgb), _ptr(grad_density), _ptr(grad_rgb), _ptr(loss), _ptr(ws),
        nws, _stream(dev)))
    return loss, rgb


def view_counts(n, box_min, box_max, cams: torch.Tensor, H: int, W: int, focal: float):
    """``dvgo_view_counts``: (counts int32 [n], lr_scale float32 [n]); cams
    [ncam, 12] device float32 (row-major R, centre)."""
    lib = load()
    dev = cams.device
    counts = torch.empty(tuple(n), dtype=torch.int32, device=dev)
    scale = torch.empty(tuple(n), dtype=torch.float32, device=dev)
    box = make_box(box_min, box_max, tuple(n))
    nws = lib.dvgo_view_counts_workspace_bytes()
    ws = torch.empty(max(nws, 256), dtype=torch.uint8, device=dev)
    check("dvgo_view_counts", lib.dvgo_view_counts(ctypes.byref(box), _ptr(cams), cams.shape[0], int(H), int(W),
                                                   float(focal), _ptr(counts), _ptr(scale), _ptr(ws), nws,
                                                   _stream(dev)))
    return counts, scale


def adam_step_scaled(p, g, m, v, lr_scale, lr, t, betas=(0.9, 0.999), eps=1e-8) -> None:
    lib = load()
    check("dvgo_adam_step_scaled", lib.dvgo_adam_step_scaled(_ptr(p), _ptr(g), _ptr(m), _ptr(v), _ptr(lr_scale),
                                                             p.numel(), float(lr), float(betas[0]), float(betas[1]),
                                                             float(eps), int(t), _stream(p.device)))
