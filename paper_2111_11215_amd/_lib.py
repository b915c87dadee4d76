"""ctypes loader for ``libdvgo.so`` and the C structs of ``include/dvgo.h``.

The library is loaded from this package directory only; if it is missing
the import of any GPU entry point fails loudly (there is no fallback).
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_void_p

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdvgo.so")

DVGO_F32, DVGO_BF16 = 0, 1
DVGO_TOY_PRE, DVGO_TOY_IN, DVGO_TOY_POST = 0, 1, 2

STATUS = {0: "DVGO_OK", -1: "DVGO_E_ARG", -2: "DVGO_E_SHAPE", -3: "DVGO_E_DTYPE",
          -4: "DVGO_E_CAPACITY", -5: "DVGO_E_HIP", -6: "DVGO_E_UNSUPPORTED"}


class Box(ctypes.Structure):
    _fields_ = [("xyz_min", c_float * 3), ("xyz_max", c_float * 3), ("n", c_int32 * 3)]


class FineFilter(ctypes.Structure):
    _fields_ = [("density", c_void_p), ("box", Box), ("raw_threshold", c_float)]


class AuxLoss(ctypes.Structure):
    _fields_ = [("w_pt_rgb", c_float), ("w_bg_entropy", c_float)]


class CoarseField(ctypes.Structure):
    _fields_ = [("density", c_void_p), ("rgb", c_void_p), ("box", Box), ("act_shift", c_float)]


class Field(ctypes.Structure):
    _fields_ = [("density", c_void_p), ("feat", c_void_p), ("feat_dtype", c_int32), ("channels", c_int32),
                ("box", Box), ("act_shift", c_float)]


class Mlp(ctypes.Structure):
    _fields_ = [("w1", c_void_p), ("b1", c_void_p), ("w2", c_void_p), ("b2", c_void_p), ("w3", c_void_p),
                ("b3", c_void_p), ("hidden", c_int32), ("precision", c_int32), ("pe_x", c_int32)]


class Prop(ctypes.Structure):
    _fields_ = [("w1", c_void_p), ("b1", c_void_p), ("w2", c_void_p), ("b2", c_void_p), ("w3", c_void_p),
                ("b3", c_void_p)]


class GridAdam(ctypes.Structure):
    _fields_ = [("density", c_void_p), ("density_m", c_void_p), ("density_v", c_void_p), ("feat", c_void_p),
                ("feat_m", c_void_p), ("feat_v", c_void_p), ("feat_shadow_bf16", c_void_p), ("lr", c_float),
                ("beta1", c_float), ("beta2", c_float), ("eps", c_float), ("t", c_int32), ("active", c_void_p)]


class AdamState(ctypes.Structure):
    _fields_ = [("param", c_void_p), ("m", c_void_p), ("v", c_void_p), ("lr", c_float), ("beta1", c_float),
                ("beta2", c_float), ("eps", c_float), ("t", c_int32)]


class Camera(ctypes.Structure):
    _fields_ = [("c2w", c_float * 9), ("origin", c_float * 3), ("H", c_int32), ("W", c_int32), ("focal", c_float)]


class DvgoError(RuntimeError):
    def __init__(self, fn: str, status: int, text: str, last: str):
        super().__init__(f"{fn} returned {STATUS.get(status, status)} ({text}) {last}".strip())
        self.status = status


P = c_void_p
# name -> (restype, argtypes)
SIGNATURES = {
    "dvgo_mlp_param_count": (c_int64, [c_int32, c_int32, c_int32]),
    "dvgo_prop_param_count": (c_int64, []),
    "dvgo_coarse_mask_build": (c_int32, [P, POINTER(Box), c_float, P, P]),
    "dvgo_sample_workspace_bytes": (c_size_t, [c_int32]),
    "dvgo_sample_rays": (c_int32, [P, P, P, c_int32, POINTER(Box), c_float, c_int32, P, POINTER(Box), P,
                                   POINTER(FineFilter), c_int32, P, P, P, P, P, P, P, P, c_int64, P, P, c_size_t, P]),
    "dvgo_sample_rays_noalloc": (c_int32, [P, P, P, c_int32, POINTER(Box), c_float, c_int32, P, POINTER(Box), P,
                                           POINTER(FineFilter), c_int32, P, P, P, P, P, P, P, P, c_int64, P, P]),
    "dvgo_render_workspace_bytes": (c_size_t, [c_int32, c_int64, c_int32, POINTER(Box)]),
    "dvgo_render_fwd": (c_int32, [POINTER(Field), POINTER(Mlp), P, P, P, P, P, P, P, P, P, P, c_int64, c_int32,
                                  c_float, POINTER(c_float), P, P, P, P, P, P, P, c_size_t, P]),
    "dvgo_render_bwd": (c_int32, [POINTER(Field), POINTER(Mlp), P, P, P, P, P, P, P, P, P, P, c_int64, c_int32,
                                  c_float, POINTER(c_float), P, P, P, P, P, P, P, P, c_size_t, P]),
    "dvgo_render_bwd_adam": (c_int32, [POINTER(Field), POINTER(Mlp), P, P, P, P, P, P, P, P, P, P, c_int64, c_int32,
                                       c_float, POINTER(c_float), P, P, P, P, POINTER(GridAdam), P, P, c_size_t, P]),
    "dvgo_train_step": (c_int32, [POINTER(Field), POINTER(Mlp), P, P, P, P, P, P, P, P, P, P, c_int64, c_int32,
                                  c_float, POINTER(c_float), P, P, P, POINTER(GridAdam), P, POINTER(AdamState),
                                  POINTER(AuxLoss), P, c_size_t, P]),
    "dvgo_photo_loss": (c_int32, [P, P, c_int32, P, P, P]),
    "dvgo_fd_reduce_f64": (c_int32, [P, P, P, c_int32, c_int32, P, P]),
    "dvgo_adam_step": (c_int32, [P, P, P, P, P, c_int64, c_float, c_float, c_float, c_float, c_int32, P]),
    "dvgo_grid_active_init": (c_int32, [P, P, P, P, c_int64, P, P]),
    "dvgo_proposal_fwd": (c_int32, [P, P, P, P, c_int32, POINTER(Box), POINTER(Prop), c_float, c_float, P, P, P,
                                    P]),
    "dvgo_proposal_bwd": (c_int32, [P, P, P, P, c_int32, POINTER(Box), POINTER(Prop), P, P, P, P, P, c_size_t, P]),
    "dvgo_proposal_bwd_adam": (c_int32, [P, P, P, P, c_int32, POINTER(Box), POINTER(Prop), P, P, P,
                                         POINTER(AdamState), P, P, c_size_t, P]),
    "dvgo_proposal_workspace_bytes": (c_size_t, [c_int32]),
    "dvgo_scene_render": (c_int32, [P, P, c_int32, POINTER(Box), P, c_int32, c_float, c_float, POINTER(c_float), P,
                                    P]),
    "dvgo_low_density_bias": (c_int32, [c_double, c_double, POINTER(c_double)]),
    "dvgo_coarse_raw_threshold": (c_int32, [c_double, c_double, c_double, POINTER(c_float)]),
    "dvgo_lr_at": (c_int32, [c_double, c_int64, c_int64, c_double, POINTER(c_double)]),
    "dvgo_pg_resolution": (c_int32, [c_int32, c_int32, c_int32, POINTER(c_int32)]),
    "dvgo_render_fwd_workspace_bytes": (c_size_t, [c_int32, c_int64, c_int32, POINTER(Box)]),
    "dvgo_render_image_workspace_bytes": (c_size_t, [c_int32, c_int32, POINTER(Box)]),
    "dvgo_render_image": (c_int32, [POINTER(Field), POINTER(Mlp), POINTER(Camera), c_float, c_int32, P, POINTER(Box),
                                    POINTER(FineFilter), POINTER(c_float), c_int32, P, P, P, P, P, P, c_size_t, P]),
    "dvgo_grid_resample": (c_int32, [P, POINTER(Box), c_int32, P, POINTER(Box), P]),
    "dvgo_coarse_workspace_bytes": (c_size_t, [c_int32]),
    "dvgo_coarse_step": (c_int32, [POINTER(CoarseField), P, P, P, P, P, P, P, P, c_int64, c_int32, c_int32, c_float,
                                   POINTER(c_float), P, c_float, c_float, P, P, P, P, P, c_size_t, P]),
    "dvgo_view_counts_workspace_bytes": (c_size_t, []),
    "dvgo_view_counts": (c_int32, [POINTER(Box), P, c_int32, c_int32, c_int32, c_float, P, P, P, c_size_t, P]),
    "dvgo_adam_step_scaled": (c_int32, [P, P, P, P, P, c_int64, c_float, c_float, c_float, c_float, c_int32, P]),
    "dvgo_toy2d_workspace_bytes": (c_size_t, [c_int32, c_int32]),
    "dvgo_toy2d_forward": (c_int32, [P, c_int32, c_int32, c_int32, c_int32, c_int32, c_float, P, P]),
    "dvgo_toy2d_loss_grad": (c_int32, [P, c_int32, c_int32, P, c_int32, c_int32, c_int32, c_float, P, P, P, c_size_t,
                                       P]),
    "dvgo_status_string": (c_char_p, [c_int32]),
    "dvgo_last_error": (c_char_p, []),
    "dvgo_version": (c_int32, []),
    "dvgo_profile_enable": (c_int32, [c_int32]),
    "dvgo_profile_read": (c_int32, [POINTER(ctypes.c_double), POINTER(c_int64)]),
}

KERNEL_IDS = {name: i for i, name in enumerate([
    "ray_setup", "morton_sort", "count_kept", "scan", "fill_kept", "coarse_mask", "pack", "ray_base", "gather",
    "mlp_fwd", "compose_fwd", "compose_bwd", "mlp_bwd", "scatter", "reduce", "photo_loss", "adam", "prop_fwd",
    "prop_bwd", "prop_reduce", "scene", "bin_count", "cell_scan", "bin_place", "grid_adam", "grid_active",
    "toy_pixel", "toy_vertex", "toy_reduce", "grid_resample", "coarse_step", "view_count"])}

_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once) and declare every signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build() "
                           "or python paper_2111_11215_amd/build.py)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(fn: str, status: int) -> None:
    if status != 0:
        lib = load()
        raise DvgoError(fn, status, lib.dvgo_status_string(status).decode(), lib.dvgo_last_error().decode())


def make_box(xyz_min, xyz_max, n=(2, 2, 2)) -> Box:
    b = Box()
    for i in range(3):
        b.xyz_min[i] = float(xyz_min[i])
        b.xyz_max[i] = float(xyz_max[i])
        b.n[i] = int(n[i])
    return b
