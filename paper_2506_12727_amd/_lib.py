"""ctypes binding of libmvgs.so: the C ABI of include/mvgs.h under the same names.

Argument marshalling only: every step of the rasterizer runs in the library's HIP kernels.
Loading fails loudly when the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmvgs.so")

MVGS_OK = 0
MVGS_EINVAL = -1
MVGS_ENOMEM = -2
MVGS_ECAPACITY = -3
MVGS_EHIP = -4
MVGS_ERETRY = -5
MVGS_MAX_VIEWS = 65535
MVGS_MAX_TILES_PER_VIEW = 65536
MVGS_NOALLOC_SCRATCH_BYTES = 32 * 1024 * 1024

EXPORTED = ["mvgs_create", "mvgs_destroy", "mvgs_forward", "mvgs_loss", "mvgs_backward", "mvgs_frame_release",
            "mvgs_frame_info", "mvgs_export_binning", "mvgs_export_transmittance", "mvgs_status_string",
            "mvgs_last_error", "mvgs_profile_enable", "mvgs_profile_read", "mvgs_profile_reset",
            "mvgs_stage_name", "mvgs_frame_work", "mvgs_set_workspace_limit", "mvgs_memory_held",
            "mvgs_frame_workspace", "mvgs_forward_partial", "mvgs_subsample", "mvgs_frame_check",
            "mvgs_frame_set_cameras", "mvgs_loss_3d", "mvgs_export_depth", "mvgs_adapt_density",
            "mvgs_adam_step", "mvgs_gather_rows", "mvgs_grad_moments", "mvgs_frame_merge",
            "mvgs_frame_void_word", "mvgs_count_views", "mvgs_workspace_bound",
            "mvgs_frame_sort_info", "mvgs_loss_noalloc"]
MVGS_PARTIAL_COMPACT = 0
MVGS_PARTIAL_MASKED = 1
MVGS_STAGE_COUNT = 10
MVGS_WORK_FORWARD = 0
MVGS_WORK_LOSS = 1
MVGS_WORK_LOSS_DSSIM = 2
MVGS_WORK_BACKWARD = 4

# allocator callbacks of mvgs_options
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class mvgs_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("bg", C.c_float * 3)]


class mvgs_gaussians(C.Structure):
    _fields_ = [("P", C.c_int64), ("sh_degree", C.c_int32), ("means", C.c_void_p), ("scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacities", C.c_void_p), ("sh", C.c_void_p)]


class mvgs_grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p), ("opacities", C.c_void_p),
                ("sh", C.c_void_p)]


class mvgs_densify(C.Structure):
    _fields_ = [("e1", C.c_void_p), ("e2", C.c_void_p), ("count", C.c_void_p)]


class mvgs_options(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("pixels_per_lane", C.c_int32),
                ("reserved0", C.c_int32), ("workspace_limit", C.c_int64), ("capacity_records", C.c_int64),
                ("capacity_pairs", C.c_int64), ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", C.c_void_p)]


class mvgs_adc_params(C.Structure):
    _fields_ = [("split_threshold", C.c_float), ("clone_threshold", C.c_float), ("dense_scale", C.c_float),
                ("min_opacity", C.c_float)]


class mvgs_gaussians_out(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p), ("opacities", C.c_void_p),
                ("sh", C.c_void_p)]


class mvgs_adam_params(C.Structure):
    _fields_ = [("lr_means", C.c_float), ("lr_scales", C.c_float), ("lr_quats", C.c_float),
                ("lr_opacities", C.c_float), ("lr_sh_dc", C.c_float), ("lr_sh_rest", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("step", C.c_int32),
                ("step_dev", C.c_void_p), ("skip_dev", C.c_void_p)]


class MvgsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"mvgs status {status}: {message}")
        self.status = status


_LIB = None


def lib():
    """Load libmvgs.so. Raises if it is missing: build it with paper_2506_12727_amd/build.py."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: the HIP library must be built (python -c "
                           "'import __graft_entry__ as g; g.build()') before the GPU path can run")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    L.mvgs_create.argtypes = [C.POINTER(vp), C.POINTER(mvgs_options)]
    L.mvgs_create.restype = C.c_int
    L.mvgs_destroy.argtypes = [vp]
    L.mvgs_destroy.restype = None
    L.mvgs_forward.argtypes = [vp, vp, C.POINTER(mvgs_gaussians), C.POINTER(mvgs_camera), i32, vp, C.POINTER(vp)]
    L.mvgs_forward.restype = C.c_int
    L.mvgs_loss.argtypes = [vp, vp, C.POINTER(mvgs_camera), i32, vp, vp, f32, f32, vp, vp]
    L.mvgs_loss.restype = C.c_int
    L.mvgs_loss_noalloc.argtypes = [vp, vp, C.POINTER(mvgs_camera), i32, vp, vp, f32, f32, vp, vp]
    L.mvgs_loss_noalloc.restype = C.c_int
    L.mvgs_backward.argtypes = [vp, vp, C.POINTER(mvgs_gaussians), vp, vp, C.POINTER(mvgs_grads),
                                C.POINTER(mvgs_densify)]
    L.mvgs_backward.restype = C.c_int
    L.mvgs_frame_release.argtypes = [vp, vp]
    L.mvgs_frame_release.restype = C.c_int
    L.mvgs_frame_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.mvgs_frame_info.restype = C.c_int
    L.mvgs_export_binning.argtypes = [vp, vp, vp, vp, vp, vp]
    L.mvgs_export_binning.restype = C.c_int
    L.mvgs_export_transmittance.argtypes = [vp, vp, vp, vp]
    L.mvgs_export_transmittance.restype = C.c_int
    L.mvgs_status_string.argtypes = [C.c_int]
    L.mvgs_status_string.restype = C.c_char_p
    L.mvgs_last_error.argtypes = [vp]
    L.mvgs_last_error.restype = C.c_char_p
    L.mvgs_profile_enable.argtypes = [vp, C.c_int]
    L.mvgs_profile_enable.restype = C.c_int
    L.mvgs_profile_read.argtypes = [vp, vp, vp]
    L.mvgs_profile_read.restype = C.c_int
    L.mvgs_profile_reset.argtypes = [vp]
    L.mvgs_profile_reset.restype = C.c_int
    L.mvgs_stage_name.argtypes = [C.c_int]
    L.mvgs_stage_name.restype = C.c_char_p
    L.mvgs_frame_work.argtypes = [vp, vp, vp, vp]
    L.mvgs_frame_work.restype = C.c_int
    L.mvgs_set_workspace_limit.argtypes = [vp, i64]
    L.mvgs_set_workspace_limit.restype = C.c_int
    L.mvgs_memory_held.argtypes = [vp, C.POINTER(i64)]
    L.mvgs_memory_held.restype = C.c_int
    L.mvgs_frame_workspace.argtypes = [vp, C.POINTER(i64)]
    L.mvgs_frame_workspace.restype = C.c_int
    L.mvgs_forward_partial.argtypes = [vp, vp, C.POINTER(mvgs_gaussians), C.POINTER(mvgs_camera), i32, vp, vp, i64,
                                       i32, vp, C.POINTER(vp)]
    L.mvgs_forward_partial.restype = C.c_int
    L.mvgs_subsample.argtypes = [vp, vp, C.POINTER(mvgs_camera), i32, vp, vp, vp]
    L.mvgs_subsample.restype = C.c_int
    L.mvgs_frame_check.argtypes = [vp, vp, vp]
    L.mvgs_frame_check.restype = C.c_int
    L.mvgs_frame_set_cameras.argtypes = [vp, vp, C.POINTER(mvgs_camera), i32]
    L.mvgs_frame_set_cameras.restype = C.c_int
    L.mvgs_loss_3d.argtypes = [vp, vp, vp, vp, vp, f32, f32, vp, vp]
    L.mvgs_loss_3d.restype = C.c_int
    L.mvgs_frame_sort_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
    L.mvgs_frame_sort_info.restype = C.c_int
    L.mvgs_count_views.argtypes = [vp, vp, C.POINTER(mvgs_gaussians), C.POINTER(mvgs_camera), i32, vp, vp]
    L.mvgs_count_views.restype = C.c_int
    L.mvgs_workspace_bound.argtypes = [vp, C.POINTER(mvgs_camera), i32, i64, i64, i64, i32, C.POINTER(i64)]
    L.mvgs_workspace_bound.restype = C.c_int
    L.mvgs_export_depth.argtypes = [vp, vp, vp, vp]
    L.mvgs_export_depth.restype = C.c_int
    L.mvgs_adapt_density.argtypes = [vp, vp, C.POINTER(mvgs_gaussians), vp, vp, vp, vp, C.POINTER(mvgs_adc_params),
                               C.POINTER(mvgs_gaussians_out), vp, i64, C.POINTER(i64)]
    L.mvgs_adapt_density.restype = C.c_int
    L.mvgs_adam_step.argtypes = [vp, vp, i64, C.c_int32, C.POINTER(mvgs_gaussians_out), C.POINTER(mvgs_grads), vp,
                                 C.POINTER(mvgs_adam_params)]
    L.mvgs_adam_step.restype = C.c_int
    L.mvgs_frame_void_word.argtypes = [vp, C.POINTER(vp)]
    L.mvgs_frame_void_word.restype = C.c_int
    L.mvgs_gather_rows.argtypes = [vp, vp, vp, i64, i64, vp, vp]
    L.mvgs_gather_rows.restype = C.c_int
    L.mvgs_grad_moments.argtypes = [vp, vp, i64, C.c_int32, C.POINTER(mvgs_grads), vp, vp]
    L.mvgs_grad_moments.restype = C.c_int
    L.mvgs_frame_merge.argtypes = [vp, vp, vp, vp, i32, vp]
    L.mvgs_frame_merge.restype = C.c_int
    _LIB = L
    return L


def check(status: int, ctx=None) -> None:
    if status != MVGS_OK:
        L = lib()
        msg = L.mvgs_status_string(status).decode()
        if ctx:
            detail = L.mvgs_last_error(ctx).decode()
            if detail:
                msg = f"{msg}: {detail}"
        raise MvgsError(status, msg)


def ptr_array(ptrs) -> C.Array:
    return (C.c_void_p * len(ptrs))(*[int(p) for p in ptrs])


def make_camera(width, height, fx, fy, cx, cy, R, t, bg=(0.0, 0.0, 0.0)) -> mvgs_camera:
    c = mvgs_camera()
    c.width, c.height = int(width), int(height)
    c.fx, c.fy, c.cx, c.cy = float(fx), float(fy), float(cx), float(cy)
    Rf = [float(x) for x in list(R.reshape(-1) if hasattr(R, "reshape") else R)]
    tf = [float(x) for x in list(t.reshape(-1) if hasattr(t, "reshape") else t)]
    bf = [float(x) for x in list(bg.reshape(-1) if hasattr(bg, "reshape") else bg)]
    c.R = (C.c_float * 9)(*Rf)
    c.t = (C.c_float * 3)(*tf)
    c.bg = (C.c_float * 3)(*bf)
    return c


def camera_array(cams) -> C.Array:
    arr = (mvgs_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = c if isinstance(c, mvgs_camera) else make_camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.R,
                                                                   c.t, c.bg)
    return arr
