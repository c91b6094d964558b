"""ctypes binding of ``libh4dgs.so`` (argument marshalling only).

Every entry point declared in ``include/h4dgs.h`` has a Python twin of the same
name here.  Nothing here computes any part of the rasterizer: the library runs
every step on the GPU.  If the library is missing the import of this module
succeeds but the first call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libh4dgs.so")

MAX_VIEWS = 32

H4D_OK = 0
H4D_ERR_INVALID_ARG = 1
H4D_ERR_CAPACITY = 2
H4D_ERR_HIP = 3
H4D_ERR_NONFINITE = 4
H4D_ERR_UNSUPPORTED = 5
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "CAPACITY", 3: "HIP", 4: "NONFINITE", 5: "UNSUPPORTED"}

EXPORTS = (
    "h4dgs_create", "h4dgs_destroy", "h4dgs_last_error", "h4dgs_version", "h4dgs_workspace_size",
    "h4dgs_render_fwd", "h4dgs_render_infer", "h4dgs_render_bwd", "h4dgs_check", "h4dgs_rasterize_splats",
    "h4dgs_convert_scratch_bytes", "h4dgs_convert_static", "h4dgs_adam", "h4dgs_l1_loss_grad",
    "h4dgs_profile", "h4dgs_profile_read", "h4dgs_stats", "h4dgs_stats_read", "h4dgs_radix_hist_words",
    "h4dgs_radix_pass_check", "h4dgs_render_infer_noalloc", "h4dgs_convert_moments", "h4dgs_render_bwd_stats",
    "h4dgs_densify_scratch_bytes", "h4dgs_densify", "h4dgs_gather_rows", "h4dgs_adam_masked", "h4dgs_tile_lists",
)

NOALLOC_BYTES = 256 << 20  # H4DGS_NOALLOC_BYTES

STAGES = ("preprocess", "depth_sort", "binning", "blend_fwd", "blend_bwd", "preprocess_bwd", "adam", "loss")


class H4DError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"h4dgs error {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class G3D(C.Structure):
    _fields_ = [("n", C.c_int32)] + [(k, C.c_void_p) for k in ("mean", "log_scale", "quat", "opacity", "sh")]


class G4D(C.Structure):
    _fields_ = [("n", C.c_int32)] + [(k, C.c_void_p) for k in
                                     ("mean", "mean_t", "log_scale", "quat_l", "quat_r", "opacity", "sh")] + \
               [("sh_t_degree", C.c_int32), ("sh_t_period", C.c_float), ("sh_t", C.c_void_p)]


class View(C.Structure):
    _fields_ = [("world_to_cam", C.c_float * 12), ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32), ("t", C.c_float),
                ("bg", C.c_float * 3)]


class SetStats(C.Structure):
    _fields_ = [("grad_norm", C.c_void_p), ("visible", C.c_void_p), ("step_visible", C.c_void_p)]


class DensifyParams(C.Structure):
    _fields_ = [("grad_threshold", C.c_float), ("split_n", C.c_int32), ("log_dense_scale", C.c_double),
                ("opacity_logit_min", C.c_double), ("log_max_scale", C.c_double), ("log_shrink", C.c_double)]


class Config(C.Structure):
    _fields_ = [("tile", C.c_int32), ("chunk", C.c_int32), ("batched", C.c_int32), ("cull", C.c_int32),
                ("pair_capacity", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2505_13215_amd.build.build() "
                          "(there is no non-GPU fallback)")
    L = C.CDLL(path)
    vp, i32, i64, sz, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_float
    P = C.POINTER
    L.h4dgs_create.argtypes = [P(vp)]
    L.h4dgs_destroy.argtypes = [vp]
    L.h4dgs_last_error.argtypes = [vp]
    L.h4dgs_last_error.restype = C.c_char_p
    L.h4dgs_version.restype = C.c_char_p
    L.h4dgs_workspace_size.argtypes = [vp, i32, i32, vp, i32, vp, P(sz), P(sz)]
    L.h4dgs_render_fwd.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, sz, vp, sz, vp]
    L.h4dgs_render_infer.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, sz, vp, sz, vp]
    L.h4dgs_render_infer_noalloc.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp]
    L.h4dgs_render_bwd.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, sz, vp, sz, vp, vp, vp]
    L.h4dgs_check.argtypes = [vp, vp, sz, P(i64), vp]
    L.h4dgs_rasterize_splats.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp,
                                         vp, sz, vp, sz, vp]
    L.h4dgs_convert_scratch_bytes.argtypes = [i32]
    L.h4dgs_convert_scratch_bytes.restype = sz
    L.h4dgs_convert_static.argtypes = [vp, vp, vp, f32, vp, vp, vp, P(i32), P(i32), vp, sz, vp]
    L.h4dgs_convert_moments.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.h4dgs_render_bwd_stats.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, sz, vp, sz, vp, vp, vp, vp, vp]
    L.h4dgs_densify_scratch_bytes.argtypes = [i32, i32]
    L.h4dgs_densify_scratch_bytes.restype = sz
    L.h4dgs_densify.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, P(i32), P(i32), vp, sz, vp]
    L.h4dgs_gather_rows.argtypes = [vp, vp, vp, vp, i32, vp, i32, vp, vp, vp]
    L.h4dgs_adam_masked.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, C.c_double, C.c_double, C.c_double,
                                    i32, vp]
    L.h4dgs_adam.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, C.c_double, C.c_double, C.c_double, i32, vp]
    L.h4dgs_l1_loss_grad.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    L.h4dgs_profile.argtypes = [vp, i32]
    L.h4dgs_profile_read.argtypes = [vp, vp, vp]
    L.h4dgs_stats.argtypes = [vp, i32]
    L.h4dgs_stats_read.argtypes = [vp, vp, sz, vp, vp]
    L.h4dgs_radix_hist_words.argtypes = [C.c_uint64, i32, i32, i32]
    L.h4dgs_radix_hist_words.restype = sz
    L.h4dgs_radix_pass_check.argtypes = [C.c_uint64, i32, i32, i32, sz, sz]
    for name in EXPORTS:
        if name not in ("h4dgs_last_error", "h4dgs_version", "h4dgs_convert_scratch_bytes", "h4dgs_radix_hist_words",
                        "h4dgs_densify_scratch_bytes"):
            getattr(L, name).restype = i32
    _lib = L
    return L


class Context:
    """Owns one ``h4d_ctx``."""

    def __init__(self):
        self.L = load()
        self.h = C.c_void_p()
        rc = self.L.h4dgs_create(C.byref(self.h))
        if rc != H4D_OK:
            raise H4DError(rc, "h4dgs_create failed")

    def check(self, rc: int):
        if rc != H4D_OK:
            msg = self.L.h4dgs_last_error(self.h)
            raise H4DError(rc, msg.decode() if msg else "")
        return rc

    def close(self):
        if self.h:
            self.L.h4dgs_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ptr_array(ptrs) -> C.Array:
    arr = (C.c_void_p * max(1, len(ptrs)))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr


def view_array(views) -> C.Array:
    arr = (View * len(views))()
    for i, v in enumerate(views):
        M = [float(x) for x in list(v.world_to_cam.reshape(-1))]
        arr[i].world_to_cam = (C.c_float * 12)(*M)
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = float(v.fx), float(v.fy), float(v.cx), float(v.cy)
        arr[i].width, arr[i].height = int(v.width), int(v.height)
        arr[i].t = float(v.t)
        arr[i].bg = (C.c_float * 3)(*[float(b) for b in v.bg])
    return arr


def version() -> str:
    return load().h4dgs_version().decode()
