"""ctypes binding of libgut.so (the C ABI in include/gut.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
libgut.  PyTorch supplies device memory and streams.  If the library has not
been built this module raises on first use; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgut.so")

GUT_OK, GUT_E_INVALID, GUT_E_CAPACITY, GUT_E_HIP, GUT_E_ADMISSION, GUT_E_UNSUPPORTED, \
    GUT_E_NOT_FOUND = range(7)
GUT_PINHOLE, GUT_FISHEYE_OPENCV = 0, 1
GUT_GLOBAL_SHUTTER, GUT_ROLLING_TOP_TO_BOTTOM = 0, 1

# Every symbol include/gut.h declares.
EXPORTS = (
    "gut_default_params", "gut_num_tiles", "gut_num_pixels", "gut_project",
    "gut_bin_workspace_bytes", "gut_bin", "gut_render", "gut_render_bwd_workspace_bytes",
    "gut_render_bwd", "gut_render_bwd_noalloc", "gut_serve_create", "gut_serve_submit", "gut_serve_poll",
    "gut_serve_wait", "gut_serve_latency", "gut_serve_stats", "gut_serve_reset_stats",
    "gut_serve_destroy", "gut_status_string", "gut_last_error",
)


class GutError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class Camera(C.Structure):
    _fields_ = [("model", C.c_int32), ("shutter", C.c_int32), ("width", C.c_int32),
                ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("k", C.c_double * 4),
                ("R0", C.c_double * 9), ("t0", C.c_double * 3),
                ("R1", C.c_double * 9), ("t1", C.c_double * 3)]


class Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("reserved", C.c_int32),
                ("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacities", C.c_void_p), ("sh", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("ut_alpha", C.c_float), ("ut_beta", C.c_float), ("ut_kappa", C.c_float),
                ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("near_plane", C.c_float), ("k_sigma_max", C.c_float),
                ("tile", C.c_int32), ("rs_iters", C.c_int32), ("bg", C.c_float * 3),
                ("kernel_degree", C.c_int32), ("kbuffer", C.c_int32), ("tile_cull", C.c_int32)]


class Projected(C.Structure):
    _fields_ = [("rect", C.c_void_p), ("tiles", C.c_void_p), ("depth", C.c_void_p),
                ("rgb", C.c_void_p), ("record", C.c_void_p), ("mean2d", C.c_void_p),
                ("cov2d", C.c_void_p), ("extent", C.c_void_p)]


class ServeMetrics(C.Structure):
    _fields_ = [("frames_per_s", C.c_double), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("mean_ms", C.c_double), ("max_ms", C.c_double), ("wall_s", C.c_double),
                ("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("batches", C.c_int64), ("cameras", C.c_int64), ("peak_bytes", C.c_int64)]


_lib = None


def lib_path() -> str:
    return LIB_PATH


def load():
    """Load libgut.so (built in-tree by paper_2412_12507_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libgut.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    st = C.c_int
    L.gut_default_params.argtypes = [vp]
    L.gut_default_params.restype = None
    L.gut_num_tiles.argtypes = [vp, i32, vp]
    L.gut_num_tiles.restype = i64
    L.gut_num_pixels.argtypes = [vp, i32]
    L.gut_num_pixels.restype = i64
    L.gut_project.argtypes = [vp, vp, i32, vp, vp, vp]
    L.gut_project.restype = st
    L.gut_bin_workspace_bytes.argtypes = [i64, vp, i32, i64]
    L.gut_bin_workspace_bytes.restype = sz
    L.gut_bin.argtypes = [vp, i64, vp, i32, vp, vp, sz, i64, vp, vp, vp, vp]
    L.gut_bin.restype = st
    L.gut_render.argtypes = [vp, i64, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.gut_render.restype = st
    L.gut_render_bwd_workspace_bytes.argtypes = [i64, i32]
    L.gut_render_bwd_workspace_bytes.restype = sz
    L.gut_render_bwd.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                 vp, vp, vp, sz, vp]
    L.gut_render_bwd.restype = st
    L.gut_render_bwd_noalloc.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp,
                                         vp, vp, vp, vp, vp]
    L.gut_render_bwd_noalloc.restype = st
    serve_sigs = {
        "gut_serve_create": [vp, vp, sz, i32, i32, vp],
        "gut_serve_submit": [vp, vp, i32, vp, vp],
        "gut_serve_poll": [vp, C.c_uint64, vp],
        "gut_serve_wait": [vp, C.c_uint64],
        "gut_serve_latency": [vp, C.c_uint64, vp],
        "gut_serve_stats": [vp, vp],
        "gut_serve_reset_stats": [vp],
        "gut_serve_destroy": [vp],
    }
    for name, args in serve_sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    L.gut_status_string.argtypes = [st]
    L.gut_status_string.restype = C.c_char_p
    L.gut_last_error.argtypes = []
    L.gut_last_error.restype = C.c_char_p
    _lib = L
    return L


def check(status: int, where: str):
    if status != GUT_OK:
        L = load()
        msg = L.gut_last_error().decode(errors="replace")
        raise GutError(status, where, f"{L.gut_status_string(status).decode()}: {msg}")


def ref(x):
    return C.cast(C.pointer(x), C.c_void_p)


def camera_struct(cam: dict) -> Camera:
    c = Camera()
    c.model = {"pinhole": GUT_PINHOLE, "fisheye": GUT_FISHEYE_OPENCV}[cam["model"]]
    c.shutter = {"global": GUT_GLOBAL_SHUTTER, "rolling": GUT_ROLLING_TOP_TO_BOTTOM}[cam["shutter"]]
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.fx, c.fy, c.cx, c.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    for i in range(4):
        c.k[i] = float(cam["k"][i])
    R0 = [float(v) for row in cam["R0"] for v in (row if hasattr(row, "__len__") else [row])]
    R1 = [float(v) for row in cam["R1"] for v in (row if hasattr(row, "__len__") else [row])]
    for i in range(9):
        c.R0[i], c.R1[i] = R0[i], R1[i]
    for i in range(3):
        c.t0[i], c.t1[i] = float(cam["t0"][i]), float(cam["t1"][i])
    return c


def camera_array(cams):
    arr = (Camera * len(cams))()
    for i, cam in enumerate(cams):
        arr[i] = camera_struct(cam)
    return arr


def params_struct(params: dict | None = None) -> Params:
    p = Params()
    load().gut_default_params(ref(p))
    for k, v in (params or {}).items():
        if k == "bg":
            for i in range(3):
                p.bg[i] = float(v[i])
        elif k in ("tile", "rs_iters", "kernel_degree", "kbuffer", "tile_cull"):
            setattr(p, k, int(v))
        else:
            setattr(p, k, float(v))
    return p
