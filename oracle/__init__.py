"""ctypes wrapper of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP path; the two meet only in the seeded inputs of ``gut_synth``.

Every function here marshals arrays and calls the C oracle; the method's
arithmetic lives in ``oracle.c`` (see its header for the paper passages each
step follows and for the readings where the paper is silent).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MAXALT = 8


FLAGS = ["-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
         "-ffp-contract=off"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (C11, FP64, OpenMP, no FMA contraction),
    for any x86-64 host (the library travels with the tree)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc"] + FLAGS + [_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def use_native() -> str:
    """Rebuild the oracle for this host's CPU (-march=native) in a temporary
    folder and load that copy instead (for timing it); returns the flags."""
    global _lib
    import tempfile
    flags = FLAGS + ["-march=native"]
    path = os.path.join(tempfile.mkdtemp(prefix="oracle_native_"), "liboracle_native.so")
    subprocess.check_call(["gcc"] + flags + [_SRC, "-o", path, "-lm"])
    L = C.CDLL(path)
    _declare(L)
    _lib = L
    return " ".join(flags)


def set_threads(n: int = 0) -> int:
    """OpenMP threads of the oracle: n > 0 sets them; returns the count in use."""
    return int(lib().ora_set_threads(int(n)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


# ----------------------------------------------------------------------------
# C structs
# ----------------------------------------------------------------------------

class Camera(C.Structure):
    _fields_ = [("model", C.c_int32), ("shutter", C.c_int32), ("width", C.c_int32),
                ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("k", C.c_double * 4),
                ("R0", C.c_double * 9), ("t0", C.c_double * 3),
                ("R1", C.c_double * 9), ("t1", C.c_double * 3)]


class Params(C.Structure):
    _fields_ = [("ut_alpha", C.c_double), ("ut_beta", C.c_double), ("ut_kappa", C.c_double),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double), ("t_min", C.c_double),
                ("near_plane", C.c_double), ("k_sigma_max", C.c_double),
                ("tile", C.c_int32), ("rs_iters", C.c_int32), ("bg", C.c_double * 3),
                ("kernel_degree", C.c_int32), ("kbuffer", C.c_int32), ("tile_cull", C.c_int32)]


class SceneS(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32),
                ("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacities", C.c_void_p), ("sh", C.c_void_p)]


class ProjS(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("cull", "mean2d", "cov2d", "rect", "tiles", "depth",
                                          "rgb", "rgb_raw", "tstar", "edge", "valid_margin",
                                          "kext")]


class Amb(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("alpha", "trans", "tau", "depth", "edge", "valid",
                                          "pixel", "diff", "clip", "order", "conic")]


class ImageS(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("rgb", "T", "n_contrib", "n_eval", "inside", "n_alt",
                                          "alt_rgb", "alt_T", "alt_nc", "alt_ne", "n_amb")]


def _declare(L):
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.ora_theta_lim.restype = d
    L.ora_theta_lim.argtypes = [vp]
    L.ora_ut_weights.argtypes = [d, d, d, vp, vp, vp]
    L.ora_ut_affine.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.ora_quat_to_rot.argtypes = [vp, vp]
    L.ora_pose.argtypes = [vp, d, vp, vp]
    L.ora_project_point.argtypes = [vp, vp, d, vp, vp, vp]
    L.ora_project_point.restype = C.c_int
    L.ora_solve_time.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp]
    L.ora_solve_time.restype = C.c_int
    L.ora_pixel_ray.argtypes = [vp, d, d, vp, vp, vp]
    L.ora_pixel_ray.restype = C.c_int
    L.ora_sh_basis.argtypes = [C.c_int, vp, vp]
    L.ora_sh_basis_grad.argtypes = [C.c_int, vp, vp]
    L.ora_particle_alpha.argtypes = [vp, vp, vp, d, vp, vp, i32, vp, vp, vp]
    L.ora_particle_alpha.restype = C.c_int
    L.ora_project_samples.argtypes = [vp, vp, C.c_int, i64, vp, vp, vp]
    L.ora_ewa.argtypes = [vp, vp, d, vp, vp, vp, d, vp, vp]
    L.ora_ewa.restype = C.c_int
    L.ora_project.argtypes = [vp, vp, vp, vp]
    L.ora_set_threads.argtypes = [C.c_int]
    L.ora_set_threads.restype = C.c_int
    L.ora_ellipse_box_qmin.argtypes = [vp, vp, d, d, d, d]
    L.ora_ellipse_box_qmin.restype = d
    L.ora_bin.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
    L.ora_bin.restype = i64
    L.ora_render.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, i32, vp, vp]
    L.ora_backward.argtypes = [vp] * 10 + [vp] * 5
    L.ora_record.argtypes = [vp] * 11
    L.ora_record.restype = i64
    L.ora_loss_frozen.argtypes = [vp] * 9
    L.ora_loss_frozen.restype = d


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _ref(x):
    return C.cast(C.pointer(x), C.c_void_p)


# ----------------------------------------------------------------------------
# Parameters, cameras, scenes
# ----------------------------------------------------------------------------

def default_params(**kw) -> dict:
    """3DGS thresholds (the paper adopts 3DGS's parameters) and the UT spread
    alpha=1, beta=2, kappa=0 of Sec. 4.4.  Threshold values are the FP32 numbers
    the GPU path receives, so both sides compare against the same values."""
    f = lambda v: float(np.float32(v))
    p = dict(ut_alpha=1.0, ut_beta=2.0, ut_kappa=0.0, alpha_min=f(1.0 / 255.0),
             alpha_max=f(0.99), t_min=f(1e-4), near_plane=f(0.2), k_sigma_max=3.0,
             tile=16, rs_iters=3, bg=(0.0, 0.0, 0.0), kernel_degree=2, kbuffer=0, tile_cull=1)
    p.update(kw)
    return p


def default_amb(**kw) -> dict:
    a = dict(alpha=1e-6, trans=1e-4, tau=1e-5, depth=1e-6, edge=2e-3, valid=1e-5, pixel=1e-9,
             diff=1e-6, clip=1e-5, order=1e-5, conic=1e-6)
    a.update(kw)
    return a


def _params(p: dict) -> Params:
    s = Params()
    for k in ("ut_alpha", "ut_beta", "ut_kappa", "alpha_min", "alpha_max", "t_min",
              "near_plane", "k_sigma_max"):
        setattr(s, k, float(p[k]))
    s.tile = int(p["tile"])
    s.rs_iters = int(p["rs_iters"])
    s.kernel_degree = int(p.get("kernel_degree", 2))
    s.kbuffer = int(p.get("kbuffer", 0))
    s.tile_cull = int(p.get("tile_cull", 1))
    for i in range(3):
        s.bg[i] = float(p["bg"][i])
    return s


def _amb(a: dict) -> Amb:
    s = Amb()
    for k, v in a.items():
        setattr(s, k, float(v))
    return s


def camera_struct(cam: dict) -> Camera:
    c = Camera()
    c.model = {"pinhole": 0, "fisheye": 1}[cam["model"]]
    c.shutter = {"global": 0, "rolling": 1}[cam["shutter"]]
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.fx, c.fy, c.cx, c.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    for i in range(4):
        c.k[i] = float(cam["k"][i])
    R0 = np.asarray(cam["R0"], np.float64).reshape(-1)
    R1 = np.asarray(cam["R1"], np.float64).reshape(-1)
    for i in range(9):
        c.R0[i], c.R1[i] = R0[i], R1[i]
    for i in range(3):
        c.t0[i], c.t1[i] = float(cam["t0"][i]), float(cam["t1"][i])
    return c


class OScene:
    """Double-precision copy of a particle set (FP32 inputs converted exactly)."""

    def __init__(self, means, scales, quats, opacities, sh, sh_degree):
        self.means = np.ascontiguousarray(means, np.float64)
        self.scales = np.ascontiguousarray(scales, np.float64)
        self.quats = np.ascontiguousarray(quats, np.float64)
        self.opacities = np.ascontiguousarray(opacities, np.float64).reshape(-1)
        self.sh = np.ascontiguousarray(sh, np.float64)
        self.sh_degree = int(sh_degree)
        self.n = self.means.shape[0]

    @classmethod
    def from_scene(cls, sc):
        return cls(sc.means, sc.scales, sc.quats, sc.opacities, sc.sh, sc.sh_degree)

    def copy(self):
        return OScene(self.means.copy(), self.scales.copy(), self.quats.copy(),
                      self.opacities.copy(), self.sh.copy(), self.sh_degree)

    def struct(self) -> SceneS:
        s = SceneS()
        s.n, s.sh_degree = self.n, self.sh_degree
        s.means, s.scales, s.quats = _p(self.means), _p(self.scales), _p(self.quats)
        s.opacities, s.sh = _p(self.opacities), _p(self.sh)
        return s


def as_oscene(scene) -> OScene:
    return scene if isinstance(scene, OScene) else OScene.from_scene(scene)


def tiles_xy(cam, params):
    t = params["tile"]
    return (cam["width"] + t - 1) // t, (cam["height"] + t - 1) // t


# ----------------------------------------------------------------------------
# Primitives (for the pins)
# ----------------------------------------------------------------------------

def theta_lim(k):
    k = np.ascontiguousarray(k, np.float64)
    return lib().ora_theta_lim(_p(k))


def ut_weights(a=1.0, b=2.0, kappa=0.0):
    lam = C.c_double()
    wm, wc = np.zeros(7), np.zeros(7)
    lib().ora_ut_weights(a, b, kappa, C.byref(lam), _p(wm), _p(wc))
    return lam.value, wm, wc


def ut_affine(mu, quat, scale, A, b, params=None):
    p = _params(params or default_params())
    mu, quat, scale = (np.ascontiguousarray(x, np.float64) for x in (mu, quat, scale))
    A, b = np.ascontiguousarray(A, np.float64), np.ascontiguousarray(b, np.float64)
    m, cv = np.zeros(2), np.zeros(3)
    lib().ora_ut_affine(_p(mu), _p(quat), _p(scale), _ref(p), _p(A), _p(b), _p(m), _p(cv))
    return m, np.array([[cv[0], cv[1]], [cv[1], cv[2]]])


def quat_to_rot(q):
    q = np.ascontiguousarray(q, np.float64)
    R = np.zeros(9)
    lib().ora_quat_to_rot(_p(q), _p(R))
    return R.reshape(3, 3)


def pose(cam, t):
    c = camera_struct(cam)
    R, cen = np.zeros(9), np.zeros(3)
    lib().ora_pose(_ref(c), float(t), _p(R), _p(cen))
    return R.reshape(3, 3), cen


def project_point(cam, x, t=0.0, params=None):
    c, p = camera_struct(cam), _params(params or default_params())
    x = np.ascontiguousarray(x, np.float64)
    v, m = np.zeros(2), C.c_double()
    ok = lib().ora_project_point(_ref(c), _ref(p), float(t), _p(x), _p(v), C.byref(m))
    return bool(ok), v, m.value


def solve_time(cam, x, iters=3, params=None):
    c, p = camera_struct(cam), _params(params or default_params())
    x = np.ascontiguousarray(x, np.float64)
    v, t, m = np.zeros(2), C.c_double(), C.c_double()
    ok = lib().ora_solve_time(_ref(c), _ref(p), int(iters), _p(x), C.byref(t), _p(v), C.byref(m))
    return bool(ok), t.value, v, m.value


def pixel_ray(cam, u, v):
    c = camera_struct(cam)
    o, d, m = np.zeros(3), np.zeros(3), C.c_double()
    ok = lib().ora_pixel_ray(_ref(c), float(u), float(v), _p(o), _p(d), C.byref(m))
    return bool(ok), o, d, m.value


def sh_basis(degree, d):
    d = np.ascontiguousarray(d, np.float64)
    Y = np.zeros((degree + 1) ** 2)
    lib().ora_sh_basis(int(degree), _p(d), _p(Y))
    return Y


def sh_basis_grad(degree, d):
    d = np.ascontiguousarray(d, np.float64)
    dY = np.zeros(((degree + 1) ** 2, 3))
    lib().ora_sh_basis_grad(int(degree), _p(d), _p(dY))
    return dY


def ellipse_box_qmin(m, A, box):
    """min over the closed box (x0, y0, x1, y1) of (v-m)^T A^-1 (v-m), A = (xx, xy, yy)."""
    m = np.ascontiguousarray(m, np.float64)
    A = np.ascontiguousarray(A, np.float64)
    return float(lib().ora_ellipse_box_qmin(_p(m), _p(A), *[float(b) for b in box]))


def particle_alpha(mu, quat, scale, opacity, o, d, kernel_degree=2):
    mu, quat, scale, o, d = (np.ascontiguousarray(x, np.float64) for x in (mu, quat, scale, o, d))
    tau, om2, a = C.c_double(), C.c_double(), C.c_double()
    ok = lib().ora_particle_alpha(_p(mu), _p(quat), _p(scale), float(opacity), _p(o), _p(d),
                                  int(kernel_degree), C.byref(tau), C.byref(om2), C.byref(a))
    return bool(ok), tau.value, om2.value, a.value


def project_samples(cam, x, iters=20, params=None):
    """World points x[m,3] through the camera as sigma points (Supp. C's
    Monte-Carlo reference); returns (v[m,2], ok[m])."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    v = np.zeros((x.shape[0], 2))
    ok = np.zeros(x.shape[0], np.int32)
    cs = camera_struct(cam)
    ps = _params(params or default_params())
    lib().ora_project_samples(C.byref(cs), C.byref(ps), int(iters), x.shape[0], _p(x), _p(v), _p(ok))
    return v, ok.astype(bool)


def ewa(cam, mu, quat, scale, t=0.0, h=1e-6, params=None):
    """EWA projection (Eq. 3) at exposure time t: (ok, mean[2], cov[2,2])."""
    mu, quat, scale = (np.ascontiguousarray(a, np.float64) for a in (mu, quat, scale))
    m, c = np.zeros(2), np.zeros(3)
    cs = camera_struct(cam)
    ps = _params(params or default_params())
    ok = lib().ora_ewa(C.byref(cs), C.byref(ps), float(t), _p(mu), _p(quat), _p(scale), float(h),
                       _p(m), _p(c))
    return bool(ok), m, np.array([[c[0], c[1]], [c[1], c[2]]])


# ----------------------------------------------------------------------------
# Pipeline
# ----------------------------------------------------------------------------

class Projection(dict):
    """Per-particle outputs of ora_project, plus the C struct that points at them."""

    def struct(self) -> ProjS:
        s = ProjS()
        for k in ProjS._fields_:
            setattr(s, k[0], _p(self[k[0]]))
        return s


def project(scene, cam, params=None) -> Projection:
    sc = as_oscene(scene)
    p = params or default_params()
    n = sc.n
    out = Projection(cull=np.zeros(n, np.int32), mean2d=np.zeros((n, 2)), cov2d=np.zeros((n, 3)),
                     rect=np.zeros((n, 4), np.int32), tiles=np.zeros(n, np.int32),
                     depth=np.zeros(n), rgb=np.zeros((n, 3)), rgb_raw=np.zeros((n, 3)),
                     tstar=np.zeros(n), edge=np.zeros((n, 4)), valid_margin=np.zeros(n),
                     kext=np.zeros(n))
    ss, cs, ps, prs = sc.struct(), camera_struct(cam), _params(p), out.struct()
    lib().ora_project(_ref(ss), _ref(cs), _ref(ps), _ref(prs))
    return out


def bin_tiles(proj: Projection, cam, params=None, amb=None):
    """Per-tile lists ordered by (depth, id).  Returns (tile_start[T+1], ids, flags);
    flags bit0 = member of the primary list, bit1 = membership undecided."""
    p = params or default_params()
    a = _amb(amb or default_amb())
    n = proj["cull"].shape[0]
    tx, ty = tiles_xy(cam, p)
    cs, ps, prs = camera_struct(cam), _params(p), proj.struct()
    total = lib().ora_bin(n, _ref(prs), _ref(cs), _ref(ps), _ref(a), None, None, None)
    ts = np.zeros(tx * ty + 1, np.int64)
    ids = np.zeros(max(total, 1), np.int32)
    fl = np.zeros(max(total, 1), np.int32)
    lib().ora_bin(n, _ref(prs), _ref(cs), _ref(ps), _ref(a), _p(ts), _p(ids), _p(fl))
    return ts, ids[:total], fl[:total]


def _clip(clip, cam):
    if clip is None:
        return None
    c = np.ascontiguousarray(clip, np.float64).reshape(-1)
    assert c.size == cam["width"] * cam["height"]
    return c


def render(scene, proj, cam, bins, params=None, amb=None, tiles=None, brute_force=False,
           alternatives=True, clip=None):
    """Render the listed tiles (default: all).  Returns a dict of per-pixel
    arrays laid out [n_tiles, tile, tile, ...]; ``to_image`` reassembles a
    full render.  clip: [H, W] hybrid-rendering clip distances (Sec. 6.2)."""
    clip = _clip(clip, cam)
    sc = as_oscene(scene)
    p = params or default_params()
    a = _amb(amb or default_amb())
    tx, ty = tiles_xy(cam, p)
    ts_ = p["tile"]
    if tiles is None:
        tiles = np.arange(tx * ty, dtype=np.int32)
    tiles = np.ascontiguousarray(tiles, np.int32)
    npx = len(tiles) * ts_ * ts_
    out = dict(rgb=np.zeros((npx, 3)), T=np.zeros(npx), n_contrib=np.zeros(npx, np.int32),
               n_eval=np.zeros(npx, np.int32), inside=np.zeros(npx, np.int32))
    if alternatives:
        out.update(n_alt=np.zeros(npx, np.int32), alt_rgb=np.zeros((npx, MAXALT, 3)),
                   alt_T=np.zeros((npx, MAXALT)), alt_nc=np.zeros((npx, MAXALT), np.int32),
                   alt_ne=np.zeros((npx, MAXALT), np.int32), n_amb=np.zeros(npx, np.int32))
    img = ImageS()
    for k, _ in ImageS._fields_:
        setattr(img, k, _p(out.get(k)))
    tstart, ids, fl = bins if bins is not None else (np.zeros(1, np.int64), np.zeros(1, np.int32),
                                                     np.zeros(1, np.int32))
    ss, cs, ps, prs = sc.struct(), camera_struct(cam), _params(p), proj.struct()
    lib().ora_render(_ref(ss), _ref(prs), _ref(cs), _ref(ps), _ref(a), _p(tstart), _p(ids),
                     _p(fl), _p(tiles), len(tiles), int(bool(brute_force)), _p(clip), _ref(img))
    out["tiles"] = tiles
    return out


def to_image(res, cam, params=None, key="rgb"):
    """Reassemble a full-tile-list render into an [H, W, ...] array."""
    p = params or default_params()
    ts_ = p["tile"]
    tx, ty = tiles_xy(cam, p)
    a = res[key]
    shp = a.shape[1:]
    a = a.reshape(ty, tx, ts_, ts_, *shp)
    a = np.moveaxis(a, 2, 1).reshape(ty * ts_, tx * ts_, *shp)
    return a[: cam["height"], : cam["width"]]


def backward(scene, proj, cam, bins, dL_drgb, dL_dT=None, params=None, clip=None):
    clip = _clip(clip, cam)
    sc = as_oscene(scene)
    p = params or default_params()
    n, K = sc.n, (sc.sh_degree + 1) ** 2
    g = dict(means=np.zeros((n, 3)), scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
             opacities=np.zeros(n), sh=np.zeros((n, K, 3)))
    dC = np.ascontiguousarray(dL_drgb, np.float64)
    dT = None if dL_dT is None else np.ascontiguousarray(dL_dT, np.float64)
    tstart, ids, fl = bins
    ss, cs, ps, prs = sc.struct(), camera_struct(cam), _params(p), proj.struct()
    lib().ora_backward(_ref(ss), _ref(prs), _ref(cs), _ref(ps), _p(tstart), _p(ids), _p(fl),
                       _p(clip), _p(dC), _p(dT), _p(g["means"]), _p(g["scales"]), _p(g["quats"]),
                       _p(g["opacities"]), _p(g["sh"]))
    return g


def record(scene, proj, cam, bins, params=None, clip=None):
    clip = _clip(clip, cam)
    sc = as_oscene(scene)
    p = params or default_params()
    tstart, ids, fl = bins
    ss, cs, ps, prs = sc.struct(), camera_struct(cam), _params(p), proj.struct()
    npx = cam["width"] * cam["height"]
    pix_start = np.zeros(npx + 1, np.int64)
    total = lib().ora_record(_ref(ss), _ref(prs), _ref(cs), _ref(ps), _p(tstart), _p(ids), _p(fl),
                             _p(clip), _p(pix_start), None, None)
    contrib = np.zeros(max(total, 1), np.int32)
    clamped = np.zeros(max(total, 1), np.int32)
    lib().ora_record(_ref(ss), _ref(prs), _ref(cs), _ref(ps), _p(tstart), _p(ids), _p(fl),
                     _p(clip), _p(pix_start), _p(contrib), _p(clamped))
    return pix_start, contrib, clamped


def loss_frozen(scene, proj, cam, rec, wC, wT=None, params=None):
    sc = as_oscene(scene)
    p = params or default_params()
    pix_start, contrib, clamped = rec
    wC = np.ascontiguousarray(wC, np.float64)
    wT = None if wT is None else np.ascontiguousarray(wT, np.float64)
    ss, cs, ps, prs = sc.struct(), camera_struct(cam), _params(p), proj.struct()
    return lib().ora_loss_frozen(_ref(ss), _ref(prs), _ref(cs), _ref(ps), _p(pix_start),
                                 _p(contrib), _p(clamped), _p(wC), _p(wT))


def render_full(scene, cam, params=None, amb=None, alternatives=True):
    """project -> bin -> render every tile; returns (proj, bins, res)."""
    p = params or default_params()
    pr = project(scene, cam, p)
    b = bin_tiles(pr, cam, p, amb)
    res = render(scene, pr, cam, b, p, amb, alternatives=alternatives)
    return pr, b, res
