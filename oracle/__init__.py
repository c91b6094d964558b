"""ctypes front end of the FP64 CPU oracle (``h4dgs_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may use this package; the product path never does.  It shares
no code with the HIP library: the only inputs both sides see are the seeded
arrays from ``scenegen``.

All functions take the float32 parameter arrays exactly as the GPU path gets
them, widen them to float64 and compute in float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "h4dgs_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

CXX_FLAGS = ["-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off"]


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (no -ffast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["g++", *CXX_FLAGS, _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _OScene(C.Structure):
    _fields_ = [("n3", C.c_int32)] + [(k, C.c_void_p) for k in ("mean3", "ls3", "q3", "op3", "sh3")] + \
               [("n4", C.c_int32)] + [(k, C.c_void_p) for k in ("mean4", "mt4", "ls4", "ql4", "qr4", "op4", "sh4")] + \
               [("sht_deg", C.c_int32), ("sht_period", C.c_double), ("sht4", C.c_void_p)]


_GRAD_FIELDS = ("mean3", "ls3", "q3", "op3", "sh3", "mean4", "mt4", "ls4", "ql4", "qr4", "op4", "sh4", "sht4")


class _OTangent(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in _GRAD_FIELDS]


class _OGrad(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in _GRAD_FIELDS]


class _OView(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("T", C.c_double * 3), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("W", C.c_int32), ("H", C.c_int32),
                ("time", C.c_double), ("bg", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        vp, i32, dbl, f32 = C.c_void_p, C.c_int32, C.c_double, C.c_float
        L.orc_render.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        L.orc_render_jvp.argtypes = [vp, vp, vp, i32, vp, vp]
        L.orc_render_bwd.argtypes = [vp, vp, i32, vp, vp, vp]
        L.orc_project.argtypes = [vp, vp, vp]
        L.orc_world.argtypes = [vp, i32, dbl, vp, vp, vp]
        L.orc_rot4.argtypes = [vp, vp, vp, vp, vp]
        L.orc_quat_to_rot.argtypes = [vp, vp]
        L.orc_mat2quat.argtypes = [vp, vp]
        L.orc_sh_basis.argtypes = [vp, vp]
        L.orc_pixels.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
        L.orc_tile_lists.argtypes = [i32, vp, vp, vp, vp, vp, i32, i32, i32, vp, vp, vp]
        L.orc_composite_records.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, i32, i32, i32, vp, vp, vp, vp]
        L.orc_convert_static.argtypes = [vp, f32, vp, vp, vp, vp]
        L.orc_adam.argtypes = [C.c_int64, vp, vp, vp, vp, dbl, dbl, dbl, dbl, i32, vp, vp, vp]
        L.orc_num_threads.restype = i32
        L.orc_local_new.argtypes = [vp, i32, vp, i32, i32, vp]
        L.orc_local_new.restype = vp
        L.orc_local_free.argtypes = [vp]
        L.orc_local_amb.argtypes = [vp, i32, vp]
        L.orc_local_grad.argtypes = [vp, vp, vp]
        L.orc_local_fd.argtypes = [vp, vp, i32, vp, dbl, vp, vp]
        L.orc_blended_at.argtypes = [vp, vp, i32, i32, vp, vp, i32, vp, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _period(scene) -> float:
    return float(getattr(scene, "time_period", 1.0))


class _SceneRef:
    """Keeps the contiguous float32 arrays alive while the C struct points at them.
    A 4D set may carry time coefficients of its colour, g4["sh_t"] = [48 D][n4]
    (D = 1 or 2), with period `period`."""

    def __init__(self, g3: dict, g4: dict, period: float = 1.0):
        self.keep = []

        def f(a):
            a = _c(a, np.float32)
            self.keep.append(a)
            return _p(a)

        self.n3 = int(np.asarray(g3["opacity"]).shape[0])
        self.n4 = int(np.asarray(g4["opacity"]).shape[0])
        sht = g4.get("sh_t")
        deg = 0 if sht is None else int(np.asarray(sht).shape[0]) // 48
        assert sht is None or (np.asarray(sht).shape[0] == 48 * deg and 1 <= deg <= 2 and period > 0)
        self.s = _OScene(self.n3, f(g3["mean"]), f(g3["log_scale"]), f(g3["quat"]), f(g3["opacity"]), f(g3["sh"]),
                         self.n4, f(g4["mean"]), f(g4["mean_t"]), f(g4["log_scale"]), f(g4["quat_l"]),
                         f(g4["quat_r"]), f(g4["opacity"]), f(g4["sh"]), deg, float(period),
                         f(sht) if sht is not None else None)

    @property
    def ref(self):
        return C.byref(self.s)


def _view(v) -> _OView:
    M = np.asarray(v.world_to_cam, np.float32).astype(np.float64)
    o = _OView()
    for i in range(9):
        o.R[i] = M[i // 3, i % 3]
    for i in range(3):
        o.T[i] = M[i, 3]
        o.bg[i] = float(np.float32(v.bg[i]))
    o.fx, o.fy = float(np.float32(v.fx)), float(np.float32(v.fy))
    o.cx, o.cy = float(np.float32(v.cx)), float(np.float32(v.cy))
    o.W, o.H = int(v.width), int(v.height)
    o.time = float(np.float32(v.t))
    return o


def render(scene, view, tile: int = 16):
    """FP64 forward of one view.  Returns dict(img[3,H,W], T[H,W], nblend[H,W],
    amb[H,W]); ``amb`` flags pixels touched by a decision within the FP32 guard band."""
    L = lib()
    sr = _SceneRef(scene.g3, scene.g4, _period(scene))
    V = _view(view)
    H, W = view.height, view.width
    img = np.zeros((3, H, W), np.float64)
    T = np.zeros((H, W), np.float64)
    nb = np.zeros((H, W), np.int32)
    amb = np.zeros((H, W), np.uint8)
    rc = L.orc_render(sr.ref, C.byref(V), tile, _p(img), _p(T), _p(nb), _p(amb))
    assert rc == 0
    return dict(img=img, T=T, nblend=nb, amb=amb.astype(bool))


def render_jvp(scene, tangent3: dict, tangent4: dict, view, tile: int = 16):
    L = lib()
    sr = _SceneRef(scene.g3, scene.g4, _period(scene))
    keep = []

    def d(a):
        if a is None:
            return None
        a = _c(a, np.float64)
        keep.append(a)
        return _p(a)

    t = _OTangent(d(tangent3.get("mean")), d(tangent3.get("log_scale")), d(tangent3.get("quat")),
                  d(tangent3.get("opacity")), d(tangent3.get("sh")), d(tangent4.get("mean")),
                  d(tangent4.get("mean_t")), d(tangent4.get("log_scale")), d(tangent4.get("quat_l")),
                  d(tangent4.get("quat_r")), d(tangent4.get("opacity")), d(tangent4.get("sh")),
                  d(tangent4.get("sh_t")))
    V = _view(view)
    img = np.zeros((3, view.height, view.width), np.float64)
    dimg = np.zeros_like(img)
    assert L.orc_render_jvp(sr.ref, C.byref(t), C.byref(V), tile, _p(img), _p(dimg)) == 0
    return img, dimg


def zeros_like_params(scene):
    g3 = {k: np.zeros(v.shape, np.float64) for k, v in scene.g3.items()}
    g4 = {k: np.zeros(v.shape, np.float64) for k, v in scene.g4.items()}
    return g3, g4


def render_bwd(scene, views, dl_dimgs, tile: int = 16, want_g2: bool = False):
    """FP64 adjoint.  Gradients are summed over ``views``.  Returns (g3, g4[, g2])
    with float64 arrays shaped like the parameters; g2 is [n_views][N][9]."""
    L = lib()
    sr = _SceneRef(scene.g3, scene.g4, _period(scene))
    g3, g4 = zeros_like_params(scene)
    G = _OGrad(_p(g3["mean"]), _p(g3["log_scale"]), _p(g3["quat"]), _p(g3["opacity"]), _p(g3["sh"]),
               _p(g4["mean"]), _p(g4["mean_t"]), _p(g4["log_scale"]), _p(g4["quat_l"]), _p(g4["quat_r"]),
               _p(g4["opacity"]), _p(g4["sh"]), _p(g4.get("sh_t")))
    N = scene.n3 + scene.n4
    g2s = []
    for v, dl in zip(views, dl_dimgs):
        V = _view(v)
        g2 = np.zeros((N, 9), np.float64)
        dl = _c(dl, np.float32)
        assert L.orc_render_bwd(sr.ref, C.byref(V), tile, _p(dl), C.byref(G), _p(g2)) == 0
        g2s.append(g2)
    if want_g2:
        return g3, g4, g2s
    return g3, g4


def project(scene, view) -> dict:
    L = lib()
    sr = _SceneRef(scene.g3, scene.g4, _period(scene))
    V = _view(view)
    N = scene.n3 + scene.n4
    out = np.zeros((N, 20), np.float64)
    assert L.orc_project(sr.ref, C.byref(V), _p(out)) == 0
    names = ["visible", "culled", "u", "v", "depth", "q00", "q01", "q11", "op", "r", "g", "b", "radius", "x0", "x1",
             "y0", "y1", "key", "margin", "pt"]
    return {n: out[:, i] for i, n in enumerate(names)}


def world(scene, g: int, t: float):
    L = lib()
    sr = _SceneRef(scene.g3, scene.g4, _period(scene))
    mu = np.zeros(3)
    Sg = np.zeros(9)
    op = np.zeros(3)
    assert L.orc_world(sr.ref, int(g), float(t), _p(mu), _p(Sg), _p(op)) == 0
    return mu, Sg.reshape(3, 3), dict(op=op[0], sigmoid=op[1], pt=op[2])


def rot4(ql, qr):
    L = lib()
    ql = _c(ql, np.float64)
    qr = _c(qr, np.float64)
    Lm, Rm, R = np.zeros(16), np.zeros(16), np.zeros(16)
    L.orc_rot4(_p(ql), _p(qr), _p(Lm), _p(Rm), _p(R))
    return Lm.reshape(4, 4), Rm.reshape(4, 4), R.reshape(4, 4)


def quat_to_rot(q):
    L = lib()
    q = _c(q, np.float64)
    R = np.zeros(9)
    L.orc_quat_to_rot(_p(q), _p(R))
    return R.reshape(3, 3)


def mat2quat(R):
    L = lib()
    R = _c(R, np.float64).reshape(-1)
    q = np.zeros(4)
    L.orc_mat2quat(_p(R), _p(q))
    return q


def sh_basis(d):
    L = lib()
    d = _c(d, np.float64)
    Y = np.zeros(16)
    L.orc_sh_basis(_p(d), _p(Y))
    return Y


def pixels(scene, view, px, py):
    """Brute-force colour of selected pixels (no tiles).  Returns (rgb[n,3], T[n], amb[n])."""
    L = lib()
    sr = _SceneRef(scene.g3, scene.g4, _period(scene))
    V = _view(view)
    px = _c(px, np.int32)
    py = _c(py, np.int32)
    n = px.shape[0]
    rgb = np.zeros((n, 3))
    T = np.zeros(n)
    amb = np.zeros(n, np.uint8)
    assert L.orc_pixels(sr.ref, C.byref(V), n, _p(px), _p(py), _p(rgb), _p(T), _p(amb)) == 0
    return rgb, T, amb.astype(bool)


def tile_lists(rec: dict, W: int, H: int, tile: int):
    """Exact per-tile sorted id lists of given screen-space splats.  Returns (start[tiles+1], ids[P])."""
    L = lib()
    n = rec["u"].shape[0]
    u, v = _c(rec["u"], np.float32), _c(rec["v"], np.float32)
    r, dpt, vis = _c(rec["radius"], np.int32), _c(rec["depth"], np.float32), _c(rec["visible"], np.uint8)
    npairs = np.zeros(1, np.int64)
    L.orc_tile_lists(n, _p(u), _p(v), _p(r), _p(dpt), _p(vis), W, H, tile, _p(npairs), None, None)
    tiles = ((W + tile - 1) // tile) * ((H + tile - 1) // tile)
    start = np.zeros(tiles + 1, np.int64)
    ids = np.zeros(int(npairs[0]), np.int32)
    L.orc_tile_lists(n, _p(u), _p(v), _p(r), _p(dpt), _p(vis), W, H, tile, _p(npairs), _p(start), _p(ids))
    return start, ids


def composite_records(rec: dict, W: int, H: int, tile: int = 16, bg=(0.0, 0.0, 0.0)):
    L = lib()
    n = rec["u"].shape[0]
    arrs = [_c(rec["u"], np.float32), _c(rec["v"], np.float32), _c(rec["conic"], np.float32),
            _c(rec["opacity"], np.float32), _c(rec["rgb"], np.float32), _c(rec["radius"], np.int32),
            _c(rec["depth"], np.float32), _c(rec["visible"], np.uint8)]
    bgv = np.asarray(bg, np.float64)
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    amb = np.zeros((H, W), np.uint8)
    L.orc_composite_records(n, *[_p(a) for a in arrs], W, H, tile, _p(bgv), _p(img), _p(T), _p(amb))
    return img, T, amb.astype(bool)


def convert_static(scene, tau: float):
    """Returns (perm[n4], n4_out, n3_out, q3d[4, n_conv])."""
    L = lib()
    sr = _SceneRef(scene.g3, scene.g4, _period(scene))
    n4 = scene.n4
    perm = np.zeros(n4, np.int32)
    n4o = np.zeros(1, np.int32)
    n3o = np.zeros(1, np.int32)
    q = np.zeros(4 * max(n4, 1), np.float64)
    assert L.orc_convert_static(sr.ref, C.c_float(tau), _p(perm), _p(n4o), _p(n3o), _p(q)) == 0
    nc = int(n3o[0]) - scene.n3
    return perm, int(n4o[0]), int(n3o[0]), q[:4 * nc].reshape(4, nc)


def adam(p, g, m, v, lr, b1, b2, eps, step):
    L = lib()
    p, g, m, v = (_c(a, np.float32) for a in (p, g, m, v))
    po, mo, vo = np.zeros(p.shape), np.zeros(p.shape), np.zeros(p.shape)
    L.orc_adam(p.size, _p(p), _p(g), _p(m), _p(v), lr, b1, b2, eps, int(step), _p(po), _p(mo), _p(vo))
    return po, mo, vo


def num_threads() -> int:
    return int(lib().orc_num_threads())


def blended_at(scene, view, px, py, cap: int = 512, tile: int = 16):
    """The Gaussians blended at the given pixels, front to back: a list per
    pixel of (merged id, blend weight alpha T) pairs."""
    L = lib()
    sr = _SceneRef(scene.g3, scene.g4, _period(scene))
    V = _view(view)
    px, py = _c(px, np.int32), _c(py, np.int32)
    n = px.shape[0]
    ids = np.zeros((n, cap), np.int32)
    w = np.zeros((n, cap), np.float64)
    cnt = np.zeros(n, np.int32)
    assert L.orc_blended_at(sr.ref, C.byref(V), tile, n, _p(px), _p(py), cap, _p(ids), _p(w), _p(cnt)) == 0
    assert cnt.max(initial=0) <= cap, "raise cap"
    return [list(zip(ids[k, :cnt[k]].tolist(), w[k, :cnt[k]].tolist())) for k in range(n)]


# Parameter order of one Gaussian's row in Local.grad / Local.fd (the ABI field order).
ROW4 = [("mean", c) for c in range(3)] + [("mean_t", None)] + [("log_scale", c) for c in range(4)] + \
    [("quat_l", c) for c in range(4)] + [("quat_r", c) for c in range(4)] + [("opacity", None)] + \
    [("sh", c) for c in range(48)]
ROW3 = [("mean", c) for c in range(3)] + [("log_scale", c) for c in range(3)] + [("quat", c) for c in range(4)] + \
    [("opacity", None)] + [("sh", c) for c in range(48)]


class Local:
    """Oracle evaluation restricted to the pixel squares of a few selected
    Gaussians (merged ids: 4D rows first, then 3D rows) in the given views, for
    scenes too large to composite whole.  The candidate lists are those of the
    whole-view path for the tiles the squares touch.

    amb(v): uint8 [H, W], bit 0 = inside a selected square, bit 1 = guard-band
    flag (the same flags ``render`` sets there).
    grad(dls): float64 [n_sel, 65], the selected Gaussians' gradients of
    sum_v <dls[v], C_v> with dls zeroed at flagged pixels (rows in ROW4 / ROW3
    order; a 3D row fills its first 59 entries).
    fd(dls, entries, hrel): central differences of the same loss for
    (selection index, row index) entries, float64, and an ok flag (False where a
    move changes a discrete decision)."""

    def __init__(self, scene, views, sel, tile: int = 16):
        L = lib()
        self._sr = _SceneRef(scene.g3, scene.g4, _period(scene))
        self._views = (_OView * len(views))(*[_view(v) for v in views])
        self.views = list(views)
        self.sel = _c(sel, np.int32)
        self.n4 = scene.n4
        self.h = L.orc_local_new(self._sr.ref, len(views), self._views, tile, int(self.sel.size), _p(self.sel))
        if not self.h:
            raise ValueError("orc_local_new rejected its arguments")

    def _dls(self, dls):
        keep = [_c(d, np.float32) for d in dls]
        arr = (C.c_void_p * len(keep))(*[a.ctypes.data for a in keep])
        return keep, arr

    def amb(self, v: int) -> np.ndarray:
        view = self.views[v]
        out = np.zeros((view.height, view.width), np.uint8)
        assert lib().orc_local_amb(self.h, v, _p(out)) == 0
        return out

    def grad(self, dls) -> np.ndarray:
        keep, arr = self._dls(dls)
        rows = np.zeros((self.sel.size, 65), np.float64)
        assert lib().orc_local_grad(self.h, arr, _p(rows)) == 0
        return rows

    def fd(self, dls, entries, hrel: float = 1e-6):
        keep, arr = self._dls(dls)
        ent = _c(entries, np.int32).reshape(-1, 2)
        fd = np.zeros(ent.shape[0], np.float64)
        ok = np.zeros(ent.shape[0], np.int32)
        assert lib().orc_local_fd(self.h, arr, ent.shape[0], _p(ent), float(hrel), _p(fd), _p(ok)) == 0
        return fd, ok.astype(bool)

    def close(self):
        if getattr(self, "h", None):
            lib().orc_local_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
