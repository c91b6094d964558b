"""PyTorch front end: device memory, streams and one ``torch.autograd.Function``.

PyTorch only allocates buffers and supplies the current HIP stream; every
stage of the rasterizer runs inside ``libh4dgs.so``.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L

G3_KEYS = ("mean", "log_scale", "quat", "opacity", "sh")
G4_KEYS = ("mean", "mean_t", "log_scale", "quat_l", "quat_r", "opacity", "sh")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


def _chk(t: torch.Tensor, name: str) -> torch.Tensor:
    if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous float32 CUDA tensor, got {t.dtype} on {t.device}")
    return t


def g3_struct(g3: dict, mut=False):
    n = int(g3["opacity"].shape[0])
    for k in G3_KEYS:
        _chk(g3[k], "g3." + k)
    return L.G3D(n, *[_ptr(g3[k]) for k in G3_KEYS])


def g4_keys(g4: dict) -> tuple:
    """The 4D set's arrays: G4_KEYS, and "sh_t" (time coefficients of the
    colour, [48 D][n]) when the set has them."""
    return G4_KEYS + (("sh_t",) if "sh_t" in g4 else ())


def time_degree(g4: dict) -> int:
    t = g4.get("sh_t")
    if t is None:
        return 0
    if t.dim() != 2 or t.shape[0] % 48 or t.shape[1] != g4["opacity"].shape[0]:
        raise ValueError("g4.sh_t: expected [48 D, n4]")
    return int(t.shape[0]) // 48


def g4_struct(g4: dict, period: float = 1.0, n: int = None):
    """Descriptor of a 4D set (or of a parameter-shaped mirror of one, e.g.
    gradients or moments, whose row stride is n)."""
    n = int(g4["opacity"].shape[0]) if n is None else int(n)
    for k in g4_keys(g4):
        _chk(g4[k], "g4." + k)
    deg = time_degree(g4)
    return L.G4D(n, *[_ptr(g4[k]) for k in G4_KEYS], deg, float(period), _ptr(g4["sh_t"]) if deg else None)


def _stats_struct(d: dict, n: int) -> L.SetStats:
    def get(key, dtype):
        t = d.get(key)
        if t is None:
            return C.c_void_p(0)
        if t.device.type != "cuda" or t.dtype != dtype or t.numel() != n or not t.is_contiguous():
            raise ValueError(f"stats {key}: expected {n} contiguous {dtype} CUDA elements")
        return _ptr(t)
    return L.SetStats(get("grad_norm", torch.float32), get("visible", torch.float32),
                      get("step_visible", torch.uint8))


def new_stats(n3: int, n4: int, device="cuda") -> tuple:
    """Zeroed per-Gaussian statistics (grad_norm, visible, step_visible) of both sets."""
    return tuple({"grad_norm": torch.zeros(n, device=device), "visible": torch.zeros(n, device=device),
                  "step_visible": torch.zeros(n, dtype=torch.uint8, device=device)} for n in (n3, n4))


def to_device(d: dict, device="cuda") -> dict:
    return {k: torch.as_tensor(v, dtype=torch.float32, device=device).contiguous() for k, v in d.items()}


@dataclass
class FwdHandle:
    generation: int
    views: object      # ctypes View array
    n_views: int
    cfg: L.Config
    n3: int
    n4: int
    state: torch.Tensor
    images: list
    differentiable: bool = True  # False after an inference render


# Launch configuration of the training step (tile edge in pixels, splats staged
# per LDS chunk); images do not depend on either.
DEFAULT_TILE = 16
DEFAULT_CHUNK = 64


class Rasterizer:
    """Owns a context, the launch configuration and the workspace tensors.

    ``check`` selects when the pair-capacity status is read back: "eager" (after
    every forward, one stream synchronisation, re-rendering with a larger
    capacity on overflow) or "deferred" (read back by ``verify()``; a forward
    whose pairs did not fit raises there).  ``batched`` processes all views of
    a call in one launch per stage instead of one view after another (same
    kernels, bit-identical images).  ``cull`` leaves a splat out of the tiles
    in which no pixel can reach alpha >= 1/255 (images unchanged)."""

    def __init__(self, tile: int = DEFAULT_TILE, chunk: int = DEFAULT_CHUNK, pair_capacity: int = 1 << 22,
                 growth: float = 1.3, check: str = "eager", batched: bool = False, cull: bool = True,
                 time_period: float = 1.0):
        self.ctx = L.Context()
        self.time_period = float(time_period)  # period of the 4D colour's time terms
        self.tile, self.chunk = int(tile), int(chunk)
        self.batched = bool(batched)
        self.cull = bool(cull)
        self.capacity = int(pair_capacity)
        self.growth = float(growth)
        self.check_mode = check
        self._state = None
        self._scratch = None
        self._gen = 0
        self._pending = None
        self.last_pairs = 0

    # -- workspace -------------------------------------------------------------
    def config(self) -> L.Config:
        return L.Config(self.tile, self.chunk, int(self.batched), int(self.cull), self.capacity)

    def sizes(self, n3: int, n4: int, views_arr, n_views: int):
        st, sc = C.c_size_t(), C.c_size_t()
        cfg = self.config()
        self.ctx.check(self.ctx.L.h4dgs_workspace_size(self.ctx.h, n3, n4, views_arr, n_views, C.byref(cfg),
                                                       C.byref(st), C.byref(sc)))
        return int(st.value), int(sc.value)

    def _ensure(self, n3, n4, views_arr, n_views):
        st, sc = self.sizes(n3, n4, views_arr, n_views)
        if self._state is None or self._state.numel() < st:
            self._state = torch.empty(max(st, 256), dtype=torch.uint8, device="cuda")
        if self._scratch is None or self._scratch.numel() < sc:
            self._scratch = torch.empty(max(sc, 256), dtype=torch.uint8, device="cuda")

    # -- forward / backward -----------------------------------------------------
    def infer(self, g3: dict, g4: dict, views) -> FwdHandle:
        """Inference render: the same images as ``forward`` without the state
        the adjoint reads (its handle cannot be passed to ``backward``)."""
        return self.forward(g3, g4, views, _keep=False)

    def forward(self, g3: dict, g4: dict, views, _keep: bool = True) -> FwdHandle:
        if self._pending is not None and self.check_mode == "eager":
            self._pending = None
        s3, s4 = g3_struct(g3), g4_struct(g4, self.time_period)
        n_views = len(views)
        va = L.view_array(views)
        images = [torch.empty((3, v.height, v.width), dtype=torch.float32, device="cuda") for v in views]
        for _attempt in range(3):
            self._ensure(s3.n, s4.n, va, n_views)
            cfg = self.config()
            imgs = L.ptr_array([im.data_ptr() for im in images])
            entry = self.ctx.L.h4dgs_render_fwd if _keep else self.ctx.L.h4dgs_render_infer
            self.ctx.check(entry(
                self.ctx.h, C.byref(s3), C.byref(s4), va, n_views, C.byref(cfg), imgs, _ptr(self._state),
                self._state.numel(), _ptr(self._scratch), self._scratch.numel(), _stream()))
            self._gen += 1
            h = FwdHandle(self._gen, va, n_views, cfg, s3.n, s4.n, self._state, images, bool(_keep))
            if self.check_mode != "eager":
                self._pending = h
                return h
            need = C.c_int64()
            rc = self.ctx.L.h4dgs_check(self.ctx.h, _ptr(self._state), self._state.numel(), C.byref(need), _stream())
            self.last_pairs = int(need.value)
            if rc == L.H4D_OK:
                return h
            if rc != L.H4D_ERR_CAPACITY:
                self.ctx.check(rc)
            self.capacity = int(need.value * self.growth) + 1024
        raise L.H4DError(L.H4D_ERR_CAPACITY, "pair capacity kept overflowing")

    def verify(self) -> int:
        """Synchronise and read the status of the last forward; returns its pair count."""
        if self._state is None:
            return 0
        need = C.c_int64()
        rc = self.ctx.L.h4dgs_check(self.ctx.h, _ptr(self._state), self._state.numel(), C.byref(need), _stream())
        self.last_pairs = int(need.value)
        if rc == L.H4D_ERR_CAPACITY:
            self.capacity = int(need.value * self.growth) + 1024
        self.ctx.check(rc)
        return self.last_pairs

    def backward(self, h: FwdHandle, g3: dict, g4: dict, dl_images, out=None, stats=None) -> tuple:
        """Gradients of every raw parameter; ``out`` = (gr3, gr4) dicts to fill in
        place; ``stats`` = (st3, st4) dicts of per-Gaussian statistics to
        accumulate (keys grad_norm, visible: float32 [n]; step_visible: uint8
        [n]; any may be missing)."""
        if h.generation != self._gen:
            raise RuntimeError("backward must follow its own forward (the workspace was reused)")
        if not h.differentiable:
            raise RuntimeError("an inference render keeps no state for the backward")
        s3, s4 = g3_struct(g3), g4_struct(g4, self.time_period)
        if out is None:
            gr3 = {k: torch.empty_like(g3[k]) for k in G3_KEYS}
            gr4 = {k: torch.empty_like(g4[k]) for k in g4_keys(g4)}
        else:
            gr3, gr4 = out
            for k in G3_KEYS:
                _chk(gr3[k], "grad3." + k)
        m3 = L.G3D(s3.n, *[_ptr(gr3[k]) for k in G3_KEYS])
        m4 = g4_struct(gr4, self.time_period, n=s4.n)
        dl = [_chk(d, "dl_dimage") for d in dl_images]
        arr = L.ptr_array([d.data_ptr() for d in dl])
        if stats is None:
            self.ctx.check(self.ctx.L.h4dgs_render_bwd(
                self.ctx.h, C.byref(s3), C.byref(s4), h.views, h.n_views, C.byref(h.cfg), arr, _ptr(h.state),
                h.state.numel(), _ptr(self._scratch), self._scratch.numel(), C.byref(m3), C.byref(m4), _stream()))
        else:
            st = [_stats_struct(d, n) for d, n in zip(stats, (s3.n, s4.n))]
            self.ctx.check(self.ctx.L.h4dgs_render_bwd_stats(
                self.ctx.h, C.byref(s3), C.byref(s4), h.views, h.n_views, C.byref(h.cfg), arr, _ptr(h.state),
                h.state.numel(), _ptr(self._scratch), self._scratch.numel(), C.byref(m3), C.byref(m4),
                C.byref(st[0]), C.byref(st[1]), _stream()))
        return gr3, gr4


    def tile_lists(self, h: FwdHandle) -> tuple:
        """The tile lists of forward `h` (the last one on this rasterizer):
        (ids, ranges[total tiles, 2]); tile t's depth-ordered splat ids (into the
        merged set [4D | 3D]) are ids[ranges[t, 0]:ranges[t, 1]], tiles of the
        views one after another."""
        if h.generation != self._gen:
            raise RuntimeError("tile_lists must follow its own forward (the workspace was reused)")
        t = h.cfg.tile
        tiles = sum(((h.views[k].width + t - 1) // t) * ((h.views[k].height + t - 1) // t) for k in range(h.n_views))
        cap = max(1, h.cfg.pair_capacity)
        ranges = torch.empty((tiles, 2), dtype=torch.int64, device="cuda")
        for _ in range(2):
            ids = torch.empty(cap, dtype=torch.int32, device="cuda")
            self.ctx.check(self.ctx.L.h4dgs_tile_lists(
                self.ctx.h, h.n3, h.n4, h.views, h.n_views, C.byref(h.cfg), _ptr(h.state), h.state.numel(),
                _ptr(self._scratch), self._scratch.numel(), _ptr(ids), C.c_uint64(cap), _ptr(ranges), _stream()))
            total = int(ranges[-1, 1]) if tiles else 0
            if total <= cap:
                return ids, ranges
            cap = total  # a shared static list counts once per view: make room and write again
        raise RuntimeError("tile lists kept growing")

    # -- instrumentation -----------------------------------------------------------
    def profile(self, enable=True):
        """Event timing of later calls: False / 0 off, True / 1 every stage
        (event pairs between stages), 2 the blending kernels only, from their
        own dispatch timestamps (no added stream commands), 3 / 4 the forward /
        backward blending kernel only."""
        self.ctx.check(self.ctx.L.h4dgs_profile(self.ctx.h, int(enable)))

    def profile_read(self) -> dict:
        """{stage: (total_ms, launches)} since the previous read (synchronises)."""
        n = len(L.STAGES)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        self.ctx.check(self.ctx.L.h4dgs_profile_read(self.ctx.h, ms, cnt))
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(L.STAGES)}

    def stats(self, enable: bool = True):
        self.ctx.check(self.ctx.L.h4dgs_stats(self.ctx.h, int(bool(enable))))

    def stats_read(self) -> dict:
        out = (C.c_int64 * 7)()
        self.ctx.check(self.ctx.L.h4dgs_stats_read(self.ctx.h, _ptr(self._state), self._state.numel(), out,
                                                   _stream()))
        return dict(fwd_eval=int(out[0]), fwd_blend=int(out[1]), bwd_eval=int(out[2]), bwd_blend=int(out[3]),
                    list_entries=int(out[4]), traversed=int(out[5]), onscreen=int(out[6]))


def l1_loss_grad(rast: Rasterizer, images, targets, views, dl_out, loss: torch.Tensor = None):
    """dl_out[v] = sign(images[v] - targets[v]) / (3 W H n_views); loss (1-element
    float32 CUDA tensor, optional) = mean over views of the mean absolute error."""
    n = len(images)
    va = L.view_array(views)
    rast.ctx.check(rast.ctx.L.h4dgs_l1_loss_grad(
        rast.ctx.h, n, L.ptr_array([_chk(i, "image").data_ptr() for i in images]),
        L.ptr_array([_chk(t, "target").data_ptr() for t in targets]), va,
        L.ptr_array([_chk(d, "dl").data_ptr() for d in dl_out]), _ptr(loss) if loss is not None else None,
        _stream()))


class H4DGSRender(torch.autograd.Function):
    """images = render(parameters); backward calls the library's adjoint."""

    @staticmethod
    def forward(ctx, rast: Rasterizer, views, *params):
        g3 = dict(zip(G3_KEYS, params[:5]))
        g4 = dict(zip(G4_KEYS + ("sh_t",), params[5:]))
        h = rast.forward(g3, g4, views)
        ctx.rast, ctx.h = rast, h
        ctx.save_for_backward(*params)
        return tuple(h.images)

    @staticmethod
    def backward(ctx, *dl):
        params = ctx.saved_tensors
        g3 = dict(zip(G3_KEYS, params[:5]))
        g4 = dict(zip(G4_KEYS + ("sh_t",), params[5:]))
        dls = [d.contiguous() if d is not None else torch.zeros_like(im) for d, im in zip(dl, ctx.h.images)]
        gr3, gr4 = ctx.rast.backward(ctx.h, g3, g4, dls)
        return (None, None, *[gr3[k] for k in G3_KEYS], *[gr4[k] for k in g4_keys(g4)])


def render(rast: Rasterizer, g3: dict, g4: dict, views) -> tuple:
    """Differentiable render of ``views``; returns one [3, H, W] image per view."""
    return H4DGSRender.apply(rast, list(views), *[g3[k] for k in G3_KEYS], *[g4[k] for k in g4_keys(g4)])


# -- other entry points ------------------------------------------------------------

def render_infer_noalloc(rast: Rasterizer, g3: dict, g4: dict, views, images=None, status=None):
    """Inference render whose state and scratch live in the library's fixed
    per-GPU workspace (``h4dgs_render_infer_noalloc``): the caller passes only
    inputs and outputs.  ``images`` (one [3, H, W] float32 tensor per view)
    and ``status`` (a 2-element int64 tensor receiving the status flags and the
    pair count) are allocated here when not given.  Returns (images, status)."""
    s3, s4 = g3_struct(g3), g4_struct(g4, rast.time_period)
    va = L.view_array(views)
    if images is None:
        images = [torch.empty((3, v.height, v.width), dtype=torch.float32, device="cuda") for v in views]
    for im, v in zip(images, views):
        if tuple(im.shape) != (3, v.height, v.width):
            raise ValueError(f"image shape {tuple(im.shape)} does not match the view's {(3, v.height, v.width)}")
        _chk(im, "image")
    if status is None:
        status = torch.empty(2, dtype=torch.int64, device="cuda")
    if status.dtype != torch.int64 or status.numel() < 2 or not status.is_cuda:
        raise ValueError("status: expected at least 2 int64 CUDA elements")
    cfg = rast.config()
    imgs = L.ptr_array([im.data_ptr() for im in images])
    rast.ctx.check(rast.ctx.L.h4dgs_render_infer_noalloc(rast.ctx.h, C.byref(s3), C.byref(s4), va, len(views),
                                                         C.byref(cfg), imgs, _ptr(status), _stream()))
    return images, status


def rasterize_splats(rast: Rasterizer, sp: dict, width: int, height: int, bg=(0.0, 0.0, 0.0)):
    """Binning, sorting and blending of given screen-space splats.  Returns
    (image[3,H,W], T[H,W], ids, ranges[tiles, 2]); tile t's depth-ordered list
    is ids[ranges[t, 0]:ranges[t, 1]]."""
    n = int(sp["u"].shape[0])
    dev = "cuda"
    t = {k: torch.as_tensor(v, device=dev).contiguous() for k, v in sp.items()}
    t["radius"] = t["radius"].to(torch.int32)
    t["visible"] = t["visible"].to(torch.uint8)
    image = torch.empty((3, height, width), dtype=torch.float32, device=dev)
    T = torch.empty((height, width), dtype=torch.float32, device=dev)
    bgv = (C.c_float * 3)(*[float(b) for b in bg])
    from scenegen import View  # a plain camera container (no rendering arithmetic)
    import numpy as np
    v = View(np.eye(3, 4, dtype=np.float32), 1.0, 1.0, 0.0, 0.0, width, height, 0.0, tuple(bg))
    va = L.view_array([v])
    for _ in range(3):
        rast._ensure(n, 0, va, 1)
        cfg = rast.config()
        ids = torch.empty(max(1, rast.capacity), dtype=torch.int32, device=dev)
        tiles = ((width + rast.tile - 1) // rast.tile) * ((height + rast.tile - 1) // rast.tile)
        ranges = torch.empty((tiles, 2), dtype=torch.int64, device=dev)
        rast.ctx.check(rast.ctx.L.h4dgs_rasterize_splats(
            rast.ctx.h, n, _ptr(t["u"]), _ptr(t["v"]), _ptr(t["conic"]), _ptr(t["opacity"]), _ptr(t["rgb"]),
            _ptr(t["radius"]), _ptr(t["depth"]), _ptr(t["visible"]), width, height, bgv, C.byref(cfg), _ptr(image),
            _ptr(T), _ptr(ids), _ptr(ranges), _ptr(rast._state), rast._state.numel(), _ptr(rast._scratch),
            rast._scratch.numel(), _stream()))
        need = C.c_int64()
        rc = rast.ctx.L.h4dgs_check(rast.ctx.h, _ptr(rast._state), rast._state.numel(), C.byref(need), _stream())
        if rc == L.H4D_OK:
            return image, T, ids, ranges
        if rc != L.H4D_ERR_CAPACITY:
            rast.ctx.check(rc)
        rast.capacity = int(need.value * rast.growth) + 1024
    raise L.H4DError(L.H4D_ERR_CAPACITY, "pair capacity kept overflowing")


def _set_buffers(n3: int, n4: int, dev="cuda", deg4: int = 0):
    """Uninitialised parameter-shaped arrays for n3 3D and n4 4D rows (with
    time coefficients of degree deg4 for the 4D set)."""
    o3 = {"mean": torch.empty((3, n3), device=dev), "log_scale": torch.empty((3, n3), device=dev),
          "quat": torch.empty((4, n3), device=dev), "opacity": torch.empty(n3, device=dev),
          "sh": torch.empty((48, n3), device=dev)}
    o4 = {"mean": torch.empty((3, n4), device=dev), "mean_t": torch.empty(n4, device=dev),
          "log_scale": torch.empty((4, n4), device=dev), "quat_l": torch.empty((4, n4), device=dev),
          "quat_r": torch.empty((4, n4), device=dev), "opacity": torch.empty(n4, device=dev),
          "sh": torch.empty((48, n4), device=dev)}
    if deg4:
        o4["sh_t"] = torch.empty((48 * deg4, n4), device=dev)
    return o3, o4


def _first_rows(d: dict, k: int) -> dict:
    return {name: (v[..., :k] if v.dim() == 2 else v[:k]).contiguous() for name, v in d.items()}


def convert_static(rast: Rasterizer, g3: dict, g4: dict, tau: float, moments=()):
    """Static identification + 4D->3D conversion.  Returns (g3', g4', perm);
    with ``moments`` (pairs (m3, m4) of parameter-shaped arrays, e.g. Adam's
    first and second moments) also the list of the moved pairs."""
    s3, s4 = g3_struct(g3), g4_struct(g4, rast.time_period)
    n3, n4 = s3.n, s4.n
    dev = "cuda"
    cap3 = n3 + n4
    deg = time_degree(g4)
    o3, o4 = _set_buffers(cap3, n4, dev, deg)
    m3 = L.G3D(cap3, *[_ptr(o3[k]) for k in G3_KEYS])
    m4 = g4_struct(o4, rast.time_period, n=n4)
    perm = torch.empty(max(1, n4), dtype=torch.int32, device=dev)
    nsc = int(rast.ctx.L.h4dgs_convert_scratch_bytes(n4))
    scratch = torch.empty(max(256, nsc), dtype=torch.uint8, device=dev)
    n4o, n3o = C.c_int32(), C.c_int32()
    rast.ctx.check(rast.ctx.L.h4dgs_convert_static(
        rast.ctx.h, C.byref(s4), C.byref(s3), C.c_float(tau), C.byref(m4), C.byref(m3), _ptr(perm), C.byref(n4o),
        C.byref(n3o), _ptr(scratch), scratch.numel(), _stream()))
    k3, k4 = n3o.value, n4o.value
    g3n, g4n = _first_rows(o3, k3), _first_rows(o4, k4)
    if not moments:
        return g3n, g4n, perm[:n4]
    moved = []
    for a3, a4 in moments:
        b3, b4 = _set_buffers(cap3, n4, dev, time_degree(a4))
        rast.ctx.check(rast.ctx.L.h4dgs_convert_moments(
            rast.ctx.h, C.byref(g4_struct(a4, rast.time_period)), C.byref(g3_struct(a3)), _ptr(perm),
            C.byref(g4_struct(b4, rast.time_period, n=n4)), C.byref(L.G3D(cap3, *[_ptr(b3[k]) for k in G3_KEYS])),
            _stream()))
        moved.append((_first_rows(b3, k3), _first_rows(b4, k4)))
    return g3n, g4n, perm[:n4], moved


def densify(rast: Rasterizer, g3: dict, g4: dict, stats3: dict, stats4: dict, noise3: torch.Tensor,
            noise4: torch.Tensor, p3: L.DensifyParams, p4: L.DensifyParams, moments=()):
    """Clone / split / prune of each set (h4dgs_densify).  noise3: float32
    [split_n, 3, n3], noise4: [split_n, 4, n4] standard normal draws.  Returns
    (g3', g4', src3, src4[, moved]) where moved lists the moment pairs
    (m3, m4) gathered to the new rows (zeros for new rows)."""
    s3, s4 = g3_struct(g3), g4_struct(g4, rast.time_period)
    n3, n4 = s3.n, s4.n
    cap3, cap4 = n3 * max(2, p3.split_n), n4 * max(2, p4.split_n)
    o3, o4 = _set_buffers(cap3, cap4, deg4=time_degree(g4))
    src3 = torch.empty(max(1, cap3), dtype=torch.int32, device="cuda")
    src4 = torch.empty(max(1, cap4), dtype=torch.int32, device="cuda")
    nsc = int(rast.ctx.L.h4dgs_densify_scratch_bytes(n3, n4))
    scratch = torch.empty(max(256, nsc), dtype=torch.uint8, device="cuda")
    st3, st4 = _stats_struct(stats3, n3), _stats_struct(stats4, n4)
    n3o, n4o = C.c_int32(), C.c_int32()
    for t, shape in ((noise3, (p3.split_n, 3, n3)), (noise4, (p4.split_n, 4, n4))):
        if tuple(t.shape) != shape or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"noise: expected a contiguous float32 CUDA tensor of shape {shape}")
    rast.ctx.check(rast.ctx.L.h4dgs_densify(
        rast.ctx.h, C.byref(s3), C.byref(s4), C.byref(st3), C.byref(st4), _ptr(noise3), _ptr(noise4),
        C.byref(p3), C.byref(p4), C.byref(L.G3D(cap3, *[_ptr(o3[k]) for k in G3_KEYS])),
        C.byref(g4_struct(o4, rast.time_period, n=cap4)), _ptr(src3), _ptr(src4), C.byref(n3o), C.byref(n4o),
        _ptr(scratch), scratch.numel(), _stream()))
    k3, k4 = n3o.value, n4o.value
    out = [_first_rows(o3, k3), _first_rows(o4, k4), src3[:k3].clone(), src4[:k4].clone()]
    if not moments:
        return tuple(out)
    moved = []
    for a3, a4 in moments:
        b3, b4 = _set_buffers(k3, k4, deg4=time_degree(a4))
        rast.ctx.check(rast.ctx.L.h4dgs_gather_rows(
            rast.ctx.h, C.byref(g3_struct(a3)), C.byref(g4_struct(a4, rast.time_period)), _ptr(src3), k3, _ptr(src4),
            k4, C.byref(L.G3D(k3, *[_ptr(b3[k]) for k in G3_KEYS])), C.byref(g4_struct(b4, rast.time_period, n=k4)),
            _stream()))
        moved.append((b3, b4))
    return tuple(out) + (moved,)


class CapturedStep:
    """forward -> L1 loss gradient -> backward over a fixed view set, captured
    once in a HIP graph and replayed.  Parameters, targets and gradient
    buffers are read and written in place, so a replay sees their current
    contents.  The workspace is sized by one eager step first; the capacity
    status of a replay is read by ``verify()`` (a replay whose pairs did not
    fit raises there: capture again)."""

    def __init__(self, rast: Rasterizer, g3: dict, g4: dict, views, targets, grads):
        self.rast, self.g3, self.g4, self.views = rast, g3, g4, list(views)
        self.targets = list(targets)
        self.gr3, self.gr4 = grads
        self.dls = [torch.empty((3, v.height, v.width), dtype=torch.float32, device="cuda") for v in self.views]
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        rast.check_mode = "eager"
        self._body()  # sizes the workspace and the capacity
        torch.cuda.synchronize()
        rast.check_mode = "deferred"
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._body()  # warm-up on the capture stream
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(self.graph):
            self.images = self._body()

    def _body(self):
        h = self.rast.forward(self.g3, self.g4, self.views)
        l1_loss_grad(self.rast, h.images, self.targets, self.views, self.dls, self.loss)
        self.rast.backward(h, self.g3, self.g4, self.dls, out=(self.gr3, self.gr4))
        return h.images

    def replay(self):
        self.graph.replay()

    def verify(self) -> int:
        return self.rast.verify()


def adam_step(rast: Rasterizer, params, grads, ms, vs, lrs, step: int, betas=(0.9, 0.999), eps=1e-8,
              masks=None):
    """One Adam step over lists of float32 CUDA tensors (in place on params,
    ms, vs).  masks: optional list of (uint8 [rows] CUDA tensor or None) per
    parameter: only the rows (Gaussians) whose mask is set are updated."""
    n = len(params)
    if masks is not None:
        for i in range(0, n, 16):
            sl = slice(i, min(n, i + 16))
            P, G, M, V, K = params[sl], grads[sl], ms[sl], vs[sl], masks[sl]
            k = len(P)
            sizes = (C.c_int64 * k)(*[int(p.numel()) for p in P])
            rows = (C.c_int64 * k)(*[int(mk.numel()) if mk is not None else 0 for mk in K])
            lr = (C.c_float * k)(*[float(x) for x in lrs[sl]])
            mp = L.ptr_array([mk.data_ptr() if mk is not None and mk.numel() else 0 for mk in K])
            rast.ctx.check(rast.ctx.L.h4dgs_adam_masked(
                rast.ctx.h, k, L.ptr_array([p.data_ptr() for p in P]), L.ptr_array([g.data_ptr() for g in G]),
                L.ptr_array([m.data_ptr() for m in M]), L.ptr_array([v.data_ptr() for v in V]), sizes, lr, mp, rows,
                C.c_double(betas[0]), C.c_double(betas[1]), C.c_double(eps), int(step), _stream()))
        return
    for i in range(0, n, 16):
        sl = slice(i, min(n, i + 16))
        P, G, M, V = params[sl], grads[sl], ms[sl], vs[sl]
        k = len(P)
        sizes = (C.c_int64 * k)(*[int(p.numel()) for p in P])
        lr = (C.c_float * k)(*[float(x) for x in lrs[sl]])
        rast.ctx.check(rast.ctx.L.h4dgs_adam(
            rast.ctx.h, k, L.ptr_array([p.data_ptr() for p in P]), L.ptr_array([g.data_ptr() for g in G]),
            L.ptr_array([m.data_ptr() for m in M]), L.ptr_array([v.data_ptr() for v in V]), sizes, lr,
            C.c_double(betas[0]), C.c_double(betas[1]), C.c_double(eps), int(step), _stream()))
