"""The C-ABI library on the host: it loads, exports every declared entry point,
sizes workspaces and rejects bad arguments before touching a GPU (no GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import scenegen as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "h4dgs.h")


@pytest.fixture(scope="module")
def L():
    from paper_2505_13215_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2505_13215_amd import build
        build.build()
    return _lib


def declared_entry_points():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(h4dgs_\w+)\s*\(", txt)))


def test_header_declares_the_expected_calls():
    names = declared_entry_points()
    for must in ("h4dgs_render_fwd", "h4dgs_render_bwd", "h4dgs_convert_static", "h4dgs_workspace_size"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    lib = L.load()
    for name in declared_entry_points():
        assert hasattr(lib, name), name
    assert set(declared_entry_points()) == set(L.EXPORTS)


def test_version(L):
    assert "gfx950" in L.version()


def _cfg(L, tile=16, chunk=256, batched=0, cap=1 << 20):
    return L.Config(tile, chunk, batched, 0, cap)


def _ctx(L):
    return L.Context()


def _views(L, n=1, W=128, H=96):
    v = sg.tiny_scene(n3=1, n4=1, width=W, height=H).views[0]
    return L.view_array([v] * n)


def test_workspace_size_grows_with_inputs(L):
    c = _ctx(L)
    st, sc = C.c_size_t(), C.c_size_t()
    va = _views(L)
    cfg = _cfg(L)
    assert c.L.h4dgs_workspace_size(c.h, 1000, 1000, va, 1, C.byref(cfg), C.byref(st), C.byref(sc)) == 0
    s1, k1 = st.value, sc.value
    assert c.L.h4dgs_workspace_size(c.h, 4000, 1000, va, 1, C.byref(cfg), C.byref(st), C.byref(sc)) == 0
    assert st.value > s1 and sc.value > k1
    cfg2 = _cfg(L, cap=1 << 22)
    assert c.L.h4dgs_workspace_size(c.h, 1000, 1000, va, 1, C.byref(cfg2), C.byref(st), C.byref(sc)) == 0
    assert st.value > s1
    va2 = _views(L, 2)
    assert c.L.h4dgs_workspace_size(c.h, 1000, 1000, va2, 2, C.byref(cfg), C.byref(st), C.byref(sc)) == 0
    # per view: 64 B records for every Gaussian, 20 B of per-pixel state
    assert st.value >= s1 + 2000 * 64 + 128 * 96 * 20


def _distinct_views(L, n=4, W=128, H=96):
    v = sg.tiny_scene(n3=1, n4=1, width=W, height=H).views[0]
    out = []
    for k in range(n):
        M = v.world_to_cam.copy()
        M[0, 3] += 0.01 * k
        out.append(sg.View(M, v.fx, v.fy, v.cx, v.cy, W, H, 0.5, v.bg))
    return L.view_array(out)


def test_batched_workspace(L):
    """Batched mode keeps the same state (kept from forward to backward) and
    needs per-pass scratch for every view of the call at once."""
    c = _ctx(L)
    st, sc = C.c_size_t(), C.c_size_t()
    va = _distinct_views(L, 4)
    assert c.L.h4dgs_workspace_size(c.h, 3000, 1000, va, 4, C.byref(_cfg(L)), C.byref(st), C.byref(sc)) == 0
    s_single, k_single = st.value, sc.value
    assert c.L.h4dgs_workspace_size(c.h, 3000, 1000, va, 4, C.byref(_cfg(L, batched=1)), C.byref(st),
                                    C.byref(sc)) == 0
    assert st.value == s_single
    assert sc.value >= k_single
    # depth keys, ids and their sort buffers for all four views
    assert sc.value >= 4 * 4000 * 16


def test_shared_static_binning_workspace(L):
    """Four views of one camera in a batched call bin the 3D Gaussians once,
    on a super-tile grid of their own: the state grows by that grid's list
    ranges (16 bytes per super-tile: 128 x 96 pixels at 16-pixel tiles is 2 x 2
    super-tiles of 64 pixels, rounded up to the workspace's 256-byte
    alignment, or absorbed by the 2 MiB alignment of the per-pixel arrays that
    follow them); the scratch does not grow (its depth sorts are over fewer
    keys)."""
    c = _ctx(L)
    st, sc = C.c_size_t(), C.c_size_t()
    assert c.L.h4dgs_workspace_size(c.h, 3000, 1000, _distinct_views(L, 4), 4, C.byref(_cfg(L, batched=1)),
                                    C.byref(st), C.byref(sc)) == 0
    s_distinct, k_distinct = st.value, sc.value
    assert c.L.h4dgs_workspace_size(c.h, 3000, 1000, _views(L, 4), 4, C.byref(_cfg(L, batched=1)), C.byref(st),
                                    C.byref(sc)) == 0
    assert 0 <= st.value - s_distinct <= (1 << 21) + 256 and sc.value <= k_distinct
    # no 3D Gaussians: nothing to share
    assert c.L.h4dgs_workspace_size(c.h, 0, 4000, _views(L, 4), 4, C.byref(_cfg(L, batched=1)), C.byref(st),
                                    C.byref(sc)) == 0
    s0 = st.value
    assert c.L.h4dgs_workspace_size(c.h, 0, 4000, _distinct_views(L, 4), 4, C.byref(_cfg(L, batched=1)),
                                    C.byref(st), C.byref(sc)) == 0
    assert st.value == s0


def test_views_beyond_one_pass_of_super_tiles_are_refused(L):
    """A view's super-tiles must fit one pass's 16-bit key range: 8200 x 8200
    pixels at 8-pixel tiles (257 x 257 super-tiles of 32 pixels) is refused
    before anything is enqueued, 8192 x 8192 is accepted."""
    c = _ctx(L)
    st, sc = C.c_size_t(), C.c_size_t()
    ok = c.L.h4dgs_workspace_size(c.h, 10, 10, _views(L, 1, 8192, 8192), 1, C.byref(_cfg(L, tile=8)), C.byref(st),
                                  C.byref(sc))
    assert ok == L.H4D_OK
    bad = c.L.h4dgs_workspace_size(c.h, 10, 10, _views(L, 1, 8200, 8200), 1, C.byref(_cfg(L, tile=8)),
                                   C.byref(st), C.byref(sc))
    assert bad == L.H4D_ERR_UNSUPPORTED
    assert "super-tiles" in c.L.h4dgs_last_error(c.h).decode()


def test_batched_pass_size_limit(L):
    """A batched pass indexes (view, Gaussian) pairs with 32-bit integers."""
    c = _ctx(L)
    st, sc = C.c_size_t(), C.c_size_t()
    va = _views(L, 3)
    n = 1 << 30
    assert c.L.h4dgs_workspace_size(c.h, n, 0, va, 3, C.byref(_cfg(L)), C.byref(st), C.byref(sc)) == 0
    rc = c.L.h4dgs_workspace_size(c.h, n, 0, va, 3, C.byref(_cfg(L, batched=1)), C.byref(st), C.byref(sc))
    assert rc == L.H4D_ERR_INVALID_ARG
    assert b"batched" in c.L.h4dgs_last_error(c.h)
    rc = c.L.h4dgs_workspace_size(c.h, 10, 0, va, 3, C.byref(_cfg(L, batched=2)), C.byref(st), C.byref(sc))
    assert rc == L.H4D_ERR_INVALID_ARG
    cfg = _cfg(L)
    cfg.cull = 2
    assert c.L.h4dgs_workspace_size(c.h, 10, 0, va, 3, C.byref(cfg), C.byref(st), C.byref(sc)) == L.H4D_ERR_INVALID_ARG
    assert b"cull" in c.L.h4dgs_last_error(c.h)


@pytest.mark.parametrize("tile,chunk", [(7, 256), (16, 100), (64, 256), (0, 0)])
def test_bad_tile_or_chunk_rejected(L, tile, chunk):
    c = _ctx(L)
    st, sc = C.c_size_t(), C.c_size_t()
    cfg = _cfg(L, tile, chunk)
    rc = c.L.h4dgs_workspace_size(c.h, 10, 10, _views(L), 1, C.byref(cfg), C.byref(st), C.byref(sc))
    assert rc == L.H4D_ERR_INVALID_ARG
    assert b"tile" in c.L.h4dgs_last_error(c.h)


@pytest.mark.parametrize("nv", [0, 33])
def test_view_count_rejected(L, nv):
    c = _ctx(L)
    st, sc = C.c_size_t(), C.c_size_t()
    cfg = _cfg(L)
    va = _views(L, max(nv, 1))
    assert c.L.h4dgs_workspace_size(c.h, 10, 10, va, nv, C.byref(cfg), C.byref(st), C.byref(sc)) == 1


def test_bad_view_rejected(L):
    c = _ctx(L)
    st, sc = C.c_size_t(), C.c_size_t()
    cfg = _cfg(L)
    va = _views(L)
    va[0].width = 0
    assert c.L.h4dgs_workspace_size(c.h, 10, 10, va, 1, C.byref(cfg), C.byref(st), C.byref(sc)) == 1
    va = _views(L)
    va[0].fx = float("nan")
    assert c.L.h4dgs_workspace_size(c.h, 10, 10, va, 1, C.byref(cfg), C.byref(st), C.byref(sc)) == 1


def _sets(L, n3=4, n4=4, null=False):
    fake = C.c_void_p(0 if null else 0x1000)  # never dereferenced: argument checks fail first
    g3 = L.G3D(n3, fake, fake, fake, fake, fake)
    g4 = L.G4D(n4, fake, fake, fake, fake, fake, fake, fake)
    return g3, g4


def test_render_fwd_rejects_null_arrays_on_the_host(L):
    c = _ctx(L)
    g3, g4 = _sets(L, null=True)
    cfg = _cfg(L)
    imgs = L.ptr_array([0x1000])
    rc = c.L.h4dgs_render_fwd(c.h, C.byref(g3), C.byref(g4), _views(L), 1, C.byref(cfg), imgs, C.c_void_p(0x1000),
                              1 << 30, C.c_void_p(0x1000), 1 << 30, None)
    assert rc == L.H4D_ERR_INVALID_ARG


def test_render_fwd_rejects_small_workspace(L):
    c = _ctx(L)
    g3, g4 = _sets(L)
    cfg = _cfg(L)
    imgs = L.ptr_array([0x1000])
    rc = c.L.h4dgs_render_fwd(c.h, C.byref(g3), C.byref(g4), _views(L), 1, C.byref(cfg), imgs, C.c_void_p(0x1000),
                              16, C.c_void_p(0x1000), 1 << 30, None)
    assert rc == L.H4D_ERR_INVALID_ARG and b"state too small" in c.L.h4dgs_last_error(c.h)


def test_render_bwd_rejects_mismatched_gradient_counts(L):
    c = _ctx(L)
    g3, g4 = _sets(L)
    gr3, gr4 = _sets(L, n3=5)
    cfg = _cfg(L)
    dls = L.ptr_array([0x1000])
    rc = c.L.h4dgs_render_bwd(c.h, C.byref(g3), C.byref(g4), _views(L), 1, C.byref(cfg), dls, C.c_void_p(0x1000),
                              1 << 30, C.c_void_p(0x1000), 1 << 30, C.byref(gr3), C.byref(gr4), None)
    assert rc == L.H4D_ERR_INVALID_ARG


def test_negative_counts_rejected(L):
    c = _ctx(L)
    g3, g4 = _sets(L, n3=-1)
    cfg = _cfg(L)
    rc = c.L.h4dgs_render_fwd(c.h, C.byref(g3), C.byref(g4), _views(L), 1, C.byref(cfg), L.ptr_array([0x1000]),
                              C.c_void_p(0x1000), 1 << 30, C.c_void_p(0x1000), 1 << 30, None)
    assert rc == L.H4D_ERR_INVALID_ARG


def test_convert_static_argument_checks(L):
    c = _ctx(L)
    g3, g4 = _sets(L)
    o3, o4 = _sets(L, n3=8, n4=4)
    n4o, n3o = C.c_int32(), C.c_int32()
    rc = c.L.h4dgs_convert_static(c.h, C.byref(g4), C.byref(g3), C.c_float(0.0), C.byref(o4), C.byref(o3),
                                  C.c_void_p(0x1000), C.byref(n4o), C.byref(n3o), C.c_void_p(0x1000), 1 << 20, None)
    assert rc == L.H4D_ERR_INVALID_ARG  # tau must be > 0
    small3, _ = _sets(L, n3=7)
    rc = c.L.h4dgs_convert_static(c.h, C.byref(g4), C.byref(g3), C.c_float(0.5), C.byref(o4), C.byref(small3),
                                  C.c_void_p(0x1000), C.byref(n4o), C.byref(n3o), C.c_void_p(0x1000), 1 << 20, None)
    assert rc == L.H4D_ERR_CAPACITY


def test_convert_scratch_bytes_monotone(L):
    lib = L.load()
    assert lib.h4dgs_convert_scratch_bytes(1000) < lib.h4dgs_convert_scratch_bytes(100000)


def test_adam_argument_checks(L):
    c = _ctx(L)
    one = (C.c_int64 * 1)(10)
    lr = (C.c_float * 1)(1e-3)
    arr = L.ptr_array([0x1000])
    assert c.L.h4dgs_adam(c.h, 17, arr, arr, arr, arr, one, lr, 0.9, 0.999, 1e-8, 1, None) == 1
    assert c.L.h4dgs_adam(c.h, 1, arr, arr, arr, arr, one, lr, 0.9, 0.999, 1e-8, 0, None) == 1
    assert c.L.h4dgs_adam(c.h, 1, arr, arr, arr, arr, one, lr, 1.0, 0.999, 1e-8, 1, None) == 1


def test_null_context(L):
    lib = L.load()
    st, sc = C.c_size_t(), C.c_size_t()
    assert lib.h4dgs_workspace_size(None, 1, 1, None, 1, None, C.byref(st), C.byref(sc)) == 1
    assert lib.h4dgs_last_error(None) == b"null context"


def test_profile_levels(L):
    c = _ctx(L)
    for level in (0, 1, 2, 3, 4, 0):
        assert c.L.h4dgs_profile(c.h, level) == 0
    for level in (-1, 5):
        assert c.L.h4dgs_profile(c.h, level) == 1
        assert b"profile level" in c.L.h4dgs_last_error(c.h)
    ms = (C.c_double * 8)()
    n = (C.c_int64 * 8)()
    assert c.L.h4dgs_profile_read(c.h, ms, n) == 0
    assert list(n) == [0] * 8


def test_radix_pass_buffer_check_on_the_host(L):
    """The host-side check every radix pass of the binning goes through before
    launch: exactly sized buffers pass, one word less of histogram or digit
    totals fails (the launcher then enqueues nothing), and so do digit widths
    outside [1, 11] or more than 8 bits with 2 keys per thread."""
    lib = L.load()
    for cap, nseg, bits, items in [(250_000, 1, 8, 2), (250_000, 32, 8, 2), (26_000_000, 1, 11, 8),
                                   (5_000, 1, 6, 8), (0, 1, 9, 8), (1, 3, 1, 8)]:
        need = lib.h4dgs_radix_hist_words(cap, nseg, bits, items)
        tot = (1 << bits) * max(1, nseg)
        assert need >= (1 << bits) * max(1, nseg)
        assert lib.h4dgs_radix_pass_check(cap, nseg, bits, items, need, tot) == L.H4D_OK
        assert lib.h4dgs_radix_pass_check(cap, nseg, bits, items, need - 1, tot) == L.H4D_ERR_INVALID_ARG
        assert lib.h4dgs_radix_pass_check(cap, nseg, bits, items, need, tot - 1) == L.H4D_ERR_INVALID_ARG
    # the failure that once happened: a histogram sized for 6-bit digits, used
    # by an 11-bit pass over the same keys
    small = lib.h4dgs_radix_hist_words(3_000_000, 1, 6, 8)
    assert lib.h4dgs_radix_pass_check(3_000_000, 1, 11, 8, small, 1 << 11) == L.H4D_ERR_INVALID_ARG
    for bits, items in [(0, 8), (12, 8), (9, 2), (8, 4)]:
        assert lib.h4dgs_radix_pass_check(1000, 1, bits, items, 1 << 40, 1 << 40) == L.H4D_ERR_INVALID_ARG
