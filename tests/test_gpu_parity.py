"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars (from the method's arithmetic, see the design notes):
  * images: max |C_gpu - C_oracle| <= 1e-4 over pixels whose oracle decisions
    are all outside the FP32 guard band; flagged pixels < 1e-3 of the image;
  * gradients: per parameter group ||g - g_ref|| <= 1e-3 ||g_ref||, and per
    element |g - g_ref| <= 1e-3 |g_ref| + 1e-3 rms(g_ref) for every Gaussian whose
    square holds no flagged pixel;
  * tile lists, sort order, ranges and the static conversion: bit-exact on the
    same inputs.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from parity_util import IMG_TOL, GRAD_TOL, check_image as _check_image, flagged_gaussians as _flagged_gaussians
from parity_util import check_grads as _check_grads, mask_flagged


@pytest.fixture(scope="module")
def h4d():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_13215_amd as m
    m._lib.load()
    return m


def _render(h4d, scene, views, tile=16, chunk=256, cap=1 << 20):
    rast = h4d.Rasterizer(tile=tile, chunk=chunk, pair_capacity=cap)
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    h = rast.forward(g3, g4, views)
    torch.cuda.synchronize()
    return rast, g3, g4, h


# ---------------------------------------------------------------------------
# forward
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(128, 96), (77, 45), (200, 150)])
def test_forward_matches_oracle(h4d, shape):
    W, H = shape
    print(f"[forward parity] {W}x{H}", flush=True)
    scene = sg.tiny_scene(width=W, height=H)
    v = scene.views[0]
    _, _, _, h = _render(h4d, scene, [v])
    ref = oracle.render(scene, v)
    _check_image(h.images[0].cpu().numpy(), ref["img"], ref["amb"])


def test_forward_mid_scene_many_tiles(h4d):
    print("[forward parity] 20k Gaussians, 333x250", flush=True)
    scene = sg.multiview_scene(n_total=20_000, width=333, height=250, seed=3)
    v = scene.views[7].with_time(0.41)
    rast, g3, g4, h = _render(h4d, scene, [v])
    ref = oracle.render(scene, v)
    _check_image(h.images[0].cpu().numpy(), ref["img"], ref["amb"])


def test_forward_background_and_time(h4d):
    scene = sg.tiny_scene(n3=400, n4=600, width=96, height=64, seed=4)
    v0 = scene.views[0]
    v = sg.View(v0.world_to_cam, v0.fx, v0.fy, v0.cx, v0.cy, v0.width, v0.height, 0.23, (0.2, 0.6, 1.0))
    _, _, _, h = _render(h4d, scene, [v])
    ref = oracle.render(scene, v)
    _check_image(h.images[0].cpu().numpy(), ref["img"], ref["amb"])


@pytest.mark.parametrize("n3,n4", [(0, 500), (500, 0), (0, 0)])
def test_forward_single_set_and_empty(h4d, n3, n4):
    scene = sg.tiny_scene(n3=n3, n4=n4, width=64, height=48, seed=2)
    v = sg.View(scene.views[0].world_to_cam, scene.views[0].fx, scene.views[0].fy, 32.0, 24.0, 64, 48, 0.5,
                (0.1, 0.2, 0.3))
    _, _, _, h = _render(h4d, scene, [v])
    ref = oracle.render(scene, v)
    _check_image(h.images[0].cpu().numpy(), ref["img"], ref["amb"])


@pytest.mark.parametrize("shape", [(32767, 7), (5, 32767), (1, 1), (17, 1)])
def test_forward_extreme_image_sizes(h4d, shape):
    """Largest accepted image edge (32767), one-pixel images, ragged single tiles."""
    W, H = shape
    print(f"[forward parity] {W}x{H}", flush=True)
    scene = sg.tiny_scene(n3=600, n4=600, seed=11)
    v0 = scene.views[0]
    v = sg.View(v0.world_to_cam, 300.0, 300.0, W / 2.0, H / 2.0, W, H, 0.5, (0.2, 0.3, 0.4))
    _, _, _, h = _render(h4d, scene, [v], cap=1 << 22)
    ref = oracle.render(scene, v)
    _check_image(h.images[0].cpu().numpy(), ref["img"], ref["amb"])


def test_forward_everything_behind_camera(h4d):
    scene = sg.tiny_scene(n3=200, n4=200, width=64, height=48, seed=6)
    v0 = scene.views[0]
    M = v0.world_to_cam.copy()
    M[:, :3] = -M[:, :3]  # look away from the scene
    M[2, 3] = -3.0
    v = sg.View(M, v0.fx, v0.fy, v0.cx, v0.cy, 64, 48, 0.5, (0.3, 0.3, 0.3))
    _, _, _, h = _render(h4d, scene, [v])
    img = h.images[0].cpu().numpy()
    assert np.array_equal(img, np.broadcast_to(np.float32([0.3, 0.3, 0.3])[:, None, None], img.shape))


def test_forward_is_deterministic(h4d):
    scene = sg.tiny_scene()
    v = scene.views[0]
    rast, g3, g4, h1 = _render(h4d, scene, [v])
    a = h1.images[0].clone()
    h2 = rast.forward(g3, g4, [v])
    assert torch.equal(a, h2.images[0])


def test_images_do_not_depend_on_tile_chunk_or_cull(h4d):
    scene = sg.tiny_scene(width=111, height=70, seed=8)
    v = scene.views[0]
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    base = None
    for tile in (8, 16, 32):
        for chunk in (64, 128, 256, 512):
            for cull in (False, True):
                rast = h4d.Rasterizer(tile=tile, chunk=chunk, pair_capacity=1 << 20, cull=cull)
                img = rast.forward(g3, g4, [v]).images[0].cpu()
                if base is None:
                    base = img
                else:
                    assert torch.equal(img, base), (tile, chunk, cull)


def test_capacity_overflow_is_detected_and_recovered(h4d):
    scene = sg.tiny_scene()
    v = scene.views[0]
    rast, g3, g4, h = _render(h4d, scene, [v], cap=64)
    assert rast.capacity > 64 and rast.last_pairs > 64
    ref = oracle.render(scene, v)
    _check_image(h.images[0].cpu().numpy(), ref["img"], ref["amb"])


# ---------------------------------------------------------------------------
# stages on identical screen-space inputs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("tile", [8, 16, 32])
def test_tile_lists_and_ranges_bit_exact(h4d, tile):
    W, H = 203, 131
    rec = sg.synthetic_records(3000, W, H, seed=21, max_radius=40)
    rast = h4d.Rasterizer(tile=tile, chunk=256, pair_capacity=1 << 20, cull=False)
    img, T, ids, ranges = h4d.rasterize_splats(rast, rec, W, H)
    start, ref_ids = oracle.tile_lists(rec, W, H, tile)
    ids = ids.cpu().numpy()
    rg = ranges.cpu().numpy()
    tiles = len(start) - 1
    assert rg.shape[0] == tiles
    for t in range(tiles):
        got = ids[rg[t, 0]:rg[t, 1]]
        assert np.array_equal(got, ref_ids[start[t]:start[t + 1]]), t


@pytest.mark.parametrize("tile,W,H,n,max_radius", [(8, 203, 131, 3000, 40), (16, 203, 131, 3000, 40),
                                                   (32, 203, 131, 3000, 40), (8, 400, 300, 1200, 150),
                                                   (16, 640, 480, 800, 300)])
def test_culled_tile_lists_drop_only_tiles_without_blending(h4d, tile, W, H, n, max_radius):
    """With cull, each tile's list is an order-preserving subset of the
    square-overlap list, every dropped splat stays below alpha = 1/255 at
    every pixel centre of the tile inside its square (checked in FP64), and the
    image is bit-identical to the unculled one.  The larger radii give splats
    taller than the binning's table of per-row tile spans (more than 16 tile
    rows), whose tiles are tested per coarse entry."""
    print(f"[culled lists] tile {tile} {W}x{H} n={n} r<={max_radius}", flush=True)
    rec = sg.synthetic_records(n, W, H, seed=23, max_radius=max_radius)
    full = h4d.Rasterizer(tile=tile, chunk=128, pair_capacity=1 << 20, cull=False)
    img0, T0, _, _ = h4d.rasterize_splats(full, rec, W, H)
    rast = h4d.Rasterizer(tile=tile, chunk=128, pair_capacity=1 << 20, cull=True)
    img1, T1, ids, ranges = h4d.rasterize_splats(rast, rec, W, H)
    assert torch.equal(img0, img1) and torch.equal(T0, T1)
    start, ref_ids = oracle.tile_lists(rec, W, H, tile)
    ids = ids.cpu().numpy()
    rg = ranges.cpu().numpy()
    u, v = rec["u"].astype(np.float64), rec["v"].astype(np.float64)
    c0, c1, c2 = (rec["conic"][i].astype(np.float64) for i in range(3))
    op, r = rec["opacity"].astype(np.float64), rec["radius"].astype(np.int64)
    tiles_x = (W + tile - 1) // tile
    kept = dropped = 0
    for t in range(len(start) - 1):
        got = ids[rg[t, 0]:rg[t, 1]]
        ref = ref_ids[start[t]:start[t + 1]]
        # order-preserving subset: matching ids appear in the same relative order
        where = {g: i for i, g in enumerate(ref)}
        idx = np.array([where[g] for g in got], dtype=np.int64)
        assert np.all(np.diff(idx) > 0), t
        kept += len(got)
        tx, ty = t % tiles_x, t // tiles_x
        for g in np.setdiff1d(ref, got):
            dropped += 1
            xa = max(tx * tile, int(np.ceil(u[g] - r[g] - 0.5)), 0)
            xb = min(tx * tile + tile - 1, int(np.floor(u[g] + r[g] - 0.5)), W - 1)
            ya = max(ty * tile, int(np.ceil(v[g] - r[g] - 0.5)), 0)
            yb = min(ty * tile + tile - 1, int(np.floor(v[g] + r[g] - 0.5)), H - 1)
            X, Y = np.meshgrid(np.arange(xa, xb + 1) + 0.5 - u[g], np.arange(ya, yb + 1) + 0.5 - v[g])
            alpha = op[g] * np.exp(-0.5 * (c0[g] * X * X + 2.0 * c1[g] * X * Y + c2[g] * Y * Y))
            assert alpha.max() < 1.0 / 255.0, (t, g)
    assert dropped > 0.05 * (kept + dropped), "culling removed almost nothing"


def test_composite_on_shared_splats(h4d):
    W, H = 150, 100
    rec = sg.synthetic_records(2500, W, H, seed=22, max_radius=30)
    rast = h4d.Rasterizer(tile=16, chunk=256, pair_capacity=1 << 20)
    img, T, _, _ = h4d.rasterize_splats(rast, rec, W, H, bg=(0.5, 0.25, 0.125))
    ref, Tref, amb = oracle.composite_records(rec, W, H, tile=16, bg=(0.5, 0.25, 0.125))
    _check_image(img.cpu().numpy(), ref, amb)
    assert np.abs(T.cpu().numpy() - Tref)[~amb].max() <= 1e-4


# ---------------------------------------------------------------------------
# backward
# ---------------------------------------------------------------------------

def _grads_gpu(h4d, scene, views, dls, tile=16, chunk=256):
    rast = h4d.Rasterizer(tile=tile, chunk=chunk, pair_capacity=1 << 20)
    g3 = {k: v.requires_grad_(True) for k, v in h4d.to_device(scene.g3).items()}
    g4 = {k: v.requires_grad_(True) for k, v in h4d.to_device(scene.g4).items()}
    imgs = h4d.render(rast, g3, g4, views)
    loss = sum((im * torch.as_tensor(d, device="cuda")).sum() for im, d in zip(imgs, dls))
    loss.backward()
    torch.cuda.synchronize()
    return {k: g3[k].grad for k in g3}, {k: g4[k].grad for k in g4}


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_oracle(h4d, seed):
    print(f"[backward parity] tiny seed {seed}", flush=True)
    scene = sg.tiny_scene(seed=seed)
    v = scene.views[0]
    dl = sg.upstream_grads([v], seed=10 + seed)
    gr3, gr4 = _grads_gpu(h4d, scene, [v], dl)
    r3, r4 = oracle.render_bwd(scene, [v], dl)
    amb = oracle.render(scene, v)["amb"]
    _check_grads(scene, gr3, gr4, r3, r4, _flagged_gaussians(scene, v, amb))


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_all_gaussians_masked_upstream(h4d, seed):
    """Upstream gradients zeroed at guard-band pixels: every Gaussian is checked."""
    scene = sg.tiny_scene(seed=seed)
    v = scene.views[0]
    amb = oracle.render(scene, v)["amb"]
    dl = [mask_flagged(sg.upstream_grads([v], seed=20 + seed)[0], amb)]
    gr3, gr4 = _grads_gpu(h4d, scene, [v], dl)
    r3, r4 = oracle.render_bwd(scene, [v], dl)
    _check_grads(scene, gr3, gr4, r3, r4, np.zeros(scene.n3 + scene.n4, bool))


def test_backward_l1_loss_and_background(h4d):
    scene = sg.tiny_scene(n3=700, n4=900, width=100, height=80, seed=5)
    v0 = scene.views[0]
    v = sg.View(v0.world_to_cam, v0.fx, v0.fy, 50.0, 40.0, 100, 80, 0.7, (0.3, 0.1, 0.9))
    ref = oracle.render(scene, v)
    target = sg.target_images([v], seed=1)[0]
    # the L1 gradient sign is taken from the oracle image, so both sides get the same dL/dC
    dl = (np.sign(ref["img"] - target) / (3 * v.width * v.height)).astype(np.float32)
    gr3, gr4 = _grads_gpu(h4d, scene, [v], [dl])
    r3, r4 = oracle.render_bwd(scene, [v], [dl])
    _check_grads(scene, gr3, gr4, r3, r4, _flagged_gaussians(scene, v, ref["amb"]))


def test_multi_view_gradients_are_sums(h4d):
    scene = sg.tiny_scene(seed=3)
    v0 = scene.views[0]
    views = [v0.with_time(0.2), v0.with_time(0.7)]
    dls = sg.upstream_grads(views, seed=4)
    both3, both4 = _grads_gpu(h4d, scene, views, dls)
    a3, a4 = _grads_gpu(h4d, scene, views[:1], dls[:1])
    b3, b4 = _grads_gpu(h4d, scene, views[1:], dls[1:])
    for k in both4:
        s = (a4[k] + b4[k]).double()
        assert torch.allclose(both4[k].double(), s, rtol=1e-5, atol=1e-6 * float(s.abs().max()) + 1e-12), k
    for k in both3:
        s = (a3[k] + b3[k]).double()
        assert torch.allclose(both3[k].double(), s, rtol=1e-5, atol=1e-6 * float(s.abs().max()) + 1e-12), k


@pytest.mark.parametrize("tile,chunk", [(8, 128), (32, 512)])
def test_backward_other_tile_shapes(h4d, tile, chunk):
    scene = sg.tiny_scene(seed=7, width=90, height=70)
    v = scene.views[0]
    dl = sg.upstream_grads([v], seed=5)
    gr3, gr4 = _grads_gpu(h4d, scene, [v], dl, tile=tile, chunk=chunk)
    r3, r4 = oracle.render_bwd(scene, [v], dl)
    amb = oracle.render(scene, v)["amb"]
    _check_grads(scene, gr3, gr4, r3, r4, _flagged_gaussians(scene, v, amb))


# ---------------------------------------------------------------------------
# static conversion and Adam
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("frac", [0.0, 0.5, 0.9, 1.0])
def test_convert_static_bit_exact(h4d, frac):
    rng = np.random.default_rng(int(frac * 10))
    g4 = sg.draw_4d(rng, 3000, 2.0, static_fraction=frac, tau=0.5)
    g3 = sg.draw_3d(rng, 1000, 2.0)
    scene = sg.Scene(g3, g4)
    rast = h4d.Rasterizer()
    n3, n4, perm = None, None, None
    o3, o4, perm = h4d.convert_static(rast, h4d.to_device(g3), h4d.to_device(g4), 0.5)
    rperm, rn4, rn3, rq = oracle.convert_static(scene, 0.5)
    assert np.array_equal(perm.cpu().numpy(), rperm)
    assert o4["opacity"].shape[0] == rn4 and o3["opacity"].shape[0] == rn3
    keep = np.nonzero(rperm >= 0)[0]
    conv = np.nonzero(rperm < 0)[0]
    for k in ("mean", "mean_t", "log_scale", "quat_l", "quat_r", "opacity", "sh"):
        assert np.array_equal(o4[k].cpu().numpy(), g4[k][..., keep]), k
    for k in ("mean", "log_scale", "quat", "opacity", "sh"):
        assert np.array_equal(o3[k].cpu().numpy()[..., :1000], g3[k]), k
    assert np.array_equal(o3["mean"].cpu().numpy()[:, 1000:], g4["mean"][:, conv])
    assert np.array_equal(o3["log_scale"].cpu().numpy()[:, 1000:], g4["log_scale"][:3, conv])
    assert np.array_equal(o3["opacity"].cpu().numpy()[1000:], g4["opacity"][conv])
    assert np.array_equal(o3["sh"].cpu().numpy()[:, 1000:], g4["sh"][:, conv])
    q = o3["quat"].cpu().numpy()[:, 1000:].astype(np.float64)
    if q.shape[1]:
        qn = q / np.linalg.norm(q, axis=0)
        rn = rq / np.linalg.norm(rq, axis=0)
        assert np.abs(qn - rn).max() <= 1e-6


def test_convert_moments_follow_the_rows(h4d):
    """Two moment sets (Adam's m and v) moved with the conversion of a small
    mixed scene: bit-exact against a host gather driven by the oracle's
    permutation (converted rows keep the moments of their copied fields and
    start their quaternion's at zero)."""
    from test_gpu_fullsize_convert_adam import _moved_moments
    rng = np.random.default_rng(17)
    g4 = sg.draw_4d(rng, 2000, 2.0, static_fraction=0.4, tau=0.5)
    g3 = sg.draw_3d(rng, 700, 2.0)
    scene = sg.Scene(g3, g4)
    moms = [({k: rng.normal(size=v.shape).astype(np.float32) for k, v in g3.items()},
             {k: rng.normal(size=v.shape).astype(np.float32) for k, v in g4.items()}) for _ in range(2)]
    rperm, rn4, rn3, _ = oracle.convert_static(scene, 0.5)
    rast = h4d.Rasterizer()
    _, _, perm, moved = h4d.convert_static(rast, h4d.to_device(g3), h4d.to_device(g4), 0.5,
                                           moments=[(h4d.to_device(a), h4d.to_device(b)) for a, b in moms])
    assert np.array_equal(perm.cpu().numpy(), rperm) and (rperm < 0).sum() > 100
    for (m3, m4), (g3m, g4m) in zip(moms, moved):
        w3, w4 = _moved_moments(m3, m4, rperm)
        for k in w4:
            assert np.array_equal(g4m[k].cpu().numpy(), w4[k]), k
        for k in w3:
            assert np.array_equal(g3m[k].cpu().numpy(), w3[k]), k


def test_convert_static_empty_sets(h4d):
    rast = h4d.Rasterizer()
    g3 = sg.draw_3d(np.random.default_rng(0), 10, 1.0)
    o3, o4, perm = h4d.convert_static(rast, h4d.to_device(g3), h4d.to_device(sg.empty_4d()), 0.5)
    assert o4["opacity"].shape[0] == 0 and o3["opacity"].shape[0] == 10
    assert torch.equal(o3["sh"].cpu(), torch.as_tensor(g3["sh"]))


def test_adam_matches_oracle(h4d):
    rng = np.random.default_rng(1)
    rast = h4d.Rasterizer()
    sizes = [1000, 3, 4096, 77]
    P = [rng.normal(size=n).astype(np.float32) for n in sizes]
    M = [np.zeros(n, np.float32) for n in sizes]
    V = [np.zeros(n, np.float32) for n in sizes]
    lrs = [1e-3, 5e-2, 2.5e-3, 1.6e-4]
    tp = [torch.as_tensor(p, device="cuda") for p in P]
    tm = [torch.as_tensor(m, device="cuda") for m in M]
    tv = [torch.as_tensor(v, device="cuda") for v in V]
    eps32 = 2.0 ** -24
    for step in range(1, 4):
        G = [rng.normal(size=n).astype(np.float32) for n in sizes]
        tg = [torch.as_tensor(g, device="cuda") for g in G]
        prev = [(tp[i].cpu().numpy().astype(np.float64), tm[i].cpu().numpy().astype(np.float64),
                 tv[i].cpu().numpy().astype(np.float64)) for i in range(len(sizes))]
        refs = [oracle.adam(tp[i].cpu().numpy(), G[i], tm[i].cpu().numpy(), tv[i].cpu().numpy(), lrs[i], 0.9, 0.999,
                            1e-8, step) for i in range(len(sizes))]
        h4d.adam_step(rast, tp, tg, tm, tv, lrs, step)
        torch.cuda.synchronize()
        for i in range(len(sizes)):
            po, mo, vo = refs[i]
            p0, m0, v0 = prev[i]
            g = G[i].astype(np.float64)
            # float32 rounding bounds of each update (m may cancel, v cannot)
            mtol = 4 * eps32 * (0.9 * np.abs(m0) + 0.1 * np.abs(g)) + 1e-30
            assert (np.abs(tm[i].cpu().numpy() - mo) <= mtol).all()
            assert np.allclose(tv[i].cpu().numpy(), vo, rtol=8 * eps32, atol=0)
            c1, c2 = 1 - 0.9 ** step, 1 - 0.999 ** step
            upd = lrs[i] * (np.abs(mo) / c1) / (np.sqrt(vo / c2) + 1e-8)
            ptol = 4 * eps32 * np.abs(p0) + 8 * eps32 * upd + lrs[i] * mtol / c1 / (np.sqrt(vo / c2) + 1e-8)
            assert (np.abs(tp[i].cpu().numpy() - po) <= ptol + 1e-12).all()


@pytest.mark.parametrize("sizes", [[(128, 96)], [(77, 45), (31, 17), (1, 1)], [(1352, 1014)]])
def test_l1_loss_gradient(h4d, sizes):
    """dL/dC = sign(C - target) / (3 W H V) exactly (sign(0) = 0, including the
    scalar tail of an odd pixel count); the loss is the mean over views of the
    per-view mean absolute error."""
    rng = np.random.default_rng(len(sizes))
    rast = h4d.Rasterizer()
    views, imgs, tgts = [], [], []
    for (W, H) in sizes:
        views.append(sg.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), W, H))
        img = rng.uniform(0, 1, size=(3, H, W)).astype(np.float32)
        tgt = rng.uniform(0, 1, size=(3, H, W)).astype(np.float32)
        tgt.reshape(-1)[::7] = img.reshape(-1)[::7]  # ties
        imgs.append(img)
        tgts.append(tgt)
    ti = [torch.as_tensor(a, device="cuda") for a in imgs]
    tt = [torch.as_tensor(a, device="cuda") for a in tgts]
    dl = [torch.empty_like(a) for a in ti]
    loss = torch.full((1,), 123.0, device="cuda")
    h4d.l1_loss_grad(rast, ti, tt, views, dl, loss)
    torch.cuda.synchronize()
    V = len(sizes)
    ref_loss = 0.0
    for a, b, d in zip(imgs, tgts, dl):
        scale = np.float32(1.0 / (a.size * V))
        expect = np.sign(a - b).astype(np.float32) * scale
        assert np.array_equal(d.cpu().numpy(), expect)
        ref_loss += np.abs(a.astype(np.float64) - b).mean() / V
    assert abs(float(loss) - ref_loss) <= 1e-5 * ref_loss


# ---------------------------------------------------------------------------
# raw (non-unit) quaternions: the normalisation and its 1/|q| adjoint
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_raw_quaternions_forward_and_backward(h4d, seed):
    """Quaternion columns (q, q_l, q_r) scaled by seeded factors in [0.3, 3]
    as training leaves them after an optimiser step: the image against the
    oracle, and every gradient (upstream zeroed at flagged pixels) against the
    oracle's adjoint of the same raw arrays, which carries the 1/|q| factor
    and the projection onto the tangent of the unit sphere."""
    print(f"[raw quaternions] tiny seed {seed}", flush=True)
    scene = sg.raw_quaternion_norms(sg.tiny_scene(seed=seed), seed=30 + seed, lo=0.3, hi=3.0)
    for k in ("quat_l", "quat_r"):
        nrm = np.linalg.norm(scene.g4[k].astype(np.float64), axis=0)
        assert nrm.min() < 0.5 and nrm.max() > 2.0
    v = scene.views[0]
    ref = oracle.render(scene, v)
    _, _, _, h = _render(h4d, scene, [v])
    _check_image(h.images[0].cpu().numpy(), ref["img"], ref["amb"])
    dl = [mask_flagged(sg.upstream_grads([v], seed=40 + seed)[0], ref["amb"])]
    gr3, gr4 = _grads_gpu(h4d, scene, [v], dl)
    r3, r4 = oracle.render_bwd(scene, [v], dl)
    _check_grads(scene, gr3, gr4, r3, r4, np.zeros(scene.n3 + scene.n4, bool))
    # the quaternion gradients are tangent to the sphere at q: <q, dL/dq> = 0
    for gr, keys in ((gr4, ("quat_l", "quat_r")), (gr3, ("quat",))):
        for k in keys:
            g = gr[k].cpu().numpy().astype(np.float64)
            q = (scene.g4 if gr is gr4 else scene.g3)[k].astype(np.float64)
            dot = np.abs((g * q).sum(0))
            assert dot.max() <= 1e-5 * np.abs(g).max() * np.abs(q).max(), k


# ---------------------------------------------------------------------------
# opacities that reach the 0.99 alpha clamp
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("tile,chunk", [(16, 64), (8, 64), (32, 256)])
def test_clamped_alpha_forward_and_backward(h4d, tile, chunk):
    """Half of the 3D Gaussians (and of the 4D ones) get opacity logits of 5-7
    (opacity 0.993-0.999), so that pairs near their centres take the 0.99
    alpha clamp (Sec. 4.3, the 3DGS-lineage blending constants) and carry no
    gradient through it, while pairs further out and the other Gaussians
    blend unclamped; the adjoint runs its clamp test only for splats whose
    opacity can reach the clamp.  Image and every gradient against the oracle
    (upstream zeroed at flagged pixels)."""
    print(f"[clamped alpha] tile {tile} chunk {chunk}", flush=True)
    scene = sg.tiny_scene(seed=7)
    rng = np.random.default_rng(77)
    g3, g4 = dict(scene.g3), dict(scene.g4)
    for d in (g3, g4):
        op = d["opacity"].astype(np.float64).copy()
        hi = rng.random(op.shape[0]) < 0.5
        op[hi] = rng.uniform(5.0, 7.0, size=int(hi.sum()))
        d["opacity"] = op.astype(np.float32)
    scene = sg.Scene(g3, g4, list(scene.views), name=scene.name + "_opaque", time_period=scene.time_period)
    v = scene.views[0]
    # pairs whose alpha the clamp cuts (pixel centres next to a splat centre,
    # from the oracle's projection, occlusion aside)
    P = oracle.project(scene, v)
    n_clamped = 0
    for g in np.nonzero((P["visible"] > 0) & (P["culled"] == 0) & (P["op"] > 0.99))[0]:
        i, j = np.meshgrid(np.arange(-2, 3) + np.floor(P["u"][g]), np.arange(-2, 3) + np.floor(P["v"][g]))
        dx, dy = i + 0.5 - P["u"][g], j + 0.5 - P["v"][g]
        pw = -0.5 * (P["q00"][g] * dx * dx + 2 * P["q01"][g] * dx * dy + P["q11"][g] * dy * dy)
        n_clamped += int((P["op"][g] * np.exp(pw) > 0.99).sum())
    assert n_clamped > 50, n_clamped
    ref = oracle.render(scene, v)
    _, _, _, h = _render(h4d, scene, [v], tile=tile, chunk=chunk)
    _check_image(h.images[0].cpu().numpy(), ref["img"], ref["amb"])
    dl = [mask_flagged(sg.upstream_grads([v], seed=50)[0], ref["amb"])]
    gr3, gr4 = _grads_gpu(h4d, scene, [v], dl, tile=tile, chunk=chunk)
    r3, r4 = oracle.render_bwd(scene, [v], dl)
    _check_grads(scene, gr3, gr4, r3, r4, np.zeros(scene.n3 + scene.n4, bool))
