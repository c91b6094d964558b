"""Batched mode (all views of a call in one launch per stage) against views
processed one after another, and graph-captured training steps, through the
C ABI.  Both modes run the same kernels over different view ranges, so the
forward must be bit-identical; gradients differ only by the order of
floating-point atomic additions."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from parity_util import check_image, check_pixels, sample_pixels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h4d():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_13215_amd as m
    m._lib.load()
    return m


def _views():
    """Three cameras of different image sizes (ragged tiles), times and backgrounds."""
    return [sg.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 128, 96, t=0.3, bg=(0.1, 0.2, 0.3)),
            sg.look_at((1.0, 0.5, -2.8), (0.0, 0.0, 0.0), 77, 45, t=0.6, bg=(0.0, 0.0, 0.0)),
            sg.look_at((-0.8, -0.3, -3.2), (0.1, 0.0, 0.0), 200, 150, fov_x_deg=50.0, t=0.9, bg=(0.5, 0.5, 0.5))]


def _render(h4d, scene, views, batched, tile=16, chunk=128, cap=1 << 20):
    rast = h4d.Rasterizer(tile=tile, chunk=chunk, pair_capacity=cap, batched=batched)
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    h = rast.forward(g3, g4, views)
    torch.cuda.synchronize()
    return rast, g3, g4, h


@pytest.mark.parametrize("tile,chunk", [(16, 128), (8, 64), (32, 256)])
def test_batched_forward_is_bit_identical_to_single_view(h4d, tile, chunk):
    print(f"[batched forward] tile {tile} chunk {chunk}", flush=True)
    scene = sg.tiny_scene(seed=12)
    views = _views()
    r1, _, _, h1 = _render(h4d, scene, views, False, tile, chunk)
    r2, _, _, h2 = _render(h4d, scene, views, True, tile, chunk)
    assert r1.last_pairs == r2.last_pairs
    for a, b in zip(h1.images, h2.images):
        assert torch.equal(a, b)


def test_batched_forward_matches_oracle(h4d):
    scene = sg.tiny_scene(seed=13)
    views = _views()
    _, _, _, h = _render(h4d, scene, views, True)
    for v, img in zip(views, h.images):
        ref = oracle.render(scene, v)
        check_image(img.cpu().numpy(), ref["img"], ref["amb"])


def test_batched_backward_matches_single_view(h4d):
    scene = sg.tiny_scene(seed=14)
    views = _views()
    dls = [torch.as_tensor(d, device="cuda") for d in sg.upstream_grads(views, seed=6)]
    out = []
    for batched in (False, True):
        rast, g3, g4, h = _render(h4d, scene, views, batched)
        gr3, gr4 = rast.backward(h, g3, g4, dls)
        torch.cuda.synchronize()
        out.append((gr3, gr4))
    (a3, a4), (b3, b4) = out
    for a, b in [(a3[k], b3[k]) for k in a3] + [(a4[k], b4[k]) for k in a4]:
        scale = float(a.abs().max()) + 1e-30
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-6 * scale)


def test_batched_capacity_overflow_is_recovered(h4d):
    scene = sg.tiny_scene(seed=15)
    views = _views()
    r1, _, _, h1 = _render(h4d, scene, views, False)
    r2, _, _, h2 = _render(h4d, scene, views, True, cap=256)
    assert r2.capacity > 256
    for a, b in zip(h1.images, h2.images):
        assert torch.equal(a, b)


@pytest.mark.parametrize("batched", [False, True])
def test_captured_step_replays_match_eager(h4d, batched):
    """A captured fwd -> L1 -> bwd replayed several times, with eager work and
    synchronisations in between, gives what the eager step gives."""
    print(f"[captured step] batched={batched}", flush=True)
    scene = sg.tiny_scene(seed=16)
    views = _views()
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    targets = [torch.as_tensor(t, device="cuda") for t in sg.target_images(views, seed=3)]
    # eager reference
    ref_rast = h4d.Rasterizer(batched=batched)
    h = ref_rast.forward(g3, g4, views)
    dls = [torch.empty_like(t) for t in targets]
    loss = torch.zeros(1, device="cuda")
    h4d.l1_loss_grad(ref_rast, h.images, targets, views, dls, loss)
    ref3, ref4 = ref_rast.backward(h, g3, g4, dls)
    torch.cuda.synchronize()
    ref_imgs = [im.clone() for im in h.images]
    ref_loss = float(loss)

    gr3 = {k: torch.empty_like(v) for k, v in g3.items()}
    gr4 = {k: torch.empty_like(v) for k, v in g4.items()}
    step = h4d.CapturedStep(h4d.Rasterizer(batched=batched), g3, g4, views, targets, (gr3, gr4))
    for rep in range(3):
        for k in gr3:
            gr3[k].fill_(float("nan"))
        step.replay()
        step.verify()
        for a, b in zip(step.images, ref_imgs):
            assert torch.equal(a, b), rep
        assert abs(float(step.loss) - ref_loss) <= 1e-6 * max(1.0, abs(ref_loss)), rep
        for a, b in [(gr3[k], ref3[k]) for k in gr3] + [(gr4[k], ref4[k]) for k in gr4]:
            scale = float(b.abs().max()) + 1e-30
            assert torch.allclose(a, b, rtol=1e-5, atol=1e-6 * scale), rep
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()  # unrelated eager work


def test_batched_multi_pass_super_tile_sort_is_bit_identical(h4d):
    """Three 1600x1200 views at 8-px tiles: 1900 super-tiles each, so the
    batched pass (5700 super-tiles) sorts its coarse entries in two radix passes
    (the first of which drops entries whose tile mask is empty) while each view
    alone needs one."""
    print("[batched forward] two-pass super-tile sort", flush=True)
    scene = sg.multiview_scene(n_total=20_000, width=1600, height=1200, seed=8)
    views = [scene.views[2].with_time(0.2), scene.views[9].with_time(0.5), scene.views[15].with_time(0.8)]
    r1, _, _, h1 = _render(h4d, scene, views, False, tile=8, chunk=64, cap=1 << 24)
    r2, _, _, h2 = _render(h4d, scene, views, True, tile=8, chunk=64, cap=1 << 24)
    assert r1.last_pairs == r2.last_pairs
    for a, b in zip(h1.images, h2.images):
        assert torch.equal(a, b)
    for v, img in zip(views, h2.images):
        ref = oracle.render(scene, v)
        check_image(img.cpu().numpy(), ref["img"], ref["amb"])


def test_two_pass_super_tile_sort_single_view_is_tile_independent(h4d):
    """One 2100x1600 view at 8-px tiles has 3300 super-tiles, more than one
    11-bit radix pass holds, so its coarse entries take two passes (the first
    dropping empty masks); at 16-px tiles the same view takes one.  Images do
    not depend on the tile size, so both must agree bit for bit."""
    print("[single view] two-pass super-tile sort", flush=True)
    scene = sg.multiview_scene(n_total=20_000, width=2100, height=1600, seed=9)
    views = [scene.views[4].with_time(0.35)]
    _, _, _, h8 = _render(h4d, scene, views, False, tile=8, chunk=64, cap=1 << 24)
    _, _, _, h16 = _render(h4d, scene, views, False, tile=16, chunk=64, cap=1 << 24)
    assert torch.equal(h8.images[0], h16.images[0])
    ref = oracle.render(scene, views[0])
    check_image(h8.images[0].cpu().numpy(), ref["img"], ref["amb"])


def test_views_whose_super_tile_sorts_differ_in_digit_width(h4d):
    """Views one after another, one 2100x1600 (3300 super-tiles at 8-px tiles:
    two 6-bit radix passes) and one 1600x1200 (1900: one 11-bit pass).  The
    sort's histogram must hold the widest digit of any view, not the digit of
    the view with the most super-tiles; each image equals that view rendered
    alone."""
    print("[views one after another] 6-bit and 11-bit super-tile sorts", flush=True)
    scene = sg.multiview_scene(n_total=20_000, width=2100, height=1600, seed=10)
    a = scene.views[3].with_time(0.4)
    k = 1600.0 / 2100.0
    b = sg.View(a.world_to_cam.copy(), a.fx * k, a.fy * k, 800.0, 600.0, 1600, 1200, 0.7, (0.2, 0.1, 0.0))
    _, _, _, hab = _render(h4d, scene, [a, b], False, tile=8, chunk=64, cap=1 << 24)
    _, _, _, ha = _render(h4d, scene, [a], False, tile=8, chunk=64, cap=1 << 24)
    _, _, _, hb = _render(h4d, scene, [b], False, tile=8, chunk=64, cap=1 << 24)
    assert torch.equal(hab.images[0], ha.images[0])
    assert torch.equal(hab.images[1], hb.images[0])


def test_batched_pass_with_many_count_workgroups(h4d):
    """Two views of 300k Gaussians in one batched pass: 600k depth-ordered
    Gaussians, more than 2048 count workgroups, so the coarse offsets take the
    separate top-level scan; each image equals that view rendered alone (whose
    300k Gaussians take the in-kernel scan)."""
    print("[batched forward] many count workgroups", flush=True)
    scene = sg.multiview_scene(n_total=300_000, width=320, height=240, seed=11)
    views = [scene.views[1].with_time(0.3), scene.views[12].with_time(0.6)]
    r1, _, _, h1 = _render(h4d, scene, views, False, tile=16, chunk=64, cap=1 << 24)
    r2, _, _, h2 = _render(h4d, scene, views, True, tile=16, chunk=64, cap=1 << 24)
    assert r1.last_pairs == r2.last_pairs
    for a, b in zip(h1.images, h2.images):
        assert torch.equal(a, b)
    for v, img in zip(views, h2.images):
        ref = oracle.render(scene, v)
        check_image(img.cpu().numpy(), ref["img"], ref["amb"])


def test_batched_full_size_matches_single_view(h4d):
    """The batched workload at full size: 1M Gaussians (80 % static), 8 cameras
    (four at 1352x1014, four at 2704x2028) x 4 times = 32 views, 109.7 Mpix,
    in one pass, the 3D Gaussians binned once per camera.  Images
    bit-identical to the views rendered one after another
    at the default tile and chunk; gradients equal up to the order of the
    floating-point atomic sums, compared normwise per parameter array (a
    reordered sum of float32 terms differs by a few units of rounding of the
    sum of their magnitudes, which single entries with cancellation can exceed
    relative to their own size)."""
    print("[batched full size] 1M Gaussians, 32 views", flush=True)
    scene = sg.batched_scene()
    views = sg.batched_views(scene)
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    dls = [torch.randn((3, v.height, v.width), generator=gen, device="cuda") * 1e-3 for v in views]
    out = []
    for batched in (False, True):
        rast = h4d.Rasterizer(batched=batched)
        h = rast.forward(g3, g4, views)
        gr3, gr4 = rast.backward(h, g3, g4, dls)
        torch.cuda.synchronize()
        out.append((rast.last_pairs, [im.clone() for im in h.images], gr3, gr4))
        del h, rast
        torch.cuda.empty_cache()
    (p1, im1, a3, a4), (p2, im2, b3, b4) = out
    # the batched call bins the 3D Gaussians once per camera (8, not 32 times)
    assert p1 > 0 and 0 < p2 < p1
    assert float(a3["opacity"].norm()) > 0 and float(a4["opacity"].norm()) > 0
    for v, (a, b) in enumerate(zip(im1, im2)):
        assert torch.equal(a, b), v
    for k in a3:
        assert float((a3[k] - b3[k]).norm()) <= 1e-5 * float(a3[k].norm()) + 1e-30, k
    for k in a4:
        assert float((a4[k] - b4[k]).norm()) <= 1e-5 * float(a4[k].norm()) + 1e-30, k
    # every one of the 32 batched views against the oracle's per-pixel brute
    # force over all 1M Gaussians: corners, ragged last tile row and column,
    # random pixels
    print("[batched full size] sampled pixels of the 32 views against the oracle", flush=True)
    for k, (v, img) in enumerate(zip(views, im2)):
        xs, ys = sample_pixels(v.width, v.height, 40, seed=100 + k)
        check_pixels(scene, v, img.cpu().numpy(), xs, ys)


def test_batched_call_beyond_one_pass_of_super_tiles(h4d):
    """Five 4096x4096 views at 8-pixel tiles: 16384 super-tiles each, 81920 in
    the call, more than the 65536 one pass's keys can number (their upper half
    carries the tile mask).  The batched call splits into passes of four views
    and one; its images must equal the views rendered one after another bit for
    bit, its gradients normwise up to the order of the atomic sums."""
    print("[batched call in two passes] 5 views 4096x4096, tile 8", flush=True)
    scene = sg.tiny_scene(seed=31)
    views = [sg.look_at((0.3 * k - 0.6, 0.1 * k, -3.0), (0.0, 0.0, 0.0), 4096, 4096, t=0.15 + 0.17 * k)
             for k in range(5)]
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(9)
    dls = [torch.randn((3, v.height, v.width), generator=gen, device="cuda") * 1e-6 for v in views]
    out = []
    for batched in (False, True):
        rast = h4d.Rasterizer(tile=8, chunk=64, batched=batched)
        h = rast.forward(g3, g4, views)
        gr3, gr4 = rast.backward(h, g3, g4, dls)
        torch.cuda.synchronize()
        out.append(([im.clone() for im in h.images], gr3, gr4))
        del h, rast
        torch.cuda.empty_cache()
    (im1, a3, a4), (im2, b3, b4) = out
    for v, (a, b) in enumerate(zip(im1, im2)):
        assert torch.equal(a, b), v
    for k, (v, img) in enumerate(zip(views, im2)):
        xs, ys = sample_pixels(v.width, v.height, 1500, seed=200 + k, tile=8)
        check_pixels(scene, v, img.cpu().numpy(), xs, ys)
    assert float(a3["opacity"].norm()) > 0 and float(a4["opacity"].norm()) > 0
    for k in a3:
        assert float((a3[k] - b3[k]).norm()) <= 1e-5 * float(a3[k].norm()) + 1e-30, k
    for k in a4:
        assert float((a4[k] - b4[k]).norm()) <= 1e-5 * float(a4[k].norm()) + 1e-30, k
