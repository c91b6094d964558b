"""Shared static binning: a batched call whose views repeat a camera at several
times projects, sorts and bins the 3D Gaussians once per camera (they do not
depend on t, Sec. 3.2 / Sec. 4), and each view's tiles merge that list with the
view's own 4D list by depth.  Against the views rendered one after another
(every view binning both sets together) and the oracle:

* images bit-identical to the views one after another, and within the image
  bar of the oracle;
* every tile list, as the blending kernels walk it, identical to the
  one-view list (which the tile-list tests pin to the oracle);
* gradients and per-Gaussian statistics equal to the one-view ones up to the
  order of floating-point atomic additions, and within the gradient bar of
  the oracle;
* the counting mode's workload counts (list entries, traversed entries,
  on-screen pairs, blends) equal;
* groups that are not contiguous in the view order, a camera that is not
  repeated, all-3D and all-4D sets, 8/16/32-pixel tiles, captured replays.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg
from parity_util import check_grads, check_image, mask_flagged

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
    """Two cameras at three times each and one camera alone, interleaved."""
    a = sg.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 128, 96, t=0.2, bg=(0.1, 0.2, 0.3))
    b = sg.look_at((1.0, 0.5, -2.8), (0.0, 0.0, 0.0), 77, 45, t=0.2)
    c = sg.look_at((-0.8, -0.3, -3.2), (0.1, 0.0, 0.0), 200, 150, fov_x_deg=50.0, t=0.4, bg=(0.5, 0.5, 0.5))
    return [a, b, a.with_time(0.5), c, b.with_time(0.55), a.with_time(0.8), b.with_time(0.9)]


def _pair(h4d, scene, views, tile=16, chunk=64):
    """(one after another, batched) renders of the same inputs."""
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    out = []
    for batched in (False, True):
        rast = h4d.Rasterizer(tile=tile, chunk=chunk, pair_capacity=1 << 20, batched=batched)
        h = rast.forward(g3, g4, views)
        torch.cuda.synchronize()
        out.append((rast, h))
    return g3, g4, out


def _same_lists(ra, ha, rb, hb):
    ia, ga = ra.tile_lists(ha)
    ib, gb = rb.tile_lists(hb)
    torch.cuda.synchronize()
    ia, ga, ib, gb = ia.cpu().numpy(), ga.cpu().numpy(), ib.cpu().numpy(), gb.cpu().numpy()
    assert ga.shape == gb.shape
    la, lb = ga[:, 1] - ga[:, 0], gb[:, 1] - gb[:, 0]
    assert np.array_equal(la, lb)
    assert la.sum() > 1000
    for t in np.nonzero(la)[0]:
        assert np.array_equal(ia[ga[t, 0]:ga[t, 1]], ib[gb[t, 0]:gb[t, 1]]), t


@pytest.mark.parametrize("tile,chunk", [(16, 64), (8, 128), (32, 256)])
def test_shared_static_images_and_lists_equal_one_view_at_a_time(h4d, tile, chunk):
    print(f"[shared static] tile {tile} chunk {chunk}", flush=True)
    scene = sg.tiny_scene(n3=1500, n4=1000, seed=71)
    views = _views()
    _, _, ((r1, h1), (r2, h2)) = _pair(h4d, scene, views, tile, chunk)
    for a, b in zip(h1.images, h2.images):
        assert torch.equal(a, b)
    _same_lists(r1, h1, r2, h2)


def test_shared_static_images_match_the_oracle(h4d):
    scene = sg.tiny_scene(n3=1500, n4=1000, seed=72)
    views = _views()
    _, _, (_, (_, h)) = _pair(h4d, scene, views)
    for v, img in zip(views, h.images):
        ref = oracle.render(scene, v)
        check_image(img.cpu().numpy(), ref["img"], ref["amb"])


@pytest.mark.parametrize("n3,n4", [(2000, 0), (0, 2000), (1, 1500)])
def test_shared_static_edge_sets(h4d, n3, n4):
    """All-3D (nothing per view but the shared lists), all-4D (nothing to
    share: the plain batched path) and a single 3D Gaussian."""
    print(f"[shared static] n3={n3} n4={n4}", flush=True)
    scene = sg.tiny_scene(n3=n3, n4=n4, seed=73)
    views = _views()
    _, _, ((r1, h1), (r2, h2)) = _pair(h4d, scene, views)
    for a, b in zip(h1.images, h2.images):
        assert torch.equal(a, b)
    if n3 + n4 > 100:
        _same_lists(r1, h1, r2, h2)


def test_shared_static_gradients_and_statistics(h4d):
    scene = sg.tiny_scene(n3=1500, n4=1000, seed=74)
    views = _views()
    dls = []
    for k, v in enumerate(views):
        amb = oracle.render(scene, v)["amb"]
        dls.append(mask_flagged(sg.upstream_grads([v], seed=80 + k)[0], amb))
    g3, g4, runs = _pair(h4d, scene, views)
    td = [torch.as_tensor(d, device="cuda") for d in dls]
    got = []
    for rast, h in runs:
        st = h4d.new_stats(scene.n3, scene.n4)
        gr3, gr4 = rast.backward(h, g3, g4, td, stats=st)
        torch.cuda.synchronize()
        got.append((gr3, gr4, st))
    (a3, a4, sa), (b3, b4, sb) = got
    for a, b in [(a3[k], b3[k]) for k in a3] + [(a4[k], b4[k]) for k in a4]:
        scale = float(a.abs().max()) + 1e-30
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-6 * scale)
    for s_a, s_b in zip(sa, sb):
        assert torch.equal(s_a["visible"], s_b["visible"]) and torch.equal(s_a["step_visible"], s_b["step_visible"])
        scale = float(s_a["grad_norm"].abs().max()) + 1e-30
        assert torch.allclose(s_a["grad_norm"], s_b["grad_norm"], rtol=1e-5, atol=1e-6 * scale)
    r3, r4 = oracle.render_bwd(scene, views, dls)
    check_grads(scene, b3, b4, r3, r4, np.zeros(scene.n3 + scene.n4, bool))


def test_shared_static_counts_equal(h4d):
    """The counting mode sees the same work either way: every view's lists,
    traversals, blends and on-screen pairs (a shared 3D record counts once per
    view)."""
    scene = sg.tiny_scene(n3=1500, n4=1000, seed=75)
    views = _views()
    dls = [torch.as_tensor(d, device="cuda") for d in sg.upstream_grads(views, seed=9)]
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    counts = []
    for batched in (False, True):
        rast = h4d.Rasterizer(pair_capacity=1 << 20, batched=batched)
        rast.forward(g3, g4, views)  # sizes the workspace
        rast.stats(True)
        h = rast.forward(g3, g4, views)
        rast.backward(h, g3, g4, dls)
        counts.append(rast.stats_read())
        rast.stats(False)
    assert counts[0] == counts[1], counts
    assert counts[0]["traversed"] > 0 and counts[0]["onscreen"] > 0


def test_shared_static_captured_replays(h4d):
    scene = sg.tiny_scene(n3=1500, n4=1000, seed=76)
    views = _views()
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    targets = [torch.as_tensor(t, device="cuda") for t in sg.target_images(views, seed=4)]
    ref = h4d.Rasterizer(batched=False)
    h = ref.forward(g3, g4, views)
    dls = [torch.empty_like(t) for t in targets]
    h4d.l1_loss_grad(ref, h.images, targets, views, dls, None)
    ref3, ref4 = ref.backward(h, g3, g4, dls)
    torch.cuda.synchronize()
    ref_imgs = [im.clone() for im in h.images]
    gr3 = {k: torch.empty_like(v) for k, v in g3.items()}
    gr4 = {k: torch.empty_like(v) for k, v in g4.items()}
    step = h4d.CapturedStep(h4d.Rasterizer(batched=True), g3, g4, views, targets, (gr3, gr4))
    for rep in range(3):
        step.replay()
        step.verify()
        for a, b in zip(step.images, ref_imgs):
            assert torch.equal(a, b), rep
        for a, b in [(gr3[k], ref3[k]) for k in gr3] + [(gr4[k], ref4[k]) for k in gr4]:
            scale = float(b.abs().max()) + 1e-30
            assert torch.allclose(a, b, rtol=1e-5, atol=1e-6 * scale), rep
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()


@pytest.mark.parametrize("batched", [False, True])
def test_repeated_backward_gives_the_same_gradients(h4d, batched):
    """The forward zeroes the gradient records its pairs use and the backward
    accumulates into them: a second backward on the same forward (with and
    without statistics) clears them first and gives the same gradients, and
    the shared static binning's summed 3D records (no statistics) stay within
    the oracle's bar."""
    print(f"[repeated backward] batched={batched}", flush=True)
    scene = sg.tiny_scene(n3=1500, n4=1000, seed=77)
    views = _views()
    dls = []
    for k, v in enumerate(views):
        amb = oracle.render(scene, v)["amb"]
        dls.append(mask_flagged(sg.upstream_grads([v], seed=90 + k)[0], amb))
    td = [torch.as_tensor(d, device="cuda") for d in dls]
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    rast = h4d.Rasterizer(batched=batched)
    h = rast.forward(g3, g4, views)
    runs = [rast.backward(h, g3, g4, td), rast.backward(h, g3, g4, td, stats=h4d.new_stats(scene.n3, scene.n4)),
            rast.backward(h, g3, g4, td)]
    torch.cuda.synchronize()
    a3, a4 = runs[0]
    for b3, b4 in runs[1:]:
        for a, b in [(a3[k], b3[k]) for k in a3] + [(a4[k], b4[k]) for k in a4]:
            scale = float(a.abs().max()) + 1e-30
            assert torch.allclose(a, b, rtol=1e-5, atol=1e-6 * scale)
    r3, r4 = oracle.render_bwd(scene, views, dls)
    check_grads(scene, a3, a4, r3, r4, np.zeros(scene.n3 + scene.n4, bool))
