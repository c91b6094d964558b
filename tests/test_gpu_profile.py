"""Event timing levels of the library (h4dgs_profile): level 1 brackets every
stage with events, level 2 times only the blending kernels from their own
dispatch; neither changes the rendered image."""
import pytest

import scenegen as sg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h4d():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_13215_amd as m
    m._lib.load()
    return m


def _step(h4d, rast, g3, g4, views):
    h = rast.forward(g3, g4, views)
    dls = [torch.ones_like(im) for im in h.images]
    rast.backward(h, g3, g4, dls)
    torch.cuda.synchronize()
    return [im.clone() for im in h.images]


@pytest.mark.parametrize("batched", [False, True])
def test_profile_levels_report_the_right_stages(h4d, batched):
    print(f"[profile levels] batched={batched}", flush=True)
    scene = sg.multiview_scene(n_total=4000, width=160, height=120, seed=4)
    views = scene.views[:3]
    rast = h4d.Rasterizer(tile=16, chunk=64, pair_capacity=1 << 20, batched=batched)
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    ref = _step(h4d, rast, g3, g4, views)
    n_blend = 1 if batched else len(views)

    rast.profile(2)
    got2 = _step(h4d, rast, g3, g4, views)
    p2 = rast.profile_read()
    rast.profile(4)
    _step(h4d, rast, g3, g4, views)
    p4 = rast.profile_read()
    rast.profile(1)
    got1 = _step(h4d, rast, g3, g4, views)
    p1 = rast.profile_read()
    rast.profile(0)
    _step(h4d, rast, g3, g4, views)
    p0 = rast.profile_read()

    for a, b, c in zip(ref, got2, got1):
        assert torch.equal(a, b) and torch.equal(a, c)
    for k, (ms, n) in p2.items():
        if k in ("blend_fwd", "blend_bwd"):
            assert n == n_blend and ms > 0.0, (k, ms, n)
        else:
            assert n == 0 and ms == 0.0, (k, ms, n)
    for k, (ms, n) in p4.items():
        if k == "blend_bwd":
            assert n == n_blend and ms > 0.0, (k, ms, n)
        else:
            assert n == 0 and ms == 0.0, (k, ms, n)
    for k in ("preprocess", "depth_sort", "binning", "blend_fwd", "blend_bwd", "preprocess_bwd"):
        assert p1[k][1] >= 1 and p1[k][0] > 0.0, (k, p1[k])
    assert all(n == 0 for _, n in p0.values())


def test_counting_mode_counts_match_the_oracle(h4d):
    """The counting variants' workload counts against the oracle's definition
    on a scene with no guard-band pixel (every blend decision agrees): blends
    (the sum of per-pixel blend counts, equal in the adjoint), on-screen
    records (visible Gaussians whose pixel square meets the image), tile-list
    entries (without culling: every (Gaussian, tile) pair whose square meets
    the tile) and traversed entries (per tile, the list position of the last
    splat any of its pixels blends)."""
    import numpy as np
    import oracle
    scene = sg.tiny_scene(seed=18, width=150, height=100)
    v = scene.views[0]
    ref = oracle.render(scene, v)
    assert not ref["amb"].any()
    tile = 16
    rast = h4d.Rasterizer(tile=tile, chunk=64, pair_capacity=1 << 20, cull=False)
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    rast.stats(True)
    h = rast.forward(g3, g4, [v])
    rast.backward(h, g3, g4, [torch.ones_like(h.images[0])])
    c = rast.stats_read()
    rast.stats(False)
    pr = oracle.project(scene, v)
    on = (pr["visible"] > 0) & (pr["x0"] <= pr["x1"]) & (pr["y0"] <= pr["y1"])
    assert c["onscreen"] == int(on.sum())
    assert c["fwd_blend"] == int(ref["nblend"].sum()) == c["bwd_blend"]
    tiles_x, tiles_y = (v.width + tile - 1) // tile, (v.height + tile - 1) // tile
    lists = [[] for _ in range(tiles_x * tiles_y)]
    order = np.lexsort((np.arange(on.size), pr["key"]))  # by depth key, then id
    for g in order[on[order]]:
        for ty in range(int(pr["y0"][g]) // tile, int(pr["y1"][g]) // tile + 1):
            for tx in range(int(pr["x0"][g]) // tile, int(pr["x1"][g]) // tile + 1):
                lists[ty * tiles_x + tx].append(int(g))
    assert c["list_entries"] == sum(len(lst) for lst in lists)
    ys, xs = np.mgrid[0:v.height, 0:v.width]
    xs, ys = xs.ravel().astype(np.int32), ys.ravel().astype(np.int32)
    last = np.zeros(len(lists), np.int64)
    pos = [{g: i for i, g in enumerate(lst)} for lst in lists]
    for x, y, bl in zip(xs, ys, oracle.blended_at(scene, v, xs, ys, cap=1024)):
        if bl:
            t = (y // tile) * tiles_x + x // tile
            last[t] = max(last[t], pos[t][bl[-1][0]] + 1)
    assert c["traversed"] == int(last.sum())
