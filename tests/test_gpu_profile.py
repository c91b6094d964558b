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
