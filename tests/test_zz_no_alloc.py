"""The allocation-free inference render (h4dgs_render_infer_noalloc) against
render_infer, through the C ABI: two calls in a row on the library's fixed
workspace, the second with a smaller input (fewer Gaussians, other view
sizes), each bit-identical to render_infer with caller-owned buffers (same
kernels, same launch configuration); the status words it writes; a pair
overflow reported through them; and a call too large for the fixed workspace
refused on the host before anything is enqueued."""
import numpy as np
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


def _compare(h4d, scene, views, batched):
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    rast = h4d.Rasterizer(batched=batched)
    ref = [im.clone() for im in rast.infer(g3, g4, views).images]
    pairs = rast.last_pairs
    # fill the outputs with NaN first: every pixel must be written
    out = [torch.full_like(im, float("nan")) for im in ref]
    imgs, status = h4d.render_infer_noalloc(rast, g3, g4, views, images=out)
    torch.cuda.synchronize()
    for a, b in zip(ref, imgs):
        assert torch.equal(a, b)
    st = status.cpu().numpy()
    assert st[0] == 0 and st[1] == pairs
    return rast


@pytest.mark.parametrize("batched", [False, True])
def test_noalloc_two_calls_match_render_infer(h4d, batched):
    print(f"[noalloc] two calls, batched={batched}", flush=True)
    big = sg.tiny_scene(seed=51)
    views = [sg.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 200, 150, t=0.3, bg=(0.1, 0.2, 0.3)),
             sg.look_at((1.0, 0.5, -2.8), (0.0, 0.0, 0.0), 128, 96, t=0.6)]
    _compare(h4d, big, views, batched)
    small = sg.tiny_scene(n3=300, n4=200, seed=52)
    _compare(h4d, small, [sg.look_at((-0.8, -0.3, -3.2), (0.1, 0.0, 0.0), 77, 45, t=0.9)], batched)


def test_noalloc_reports_pair_overflow(h4d):
    print("[noalloc] pair overflow", flush=True)
    scene = sg.tiny_scene(seed=53)
    v = scene.views[0]
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    rast = h4d.Rasterizer()
    rast.infer(g3, g4, [v])
    need = rast.last_pairs
    small = h4d.Rasterizer(pair_capacity=64)
    _, status = h4d.render_infer_noalloc(small, g3, g4, [v])
    st = status.cpu().numpy()
    assert st[0] & 1 and st[1] == need
    # the next call with room clears the flag
    _, status = h4d.render_infer_noalloc(rast, g3, g4, [v])
    st = status.cpu().numpy()
    assert st[0] == 0 and st[1] == need


def test_noalloc_rejects_calls_beyond_its_workspace(h4d):
    scene = sg.tiny_scene(n3=10, n4=10, seed=54)
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    v = sg.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 64, 48)
    # 8 bytes of state per coarse entry, one entry per 16 pair slots
    rast = h4d.Rasterizer(pair_capacity=2 * h4d._lib.NOALLOC_BYTES + 4096)
    st, sc = rast.sizes(10, 10, h4d._lib.view_array([v]), 1)
    assert st > h4d._lib.NOALLOC_BYTES
    with pytest.raises(h4d.H4DError) as e:
        h4d.render_infer_noalloc(rast, g3, g4, [v])
    assert e.value.code == h4d._lib.H4D_ERR_CAPACITY
    assert "fixed workspace" in str(e.value)
