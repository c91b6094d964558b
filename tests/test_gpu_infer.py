"""The inference render (render_infer): against the oracle, and the training
forward's images bit for bit, with or without batching, at the small views and
at the training-step workload (whose whole image is compared with the oracle in
the full-size tests), and no backward from its handle."""
import pytest

import oracle
import scenegen as sg
from parity_util import check_image

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h4d():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_13215_amd as m
    m._lib.load()
    return m


@pytest.mark.parametrize("batched", [False, True])
def test_infer_images_equal_forward(h4d, batched):
    print(f"[infer] small views, batched={batched}", flush=True)
    scene = sg.tiny_scene(seed=41)
    views = [sg.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 128, 96, t=0.3, bg=(0.1, 0.2, 0.3)),
             sg.look_at((1.0, 0.5, -2.8), (0.0, 0.0, 0.0), 77, 45, t=0.6),
             sg.look_at((-0.8, -0.3, -3.2), (0.1, 0.0, 0.0), 200, 150, t=0.9)]
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    rast = h4d.Rasterizer(batched=batched)
    ref = [im.clone() for im in rast.forward(g3, g4, views).images]
    h = rast.infer(g3, g4, views)
    for a, b in zip(ref, h.images):
        assert torch.equal(a, b)
    for v, img in zip(views, h.images):
        o = oracle.render(scene, v)
        check_image(img.cpu().numpy(), o["img"], o["amb"])
    with pytest.raises(RuntimeError):
        rast.backward(h, g3, g4, [torch.zeros_like(im) for im in h.images])


def test_infer_training_step_workload(h4d):
    print("[infer] 250k Gaussians, 1352x1014", flush=True)
    scene = sg.multiview_scene()
    views = [s[0] for s in sg.view_schedule(scene, 2, 1, seed=4)]
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    rast = h4d.Rasterizer()
    for v in views:
        ref = rast.forward(g3, g4, [v]).images[0].clone()
        got = rast.infer(g3, g4, [v]).images[0]
        assert torch.equal(ref, got)
