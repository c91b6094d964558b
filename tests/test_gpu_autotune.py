"""The autotuner on the GPU: every candidate launch configuration runs the
training step, the pick is one of them, and the images under the pick are
bit-identical to those under the default configuration."""
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


@pytest.mark.parametrize("batched", [False, True])
def test_autotuner_pick_is_accuracy_neutral(h4d, batched):
    print(f"[autotune] batched={batched}", flush=True)
    scene = sg.tiny_scene(seed=21)
    views = [sg.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 128, 96, t=0.3),
             sg.look_at((1.0, 0.5, -2.8), (0.0, 0.0, 0.0), 77, 45, t=0.6),
             sg.look_at((-0.8, -0.3, -3.2), (0.1, 0.0, 0.0), 200, 150, t=0.9)]
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    tuner = h4d.Autotuner(steps=2, warmup=1)
    pick = tuner.pick(g3, g4, views, batched)
    assert pick in h4d.CANDIDATES
    assert set(tuner.last_timings) == set(h4d.CANDIDATES)
    assert all(ms > 0.0 for ms in tuner.last_timings.values())
    assert tuner.pick(g3, g4, views, batched) == pick  # cached
    ref = h4d.Rasterizer(batched=batched).forward(g3, g4, views).images
    ref = [im.clone() for im in ref]
    got = h4d.Rasterizer(tile=pick[0], chunk=pick[1], batched=batched).forward(g3, g4, views).images
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
