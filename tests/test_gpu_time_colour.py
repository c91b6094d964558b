"""Time-varying colour of 4D Gaussians (degree 1 and 2 cosine terms of the
4D spherindrical harmonics) through the C ABI against the oracle: images at
several times, every gradient (including the time coefficients and mean_t's
share through them), and the static conversion and densification carrying
the time coefficients of the 4D rows they keep or copy."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from oracle import densify as od
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


@pytest.mark.parametrize("degree,period", [(1, 1.0), (2, 0.8)])
def test_time_colour_forward_and_backward(h4d, degree, period):
    print(f"[time colour] degree {degree}, period {period}", flush=True)
    scene = sg.with_time_colour(sg.tiny_scene(seed=91), degree=degree, period=period, seed=92)
    rast = h4d.Rasterizer(time_period=period)
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    for t in (0.15, 0.6):
        v = scene.views[0].with_time(t)
        ref = oracle.render(scene, v)
        img = rast.forward(g3, g4, [v]).images[0].cpu().numpy()
        check_image(img, ref["img"], ref["amb"])
        dl = mask_flagged(sg.upstream_grads([v], seed=93)[0], ref["amb"])
        h = rast.forward(g3, g4, [v])
        gr3, gr4 = rast.backward(h, g3, g4, [torch.as_tensor(dl, device="cuda")])
        torch.cuda.synchronize()
        r3, r4 = oracle.render_bwd(scene, [v], [dl])
        check_grads(scene, gr3, gr4, r3, r4, np.zeros(scene.n3 + scene.n4, bool))
        g = gr4["sh_t"].cpu().numpy().astype(np.float64)
        r = r4["sh_t"]
        assert np.linalg.norm(r) > 0
        assert np.linalg.norm(g - r) <= 1e-3 * np.linalg.norm(r)
        rms = np.sqrt(np.mean(r * r))
        assert np.all(np.abs(g - r) <= 1e-3 * np.abs(r) + 1e-3 * rms)


def test_conversion_and_densification_carry_time_coefficients(h4d):
    rng = np.random.default_rng(94)
    g4 = sg.draw_4d(rng, 3000, 2.0, static_fraction=0.4, tau=0.5)
    g3 = sg.draw_3d(rng, 500, 2.0)
    g4["sh_t"] = rng.normal(0, 0.3, size=(96, 3000)).astype(np.float32)
    scene = sg.Scene(g3, g4)
    rast = h4d.Rasterizer()
    o3, o4, perm = h4d.convert_static(rast, h4d.to_device(g3), h4d.to_device(g4), 0.5)
    rperm, rn4, rn3, _ = oracle.convert_static(scene, 0.5)
    assert np.array_equal(perm.cpu().numpy(), rperm)
    keep = np.nonzero(rperm >= 0)[0]
    assert np.array_equal(o4["sh_t"].cpu().numpy(), g4["sh_t"][:, keep])
    assert "sh_t" not in o3
    # densification copies them to clones and children
    vis = rng.integers(0, 3, 3000).astype(np.float32)
    grad = (rng.exponential(2e-4, 3000) * vis).astype(np.float32)
    noise3 = np.zeros((2, 3, 500), np.float32)
    noise4 = rng.normal(size=(2, 4, 3000)).astype(np.float32)
    p = h4d._lib.DensifyParams(2e-4, 2, -2.9, math.log(0.005 / 0.995), float("inf"), math.log(1.6))
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    zeros3 = {"grad_norm": dev(np.zeros(500, np.float32)), "visible": dev(np.zeros(500, np.float32))}
    _, d4, _, src4 = h4d.densify(rast, h4d.to_device(g3), h4d.to_device(g4), zeros3,
                                 {"grad_norm": dev(grad), "visible": dev(vis)}, dev(noise3), dev(noise4), p, p)
    want, wsrc, info = od.densify_set(g4, True, grad, vis, noise4, thr=p.grad_threshold, log_dense=-2.9,
                                      logit_min=math.log(0.005 / 0.995), log_max_scale=float("inf"), split_n=2,
                                      log_shrink=math.log(1.6))
    assert info["clone"] > 0 and info["split"] > 0
    assert np.array_equal(src4.cpu().numpy(), wsrc)
    assert np.array_equal(d4["sh_t"].cpu().numpy(), want["sh_t"])
