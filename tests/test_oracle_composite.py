"""Pins of the oracle's binning, ordering and front-to-back blending (Alg. 1,
Eq. 3) against brute force and invariants (no GPU)."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg


def test_tile_path_equals_per_pixel_brute_force(tiny):
    v = tiny.views[0]
    out = oracle.render(tiny, v)
    rng = np.random.default_rng(0)
    px = rng.integers(0, v.width, 400)
    py = rng.integers(0, v.height, 400)
    rgb, T, _ = oracle.pixels(tiny, v, px, py)
    # same candidates in the same (depth key, id) order: bit-identical in FP64
    assert np.array_equal(rgb.T, out["img"][:, py, px])
    assert np.array_equal(T, out["T"][py, px])


@pytest.mark.parametrize("B", [8, 32])
def test_image_does_not_depend_on_tile_size(tiny, B):
    v = tiny.views[0]
    a = oracle.render(tiny, v, tile=16)
    b = oracle.render(tiny, v, tile=B)
    assert np.array_equal(a["img"], b["img"]) and np.array_equal(a["T"], b["T"])


def _white(scene):
    """Same geometry, every Gaussian coloured exactly (1, 1, 1)."""
    g3 = dict(scene.g3)
    g4 = dict(scene.g4)
    for g in (g3, g4):
        sh = np.zeros_like(g["sh"])
        sh[0:3] = np.float32(math.sqrt(math.pi))  # Y00 = 1/(2 sqrt(pi)): raw colour 0.5 + 0.5
        g["sh"] = sh
    return sg.Scene(g3, g4, scene.views)


def test_blend_weights_sum_to_one_minus_transmittance(tiny):
    v = tiny.views[0]
    out = oracle.render(_white(tiny), v)
    T = out["T"]
    # sum_k alpha_k T_k = 1 - T_final for a white scene on a black background
    assert np.allclose(out["img"], (1 - T)[None], atol=1e-13)
    assert (T <= 1).all() and (T >= 1e-4).all()


def test_background_enters_through_final_transmittance(tiny):
    v = tiny.views[0]
    a = oracle.render(tiny, v)
    vb = sg.View(v.world_to_cam, v.fx, v.fy, v.cx, v.cy, v.width, v.height, v.t, (0.25, 0.5, 1.0))
    b = oracle.render(tiny, vb)
    bg = np.array([0.25, 0.5, 1.0])[:, None, None]
    assert np.allclose(b["img"] - a["img"], a["T"][None] * bg, atol=1e-14)


def test_transmittance_never_drops_below_stop_threshold():
    # an opaque stack: the stop rule must leave T >= 1e-4 and keep the offender out
    n = 40
    g3 = dict(mean=np.zeros((3, n), np.float32) + np.array([[0.0], [0.0], [0.0]], np.float32),
              log_scale=np.full((3, n), math.log(0.3), np.float32),
              quat=np.tile(np.array([[1.0], [0], [0], [0]], np.float32), (1, n)),
              opacity=np.full(n, 6.0, np.float32), sh=np.zeros((48, n), np.float32))
    g3["mean"][2] = np.linspace(-0.5, 0.5, n, dtype=np.float32)
    v = sg.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 32, 24)
    out = oracle.render(sg.Scene(g3, sg.empty_4d(), [v]), v)
    T = out["T"]
    assert T.min() >= 1e-4
    # near the centre every Gaussian has alpha ~0.98: two are blended and the
    # third, which would take T below 1e-4, is refused
    assert out["nblend"][12, 16] == 2 and 1e-4 <= T[12, 16] < 1e-3


def test_guard_band_is_small(tiny):
    out = oracle.render(tiny, tiny.views[0])
    assert out["amb"].mean() < 1e-3


def _brute_lists(rec, W, H, B):
    tx, ty = -(-W // B), -(-H // B)
    lists = [[] for _ in range(tx * ty)]
    order = sorted(range(len(rec["u"])), key=lambda g: (float(rec["depth"][g]), g))
    for g in order:
        if not rec["visible"][g]:
            continue
        u, v, r = float(rec["u"][g]), float(rec["v"][g]), int(rec["radius"][g])
        # pixels i with |i + 0.5 - u| <= r
        xs = [i for i in range(W) if abs(i + 0.5 - u) <= r]
        ys = [j for j in range(H) if abs(j + 0.5 - v) <= r]
        if not xs or not ys:
            continue
        for t in range(tx * ty):
            x0, y0 = (t % tx) * B, (t // tx) * B
            if any(x0 <= i < x0 + B for i in xs) and any(y0 <= j < y0 + B for j in ys):
                lists[t].append(g)
    return lists


@pytest.mark.parametrize("B", [8, 16, 32])
def test_tile_lists_match_brute_force(B):
    W, H = 77, 45
    rec = sg.synthetic_records(300, W, H, seed=11, max_radius=25)
    start, ids = oracle.tile_lists(rec, W, H, B)
    lists = _brute_lists(rec, W, H, B)
    assert start[-1] == sum(len(l) for l in lists)
    for t, l in enumerate(lists):
        assert list(ids[start[t]:start[t + 1]]) == l


def test_composite_records_matches_python_loop():
    W, H = 40, 30
    rec = sg.synthetic_records(150, W, H, seed=3, max_radius=15)
    img, T, _ = oracle.composite_records(rec, W, H, tile=8, bg=(0.1, 0.2, 0.3))
    order = sorted(range(150), key=lambda g: (float(rec["depth"][g]), g))
    rng = np.random.default_rng(1)
    for _ in range(60):
        i, j = int(rng.integers(0, W)), int(rng.integers(0, H))
        x, y = i + 0.5, j + 0.5
        C = np.zeros(3)
        Tt = 1.0
        for g in order:
            if not rec["visible"][g]:
                continue
            u, v, r = float(rec["u"][g]), float(rec["v"][g]), int(rec["radius"][g])
            if abs(x - u) > r or abs(y - v) > r:
                continue
            a, b, c = (float(rec["conic"][k, g]) for k in range(3))
            dx, dy = x - u, y - v
            pw = -0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy)
            if pw > 0:
                continue
            al = min(0.99, float(rec["opacity"][g]) * math.exp(pw))
            if al < 1 / 255:
                continue
            Tn = Tt * (1 - al)
            if Tn < 1e-4:
                break
            C += rec["rgb"][:, g].astype(np.float64) * al * Tt
            Tt = Tn
        C += Tt * np.array([0.1, 0.2, 0.3])
        assert np.allclose(img[:, j, i], C, atol=1e-12)
        assert abs(T[j, i] - Tt) < 1e-13
