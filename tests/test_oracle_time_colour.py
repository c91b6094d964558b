"""Pins of the oracle's time-varying colour for 4D Gaussians (the cosine
terms of 4D Gaussian splatting's colour model, which the paper inherits
through its 4D Gaussians, end of Sec. 3.2), no GPU:

* closed form: a 4D Gaussian with only DC coefficients, c_0 + sum_n c_n
  cos(2 pi n (t - mu_t) / T), shows 0.5 + Y_00 times that (clamped at 0) at any
  time, degree 1 and 2, two periods;
* zero time coefficients reproduce the plain render bit for bit;
* the hand-written adjoint of the time coefficients and of mu_t through them
  equals forward-mode AD (dual numbers) in the dot-product test, and central
  differences.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg

Y00 = 0.5 / math.sqrt(math.pi)


@pytest.mark.parametrize("degree,period", [(1, 1.0), (2, 1.0), (2, 0.7)])
def test_dc_colour_closed_form(degree, period):
    scene = sg.tiny_scene(n3=0, n4=40, width=64, height=48, seed=31)
    rng = np.random.default_rng(degree)
    g4 = dict(scene.g4)
    g4["sh"] = np.zeros_like(g4["sh"])
    c0 = rng.normal(0, 0.4, size=(3, scene.n4))
    g4["sh"][0:3] = c0
    sht = np.zeros((48 * degree, scene.n4), np.float32)
    cn = [rng.normal(0, 0.4, size=(3, scene.n4)).astype(np.float32) for _ in range(degree)]
    for n in range(degree):
        sht[48 * n:48 * n + 3] = cn[n]
    g4["sh_t"] = sht
    sc = sg.Scene(scene.g3, g4, scene.views, time_period=period)
    for t in (0.1, 0.45, 0.8):
        pr = oracle.project(sc, scene.views[0].with_time(t))
        vis = pr["visible"] > 0
        assert vis.sum() > 5
        dt = float(np.float32(t)) - g4["mean_t"].astype(np.float64)  # view times are float32
        coef = c0.astype(np.float32).astype(np.float64)
        for n in range(degree):
            coef = coef + np.cos(2 * math.pi * (n + 1) * dt / period) * cn[n].astype(np.float64)
        want = np.maximum(0.0, 0.5 + Y00 * coef)
        got = np.stack([pr["r"], pr["g"], pr["b"]])
        assert np.abs(got - want)[:, vis].max() <= 1e-12


def test_zero_time_coefficients_render_like_plain_sh():
    scene = sg.tiny_scene(seed=32, width=80, height=60)
    v = scene.views[0].with_time(0.3)
    plain = oracle.render(scene, v)
    z = sg.with_time_colour(scene, degree=2, sigma=0.0)
    with_t = oracle.render(z, v)
    assert np.array_equal(plain["img"], with_t["img"]) and np.array_equal(plain["nblend"], with_t["nblend"])


@pytest.fixture(scope="module")
def timed():
    s = sg.tiny_scene(n3=200, n4=400, width=64, height=48, seed=33)
    return sg.with_time_colour(s, degree=2, sigma=0.3, period=0.8)


@pytest.mark.parametrize("key", ["sh_t", "mean_t", "sh"])
def test_time_colour_vjp_equals_dual_jvp(timed, key):
    v = timed.views[0].with_time(0.37)
    rng = np.random.default_rng(len(key))
    ubar = rng.normal(size=(3, v.height, v.width)).astype(np.float32)
    t3, t4 = sg.param_tangents(timed, seed=12)
    keep4 = {key: t4[key]}
    _, dimg = oracle.render_jvp(timed, {}, keep4, v)
    g3, g4 = oracle.render_bwd(timed, [v], [ubar])
    lhs = float((ubar.astype(np.float64) * dimg).sum())
    rhs = float((g4[key] * keep4[key]).sum())
    assert abs(lhs) > 1e-6
    assert abs(lhs - rhs) <= 1e-9 * max(1.0, abs(lhs)), (lhs, rhs)


def test_time_colour_gradients_match_central_differences(timed):
    v = timed.views[0].with_time(0.61)
    ubar = np.random.default_rng(6).normal(size=(3, v.height, v.width))
    _, g4 = oracle.render_bwd(timed, [v], [ubar.astype(np.float32)])
    pr = oracle.project(timed, v)
    vis = np.where(pr["visible"][:timed.n4] > 0)[0]
    rng = np.random.default_rng(7)
    checked = 0
    for i in rng.choice(vis, 6, replace=False):
        for key, idx in (("sh_t", (int(rng.integers(0, 96)), i)), ("sh_t", (int(rng.integers(0, 3)), i))):
            vals = []
            for h in (1e-3, -1e-3):
                g4p = {k: a.copy() for k, a in timed.g4.items()}
                a = g4p[key].astype(np.float64)
                a[idx] += h
                g4p[key] = a.astype(np.float32)
                step = float(g4p[key][idx]) - float(timed.g4[key][idx])
                sc = sg.Scene(timed.g3, g4p, timed.views, time_period=timed.time_period)
                vals.append((float((oracle.render(sc, v)["img"] * ubar).sum()), step))
            fd = (vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1])
            # the colour is linear in the time coefficients: differences are exact up to rounding
            # (unless the clamp at 0 switches, which the tolerance would expose)
            assert abs(fd - g4[key][idx]) <= 1e-6 * max(1.0, abs(fd)), (key, idx, fd, g4[key][idx])
            checked += 1
    assert checked == 12
