"""Pins of the oracle's hand-written adjoint: forward-mode AD (dual numbers)
dot-product test and central finite differences (no GPU)."""
import zlib

import numpy as np
import pytest

import oracle
import scenegen as sg

GROUPS3 = ("mean", "log_scale", "quat", "opacity", "sh")
GROUPS4 = ("mean", "mean_t", "log_scale", "quat_l", "quat_r", "opacity", "sh")


@pytest.fixture(scope="module")
def small():
    return sg.tiny_scene(n3=300, n4=300, width=64, height=48, seed=5)


def _dot(g, t):
    return float(sum((g[k] * t[k]).sum() for k in t))


@pytest.mark.parametrize("group", [("3", k) for k in GROUPS3] + [("4", k) for k in GROUPS4])
def test_vjp_equals_dual_jvp_per_group(small, group):
    v = small.views[0]
    rng = np.random.default_rng(zlib.crc32(repr(group).encode()))
    ubar = rng.normal(size=(3, v.height, v.width)).astype(np.float32)
    t3, t4 = sg.param_tangents(small, seed=9)
    keep3 = {k: t3[k] for k in t3 if group == ("3", k)}
    keep4 = {k: t4[k] for k in t4 if group == ("4", k)}
    _, dimg = oracle.render_jvp(small, keep3, keep4, v)
    g3, g4 = oracle.render_bwd(small, [v], [ubar])
    lhs = float((ubar.astype(np.float64) * dimg).sum())
    rhs = _dot(g3, keep3) + _dot(g4, keep4)
    assert abs(lhs - rhs) <= 1e-9 * max(1.0, abs(lhs)), (lhs, rhs)
    assert abs(lhs) > 1e-6  # the direction actually moves the image


def test_vjp_equals_dual_jvp_all_parameters(tiny):
    v = tiny.views[0]
    ubar = np.random.default_rng(2).normal(size=(3, v.height, v.width)).astype(np.float32)
    t3, t4 = sg.param_tangents(tiny, seed=10)
    _, dimg = oracle.render_jvp(tiny, t3, t4, v)
    g3, g4 = oracle.render_bwd(tiny, [v], [ubar])
    lhs = float((ubar.astype(np.float64) * dimg).sum())
    rhs = _dot(g3, t3) + _dot(g4, t4)
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


def _eval(scene, v, ubar, g):
    """Loss and the decision signature (per-pixel blend counts plus the
    perturbed Gaussian's square) of one evaluation."""
    out = oracle.render(scene, v)
    pr = oracle.project(scene, v)
    sig = (out["nblend"].tobytes(), tuple(float(pr[k][g]) for k in ("visible", "radius", "x0", "x1", "y0", "y1")))
    return float((out["img"] * ubar).sum()), sig


def _perturbed(scene, which, key, idx, h):
    g3 = {k: a.copy() for k, a in scene.g3.items()}
    g4 = {k: a.copy() for k, a in scene.g4.items()}
    d = g3 if which == "3" else g4
    a = d[key].astype(np.float64)
    a[idx] += h
    d[key] = a.astype(np.float32)
    base = scene.g3 if which == "3" else scene.g4
    # the step actually taken is the float32-representable one
    return sg.Scene(g3, g4, scene.views), float(d[key][idx]) - float(base[key][idx])


def test_adjoint_matches_central_differences(small):
    """Central differences with Richardson extrapolation; a parameter whose
    perturbation changes any discrete decision (blend counts, the square) is
    skipped, because the image is discontinuous there."""
    v = small.views[0]
    ubar = np.random.default_rng(4).normal(size=(3, v.height, v.width))
    g3, g4 = oracle.render_bwd(small, [v], [ubar.astype(np.float32)])
    pr = oracle.project(small, v)
    vis = np.where(pr["visible"] > 0)[0]
    rng = np.random.default_rng(8)
    checked, skipped = 0, 0
    for _ in range(80):
        g = int(rng.choice(vis))
        if g < small.n4:
            which, i = "4", g
            key = GROUPS4[rng.integers(len(GROUPS4))]
            arr = small.g4[key]
        else:
            which, i = "3", g - small.n4
            key = GROUPS3[rng.integers(len(GROUPS3))]
            arr = small.g3[key]
        idx = (int(rng.integers(arr.shape[0])), i) if arr.ndim == 2 else (i,)
        h = 1e-3 * max(1.0, abs(float(arr[idx])))
        _, sig0 = _eval(small, v, ubar, g)
        res = []
        same = True
        for step in (h, -h, h / 2, -h / 2):
            sc, hs = _perturbed(small, which, key, idx, step)
            L, sig = _eval(sc, v, ubar, g)
            same &= sig == sig0
            res.append((L, hs))
        if not same:
            skipped += 1
            continue
        (Lp, hp), (Lm, hm), (Lp2, hp2), (Lm2, hm2) = res
        fd = (Lp - Lm) / (hp - hm)
        fd2 = (Lp2 - Lm2) / (hp2 - hm2)
        rich = fd2 + (fd2 - fd) / 3.0  # cancels the h^2 term
        ad = (g3 if which == "3" else g4)[key][idx]
        assert abs(rich - ad) <= 1e-4 * max(abs(ad), 1e-2), (which, key, idx, rich, ad)
        checked += 1
    assert checked >= 50, (checked, skipped)


def test_dual_matches_finite_difference_direction(small):
    v = small.views[0]
    t3, t4 = sg.param_tangents(small, seed=12)
    for d in list(t3.values()) + list(t4.values()):
        d *= 1e-3
    base, dimg = oracle.render_jvp(small, t3, t4, v)
    eps = 1e-2
    g3p = {k: (small.g3[k].astype(np.float64) + eps * t3[k]).astype(np.float32) for k in small.g3}
    g4p = {k: (small.g4[k].astype(np.float64) + eps * t4[k]).astype(np.float32) for k in small.g4}
    g3m = {k: (small.g3[k].astype(np.float64) - eps * t3[k]).astype(np.float32) for k in small.g3}
    g4m = {k: (small.g4[k].astype(np.float64) - eps * t4[k]).astype(np.float32) for k in small.g4}
    ip = oracle.render(sg.Scene(g3p, g4p, small.views), v)["img"]
    im = oracle.render(sg.Scene(g3m, g4m, small.views), v)["img"]
    fd = (ip - im) / (2 * eps)
    # away from discontinuities the two agree; compare the aggregate
    num = np.abs(fd - dimg).sum()
    den = np.abs(dimg).sum()
    assert num / den < 5e-2, num / den
