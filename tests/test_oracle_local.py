"""Pins of the oracle's local evaluation (the selected-Gaussian gradients and
central differences used on scenes too large to composite whole): on scenes
small enough for the whole-view oracle, its flags and gradients equal the
whole-view ones, and its central differences equal its gradients (no GPU)."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from parity_util import KEYS3, KEYS4


def _rows_from_full(scene, r3, r4, sel):
    """Rows of the selected Gaussians out of whole-scene gradient arrays."""
    rows = np.zeros((len(sel), 65))
    for s, g in enumerate(sel):
        if g < scene.n4:
            order, src, i = oracle.ROW4, r4, g
        else:
            order, src, i = oracle.ROW3, r3, g - scene.n4
        for k, (name, c) in enumerate(order):
            rows[s, k] = src[name][i] if c is None else src[name][c, i]
    return rows


@pytest.fixture(scope="module")
def setup():
    scene = sg.tiny_scene(n3=500, n4=500, width=96, height=72, seed=21)
    v0 = scene.views[0]
    views = [v0.with_time(0.35), sg.look_at((0.6, 0.3, -2.9), (0.0, 0.0, 0.0), 80, 64, t=0.7, bg=(0.2, 0.4, 0.6))]
    vis = np.zeros(scene.n3 + scene.n4, bool)
    for v in views:
        vis |= oracle.project(scene, v)["visible"] > 0
    rng = np.random.default_rng(3)
    idx = np.where(vis)[0]
    sel = np.sort(np.concatenate([rng.choice(idx[idx < scene.n4], 6, replace=False),
                                  rng.choice(idx[idx >= scene.n4], 6, replace=False)])).astype(np.int32)
    return scene, views, sel


def test_local_flags_and_gradients_equal_whole_view(setup):
    scene, views, sel = setup
    loc = oracle.Local(scene, views, sel)
    dls = []
    for k, v in enumerate(views):
        full = oracle.render(scene, v)
        amb = loc.amb(k)
        region = (amb & 1) > 0
        assert region.sum() > 100
        # the local flags are the whole-view flags on every region pixel
        assert np.array_equal((amb & 2)[region] > 0, full["amb"][region])
        dls.append(np.where(full["amb"][None], 0.0, sg.upstream_grads([v], seed=50 + k)[0]).astype(np.float32))
    r3, r4 = oracle.render_bwd(scene, views, dls)
    want = _rows_from_full(scene, r3, r4, sel)
    got = loc.grad(dls)
    scale = np.abs(want).max(axis=1, keepdims=True)
    assert np.all(scale > 0)
    assert np.abs(got - want).max() <= 1e-11 * scale.max()
    assert np.all(np.abs(got - want) <= 1e-11 * scale)
    # 3D rows leave their last six entries at zero
    assert np.all(got[sel >= scene.n4, 59:] == 0)


def test_local_central_differences_equal_gradients(setup):
    scene, views, sel = setup
    loc = oracle.Local(scene, views, sel)
    dls = sg.upstream_grads(views, seed=60)
    grad = loc.grad(dls)
    ent = [(s, k) for s in range(len(sel)) for k in range(65 if sel[s] < scene.n4 else 59)]
    fd, ok = loc.fd(dls, ent, hrel=1e-6)
    assert ok.mean() > 0.9, ok.mean()
    ad = np.array([grad[s, k] for s, k in ent])
    rowscale = np.array([np.abs(grad[s]).max() for s, _ in ent])
    err = np.abs(fd - ad)[ok]
    assert np.all(err <= 1e-5 * np.abs(ad[ok]) + 1e-7 * rowscale[ok]), err.max()
    # every parameter group of both sets was compared
    names = {(sel[s] < scene.n4, (oracle.ROW4 if sel[s] < scene.n4 else oracle.ROW3)[k][0])
             for (s, k), o in zip(ent, ok) if o}
    assert names >= {(True, k) for k in KEYS4} | {(False, k) for k in KEYS3}


def test_local_rejects_bad_selection(setup):
    scene, views, _ = setup
    with pytest.raises(ValueError):
        oracle.Local(scene, views, np.array([3, 3], np.int32))
    with pytest.raises(ValueError):
        oracle.Local(scene, views, np.array([scene.n3 + scene.n4], np.int32))


def test_blended_at_matches_whole_view(setup):
    """Per sampled pixel: the count equals the whole view's blend count, the
    weights sum to 1 - T_final and, with the records' colours, reproduce the
    whole view's pixel colour."""
    scene, views, _ = setup
    v = views[1]
    full = oracle.render(scene, v)
    pr = oracle.project(scene, v)
    rng = np.random.default_rng(7)
    px = rng.integers(0, v.width, 200).astype(np.int32)
    py = rng.integers(0, v.height, 200).astype(np.int32)
    out = oracle.blended_at(scene, v, px, py)
    rgb = np.stack([pr["r"], pr["g"], pr["b"]], 1)
    for k, lst in enumerate(out):
        i, j = px[k], py[k]
        assert len(lst) == full["nblend"][j, i]
        w = np.array([x[1] for x in lst])
        ids = np.array([x[0] for x in lst], np.int64)
        assert abs(w.sum() - (1.0 - full["T"][j, i])) <= 1e-12
        col = (w[:, None] * rgb[ids]).sum(0) + full["T"][j, i] * np.asarray(v.bg)
        assert np.abs(col - full["img"][:, j, i]).max() <= 1e-12
        # front to back
        assert np.all(np.diff(pr["key"][ids]) >= 0)
