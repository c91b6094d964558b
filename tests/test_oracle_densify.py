"""Pins of the oracle's densification and pruning (clone / split / prune per
set, Sec. 4.3, adopted from 3D Gaussian Splatting), no GPU:

* its quaternion-product rotations equal the oracle's rotation matrices
  (Eq. 2's R(q) and Eq. 4's R_l R_r), which are pinned elsewhere;
* every decision at and around its boundary on hand-built rows (the selection
  compares exactly, the large-scale and prune tests are strict), with the
  expected output rows written out by hand;
* split children: a zero draw puts a child on its parent's centre, a unit
  draw along axis k moves it by exp(ls_k) times the k-th rotation column, and
  the children of many copies of one Gaussian have the parent's covariance
  (R diag(s^2) R^T, 3D and 4D) as their sample covariance.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from oracle import densify as od

LOG_SHRINK = math.log(0.8 * 2)
INF = float("inf")


def _args(**kw):
    a = dict(thr=2e-4, log_dense=math.log(0.05), logit_min=math.log(0.005 / 0.995), log_max_scale=INF, split_n=2,
             log_shrink=LOG_SHRINK)
    a.update(kw)
    return a


def test_rotations_equal_the_oracle_matrices():
    rng = np.random.default_rng(0)
    q = rng.normal(size=(4, 20)) * rng.uniform(0.3, 3.0, size=(1, 20))
    v = rng.normal(size=(3, 20))
    got = od.rotate3(q, v)
    for i in range(20):
        assert np.allclose(got[:, i], oracle.quat_to_rot(q[:, i] / np.linalg.norm(q[:, i])) @ v[:, i], atol=1e-13)
    ql, qr = rng.normal(size=(4, 20)), rng.normal(size=(4, 20))
    v4 = rng.normal(size=(4, 20))
    got4 = od.rotate4(ql, qr, v4)
    for i in range(20):
        _, _, R4 = oracle.rot4(ql[:, i] / np.linalg.norm(ql[:, i]), qr[:, i] / np.linalg.norm(qr[:, i]))
        assert np.allclose(got4[:, i], R4 @ v4[:, i], atol=1e-13)


def _rows3(ls_max, opacity):
    """3D rows with log-scales (ls_max, ls_max - 1, ls_max - 2), identity
    rotation, given opacity logits, distinct means and SH."""
    n = len(ls_max)
    ls = np.stack([np.asarray(ls_max, np.float64) - d for d in (0.0, 1.0, 2.0)])
    return dict(mean=np.arange(3 * n, dtype=np.float32).reshape(3, n), log_scale=ls.astype(np.float32),
                quat=np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)),
                opacity=np.asarray(opacity, np.float32),
                sh=np.arange(48 * n, dtype=np.float32).reshape(48, n) * 0.01)


def test_decisions_at_their_boundaries():
    a = _args(thr=2.0 ** -12)  # exact multiples, so rows can sit on the threshold
    thr = np.float32(a["thr"])
    big = np.float32(a["log_dense"]) + np.float32(0.5)   # large
    small = np.float32(-5.0)                              # not large
    at = np.float32(a["log_dense"])                       # float32 below the FP64 log_dense: not large
    ok_op = np.float32(2.0)
    lo_op = np.float32(-6.0)                              # sigmoid < 0.005: pruned
    # row: 0 selected exactly at the threshold, small -> clone
    #      1 just below the threshold -> nothing
    #      2 count 0 (gradient but never visible) -> nothing
    #      3 selected, large -> split
    #      4 selected, at log_dense -> clone
    #      5 not selected, low opacity -> pruned
    #      6 selected, small, low opacity -> clone and original both pruned
    #      7 selected, large, low opacity -> split, children pruned
    cnt = np.float32([3, 3, 0, 2, 1, 1, 4, 2])
    grad = np.float32([thr * np.float32(3), np.nextafter(thr * np.float32(3), np.float32(0)), 1.0,
                       thr * np.float32(5), thr, 0.0, 1.0, 1.0])
    assert float(thr) * 3.0 == float(thr * np.float32(3))  # the threshold row compares exactly
    g = _rows3([small, small, small, big, at, small, small, big], [ok_op] * 5 + [lo_op] * 3)
    noise = np.zeros((2, 3, 8))
    out, src, info = od.densify_set(g, False, grad, cnt, noise, **a)
    assert info == dict(clone=3, split=2, kept=4)
    # originals 0 1 2 4 (3 and 7 split, 5 and 6 pruned), clones 0 4, children of 3 (k = 0, 1)
    assert src.tolist() == [0, 1, 2, 4, -1, -5, -4, -4]
    for r, i in enumerate([0, 1, 2, 4, 0, 4, 3, 3]):
        assert np.array_equal(out["sh"][:, r], g["sh"][:, i])
        assert out["opacity"][r] == g["opacity"][i]
    want_child_ls = (g["log_scale"][:, 3].astype(np.float64) - LOG_SHRINK).astype(np.float32)
    assert np.array_equal(out["log_scale"][:, 6], want_child_ls)
    assert np.array_equal(out["log_scale"][:, :6], g["log_scale"][:, [0, 1, 2, 4, 0, 4]])
    # zero draws: children on the parent's centre
    assert np.array_equal(out["mean"][:, 6], g["mean"][:, 3]) and np.array_equal(out["mean"][:, 7], g["mean"][:, 3])


def test_prune_by_size_is_strict_and_applies_to_children():
    a = _args(log_max_scale=-2.0)
    g = _rows3([np.float32(-2.0), np.nextafter(np.float32(-2.0), np.float32(1)), np.float32(-1.6)],
               [2.0, 2.0, 2.0])
    # rows 0, 1 not selected; row 2 split: its children shrink below the limit
    out, src, _ = od.densify_set(g, False, np.float32([0, 0, 1.0]), np.float32([1, 1, 1]), np.zeros((2, 3, 3)), **a)
    assert (-1.6 - LOG_SHRINK) <= -2.0
    assert src.tolist() == [0, -3, -3]


def test_split_offsets_follow_the_rotation_columns():
    rng = np.random.default_rng(1)
    g3 = sg.draw_3d(rng, 5, 1.0)
    g3["log_scale"][:] = np.float32(-1.0)
    a = _args(log_dense=-2.0)
    for k in range(3):
        noise = np.zeros((2, 3, 5))
        noise[1, k] = 1.0
        out, src, _ = od.densify_set(g3, False, np.ones(5, np.float32), np.ones(5, np.float32), noise, **a)
        assert src.tolist() == [-1, -2, -3, -4, -5] * 2
        for i in range(5):
            R = oracle.quat_to_rot(g3["quat"][:, i].astype(np.float64) / np.linalg.norm(g3["quat"][:, i]))
            want = g3["mean"][:, i].astype(np.float64) + math.exp(-1.0) * R[:, k]
            assert np.allclose(out["mean"][:, 5 + i], want.astype(np.float32), atol=1e-7)
            assert np.array_equal(out["mean"][:, i], g3["mean"][:, i])
    g4 = sg.draw_4d(rng, 4, 1.0)
    g4["log_scale"][:] = np.float32(-1.0)
    for k in range(4):
        noise = np.zeros((2, 4, 4))
        noise[0, k] = 1.0
        out, src, _ = od.densify_set(g4, True, np.ones(4, np.float32), np.ones(4, np.float32), noise, **a)
        for i in range(4):
            ql = g4["quat_l"][:, i].astype(np.float64)
            qr = g4["quat_r"][:, i].astype(np.float64)
            _, _, R4 = oracle.rot4(ql / np.linalg.norm(ql), qr / np.linalg.norm(qr))
            d = math.exp(-1.0) * R4[:, k]
            assert np.allclose(out["mean"][:, i], (g4["mean"][:, i] + d[:3]).astype(np.float32), atol=1e-7)
            assert np.allclose(out["mean_t"][i], np.float32(g4["mean_t"][i] + d[3]), atol=1e-7)


@pytest.mark.parametrize("four_d", [False, True])
def test_children_have_the_parent_covariance(four_d):
    rng = np.random.default_rng(2)
    n = 40_000
    one = sg.draw_4d(rng, 1, 1.0) if four_d else sg.draw_3d(rng, 1, 1.0)
    one["log_scale"] = np.float32([[-1.0], [-1.5], [-0.7]] + ([[-1.2]] if four_d else []))
    g = {k: np.repeat(v, n, axis=-1) for k, v in one.items()}
    d = 4 if four_d else 3
    noise = rng.normal(size=(2, d, n))
    out, src, _ = od.densify_set(g, four_d, np.ones(n, np.float32), np.ones(n, np.float32), noise,
                                 **_args(log_dense=-5.0))
    pos = out["mean"].astype(np.float64)
    if four_d:
        pos = np.vstack([pos, out["mean_t"][None].astype(np.float64)])
    centre = np.concatenate([one["mean"][:, 0], one["mean_t"]]) if four_d else one["mean"][:, 0]
    dev = pos - centre.astype(np.float64)[:, None]
    cov = dev @ dev.T / dev.shape[1]
    s2 = np.exp(2.0 * one["log_scale"][:, 0].astype(np.float64))
    if four_d:
        ql, qr = one["quat_l"][:, 0].astype(np.float64), one["quat_r"][:, 0].astype(np.float64)
        _, _, R = oracle.rot4(ql / np.linalg.norm(ql), qr / np.linalg.norm(qr))
    else:
        q = one["quat"][:, 0].astype(np.float64)
        R = oracle.quat_to_rot(q / np.linalg.norm(q))
    want = R @ np.diag(s2) @ R.T
    assert np.abs(cov - want).max() <= 0.03 * s2.max()
