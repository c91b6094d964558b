"""FP64 definition of adaptive densification and pruning, applied separately
to the static 3D and the dynamic 4D set (Sec. 4.3: the paper adopts the
clone / split / prune densification of 3D Gaussian Splatting and runs it on
each set on its own, with no opacity reset).

TEST INFRASTRUCTURE ONLY: the test-suite may use this module; the product
path never does.  It shares no code with the HIP library.  Rotations are
applied as quaternion products (q v q* for 3D, q_l v q_r for 4D with (x, y, z,
t) as the quaternion's (1, i, j, k) parts), not as matrices.

Definition (per set, rows i = 0 .. n-1; the readings are those the library's
header states for h4dgs_densify):
  * statistics: g_i = summed image-plane gradient norm, c_i = number of views
    in which row i was visible; selected iff c_i > 0 and g_i >= thr * c_i
    (compared exactly, in FP64);
  * L_i = largest spatial log-scale; large iff L_i > log_dense;
  * clone = selected and not large; split = selected and large;
  * a row is pruned iff opacity logit < logit_min or its largest spatial
    log-scale > log_max_scale;
  * output rows: the originals that are not split and not pruned (in order),
    then the clones (exact copies) that are not pruned (in order), then for
    k = 0 .. N-1 the k-th child of every split row (in order) that is not
    pruned; a child's log-scales (all of them) are fl32(ls - log_shrink), its
    centre (3D: mean; 4D: mean and mean_t) is the parent's plus the parent's
    rotation applied to exp(ls) * z_k (z_k: the given standard-normal draws),
    everything else copied;
  * src[r]: the original row of output r, or -(1 + parent) for a new row
    (clone or child: its optimiser moments start at zero).
"""
from __future__ import annotations

import numpy as np


def hamilton(p, q):
    """Quaternion product of [4, n] arrays (w, x, y, z)."""
    w1, x1, y1, z1 = p
    w2, x2, y2, z2 = q
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _unit(q):
    q = np.asarray(q, np.float64)
    return q / np.linalg.norm(q, axis=0, keepdims=True)


def rotate3(q, v):
    """R(q) v for [4, n] quaternions (any norm) and [3, n] vectors: q v q*."""
    qh = _unit(q)
    conj = qh * np.array([1.0, -1.0, -1.0, -1.0])[:, None]
    pv = np.vstack([np.zeros((1, v.shape[1])), v])
    return hamilton(hamilton(qh, pv), conj)[1:]


def rotate4(ql, qr, v):
    """R4 v = q_l v q_r for [4, n] vectors (x, y, z, t) (Eq. 4)."""
    return hamilton(hamilton(_unit(ql), np.asarray(v, np.float64)), _unit(qr))


def densify_set(g: dict, four_d: bool, grad, count, noise, thr: float, log_dense: float, logit_min: float,
                log_max_scale: float, split_n: int, log_shrink: float):
    """One set.  g: float32 parameter arrays (the library's layout); grad,
    count: float32 [n]; noise: [split_n, 4 (4D) or 3 (3D), n] standard normal
    draws.  Returns (out: dict of float32 arrays, src: int32 [rows])."""
    n = int(np.asarray(g["opacity"]).shape[0])
    ls = np.asarray(g["log_scale"], np.float32)
    nsp = 3
    grad64 = np.asarray(grad, np.float32).astype(np.float64)
    cnt64 = np.asarray(count, np.float32).astype(np.float64)
    sel = (cnt64 > 0) & (grad64 >= np.float64(np.float32(thr)) * cnt64)
    L = ls[:nsp].astype(np.float64).max(axis=0) if n else np.zeros(0)
    large = L > log_dense
    clone = sel & ~large
    split = sel & large
    op64 = np.asarray(g["opacity"], np.float32).astype(np.float64)

    def pruned(maxls):
        return (op64 < logit_min) | (maxls > log_max_scale)

    child_ls = (ls.astype(np.float64) - log_shrink).astype(np.float32)
    child_L = child_ls[:nsp].astype(np.float64).max(axis=0) if n else np.zeros(0)
    keep_orig = ~split & ~pruned(L)
    keep_clone = clone & ~pruned(L)
    keep_child = split & ~pruned(child_L)
    io, ic, ich = np.nonzero(keep_orig)[0], np.nonzero(keep_clone)[0], np.nonzero(keep_child)[0]
    parts, srcs = [], []
    parts.append({k: np.asarray(v)[..., io] for k, v in g.items()})
    srcs.append(io.astype(np.int64))
    parts.append({k: np.asarray(v)[..., ic] for k, v in g.items()})
    srcs.append(-1 - ic.astype(np.int64))
    s = np.exp(ls[:, ich].astype(np.float64))
    for k in range(split_n):
        z = np.asarray(noise[k], np.float64)[:, ich]
        row = {key: np.asarray(v)[..., ich].copy() for key, v in g.items()}
        row["log_scale"] = child_ls[:, ich]
        if four_d:
            d = rotate4(g["quat_l"][:, ich], g["quat_r"][:, ich], s * z)
            row["mean"] = (np.asarray(g["mean"], np.float64)[:, ich] + d[:3]).astype(np.float32)
            row["mean_t"] = (np.asarray(g["mean_t"], np.float64)[ich] + d[3]).astype(np.float32)
        else:
            d = rotate3(g["quat"][:, ich], s * z)
            row["mean"] = (np.asarray(g["mean"], np.float64)[:, ich] + d).astype(np.float32)
        parts.append(row)
        srcs.append(-1 - ich.astype(np.int64))
    out = {k: np.concatenate([p[k] for p in parts], axis=-1).astype(np.float32) for k in g}
    src = np.concatenate(srcs).astype(np.int32)
    return out, src, dict(clone=int(clone.sum()), split=int(split.sum()), kept=int(keep_orig.sum()))
