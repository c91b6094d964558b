"""Shared parity bars and helpers of the GPU tests (imported by test modules).

Bars (derived from the FP32 arithmetic of the kernels):
  * images: max |C_gpu - C_oracle| <= 1e-4 over pixels whose oracle decisions
    are all outside the FP32 guard band; flagged pixels < 1e-3 of the image;
  * gradients: per parameter group ||g - g_ref|| <= 1e-3 ||g_ref||, and per
    element |g - g_ref| <= 1e-3 |g_ref| + 1e-3 rms(g_ref) for every Gaussian
    (upstream gradients zeroed at flagged pixels), or, where the upstream
    gradient is kept everywhere, for every Gaussian whose pixel square holds
    no flagged pixel.
"""
import numpy as np

import oracle

IMG_TOL = 1e-4
GRAD_TOL = 1e-3
FLAG_FRAC = 1e-3

KEYS3 = ("mean", "log_scale", "quat", "opacity", "sh")
KEYS4 = ("mean", "mean_t", "log_scale", "quat_l", "quat_r", "opacity", "sh")


def check_image(gpu, ref, amb, tol=IMG_TOL, flag_frac=FLAG_FRAC):
    """gpu, ref: [3, H, W]; amb: [H, W] guard-band flags of the oracle."""
    assert amb.mean() < flag_frac, f"guard band flags {amb.mean():.2e} of the pixels"
    err = np.abs(gpu - ref)[:, ~amb]
    assert err.size == 0 or err.max() <= tol, f"max error {err.max():.3e} on unflagged pixels"
    return float(err.max()) if err.size else 0.0


def flagged_gaussians(scene, view, amb):
    """Gaussians whose pixel square holds a flagged pixel (summed-area table)."""
    pr = oracle.project(scene, view)
    n = scene.n3 + scene.n4
    H, W = amb.shape
    sat = np.zeros((H + 1, W + 1), np.int64)
    sat[1:, 1:] = np.cumsum(np.cumsum(amb.astype(np.int64), 0), 1)
    vis = pr["visible"] > 0
    x0 = np.clip(pr["x0"], 0, W - 1).astype(np.int64)
    x1 = np.clip(pr["x1"], 0, W - 1).astype(np.int64)
    y0 = np.clip(pr["y0"], 0, H - 1).astype(np.int64)
    y1 = np.clip(pr["y1"], 0, H - 1).astype(np.int64)
    cnt = sat[y1 + 1, x1 + 1] - sat[y0, x1 + 1] - sat[y1 + 1, x0] + sat[y0, x0]
    bad = np.zeros(n, bool)
    bad[vis] = cnt[vis] > 0
    return bad


def mask_flagged(dl, amb):
    """dL/dC with the guard-band pixels zeroed.  Pixels are independent, so a
    pixel whose upstream gradient is zero contributes exactly nothing to any
    parameter gradient on either side, and every Gaussian can then be checked
    element by element."""
    out = np.array(dl, dtype=np.float32, copy=True)
    out[:, amb] = 0.0
    return out


def check_grads(scene, gr3, gr4, r3, r4, bad, tol=GRAD_TOL):
    n4 = scene.n4
    for which, gr, rf, keys in (("4", gr4, r4, KEYS4), ("3", gr3, r3, KEYS3)):
        ok_cols = ~bad[:n4] if which == "4" else ~bad[n4:]
        for k in keys:
            g = gr[k].detach().cpu().numpy().astype(np.float64)
            r = rf[k]
            nr = np.linalg.norm(r)
            if nr == 0:
                assert np.abs(g).max(initial=0.0) == 0
                continue
            rel = np.linalg.norm(g - r) / nr
            assert rel <= tol, f"{which}D {k}: relative L2 error {rel:.2e}"
            gs, rs = g[..., ok_cols], r[..., ok_cols]
            rms = np.sqrt(np.mean(r * r))
            viol = np.abs(gs - rs) > tol * np.abs(rs) + tol * rms
            assert viol.sum() == 0, f"{which}D {k}: {viol.sum()} elements out of tolerance"


def sample_pixels(W, H, n, seed, tile=16):
    """Pixel coordinates to compare against the oracle's per-pixel brute force:
    the four corners, the centre, 16 pixels each in the last (ragged) tile row
    and column of a ``tile``-pixel tiling, and n seeded random ones."""
    rng = np.random.default_rng(seed)
    xs = [0, W - 1, 0, W - 1, W // 2]
    ys = [0, 0, H - 1, H - 1, H // 2]
    for k in range(16):
        xs.append(int(rng.integers(0, W))); ys.append(H - 1 - k % (H % tile or tile))
        xs.append(W - 1 - k % (W % tile or tile)); ys.append(int(rng.integers(0, H)))
    xs += list(rng.integers(0, W, n))
    ys += list(rng.integers(0, H, n))
    return np.asarray(xs, np.int32), np.asarray(ys, np.int32)


def check_pixels(scene, view, img, xs, ys, tol=IMG_TOL):
    """img [3, H, W] at the given pixels against oracle.pixels (brute force over
    every Gaussian); flagged pixels are skipped and must stay a small share."""
    rgb, T, amb = oracle.pixels(scene, view, xs, ys)
    ok = ~amb
    assert ok.mean() > 0.9, ok.mean()
    got = img[:, ys, xs].T
    err = np.abs(got - rgb)[ok]
    assert err.max() <= tol, err.max()
    return float(err.max())
