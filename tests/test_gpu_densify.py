"""Densification support on the GPU, through the C ABI, against the oracle:

* the backward's per-Gaussian statistics (image-plane gradient norm in
  normalised device coordinates, summed over the views that see the
  Gaussian; visible-view count; this call's visibility) against the oracle's
  screen-space adjoint and projection;
* clone / split / prune of both sets (h4dgs_densify) against the oracle's
  definition on the same inputs and draws: counts, source rows and every
  copied value bit-exact, children's log-scales bit-exact, children's centres
  within two float32 ulps (FP64 on both sides, rounded once);
* the optimiser-state gather (zeros for new rows) bit-exact;
* the visibility-masked Adam step against the oracle's Adam on the visible
  rows, the other rows untouched bit for bit.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from oracle import densify as od
from parity_util import mask_flagged

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h4d():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_13215_amd as m
    m._lib.load()
    return m


def test_backward_statistics_match_the_oracle(h4d):
    print("[densify stats] two views", flush=True)
    scene = sg.tiny_scene(seed=61)
    v0 = scene.views[0]
    views = [v0.with_time(0.3), sg.look_at((0.7, 0.2, -2.9), (0.0, 0.0, 0.0), 100, 70, t=0.65)]
    dls = []
    for k, v in enumerate(views):
        amb = oracle.render(scene, v)["amb"]
        dls.append(mask_flagged(sg.upstream_grads([v], seed=70 + k)[0], amb))
    _, _, g2s = oracle.render_bwd(scene, views, dls, want_g2=True)
    N = scene.n3 + scene.n4
    want_g, want_c = np.zeros(N), np.zeros(N)
    want_last = np.zeros(N, bool)
    for k, (v, g2) in enumerate(zip(views, g2s)):
        pr = oracle.project(scene, v)
        on = (pr["visible"] > 0) & (pr["x0"] <= pr["x1"]) & (pr["y0"] <= pr["y1"])
        want_g += np.where(on, np.hypot(g2[:, 0] * 0.5 * v.width, g2[:, 1] * 0.5 * v.height), 0.0)
        want_c += on
        want_last = want_last | on
    rast = h4d.Rasterizer(batched=True)
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    st3, st4 = h4d.new_stats(scene.n3, scene.n4)
    st3["grad_norm"] += 1.0  # accumulated onto what is there
    h = rast.forward(g3, g4, views)
    rast.backward(h, g3, g4, [torch.as_tensor(d, device="cuda") for d in dls], stats=(st3, st4))
    torch.cuda.synchronize()
    got_g = np.concatenate([st4["grad_norm"].cpu().numpy(), st3["grad_norm"].cpu().numpy() - 1.0])
    got_c = np.concatenate([st4["visible"].cpu().numpy(), st3["visible"].cpu().numpy()])
    got_s = np.concatenate([st4["step_visible"].cpu().numpy(), st3["step_visible"].cpu().numpy()])
    assert np.array_equal(got_c, want_c) and np.array_equal(got_s.astype(bool), want_last)
    assert want_c.sum() > 500
    scale = np.sqrt(np.mean(want_g ** 2))
    assert np.all(np.abs(got_g - want_g) <= 1e-3 * want_g + 1e-3 * scale + 1e-6)
    # the plain backward gives the same gradients
    a3, a4 = rast.backward(rast.forward(g3, g4, views), g3, g4, [torch.as_tensor(d, device="cuda") for d in dls])
    b3, b4 = rast.backward(rast.forward(g3, g4, views), g3, g4, [torch.as_tensor(d, device="cuda") for d in dls],
                           stats=h4d.new_stats(scene.n3, scene.n4))
    for k in a3:
        assert torch.allclose(a3[k], b3[k], rtol=1e-5, atol=1e-6 * float(a3[k].abs().max()) + 1e-30)
    for k in a4:
        assert torch.allclose(a4[k], b4[k], rtol=1e-5, atol=1e-6 * float(a4[k].abs().max()) + 1e-30)


def _params(h4d, split_n, log_dense, **kw):
    p = dict(grad_threshold=2e-4, split_n=split_n, log_dense_scale=log_dense,
             opacity_logit_min=math.log(0.005 / 0.995), log_max_scale=float("inf"), log_shrink=math.log(0.8 * split_n))
    p.update(kw)
    return h4d._lib.DensifyParams(p["grad_threshold"], p["split_n"], p["log_dense_scale"], p["opacity_logit_min"],
                                  p["log_max_scale"], p["log_shrink"]), p


@pytest.mark.parametrize("n3,n4,split_n,max_scale", [(3000, 2000, 2, float("inf")), (1500, 2500, 3, -2.2),
                                                     (0, 700, 2, float("inf")), (900, 0, 2, float("inf"))])
def test_densify_matches_the_oracle(h4d, n3, n4, split_n, max_scale):
    print(f"[densify] n3={n3} n4={n4} split_n={split_n}", flush=True)
    rng = np.random.default_rng(n3 + 7 * n4 + split_n)
    g3 = sg.draw_3d(rng, n3, 2.0)
    g4 = sg.draw_4d(rng, n4, 2.0)
    for g in (g3, g4):
        g["opacity"][rng.uniform(size=g["opacity"].shape) < 0.05] = -6.0  # some below the opacity limit
    st = []
    for n in (n3, n4):
        vis = rng.integers(0, 4, n).astype(np.float32)
        grad = (rng.exponential(2e-4, n) * vis).astype(np.float32)
        st.append((grad, vis))
    noise3 = rng.normal(size=(split_n, 3, n3)).astype(np.float32)
    noise4 = rng.normal(size=(split_n, 4, n4)).astype(np.float32)
    p3, a3 = _params(h4d, split_n, -3.0, log_max_scale=max_scale)
    p4, a4 = _params(h4d, split_n, -2.9, grad_threshold=3e-4, log_max_scale=max_scale)
    rast = h4d.Rasterizer()
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    s3 = {"grad_norm": dev(st[0][0]), "visible": dev(st[0][1])}
    s4 = {"grad_norm": dev(st[1][0]), "visible": dev(st[1][1])}
    moments = [(h4d.to_device({k: rng.normal(size=v.shape).astype(np.float32) for k, v in g3.items()}),
                h4d.to_device({k: rng.normal(size=v.shape).astype(np.float32) for k, v in g4.items()}))]
    o3, o4, src3, src4, moved = h4d.densify(rast, h4d.to_device(g3), h4d.to_device(g4), s3, s4, dev(noise3),
                                            dev(noise4), p3, p4, moments=moments)
    for g, four, (grad, vis), noise, a, o, src, which in ((g3, False, st[0], noise3, a3, o3, src3, 0),
                                                          (g4, True, st[1], noise4, a4, o4, src4, 1)):
        want, wsrc, info = od.densify_set(g, four, grad, vis, noise, thr=a["grad_threshold"],
                                          log_dense=a["log_dense_scale"], logit_min=a["opacity_logit_min"],
                                          log_max_scale=a["log_max_scale"], split_n=a["split_n"],
                                          log_shrink=a["log_shrink"])
        if g["opacity"].size:
            assert info["clone"] > 0 and info["split"] > 0, info
        assert np.array_equal(src.cpu().numpy(), wsrc)
        for k in want:
            got = o[k].cpu().numpy()
            assert got.shape == want[k].shape, k
            if k in ("mean", "mean_t"):
                assert np.all(np.abs(got - want[k]) <= 2 * np.spacing(np.abs(want[k]).astype(np.float32))), k
            else:
                assert np.array_equal(got, want[k]), k
        m_old = moments[0][which]
        m_new = moved[0][which]
        keep = wsrc >= 0
        for k in m_new:
            got = m_new[k].cpu().numpy()
            ref = m_old[k].cpu().numpy()
            assert np.array_equal(got[..., keep], ref[..., wsrc[keep]]), k
            assert not got[..., ~keep].any(), k


def test_masked_adam_updates_only_visible_rows(h4d):
    rng = np.random.default_rng(5)
    rows = [1000, 333, 64]
    comps = [3, 48, 1]
    rast = h4d.Rasterizer()
    P = [rng.normal(size=(c, r)).astype(np.float32) for c, r in zip(comps, rows)]
    M = [rng.normal(size=p.shape).astype(np.float32) * 0.1 for p in P]
    V = [np.abs(rng.normal(size=p.shape)).astype(np.float32) * 0.01 for p in P]
    G = [rng.normal(size=p.shape).astype(np.float32) for p in P]
    masks = [(rng.uniform(size=r) < 0.6).astype(np.uint8) for r in rows]
    masks[2][:] = 0
    lrs = [1e-3, 2.5e-3, 5e-2]
    tp, tm, tv = ([torch.as_tensor(a, device="cuda") for a in arr] for arr in (P, M, V))
    tg = [torch.as_tensor(a, device="cuda") for a in G]
    tk = [torch.as_tensor(k, device="cuda") for k in masks]
    step = 7
    h4d.adam_step(rast, tp, tg, tm, tv, lrs, step, masks=tk)
    torch.cuda.synchronize()
    eps32 = 2.0 ** -24
    for i in range(3):
        sel = np.broadcast_to(masks[i].astype(bool)[None, :], P[i].shape)
        po, mo, vo = oracle.adam(P[i][sel], G[i][sel], M[i][sel], V[i][sel], lrs[i], 0.9, 0.999, 1e-8, step)
        gp, gm, gv = tp[i].cpu().numpy(), tm[i].cpu().numpy(), tv[i].cpu().numpy()
        assert np.array_equal(gp[~sel], P[i][~sel]) and np.array_equal(gm[~sel], M[i][~sel])
        assert np.array_equal(gv[~sel], V[i][~sel])
        if sel.any():
            # float32 rounding bounds of each update (m may cancel, v cannot)
            m0, g0, p0 = M[i][sel].astype(np.float64), G[i][sel].astype(np.float64), P[i][sel].astype(np.float64)
            mtol = 4 * eps32 * (0.9 * np.abs(m0) + 0.1 * np.abs(g0)) + 1e-30
            assert np.all(np.abs(gm[sel] - mo) <= mtol)
            assert np.allclose(gv[sel], vo, rtol=8 * eps32, atol=0)
            c1, c2 = 1 - 0.9 ** step, 1 - 0.999 ** step
            den = np.sqrt(vo / c2) + 1e-8
            upd = lrs[i] * (np.abs(mo) / c1) / den
            ptol = 4 * eps32 * np.abs(p0) + 8 * eps32 * upd + lrs[i] * mtol / c1 / den
            assert np.all(np.abs(gp[sel] - po) <= ptol + 1e-12)
