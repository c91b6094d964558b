"""Parity of the two per-Gaussian passes at their full workload sizes, through
the C ABI:

* convert_static (Eq. 7-9) on the hybrid-ratio scenes, 500k 4D Gaussians with
  0 %, 50 % and 90 % of them above the temporal-scale threshold tau = 0.5:
  the mask, the compaction order and every copied value bit-exact against the
  oracle, the converted rotations (Eq. 9) equal up to sign and rounding;
* Adam over the parameters of a 2M-Gaussian set (1.7M 3D, 0.3M 4D: 119.8M
  scalars in twelve tensors, one flat launch), two steps, sampled entries
  (both ends of every tensor and random ones) against the oracle's update
  of the same entries (Adam is elementwise, so a sample is checked exactly as
  the whole array would be).
"""
import numpy as np
import pytest

import oracle
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


@pytest.mark.parametrize("frac", [0.0, 0.5, 0.9])
def test_convert_static_full_size(h4d, frac):
    scene = sg.hybrid_ratio_scene(frac)
    g3, g4 = scene.g3, scene.g4
    n3 = g3["opacity"].shape[0]
    rast = h4d.Rasterizer()
    o3, o4, perm = h4d.convert_static(rast, h4d.to_device(g3), h4d.to_device(g4), 0.5)
    rperm, rn4, rn3, rq = oracle.convert_static(scene, 0.5)
    assert np.array_equal(perm.cpu().numpy(), rperm)
    assert o4["opacity"].shape[0] == rn4 and o3["opacity"].shape[0] == rn3
    keep = np.nonzero(rperm >= 0)[0]
    conv = np.nonzero(rperm < 0)[0]
    # the new 3D rows follow the old ones in the 4D set's order
    assert np.array_equal(-1 - rperm[conv], np.arange(n3, n3 + conv.size))
    if frac > 0.0:
        assert conv.size > 0.5 * frac * rperm.size
    for k in ("mean", "mean_t", "log_scale", "quat_l", "quat_r", "opacity", "sh"):
        assert np.array_equal(o4[k].cpu().numpy(), g4[k][..., keep]), k
    assert np.array_equal(o3["mean"].cpu().numpy()[:, n3:], g4["mean"][:, conv])
    assert np.array_equal(o3["log_scale"].cpu().numpy()[:, n3:], g4["log_scale"][:3, conv])
    assert np.array_equal(o3["opacity"].cpu().numpy()[n3:], g4["opacity"][conv])
    assert np.array_equal(o3["sh"].cpu().numpy()[:, n3:], g4["sh"][:, conv])
    q = o3["quat"].cpu().numpy()[:, n3:].astype(np.float64)
    if q.shape[1]:
        qn = q / np.linalg.norm(q, axis=0)
        rn = rq / np.linalg.norm(rq, axis=0)
        # a rotation's quaternion is defined up to sign
        sgn = np.sign(np.sum(qn * rn, axis=0))
        assert np.abs(qn - sgn * rn).max() <= 1e-6


def _adam_sizes(n3: int = 1_700_000, n4: int = 300_000):
    # 3D: mean, log_scale, quat, opacity, sh; 4D: mean, mean_t, log_scale,
    # quat_l, quat_r, opacity, sh (degree-3 SH: 48 coefficients)
    return [3 * n3, 3 * n3, 4 * n3, n3, 48 * n3, 3 * n4, n4, 4 * n4, 4 * n4, 4 * n4, n4, 48 * n4]


def test_adam_full_size_sampled(h4d):
    sizes = _adam_sizes()
    assert sum(sizes) == 119_800_000
    lrs = [1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 1.6e-4, 1.6e-4, 5e-3, 1e-3, 1e-3, 5e-2, 2.5e-3]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    P = [torch.randn(n, generator=gen, device="cuda") for n in sizes]
    M = [torch.zeros(n, device="cuda") for n in sizes]
    V = [torch.zeros(n, device="cuda") for n in sizes]
    rng = np.random.default_rng(3)
    idx = []
    for n in sizes:
        ends = np.r_[np.arange(5), np.arange(n - 5, n)]
        idx.append(torch.as_tensor(np.unique(np.r_[ends, rng.integers(0, n, 4000)]), device="cuda"))
    rast = h4d.Rasterizer()
    eps32 = 2.0 ** -24
    for step in (1, 2):
        G = [torch.randn(n, generator=gen, device="cuda") for n in sizes]
        before = [(P[i][idx[i]].cpu().numpy(), M[i][idx[i]].cpu().numpy(), V[i][idx[i]].cpu().numpy(),
                   G[i][idx[i]].cpu().numpy()) for i in range(len(sizes))]
        h4d.adam_step(rast, P, G, M, V, lrs, step)
        torch.cuda.synchronize()
        for i in range(len(sizes)):
            p0, m0, v0, g = before[i]
            po, mo, vo = oracle.adam(p0, g, m0, v0, lrs[i], 0.9, 0.999, 1e-8, step)
            p0, m0, g = p0.astype(np.float64), m0.astype(np.float64), g.astype(np.float64)
            # float32 rounding bounds of each update (m may cancel, v cannot)
            mtol = 4 * eps32 * (0.9 * np.abs(m0) + 0.1 * np.abs(g)) + 1e-30
            assert (np.abs(M[i][idx[i]].cpu().numpy() - mo) <= mtol).all(), (step, i)
            assert np.allclose(V[i][idx[i]].cpu().numpy(), vo, rtol=8 * eps32, atol=0), (step, i)
            c1, c2 = 1 - 0.9 ** step, 1 - 0.999 ** step
            upd = lrs[i] * (np.abs(mo) / c1) / (np.sqrt(vo / c2) + 1e-8)
            ptol = 4 * eps32 * np.abs(p0) + 8 * eps32 * upd + lrs[i] * mtol / c1 / (np.sqrt(vo / c2) + 1e-8)
            assert (np.abs(P[i][idx[i]].cpu().numpy() - po) <= ptol + 1e-12).all(), (step, i)
    del P, M, V, G
    torch.cuda.empty_cache()


def _moved_moments(m3, m4, perm):
    """The moment arrays after the conversion, gathered on the host with the
    oracle's permutation: kept 4D rows in order; old 3D rows, then converted
    rows with the moments of their copied fields and zeros for the quaternion."""
    keep = np.nonzero(perm >= 0)[0]
    keep = keep[np.argsort(perm[keep])]
    conv = np.nonzero(perm < 0)[0]
    conv = conv[np.argsort(-1 - perm[conv])]
    o4 = {k: v[..., keep] for k, v in m4.items()}
    add = dict(mean=m4["mean"][:, conv], log_scale=m4["log_scale"][:3, conv],
               quat=np.zeros((4, conv.size), np.float32), opacity=m4["opacity"][conv], sh=m4["sh"][:, conv])
    o3 = {k: np.concatenate([m3[k], add[k]], axis=-1) for k in m3}
    return o3, o4


@pytest.mark.parametrize("frac", [0.5, 0.9])
def test_convert_moments_full_size(h4d, frac):
    """Adam's moments follow the conversion (500k 4D Gaussians plus 100k 3D
    ones): bit-exact against a host gather driven by the oracle's permutation,
    with zeros for the converted rows' new quaternions."""
    print(f"[convert moments] 500k, static fraction {frac}", flush=True)
    scene = sg.hybrid_ratio_scene(frac)
    rng = np.random.default_rng(int(10 * frac))
    scene.g3 = sg.draw_3d(rng, 100_000, 2.0)
    moms = []
    for _ in range(2):
        m3 = {k: rng.normal(size=v.shape).astype(np.float32) for k, v in scene.g3.items()}
        m4 = {k: rng.normal(size=v.shape).astype(np.float32) for k, v in scene.g4.items()}
        moms.append((m3, m4))
    rperm, rn4, rn3, _ = oracle.convert_static(scene, 0.5)
    rast = h4d.Rasterizer()
    o3, o4, perm, moved = h4d.convert_static(rast, h4d.to_device(scene.g3), h4d.to_device(scene.g4), 0.5,
                                             moments=[(h4d.to_device(a), h4d.to_device(b)) for a, b in moms])
    assert np.array_equal(perm.cpu().numpy(), rperm)
    for (m3, m4), (g3m, g4m) in zip(moms, moved):
        w3, w4 = _moved_moments(m3, m4, rperm)
        for k in w4:
            assert np.array_equal(g4m[k].cpu().numpy(), w4[k]), k
        for k in w3:
            assert np.array_equal(g3m[k].cpu().numpy(), w3[k]), k
        assert g3m["opacity"].shape[0] == rn3 and g4m["opacity"].shape[0] == rn4
