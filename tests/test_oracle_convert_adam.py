"""Pins of the oracle's static conversion (Sec. 4.1-4.2, Eq. 7-9) and Adam step
(no GPU)."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg


@pytest.mark.parametrize("frac", [0.0, 0.3, 1.0])
def test_convert_static_mask_order_and_counts_by_brute_force(frac):
    rng = np.random.default_rng(5)
    g4 = sg.draw_4d(rng, 500, 1.0, static_fraction=frac, tau=0.5)
    g3 = sg.draw_3d(rng, 200, 1.0)
    sc = sg.Scene(g3, g4)
    tau = 0.5
    perm, n4o, n3o, q = oracle.convert_static(sc, tau)
    keep, conv = [], []
    for i in range(500):
        # static iff exp(s_t) exceeds tau (strict), i.e. s_t > ln(tau)
        if math.exp(float(g4["log_scale"][3, i])) > tau and float(g4["log_scale"][3, i]) > math.log(tau):
            conv.append(i)
        else:
            keep.append(i)
    assert n4o == len(keep) and n3o == 200 + len(conv)
    for r, i in enumerate(keep):
        assert perm[i] == r
    for r, i in enumerate(conv):
        assert perm[i] == -(1 + 200 + r)
    assert q.shape == (4, len(conv))


def test_convert_static_threshold_is_strict():
    g4 = sg.draw_4d(np.random.default_rng(1), 3, 1.0)
    tau = np.float32(0.75)
    g4["log_scale"][3] = np.array([np.float32(math.log(tau)), np.nextafter(np.float32(math.log(tau)), np.float32(1)),
                                   np.float32(-5)], np.float32)
    # float32(ln tau) may sit on either side of ln tau; the mask follows (double)s_t > ln((double)tau)
    perm, n4o, n3o, _ = oracle.convert_static(sg.Scene(sg.empty_3d(), g4), float(tau))
    expect = [float(x) > math.log(float(tau)) for x in g4["log_scale"][3]]
    assert [p < 0 for p in perm] == expect


def test_converted_quaternion_of_a_block_diagonal_rotation_is_exact():
    rng = np.random.default_rng(3)
    kq = np.array([0.0, 0.0, 0.0, 1.0])

    def ham(p, q):
        a1, b1, c1, d1 = p
        a2, b2, c2, d2 = q
        return np.array([a1 * a2 - b1 * b2 - c1 * c2 - d1 * d2, a1 * b2 + b1 * a2 + c1 * d2 - d1 * c2,
                         a1 * c2 - b1 * d2 + c1 * a2 + d1 * b2, a1 * d2 + b1 * c2 - c1 * b2 + d1 * a2])

    n = 50
    g4 = sg.draw_4d(rng, n, 1.0)
    for i in range(n):
        ql = g4["quat_l"][:, i].astype(np.float64)
        g4["quat_r"][:, i] = (-ham(ham(kq, ql * np.array([1, -1, -1, -1])), kq)).astype(np.float32)
    g4["log_scale"][3] = 3.0
    perm, n4o, n3o, q = oracle.convert_static(sg.Scene(sg.empty_3d(), g4), 0.5)
    assert n4o == 0 and n3o == n
    for i in range(n):
        _, _, R4 = oracle.rot4(g4["quat_l"][:, i].astype(np.float64), g4["quat_r"][:, i].astype(np.float64))
        # Eq. 8 ideal case: R4 = diag(R3, 1); the quaternion reproduces R3
        assert np.allclose(oracle.quat_to_rot(q[:, i]), R4[:3, :3], atol=2e-7)
        assert abs(np.linalg.norm(q[:, i]) - 1) < 1e-6


def test_converted_quaternion_of_a_tilted_rotation_follows_the_antisymmetric_part():
    rng = np.random.default_rng(4)
    g4 = sg.draw_4d(rng, 100, 1.0)
    g4["log_scale"][3] = 3.0
    _, _, _, q = oracle.convert_static(sg.Scene(sg.empty_3d(), g4), 0.5)
    for i in range(100):
        _, _, R4 = oracle.rot4(g4["quat_l"][:, i].astype(np.float64), g4["quat_r"][:, i].astype(np.float64))
        R = R4[:3, :3]
        if 1 + np.trace(R) <= 1e-6:
            continue
        w = q[0, i]
        # 4 w^2 = 1 + tr(R) and 4 w (x, y, z) = the axial vector of R - R^T
        assert abs(4 * w * w - (1 + np.trace(R))) < 1e-12
        ax = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
        assert np.allclose(4 * w * q[1:, i], ax, atol=1e-12)


def test_adam_matches_torch_reference():
    import torch
    rng = np.random.default_rng(0)
    n = 1000
    p = rng.normal(size=n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    pt = torch.tensor(p.astype(np.float64), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        po, mo, vo = oracle.adam(p, g, m, v, 1e-2, 0.9, 0.999, 1e-8, step)
        pt.grad = torch.tensor(g.astype(np.float64))
        opt.step()
        assert np.allclose(po, pt.detach().numpy(), rtol=1e-6, atol=1e-6)
        p, m, v = (pt.detach().numpy().astype(np.float32), mo.astype(np.float32), vo.astype(np.float32))
        # keep both on the same float32 state
        with torch.no_grad():
            pt.copy_(torch.tensor(p.astype(np.float64)))
            st = opt.state[pt]
            st["exp_avg"].copy_(torch.tensor(m.astype(np.float64)))
            st["exp_avg_sq"].copy_(torch.tensor(v.astype(np.float64)))
