"""Pins of the FP64 oracle's per-Gaussian geometry against closed forms,
independent routes, brute force and library routines (no GPU).

Each test names the passage of the paper it pins.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg


def hamilton(p, q):
    """Quaternion product p*q, components (1, i, j, k)."""
    a1, b1, c1, d1 = p
    a2, b2, c2, d2 = q
    return np.array([a1 * a2 - b1 * b2 - c1 * c2 - d1 * d2,
                     a1 * b2 + b1 * a2 + c1 * d2 - d1 * c2,
                     a1 * c2 - b1 * d2 + c1 * a2 + d1 * b2,
                     a1 * d2 + b1 * c2 - c1 * b2 + d1 * a2])


def conj(q):
    return np.array([q[0], -q[1], -q[2], -q[3]])


RNG = np.random.default_rng(123)


def _unit(n=4):
    q = RNG.normal(size=n)
    return q / np.linalg.norm(q)


# --- Eq. 4 -----------------------------------------------------------------

@pytest.mark.parametrize("trial", range(20))
def test_rot4_is_rotation_and_equals_double_quaternion_product(trial):
    ql, qr = RNG.normal(size=4) * 3, RNG.normal(size=4) * 0.2  # raw (unnormalised) inputs
    L, Rr, R = oracle.rot4(ql, qr)
    assert np.allclose(R @ R.T, np.eye(4), atol=1e-14)
    assert abs(np.linalg.det(R) - 1.0) < 1e-13
    assert np.allclose(L @ L.T, np.eye(4), atol=1e-14)
    assert np.allclose(Rr @ Rr.T, np.eye(4), atol=1e-14)
    a, b = ql / np.linalg.norm(ql), qr / np.linalg.norm(qr)
    for _ in range(4):
        x = RNG.normal(size=4)  # (x, y, z, t) <-> (1, i, j, k)
        assert np.allclose(R @ x, hamilton(hamilton(a, x), b), atol=1e-13)
        assert np.allclose(L @ x, hamilton(a, x), atol=1e-13)
        assert np.allclose(Rr @ x, hamilton(x, b), atol=1e-13)


@pytest.mark.parametrize("trial", range(10))
def test_quat_to_rot_is_quaternion_conjugation(trial):
    q = RNG.normal(size=4)
    R = oracle.quat_to_rot(q)
    qh = q / np.linalg.norm(q)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-14)
    assert abs(np.linalg.det(R) - 1) < 1e-13
    v = RNG.normal(size=3)
    rv = hamilton(hamilton(qh, np.r_[0.0, v]), conj(qh))
    assert np.allclose(R @ v, rv[1:], atol=1e-13)


# --- Eq. 9 -----------------------------------------------------------------

@pytest.mark.parametrize("trial", range(20))
def test_mat2quat_round_trip(trial):
    q = _unit()
    if q[0] < 0:
        q = -q
    R = oracle.quat_to_rot(q)
    q2 = oracle.mat2quat(R)
    assert np.allclose(q2, q, atol=1e-13)


@pytest.mark.parametrize("axis", [np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), np.array([0, 0, 1.0]),
                                  np.array([1.0, 2.0, -0.5])])
def test_mat2quat_half_turn_uses_largest_component_branch(axis):
    # a rotation by pi has w = 0: 1 + trace = 0 and the printed formula divides by 0
    axis = axis / np.linalg.norm(axis)
    q = np.r_[0.0, axis]
    R = oracle.quat_to_rot(q)
    assert 1 + np.trace(R) < 1e-12
    q2 = oracle.mat2quat(R)
    assert np.allclose(oracle.quat_to_rot(q2), R, atol=1e-13)
    assert abs(np.linalg.norm(q2) - 1) < 1e-13


def test_mat2quat_near_half_turn_both_branches_agree():
    # just above / below the branch threshold the two formulas give the same rotation
    for eps in (2e-6, 5e-7):
        q = np.r_[math.sqrt(eps) / 2, _unit(3) * math.sqrt(1 - eps / 4)]
        R = oracle.quat_to_rot(q)
        q2 = oracle.mat2quat(R)
        assert np.allclose(oracle.quat_to_rot(q2), R, atol=1e-9)


# --- Eq. 2 (3D covariance) ----------------------------------------------------

def test_cov3_eigen_decomposition(tiny):
    n4 = tiny.n4
    for j in range(10):
        g = n4 + j
        _, Sg, _ = oracle.world(tiny, g, 0.5)
        s2 = np.exp(2.0 * tiny.g3["log_scale"][:, j].astype(np.float64))
        R = oracle.quat_to_rot(tiny.g3["quat"][:, j].astype(np.float64))
        w, V = np.linalg.eigh(Sg)
        assert np.allclose(np.sort(w), np.sort(s2), rtol=1e-12)
        # eigenvectors are the columns of R (up to sign)
        for k in range(3):
            v = R[:, k]
            assert np.allclose(Sg @ v, s2[k] * v, atol=1e-14)


# --- Eq. 5-6 and the temporal marginal ---------------------------------------

def _sigma4(scene, i):
    s = np.exp(scene.g4["log_scale"][:, i].astype(np.float64))
    _, _, R4 = oracle.rot4(scene.g4["quat_l"][:, i].astype(np.float64), scene.g4["quat_r"][:, i].astype(np.float64))
    return R4 @ np.diag(s * s) @ R4.T


@pytest.mark.parametrize("i", range(8))
def test_slice_matches_precision_matrix_route(tiny, i):
    Sg4 = _sigma4(tiny, i)
    mu4 = np.r_[tiny.g4["mean"][:, i].astype(np.float64), np.float64(tiny.g4["mean_t"][i])]
    for t in (0.1, 0.5, 0.93):
        mu, Sg, op = oracle.world(tiny, i, t)
        Lam = np.linalg.inv(Sg4)
        Sg_ref = np.linalg.inv(Lam[:3, :3])
        mu_ref = mu4[:3] - Sg_ref @ Lam[:3, 3] * (t - mu4[3])
        assert np.allclose(Sg, Sg_ref, rtol=1e-9, atol=1e-15)
        assert np.allclose(mu, mu_ref, rtol=1e-10, atol=1e-12)


def test_slice_matches_brute_force_conditioning():
    # a fat 4D Gaussian so that a modest grid resolves it
    g4 = dict(mean=np.array([[0.1], [-0.2], [0.05]], np.float32), mean_t=np.array([0.4], np.float32),
              log_scale=np.log(np.array([[0.3], [0.2], [0.25], [0.35]], np.float32)),
              quat_l=np.array([[0.8], [0.3], [-0.4], [0.2]], np.float32),
              quat_r=np.array([[0.5], [-0.6], [0.3], [0.5]], np.float32),
              opacity=np.zeros(1, np.float32), sh=np.zeros((48, 1), np.float32))
    sc = sg.Scene(sg.empty_3d(), g4)
    t = 0.7
    mu, Sg, op = oracle.world(sc, 0, t)
    Sg4 = _sigma4(sc, 0)
    P = np.linalg.inv(Sg4)
    mu4 = np.r_[g4["mean"][:, 0].astype(np.float64), np.float64(g4["mean_t"][0])]
    n = 81
    ax = [np.linspace(mu[k] - 6 * math.sqrt(Sg[k, k]), mu[k] + 6 * math.sqrt(Sg[k, k]), n) for k in range(3)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    d = np.stack([X - mu4[0], Y - mu4[1], Z - mu4[2], np.full_like(X, t - mu4[3])], -1)
    dens = np.exp(-0.5 * np.einsum("...i,ij,...j->...", d, P, d))
    dv = np.prod([a[1] - a[0] for a in ax])
    mass = dens.sum() * dv
    m1 = np.array([(dens * G).sum() * dv / mass for G in (X, Y, Z)])
    D = np.stack([X - m1[0], Y - m1[1], Z - m1[2]], -1)
    m2 = np.einsum("abci,abcj,abc->ij", D, D, dens) * dv / mass
    assert np.allclose(m1, mu, atol=1e-6)
    assert np.allclose(m2, Sg, rtol=1e-5, atol=1e-7)
    # integral over x of the unnormalised 4D density = (2pi)^{3/2} sqrt(det Sigma_c) p(t)
    closed = (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(Sg)) * op["pt"]
    assert abs(mass / closed - 1) < 1e-6
    # and p(t) is the unnormalised marginal exp(-(t-mu_t)^2 / (2 Sigma_44))
    assert abs(op["pt"] - math.exp(-(t - mu4[3]) ** 2 / (2 * Sg4[3, 3]))) < 1e-14
    assert abs(op["op"] - op["sigmoid"] * op["pt"]) < 1e-15


# --- SH ------------------------------------------------------------------------

def test_sh_orthonormal_by_quadrature():
    x, w = np.polynomial.legendre.leggauss(24)
    nph = 48
    phs = (np.arange(nph) + 0.5) * 2 * math.pi / nph
    G = np.zeros((16, 16))
    for ct, wt in zip(x, w):
        st = math.sqrt(1 - ct * ct)
        for ph in phs:
            Y = oracle.sh_basis(np.array([st * math.cos(ph), st * math.sin(ph), ct]))
            G += np.outer(Y, Y) * wt * (2 * math.pi / nph)
    assert np.allclose(G, np.eye(16), atol=1e-12)


def test_sh_matches_scipy_with_condon_shortley():
    import scipy.special as sp
    for _ in range(10):
        d = _unit(3)
        th, ph = math.acos(d[2]), math.atan2(d[1], d[0])
        Y = oracle.sh_basis(d)
        for l in range(4):
            for m in range(-l, l + 1):
                c = sp.sph_harm_y(l, abs(m), th, ph)
                ref = c.real if m == 0 else (math.sqrt(2) * (c.real if m > 0 else c.imag))
                assert abs(Y[l * l + l + m] - ref) < 1e-12


def test_sh_low_order_signs():
    # reading: Y_1,-1 ~ -y, Y_1,0 ~ z, Y_1,1 ~ -x  (Condon-Shortley phase)
    k = math.sqrt(3 / (4 * math.pi))
    Y = oracle.sh_basis(np.array([0.0, 0.0, 1.0]))
    assert abs(Y[0] - 0.5 / math.sqrt(math.pi)) < 1e-15 and abs(Y[2] - k) < 1e-14
    Y = oracle.sh_basis(np.array([1.0, 0.0, 0.0]))
    assert abs(Y[3] + k) < 1e-14
    Y = oracle.sh_basis(np.array([0.0, 1.0, 0.0]))
    assert abs(Y[1] + k) < 1e-14


# --- EWA projection and the camera ---------------------------------------------

def _pixel_of(view, X):
    M = view.world_to_cam.astype(np.float64)
    p = M[:, :3] @ X + M[:, 3]
    return np.array([view.fx * p[0] / p[2] + view.cx, view.fy * p[1] / p[2] + view.cy])


def test_ewa_equals_numerical_jacobian_of_the_camera(tiny):
    v = tiny.views[0]
    pr = oracle.project(tiny, v)
    checked = 0
    for g in range(0, tiny.n3 + tiny.n4, 37):
        if pr["culled"][g]:
            continue
        mu, Sg, _ = oracle.world(tiny, g, v.t)
        Jn = np.zeros((2, 3))
        for k in range(3):
            h = 1e-6
            e = np.zeros(3)
            e[k] = h
            Jn[:, k] = (_pixel_of(v, mu + e) - _pixel_of(v, mu - e)) / (2 * h)
        uv = _pixel_of(v, mu)
        if abs(uv[0] - v.cx) > 1.2 * v.width / 2 or abs(uv[1] - v.cy) > 1.2 * v.height / 2:
            continue  # the Jacobian clamp is active there
        Q = np.array([[pr["q00"][g], pr["q01"][g]], [pr["q01"][g], pr["q11"][g]]])
        S2 = np.linalg.inv(Q) - 0.3 * np.eye(2)
        assert np.allclose(S2, Jn @ Sg @ Jn.T, rtol=1e-7, atol=1e-7)
        assert np.allclose([pr["u"][g], pr["v"][g]], uv, atol=1e-9)
        checked += 1
    assert checked > 20


def test_single_isotropic_gaussian_closed_form_image():
    f = sg.look_at((0.0, 0.0, -4.0), (0.0, 0.0, 0.0), 64, 48)
    s, z, op_logit = 0.02, 4.0, 1.3
    sh = np.zeros((48, 1), np.float32)
    colour = np.array([0.9, 0.4, 0.2])
    y00 = 0.5 / math.sqrt(math.pi)
    sh[0:3, 0] = (colour - 0.5) / y00
    g3 = dict(mean=np.zeros((3, 1), np.float32), log_scale=np.full((3, 1), math.log(s), np.float32),
              quat=np.array([[1.0], [0], [0], [0]], np.float32), opacity=np.array([op_logit], np.float32), sh=sh)
    sc = sg.Scene(g3, sg.empty_4d(), [f])
    out = oracle.render(sc, f)
    sig = 1 / (1 + math.exp(-op_logit))
    s_eff = math.exp(np.float64(np.float32(math.log(s))))
    var = (f.fx * s_eff / z) ** 2 + 0.3  # isotropic: J Sigma J^T = (f s / z)^2 I, plus the dilation
    col = sh[0:3, 0].astype(np.float64) * y00 + 0.5
    # equal eigenvalues: the discriminant floor 0.1 sets the radius
    r = math.ceil(3 * math.sqrt(var + math.sqrt(0.1)))
    for j in range(48):
        for i in range(64):
            dx, dy = i + 0.5 - f.cx, j + 0.5 - f.cy
            inside = abs(dx) <= r and abs(dy) <= r
            a = min(0.99, sig * math.exp(-(dx * dx + dy * dy) / (2 * var)))
            expect = col * a if (inside and a >= 1 / 255) else np.zeros(3)
            assert np.allclose(out["img"][:, j, i], expect, atol=1e-13), (i, j)


def test_point_lands_where_the_pinhole_model_says():
    v = sg.look_at((0.3, -0.2, -4.0), (0.0, 0.1, 0.0), 96, 64)
    X = np.array([0.21, -0.13, 0.4])
    g3 = dict(mean=X[:, None].astype(np.float32), log_scale=np.full((3, 1), math.log(1e-3), np.float32),
              quat=np.array([[1.0], [0], [0], [0]], np.float32), opacity=np.array([4.0], np.float32),
              sh=np.zeros((48, 1), np.float32))
    sc = sg.Scene(g3, sg.empty_4d(), [v])
    pr = oracle.project(sc, v)
    uv = _pixel_of(v, X.astype(np.float32).astype(np.float64))
    assert abs(pr["u"][0] - uv[0]) < 1e-12 and abs(pr["v"][0] - uv[1]) < 1e-12
    img = oracle.render(sc, v)["img"].sum(0)
    j, i = np.unravel_index(np.argmax(img), img.shape)
    assert abs(i + 0.5 - uv[0]) <= 0.5 and abs(j + 0.5 - uv[1]) <= 0.5


def _single_3d(X, log_s, sh=None, quat=(1.0, 0.0, 0.0, 0.0), op_logit=2.0):
    return dict(mean=np.asarray(X, np.float64)[:, None].astype(np.float32),
                log_scale=np.asarray(log_s, np.float64)[:, None].astype(np.float32),
                quat=np.asarray(quat, np.float64)[:, None].astype(np.float32),
                opacity=np.array([op_logit], np.float32),
                sh=np.zeros((48, 1), np.float32) if sh is None else sh)


@pytest.mark.parametrize("side", [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1)])
def test_jacobian_clamp_beyond_the_field_of_view(side):
    """A Gaussian whose camera-space ratio x/z (or y/z) lies beyond 1.3 times the
    half field of view: its 2D covariance minus the dilation equals J S J^T
    with J the central-difference Jacobian of the pinhole map taken at the
    clamped point (the point of the same depth on the ray at 1.3 times the
    half field of view), and differs from the unclamped one.  (3DGS-lineage
    clamp, reading of the constants the paper inherits, Sec. 4.3.)"""
    v = sg.View(np.eye(3, 4, dtype=np.float32), 100.0, 90.0, 64.0, 48.0, 128, 96, 0.5)
    z = 3.0
    limx, limy = 1.3 * 64.0 / 100.0, 1.3 * 48.0 / 90.0
    tx = (limx * 1.4 if side[0] > 0 else -limx * 1.25) if side[0] else 0.1
    ty = (limy * 1.3 if side[1] > 0 else -limy * 1.6) if side[1] else -0.05
    X = np.array([tx * z, ty * z, z])
    ls = np.log([0.05, 0.12, 0.08])
    q = np.array([0.9, 0.2, -0.3, 0.25])
    q /= np.linalg.norm(q)
    sc = sg.Scene(_single_3d(X, ls, quat=q), sg.empty_4d(), [v])
    pr = oracle.project(sc, v)
    assert pr["culled"][0] == 0
    Q = np.array([[pr["q00"][0], pr["q01"][0]], [pr["q01"][0], pr["q11"][0]]])
    S2 = np.linalg.inv(Q) - 0.3 * np.eye(2)
    mu, Sg, _ = oracle.world(sc, 0, v.t)
    def jac_at(P):
        J = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1e-6
            J[:, k] = (_pixel_of(v, P + e) - _pixel_of(v, P - e)) / 2e-6
        return J
    xc = np.clip(mu[0] / mu[2], -limx, limx)
    yc = np.clip(mu[1] / mu[2], -limy, limy)
    Jc = jac_at(np.array([xc * mu[2], yc * mu[2], mu[2]]))
    assert np.allclose(S2, Jc @ Sg @ Jc.T, rtol=1e-7, atol=1e-9)
    Ju = jac_at(mu)
    assert not np.allclose(S2, Ju @ Sg @ Ju.T, rtol=1e-3, atol=1e-6)


def test_sh_view_direction_points_from_the_camera_to_the_gaussian():
    """A Gaussian carrying only degree-1 coefficients, seen by cameras on
    opposite sides: its colour is 0.5 + c Y_1m(d) with d the unit vector from
    the camera centre to the Gaussian (Y_1-1 = -k y, Y_10 = k z, Y_11 = -k x,
    k = sqrt(3 / (4 pi)), Condon-Shortley phase).  Reversing d flips each
    degree-1 term, so the colours of opposite cameras would swap."""
    k1 = math.sqrt(3.0 / (4.0 * math.pi))
    X = np.array([0.1, -0.2, 0.3])
    sh = np.zeros((48, 1), np.float32)
    coef = {1: (0.3, -0.1, 0.2), 2: (-0.4, 0.25, 0.1), 3: (0.15, 0.35, -0.3)}  # index l^2 + l + m -> RGB
    for idx, rgb in coef.items():
        sh[3 * idx:3 * idx + 3, 0] = rgb
    checked = 0
    for eye in [(0.1, -0.2, -2.7), (0.1, -0.2, 3.3), (-2.9, -0.2, 0.3), (3.1, -0.2, 0.3), (0.1, 2.8, 0.3),
                (0.1, -3.2, 0.3), (1.7, 1.1, -2.0)]:
        up_ok = abs(eye[1] - X[1]) < 2.0
        v = sg.look_at(eye, tuple(X), 64, 48) if up_ok else _look_at_z_up(eye, X)
        sc = sg.Scene(_single_3d(X, np.log([0.05] * 3), sh=sh), sg.empty_4d(), [v])
        pr = oracle.project(sc, v)
        Xf = X.astype(np.float32).astype(np.float64)
        M = v.world_to_cam.astype(np.float64)
        C = -M[:, :3].T @ M[:, 3]
        d = (Xf - C) / np.linalg.norm(Xf - C)
        Y = {1: -k1 * d[1], 2: k1 * d[2], 3: -k1 * d[0]}
        expect = 0.5 + sum(sh[3 * i:3 * i + 3, 0].astype(np.float64) * Y[i] for i in (1, 2, 3))
        got = np.array([pr["r"][0], pr["g"][0], pr["b"][0]])
        assert np.allclose(got, np.maximum(expect, 0.0), atol=1e-12), (eye, got, expect)
        rev = 0.5 - (expect - 0.5)
        assert not np.allclose(got, np.maximum(rev, 0.0), atol=1e-3)
        checked += 1
    assert checked == 7


def _look_at_z_up(eye, target):
    """Camera at eye looking at target with world up = +z (for views along y)."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.array([0.0, 0.0, 1.0]))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    M = np.concatenate([R, (-R @ eye)[:, None]], axis=1).astype(np.float32)
    return sg.View(M, 55.4, 55.4, 32.0, 24.0, 64, 48, 0.5)


def test_raw_quaternion_norm_leaves_image_and_scales_gradient():
    """Quaternions are normalised before use: scaling a quaternion column by
    lambda leaves the image unchanged and divides its gradient by lambda (the
    gradient is orthogonal to the quaternion), for q, q_l and q_r."""
    base = sg.tiny_scene(n3=200, n4=200, width=64, height=48, seed=9)
    raw = sg.raw_quaternion_norms(base, seed=4)
    v = base.views[0]
    a = oracle.render(base, v)["img"]
    b = oracle.render(raw, v)["img"]
    # the float32 rounding of the scaled quaternion moves the image by ~1e-7
    assert np.abs(a - b).max() < 1e-5
    dl = sg.upstream_grads([v], seed=5)
    ga3, ga4 = oracle.render_bwd(base, [v], dl)
    gb3, gb4 = oracle.render_bwd(raw, [v], dl)
    # compare on the raw scene itself: its gradient times |q| against the
    # gradient of the same scene with each column normalised in float64
    unit = sg.Scene({k: x.copy() for k, x in raw.g3.items()}, {k: x.copy() for k, x in raw.g4.items()}, raw.views)
    for d, gr_raw, gr_unit_src, keys in ((raw.g3, gb3, "3", ("quat",)), (raw.g4, gb4, "4", ("quat_l", "quat_r"))):
        for k in keys:
            q = d[k].astype(np.float64)
            nrm = np.linalg.norm(q, axis=0)
            assert nrm.min() < 0.6 and nrm.max() > 1.8
            radial = (gr_raw[k] * q).sum(0)
            assert np.abs(radial).max() <= 1e-10 * np.abs(gr_raw[k]).max() * nrm.max()
    # the gradient of the normalised scene (float64 division, rounded) times 1/|q|
    for (d, k, which) in ((raw.g3, "quat", 3), (raw.g4, "quat_l", 4), (raw.g4, "quat_r", 4)):
        q = d[k].astype(np.float64)
        (unit.g3 if which == 3 else unit.g4)[k] = (q / np.linalg.norm(q, axis=0)).astype(np.float32)
    gu3, gu4 = oracle.render_bwd(unit, [v], dl)
    for d, gr_raw, gr_unit, keys in ((raw.g3, gb3, gu3, ("quat",)), (raw.g4, gb4, gu4, ("quat_l", "quat_r"))):
        for k in keys:
            nrm = np.linalg.norm(d[k].astype(np.float64), axis=0)
            got = gr_raw[k] * nrm
            want = gr_unit[k]
            assert np.linalg.norm(got - want) <= 1e-4 * np.linalg.norm(want), k


# --- Eq. 8: the static limit ----------------------------------------------------

def _static_pair(n=60, seed=7, tilt=False):
    """4D Gaussians whose rotation is block-diagonal (q_r = -k conj(q_l) k keeps
    the time axis fixed) and whose temporal scale is huge, plus the 3D Gaussians
    that Eq. 9 makes of them."""
    rng = np.random.default_rng(seed)
    g4 = sg.draw_4d(rng, n, 1.0)
    kq = np.array([0.0, 0.0, 0.0, 1.0])
    for i in range(n):
        ql = g4["quat_l"][:, i].astype(np.float64)
        qr = -hamilton(hamilton(kq, conj(ql)), kq)
        if tilt:
            qr = qr + 0.3 * rng.normal(size=4)
        g4["quat_r"][:, i] = qr.astype(np.float32)
    g4["log_scale"][3] = 20.0
    g4["opacity"][:] = np.abs(g4["opacity"]) + 1.0
    q3 = np.zeros((4, n))
    for i in range(n):
        _, _, R4 = oracle.rot4(g4["quat_l"][:, i].astype(np.float64), g4["quat_r"][:, i].astype(np.float64))
        q3[:, i] = oracle.mat2quat(R4[:3, :3])
    g3 = dict(mean=g4["mean"].copy(), log_scale=g4["log_scale"][:3].copy(), quat=q3.astype(np.float32),
              opacity=g4["opacity"].copy(), sh=g4["sh"].copy())
    return g3, g4


def test_static_4d_renders_like_its_3d_conversion():
    g3, g4 = _static_pair()
    v = sg.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 64, 48, t=0.83)
    for i in range(g4["opacity"].shape[0]):
        _, _, R4 = oracle.rot4(g4["quat_l"][:, i].astype(np.float64), g4["quat_r"][:, i].astype(np.float64))
        assert np.allclose(R4[3], [0, 0, 0, 1], atol=1e-7) and np.allclose(R4[:3, 3], 0, atol=1e-7)
    a = oracle.render(sg.Scene(sg.empty_3d(), g4), v)["img"]
    b = oracle.render(sg.Scene(g3, sg.empty_4d()), v)["img"]
    # float32 storage of q3 and of the block-diagonal q_r limit the agreement
    assert np.abs(a - b).max() < 2e-5
    # the rendering of the 4D set does not depend on time any more
    a2 = oracle.render(sg.Scene(sg.empty_3d(), g4), v.with_time(0.11))["img"]
    assert np.abs(a - a2).max() < 1e-12


def test_tilted_4d_gaussian_moves_with_constant_velocity():
    _, g4 = _static_pair(n=5, tilt=True)
    sc = sg.Scene(sg.empty_3d(), g4)
    for i in range(5):
        _, _, R4 = oracle.rot4(g4["quat_l"][:, i].astype(np.float64), g4["quat_r"][:, i].astype(np.float64))
        vel = R4[:3, 3] / R4[3, 3]
        m0, _, _ = oracle.world(sc, i, 0.2)
        m1, _, _ = oracle.world(sc, i, 0.7)
        # with the temporal scale dominating, mu(t) moves along R4[:3,3] / R4[3,3]
        assert np.allclose((m1 - m0) / 0.5, vel, rtol=1e-6, atol=1e-8)
