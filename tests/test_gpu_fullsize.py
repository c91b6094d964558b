"""Parity at the training-step workload: 250k Gaussians (70 % static 3D, 30 %
dynamic 4D), 1352x1014 images, in the launch configuration the step is timed
in (default tile and chunk), through the C ABI.

Three independent checks per view: the whole image against the oracle's tile
pipeline, sampled pixels (corners, the ragged last tile row and column, random
ones) against the oracle's per-pixel brute force over all Gaussians, and the
full backward to every raw parameter.  At the 2M-Gaussian training workload
(4 views at 2704x2028): sampled pixels against the brute force, and the
4-view adjoint against the sum of one-view adjoints.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg
from parity_util import check_grads, check_image, mask_flagged, sample_pixels, GRAD_TOL, IMG_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h4d():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_13215_amd as m
    m._lib.load()
    return m


@pytest.fixture(scope="module")
def big():
    scene = sg.multiview_scene()
    sched = sg.view_schedule(scene, 4, 1, seed=2)
    return scene, [s[0] for s in sched]


@pytest.fixture(scope="module")
def gpu_params(h4d, big):
    scene, _ = big
    return h4d.to_device(scene.g3), h4d.to_device(scene.g4)


_sample_pixels = sample_pixels


@pytest.mark.parametrize("k", [0, 1])
def test_full_size_forward(h4d, big, gpu_params, k):
    scene, views = big
    v = views[k]
    print(f"[full-size forward] view {k}: t={v.t:.4f}", flush=True)
    g3, g4 = gpu_params
    rast = h4d.Rasterizer()
    h = rast.forward(g3, g4, [v])
    img = h.images[0].cpu().numpy()
    ref = oracle.render(scene, v)
    err = check_image(img, ref["img"], ref["amb"])
    print(f"  whole image: max err {err:.2e}, flagged {ref['amb'].mean():.2e}", flush=True)
    xs, ys = _sample_pixels(v.width, v.height, 400, seed=k)
    rgb, T, amb = oracle.pixels(scene, v, xs, ys)
    ok = ~amb
    got = img[:, ys, xs].T
    assert np.abs(got - rgb)[ok].max() <= IMG_TOL
    # the tile pipeline and the brute force agree with each other exactly in FP64
    assert np.abs(ref["img"][:, ys, xs].T - rgb)[ok].max() <= 1e-12


def test_full_size_backward(h4d, big, gpu_params):
    scene, views = big
    v = views[2]
    print(f"[full-size backward] t={v.t:.4f}", flush=True)
    g3, g4 = gpu_params
    ref = oracle.render(scene, v)
    target = sg.target_images([v], seed=7)[0]
    # L1 gradient with the sign taken from the oracle image: both sides get the same dL/dC
    dl = (np.sign(ref["img"] - target) / (3 * v.width * v.height)).astype(np.float32)
    dl = mask_flagged(dl, ref["amb"])
    rast = h4d.Rasterizer()
    h = rast.forward(g3, g4, [v])
    gr3, gr4 = rast.backward(h, g3, g4, [torch.as_tensor(dl, device="cuda")])
    torch.cuda.synchronize()
    r3, r4 = oracle.render_bwd(scene, [v], [dl])
    check_grads(scene, gr3, gr4, r3, r4, np.zeros(scene.n3 + scene.n4, bool))


def test_full_size_repeated_steps_are_stable(h4d, big, gpu_params):
    """Deferred capacity checks over consecutive views (the timed loop's mode)
    give the same images as eager renders."""
    scene, views = big
    g3, g4 = gpu_params
    eager = h4d.Rasterizer()
    refs, peak = [], 0
    for v in views:
        refs.append(eager.forward(g3, g4, [v]).images[0].clone())
        peak = max(peak, eager.last_pairs)
    rast = h4d.Rasterizer(pair_capacity=int(peak * 1.5), check="deferred")
    for v, r in zip(views, refs):
        img = rast.forward(g3, g4, [v]).images[0]
        rast.verify()
        assert torch.equal(img, r)


# -- the 2M-Gaussian training workload ---------------------------------------

@pytest.fixture(scope="module")
def train2m(h4d):
    """2M Gaussians (85 % static 3D), 2704x2028 images, a batch of 4 views."""
    scene = sg.training_scene()
    views = sg.view_schedule(scene, 1, 4, seed=3)[0]
    return scene, views, h4d.to_device(scene.g3), h4d.to_device(scene.g4)


def test_training_workload_sampled_pixels(h4d, train2m):
    """The 4-view call at the training workload's size: sampled pixels of every
    view (corners, the ragged last tile row and column, random ones) against
    the oracle's per-pixel brute force over all 2M Gaussians."""
    scene, views, g3, g4 = train2m
    print("[2M training workload] forward, 4 views at 2704x2028", flush=True)
    rast = h4d.Rasterizer()
    h = rast.forward(g3, g4, views)
    torch.cuda.synchronize()
    assert rast.last_pairs > 0
    for k, v in enumerate(views):
        img = h.images[k].cpu().numpy()
        xs, ys = _sample_pixels(v.width, v.height, 200, seed=10 + k)
        rgb, T, amb = oracle.pixels(scene, v, xs, ys)
        ok = ~amb
        assert ok.mean() > 0.9
        got = img[:, ys, xs].T
        assert np.abs(got - rgb)[ok].max() <= IMG_TOL, k


def test_training_workload_gradients_are_view_sums(h4d, train2m):
    """The 4-view backward equals the sum of the four one-view backwards (the
    adjoint is linear in dL/dC and the views share no state), compared
    normwise per parameter array since the float32 atomic sums run in another
    order."""
    scene, views, g3, g4 = train2m
    print("[2M training workload] backward, 4 views vs one at a time", flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    dls = [torch.randn((3, v.height, v.width), generator=gen, device="cuda") * 1e-4 for v in views]
    rast = h4d.Rasterizer()
    h = rast.forward(g3, g4, views)
    a3, a4 = rast.backward(h, g3, g4, dls)
    s3 = {k: torch.zeros_like(x) for k, x in a3.items()}
    s4 = {k: torch.zeros_like(x) for k, x in a4.items()}
    for v, d in zip(views, dls):
        h1 = rast.forward(g3, g4, [v])
        b3, b4 = rast.backward(h1, g3, g4, [d])
        for k in s3:
            s3[k] += b3[k]
        for k in s4:
            s4[k] += b4[k]
    torch.cuda.synchronize()
    assert float(a3["opacity"].norm()) > 0 and float(a4["opacity"].norm()) > 0
    for k in a3:
        assert float((a3[k] - s3[k]).norm()) <= 1e-5 * float(a3[k].norm()) + 1e-30, k
    for k in a4:
        assert float((a4[k] - s4[k]).norm()) <= 1e-5 * float(a4[k].norm()) + 1e-30, k


# -- raw quaternions and the inference render at the training-step workload ---

def test_full_size_raw_quaternions(h4d, big):
    """The 250k scene with every quaternion column scaled by a seeded factor
    in [0.3, 3]: the whole image against the oracle, then the backward of every
    raw parameter (L1 upstream, zeroed at flagged pixels) against the oracle's
    adjoint of the same raw arrays."""
    scene0, views = big
    scene = sg.raw_quaternion_norms(scene0, seed=8, lo=0.3, hi=3.0)
    v = views[3]
    print(f"[full-size raw quaternions] t={v.t:.4f}", flush=True)
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    rast = h4d.Rasterizer()
    h = rast.forward(g3, g4, [v])
    ref = oracle.render(scene, v)
    err = check_image(h.images[0].cpu().numpy(), ref["img"], ref["amb"])
    print(f"  whole image: max err {err:.2e}, flagged {ref['amb'].mean():.2e}", flush=True)
    target = sg.target_images([v], seed=9)[0]
    dl = (np.sign(ref["img"] - target) / (3 * v.width * v.height)).astype(np.float32)
    dl = mask_flagged(dl, ref["amb"])
    gr3, gr4 = rast.backward(h, g3, g4, [torch.as_tensor(dl, device="cuda")])
    torch.cuda.synchronize()
    r3, r4 = oracle.render_bwd(scene, [v], [dl])
    check_grads(scene, gr3, gr4, r3, r4, np.zeros(scene.n3 + scene.n4, bool))


def test_full_size_inference_render_against_oracle(h4d, big, gpu_params):
    """render_infer's whole image at the training-step workload against the
    oracle (the training forward's images are compared with it bit for bit
    elsewhere), and sampled pixels against the per-pixel brute force."""
    scene, views = big
    v = views[1].with_time(0.8)
    print(f"[full-size inference render] t={v.t:.4f}", flush=True)
    g3, g4 = gpu_params
    rast = h4d.Rasterizer()
    img = rast.infer(g3, g4, [v]).images[0].cpu().numpy()
    ref = oracle.render(scene, v)
    check_image(img, ref["img"], ref["amb"])
    xs, ys = _sample_pixels(v.width, v.height, 200, seed=21)
    rgb, T, amb = oracle.pixels(scene, v, xs, ys)
    assert np.abs(img[:, ys, xs].T - rgb)[~amb].max() <= IMG_TOL


# -- the 64-Gaussian gradient check at the 2M-Gaussian training workload ------

def _rows(scene, gr3, gr4, sel):
    """Gradient rows (oracle.ROW4 / ROW3 order) of the selected merged ids."""
    a3 = {k: x.cpu().numpy().astype(np.float64) for k, x in gr3.items()}
    a4 = {k: x.cpu().numpy().astype(np.float64) for k, x in gr4.items()}
    rows = np.zeros((len(sel), 65))
    for s, g in enumerate(sel):
        order, src, i = (oracle.ROW4, a4, g) if g < scene.n4 else (oracle.ROW3, a3, g - scene.n4)
        for k, (name, c) in enumerate(order):
            rows[s, k] = src[name][i] if c is None else src[name][c, i]
    return rows


def test_training_workload_subset_gradients_against_oracle_and_fd(h4d, train2m):
    """Gradient check of the 2M-Gaussian, 4-view training call on a seeded
    subset of 64 Gaussians (32 static 3D, 32 dynamic 4D) drawn among those
    blended at seeded sample pixels of the 4 views whose pixel squares have a
    radius of at most 128 px in every view (the oracle's cost grows with the
    squares' area).  The loss is linear in the
    images, L = sum_v <dl_v, C_v>, with dl_v a seeded upstream gradient scaled
    like the L1 loss's and zeroed at the guard-band pixels of the subset's
    squares.  The oracle evaluates it locally: its adjoint over the pixels in
    the subset's squares, and central differences for two seeded parameter
    entries per Gaussian (moves that change a discrete decision skipped).
    Checks: the oracle's differences against its adjoint (FP64), the GPU's
    gradients of all 64 rows against the oracle's adjoint at the gradient bar
    (per group and per element), and the GPU's gradients against the
    differences themselves."""
    scene, views, g3, g4 = train2m
    V = len(views)
    rng = np.random.default_rng(64)
    cand = set()
    for v in views:
        xs = rng.integers(0, v.width, 128).astype(np.int32)
        ys = rng.integers(0, v.height, 128).astype(np.int32)
        for lst in oracle.blended_at(scene, v, xs, ys, cap=2048):
            cand.update(g for g, w in lst if w > 1e-3)
    cand = np.array(sorted(cand), np.int64)
    # squares of at most 128 px radius in every view keep the local differences affordable
    rmax = np.max([np.where(p["visible"] > 0, p["radius"], 0) for p in (oracle.project(scene, v) for v in views)],
                  axis=0)
    cand = cand[rmax[cand] <= 128]
    c4, c3 = cand[cand < scene.n4], cand[cand >= scene.n4]
    assert len(c4) >= 32 and len(c3) >= 32
    sel = np.sort(np.concatenate([rng.choice(c4, 32, replace=False),
                                  rng.choice(c3, 32, replace=False)])).astype(np.int32)
    print(f"[2M training workload] local oracle over 64 Gaussians, sel[:4]={sel[:4]}", flush=True)
    loc = oracle.Local(scene, views, sel)
    dls = []
    for k, (v, d) in enumerate(zip(views, sg.upstream_grads(views, seed=65))):
        d = (d / (3.0 * v.width * v.height * V)).astype(np.float32)
        d[:, (loc.amb(k) & 2) > 0] = 0.0
        dls.append(d)
    want = loc.grad(dls)
    print("[2M training workload] GPU forward + backward, 4 views", flush=True)
    rast = h4d.Rasterizer()
    h = rast.forward(g3, g4, views)
    gr3, gr4 = rast.backward(h, g3, g4, [torch.as_tensor(d, device="cuda") for d in dls])
    torch.cuda.synchronize()
    got = _rows(scene, gr3, gr4, sel)
    is4 = sel < scene.n4
    # per parameter group over the subset: normwise and per element
    group_rms = {}
    for which, order in ((True, oracle.ROW4), (False, oracle.ROW3)):
        rows_g, rows_w = got[is4 == which], want[is4 == which]
        for name in dict.fromkeys(n for n, _ in order):
            cols = [k for k, (n, _) in enumerate(order) if n == name]
            g, w = rows_g[:, cols], rows_w[:, cols]
            nw = np.linalg.norm(w)
            assert nw > 0, (which, name)
            assert np.linalg.norm(g - w) <= GRAD_TOL * nw, (which, name, np.linalg.norm(g - w) / nw)
            rms = np.sqrt(np.mean(w * w))
            viol = np.abs(g - w) > GRAD_TOL * np.abs(w) + GRAD_TOL * rms
            assert viol.sum() == 0, (which, name, int(viol.sum()))
            group_rms[(which, name)] = rms
    assert len(group_rms) == 12
    # central differences of the oracle, two seeded entries per Gaussian
    ent = [(s, int(k)) for s in range(len(sel))
           for k in rng.choice(65 if is4[s] else 59, 2, replace=False)]
    print(f"[2M training workload] oracle central differences, {len(ent)} entries", flush=True)
    fd, ok = loc.fd(dls, ent, hrel=1e-6)
    assert ok.mean() > 0.8, ok.mean()
    ad = np.array([want[s, k] for s, k in ent])
    gp = np.array([got[s, k] for s, k in ent])
    rowscale = np.array([np.abs(want[s]).max() for s, _ in ent])
    assert np.all(np.abs(fd - ad)[ok] <= 1e-5 * np.abs(ad[ok]) + 1e-7 * rowscale[ok])
    rms = np.array([group_rms[(bool(is4[s]), (oracle.ROW4 if is4[s] else oracle.ROW3)[k][0])] for s, k in ent])
    assert np.all(np.abs(gp - fd)[ok] <= GRAD_TOL * np.abs(fd[ok]) + GRAD_TOL * rms[ok])
