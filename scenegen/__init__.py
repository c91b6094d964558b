"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws random numbers and builds pinhole cameras.  It holds none
of the rasterizer's arithmetic (no activation, rotation, slicing, projection or
compositing), so both the FP64 oracle and the HIP path can consume its arrays
without sharing any of the method's code.

Layouts (all float32, structure-of-arrays, component-major, i.e. ``a[c, i]``):

* static 3D set   : mean[3,n], log_scale[3,n], quat[4,n] (w,x,y,z),
                    opacity[n] (logit), sh[48,n] (coefficient-major: row k*3+ch)
* dynamic 4D set  : mean[3,n], mean_t[n], log_scale[4,n] (x,y,z,t),
                    quat_l[4,n] (a,b,c,d), quat_r[4,n] (p,q,r,s), opacity[n], sh[48,n]

The distributions stand in for the paper's data (Neural 3D Video: 1352x1014
frames, 18-21 cameras, 300 frames per 10 s clip, a few hundred thousand points at
initialisation; Sec. 5.1 and Sec. 5.2).  None of that data is used or reproduced.

Draw order per set is fixed: means, mean_t, spatial log-scales, temporal
log-scale, quaternion(s), opacity, SH.  The 4D set is drawn before the 3D set.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SH_COEFFS = 16  # degree 3
SH_ROWS = SH_COEFFS * 3


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _unit_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.normal(0.0, 1.0, size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def draw_4d(rng: np.random.Generator, n: int, box: float, *, static_fraction: float = 0.0,
            tau: float = 0.5) -> dict:
    """Dynamic (4D) Gaussians.  ``static_fraction`` of the rows get a temporal
    log-scale just above ln(tau) (these are the rows a static/dynamic split would
    convert); the rest get N(-2, 0.5)."""
    mean = rng.uniform(-box, box, size=(3, n))
    mean_t = rng.uniform(0.0, 1.0, size=n)
    ls_xyz = rng.normal(-3.0, 0.5, size=(3, n))
    ls_t = rng.normal(-2.0, 0.5, size=n)
    if static_fraction > 0.0:
        k = int(round(static_fraction * n))
        hi = math.log(tau) + 0.5 + rng.normal(0.0, 0.2, size=k)
        hi = np.maximum(hi, math.log(tau) + 0.05)
        ls_t[:k] = hi
    ql = _unit_quats(rng, n)
    qr = _unit_quats(rng, n)
    opacity = rng.normal(0.0, 1.0, size=n)
    sh = rng.normal(0.0, 0.3, size=(SH_ROWS, n))
    return dict(mean=_f32(mean), mean_t=_f32(mean_t), log_scale=_f32(np.vstack([ls_xyz, ls_t[None]])),
                quat_l=_f32(ql), quat_r=_f32(qr), opacity=_f32(opacity), sh=_f32(sh))


def draw_3d(rng: np.random.Generator, n: int, box: float) -> dict:
    mean = rng.uniform(-box, box, size=(3, n))
    ls = rng.normal(-3.0, 0.5, size=(3, n))
    q = _unit_quats(rng, n)
    opacity = rng.normal(0.0, 1.0, size=n)
    sh = rng.normal(0.0, 0.3, size=(SH_ROWS, n))
    return dict(mean=_f32(mean), log_scale=_f32(ls), quat=_f32(q), opacity=_f32(opacity), sh=_f32(sh))


def empty_3d() -> dict:
    return dict(mean=np.zeros((3, 0), np.float32), log_scale=np.zeros((3, 0), np.float32),
                quat=np.zeros((4, 0), np.float32), opacity=np.zeros(0, np.float32),
                sh=np.zeros((SH_ROWS, 0), np.float32))


def empty_4d() -> dict:
    return dict(mean=np.zeros((3, 0), np.float32), mean_t=np.zeros(0, np.float32),
                log_scale=np.zeros((4, 0), np.float32), quat_l=np.zeros((4, 0), np.float32),
                quat_r=np.zeros((4, 0), np.float32), opacity=np.zeros(0, np.float32),
                sh=np.zeros((SH_ROWS, 0), np.float32))


@dataclass
class View:
    """Pinhole camera + timestamp.  ``world_to_cam`` is the row-major 3x4 [R|t]
    mapping world points to camera coordinates (x right, y down, z forward)."""
    world_to_cam: np.ndarray  # (3,4) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    t: float
    bg: tuple = (0.0, 0.0, 0.0)

    def with_time(self, t: float) -> "View":
        return View(self.world_to_cam.copy(), self.fx, self.fy, self.cx, self.cy, self.width,
                    self.height, float(t), self.bg)

    def as_f32(self) -> np.ndarray:
        """Flat float32 record: R(9) t(3) fx fy cx cy t bg(3)."""
        R = self.world_to_cam[:, :3].reshape(-1)
        tr = self.world_to_cam[:, 3]
        return _f32(np.concatenate([R, tr, [self.fx, self.fy, self.cx, self.cy, self.t], list(self.bg)]))


def look_at(eye, target, width: int, height: int, fov_x_deg: float = 60.0, t: float = 0.5,
            bg=(0.0, 0.0, 0.0)) -> View:
    """Camera at ``eye`` looking at ``target`` with world up = +y; horizontal field
    of view ``fov_x_deg``; square pixels (fy = fx); principal point at the centre."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    down = np.array([0.0, -1.0, 0.0])
    r = np.cross(down, f)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])  # rows: camera axes in world coordinates
    tr = -R @ eye
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    M = np.concatenate([R, tr[:, None]], axis=1)
    return View(_f32(M), float(np.float32(fx)), float(np.float32(fx)), width / 2.0, height / 2.0,
                int(width), int(height), float(np.float32(t)), tuple(float(np.float32(b)) for b in bg))


def arc_cameras(n_cams: int, width: int, height: int, radius: float = 5.0, arc_len: float = 1.0,
                focal_scale: float = 1.0) -> list:
    """``n_cams`` cameras on a horizontal arc of the given radius about the
    origin, total arc length ``arc_len``, centred on the -z axis, all looking at
    the origin."""
    total = arc_len / radius
    cams = []
    for i in range(n_cams):
        a = -0.5 * total + (total * i / (n_cams - 1) if n_cams > 1 else 0.5 * total)
        eye = (radius * math.sin(a), 0.0, -radius * math.cos(a))
        v = look_at(eye, (0.0, 0.0, 0.0), width, height)
        if focal_scale != 1.0:
            v.fx = float(np.float32(v.fx * focal_scale))
            v.fy = float(np.float32(v.fy * focal_scale))
        cams.append(v)
    return cams


@dataclass
class Scene:
    g3: dict
    g4: dict
    views: list = field(default_factory=list)
    name: str = ""
    time_period: float = 1.0  # period of the 4D colour's cosine terms (g4["sh_t"], when present)

    @property
    def n3(self) -> int:
        return int(self.g3["opacity"].shape[0])

    @property
    def n4(self) -> int:
        return int(self.g4["opacity"].shape[0])


def frame_times(n_frames: int = 300) -> np.ndarray:
    return (np.arange(n_frames) + 0.5) / n_frames


# ---------------------------------------------------------------------------
# The five workload shapes.
# ---------------------------------------------------------------------------

def tiny_scene(n3: int = 1000, n4: int = 1000, width: int = 128, height: int = 96, t: float = 0.5,
               seed: int = 0, box: float = 1.0) -> Scene:
    """2,000 Gaussians (1,000 static + 1,000 dynamic) in U[-1,1]^3, one 128x96
    camera at (0,0,-3) looking at the origin (fov 60 deg), t = 0.5."""
    rng = np.random.default_rng(seed)
    g4 = draw_4d(rng, n4, box)
    g3 = draw_3d(rng, n3, box)
    view = look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), width, height, t=t)
    return Scene(g3, g4, [view], name=f"tiny_{n3}x3d_{n4}x4d_{width}x{height}")


def multiview_scene(n_total: int = 250_000, frac_3d: float = 0.7, width: int = 1352, height: int = 1014,
                    seed: int = 0, n_cams: int = 20) -> Scene:
    """250k Gaussians (70 % static) in a 4 m box, 20 cameras on a 1 m arc of
    radius 5 m, 1352x1014 pixels."""
    rng = np.random.default_rng(seed)
    n3 = int(round(n_total * frac_3d))
    n4 = n_total - n3
    g4 = draw_4d(rng, n4, 2.0)
    g3 = draw_3d(rng, n3, 2.0)
    return Scene(g3, g4, arc_cameras(n_cams, width, height), name=f"multiview_{n_total}")


def hybrid_ratio_scene(static_fraction: float, n_total: int = 500_000, width: int = 1352,
                       height: int = 1014, seed: int = 0, tau: float = 0.5) -> Scene:
    """500k Gaussians generated all-4D; ``static_fraction`` of them carry a
    temporal scale above tau (candidates for the static conversion)."""
    rng = np.random.default_rng(seed)
    g4 = draw_4d(rng, n_total, 2.0, static_fraction=static_fraction, tau=tau)
    return Scene(empty_3d(), g4, arc_cameras(20, width, height), name=f"hybrid_{static_fraction}")


def batched_scene(n_total: int = 1_000_000, frac_3d: float = 0.8, seed: int = 0) -> Scene:
    """1M Gaussians (80 % static); 8 cameras on the arc, cameras 0-3 at
    1352x1014 and 4-7 at 2704x2028 (focal length doubled)."""
    rng = np.random.default_rng(seed)
    n3 = int(round(n_total * frac_3d))
    g4 = draw_4d(rng, n_total - n3, 2.0)
    g3 = draw_3d(rng, n3, 2.0)
    lo = arc_cameras(8, 1352, 1014)
    hi = arc_cameras(8, 2704, 2028)
    views = lo[:4] + hi[4:]
    return Scene(g3, g4, views, name="batched_1M")


def batched_views(scene: Scene, times=(0.125, 0.375, 0.625, 0.875)) -> list:
    """8 cameras x 4 timestamps = 32 views (camera-major)."""
    return [v.with_time(t) for v in scene.views for t in times]


def training_scene(n_total: int = 2_000_000, frac_3d: float = 0.85, seed: int = 0) -> Scene:
    rng = np.random.default_rng(seed)
    n3 = int(round(n_total * frac_3d))
    g4 = draw_4d(rng, n_total - n3, 2.0)
    g3 = draw_3d(rng, n3, 2.0)
    return Scene(g3, g4, arc_cameras(20, 2704, 2028), name="training_2M")


def view_schedule(scene: Scene, steps: int, views_per_step: int = 1, seed: int = 2,
                  n_frames: int = 300) -> list:
    """Per step, ``views_per_step`` (camera, frame time) pairs drawn from the
    cameras x frames grid."""
    rng = np.random.default_rng(seed)
    times = frame_times(n_frames)
    out = []
    for _ in range(steps):
        cams = rng.integers(0, len(scene.views), size=views_per_step)
        frames = rng.integers(0, n_frames, size=views_per_step)
        out.append([scene.views[int(c)].with_time(float(times[int(f)])) for c, f in zip(cams, frames)])
    return out


def target_images(views: list, seed: int = 1) -> list:
    rng = np.random.default_rng(seed)
    return [_f32(rng.uniform(0.0, 1.0, size=(3, v.height, v.width))) for v in views]


def upstream_grads(views: list, seed: int = 3, scale: float = 1.0) -> list:
    """Random dL/dC images used to compare backward passes on identical inputs."""
    rng = np.random.default_rng(seed)
    return [_f32(scale * rng.normal(0.0, 1.0, size=(3, v.height, v.width))) for v in views]


def param_tangents(scene: Scene, seed: int = 4) -> tuple:
    """Random float64 tangent directions shaped like every parameter array."""
    rng = np.random.default_rng(seed)
    t4 = {k: rng.normal(0.0, 1.0, size=v.shape) for k, v in scene.g4.items()}
    t3 = {k: rng.normal(0.0, 1.0, size=v.shape) for k, v in scene.g3.items()}
    return t3, t4


def raw_quaternion_norms(scene: Scene, seed: int = 6, lo: float = 0.5, hi: float = 2.0) -> Scene:
    """The same scene with every quaternion column (q of the 3D set, q_l and
    q_r of the 4D set) multiplied by its own factor drawn from U[lo, hi].  The
    rasterizer takes raw quaternions and normalises them itself, so the
    rendered scene is the same up to rounding, while the normalisation and its
    adjoint (the 1/|q| factor) are exercised; training moves quaternions off the
    unit sphere after the first optimiser step."""
    rng = np.random.default_rng(seed)
    g3 = dict(scene.g3)
    g4 = dict(scene.g4)
    for d, keys in ((g4, ("quat_l", "quat_r")), (g3, ("quat",))):
        for k in keys:
            q = d[k].astype(np.float64)
            d[k] = _f32(q * rng.uniform(lo, hi, size=(1, q.shape[1])))
    return Scene(g3, g4, list(scene.views), name=scene.name + "_raw_quats", time_period=scene.time_period)


def with_time_colour(scene: Scene, degree: int = 1, seed: int = 7, sigma: float = 0.3,
                     period: float = 1.0) -> Scene:
    """The same scene whose 4D Gaussians also carry time coefficients of
    their colour, g4["sh_t"] = [48 degree][n4] ~ N(0, sigma) (the cosine terms
    of 4D Gaussian splatting's colour model), with the given period."""
    rng = np.random.default_rng(seed)
    g4 = dict(scene.g4)
    g4["sh_t"] = _f32(rng.normal(0.0, sigma, size=(48 * degree, scene.n4)))
    return Scene(dict(scene.g3), g4, list(scene.views), name=scene.name + f"_time_colour{degree}",
                 time_period=float(period))


def subset(scene: Scene, idx3, idx4) -> Scene:
    g3 = {k: np.ascontiguousarray(v[..., idx3]) for k, v in scene.g3.items()}
    g4 = {k: np.ascontiguousarray(v[..., idx4]) for k, v in scene.g4.items()}
    return Scene(g3, g4, list(scene.views), name=scene.name + "_subset", time_period=scene.time_period)


def synthetic_records(n: int, width: int, height: int, seed: int = 5, max_radius: int = 60) -> dict:
    """Screen-space splat records (as a projection stage would emit them) for
    testing the binning/sorting/compositing stages on identical inputs:
    integer-part/fraction-split centres, conic, effective opacity, colour,
    integer radius, float32 depth (with deliberate exact ties) and a
    visibility flag."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.1 * width, 1.1 * width, size=n)
    v = rng.uniform(-0.1 * height, 1.1 * height, size=n)
    sx = np.exp(rng.uniform(np.log(0.7), np.log(max_radius / 3.0), size=n))
    sy = sx * np.exp(rng.uniform(-0.7, 0.7, size=n))
    th = rng.uniform(0, np.pi, size=n)
    c, s = np.cos(th), np.sin(th)
    # a random symmetric positive-definite quadratic form with axes sx, sy
    ia, ib = 1.0 / (sx * sx), 1.0 / (sy * sy)
    qa = c * c * ia + s * s * ib
    qb = c * s * (ia - ib)
    qc = s * s * ia + c * c * ib
    radius = np.ceil(3.0 * np.maximum(sx, sy)).astype(np.int64) + rng.integers(0, 3, size=n)
    depth = rng.uniform(0.5, 8.0, size=n)
    # a few exact depth ties so the id tie-break is exercised
    k = max(1, n // 50)
    depth[rng.integers(0, n, size=k)] = depth[rng.integers(0, n, size=k)]
    opac = 1.0 / (1.0 + np.exp(-rng.normal(0.5, 1.0, size=n)))
    rgb = rng.uniform(0.0, 1.0, size=(3, n))
    visible = (rng.uniform(size=n) > 0.05).astype(np.uint8)
    return dict(u=_f32(u), v=_f32(v), conic=_f32(np.stack([qa, qb, qc])),
                opacity=_f32(opac), rgb=_f32(rgb), radius=radius.astype(np.int32),
                depth=_f32(depth), visible=visible)
