"""Training loop of the hybrid 3D/4D model on the library's entry points
(Sec. 4.3): a warm-up with the model as given (all-4D at the start), then,
every `interval` iterations up to `densify_until`, a densification stage that
densifies and prunes the 3D and the 4D set separately and re-runs the static
identification (Sec. 4.1-4.2), which moves 4D Gaussians whose temporal scale
exceeds tau into the 3D set.  Every iteration renders the step's views,
takes the L1 loss gradient, runs the backward with the per-Gaussian
statistics and applies Adam with separate learning rates for the 3D and the
4D parameter groups, updating only the Gaussians the step's views see.

This module sequences library calls and holds tensors; every per-element
step runs inside the library.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from . import _lib as L
from .render import G3_KEYS, Rasterizer, adam_step, convert_static, densify, g4_keys, l1_loss_grad, new_stats

# Learning rates per parameter array (the paper does not list its own; these
# are the magnitudes of the 3D Gaussian Splatting lineage it builds on).
LR3 = dict(mean=1.6e-4, log_scale=5e-3, quat=1e-3, opacity=5e-2, sh=2.5e-3)
LR4 = dict(mean=1.6e-4, mean_t=1.6e-4, log_scale=5e-3, quat_l=1e-3, quat_r=1e-3, opacity=5e-2, sh=2.5e-3)


@dataclass
class Schedule:
    """When the densification stages run.  The paper warms up for up to 500
    iterations, then splits and densifies every 100 iterations, densifying up
    to iteration 15,000 (Sec. 4.3, Sec. 5.2); the static identification runs
    at each stage (Sec. 4.1)."""
    warmup: int = 500
    interval: int = 100
    densify_until: int = 15000
    tau: float = 0.5

    def stage_at(self, it: int) -> bool:
        """Whether iteration `it` (1-based) ends with a densification stage."""
        return self.warmup <= it <= self.densify_until and (it - self.warmup) % self.interval == 0


@dataclass
class DensifyLimits:
    """Clone / split / prune limits of one set (3D Gaussian Splatting's
    defaults; the scene extent sets the size limits)."""
    grad_threshold: float = 2e-4
    split_n: int = 2
    dense_fraction: float = 0.01      # clone below, split above this fraction of the extent
    min_opacity: float = 0.005
    max_fraction: float = float("inf")  # prune above this fraction of the extent (inf: off)

    def params(self, extent: float) -> L.DensifyParams:
        big = math.log(self.max_fraction * extent) if math.isfinite(self.max_fraction) else float("inf")
        return L.DensifyParams(self.grad_threshold, self.split_n, math.log(self.dense_fraction * extent),
                               math.log(self.min_opacity / (1.0 - self.min_opacity)), big,
                               math.log(0.8 * self.split_n))


@dataclass
class StageReport:
    it: int
    n3_in: int
    n4_in: int
    n3_densified: int
    n4_densified: int
    n3_out: int
    n4_out: int


class Trainer:
    """Owns the parameters, gradients, Adam moments and statistics of both
    sets (float32 CUDA tensors, the library's layout)."""

    def __init__(self, g3: dict, g4: dict, extent: float, schedule: Schedule = None, lr3: dict = None,
                 lr4: dict = None, limits3: DensifyLimits = None, limits4: DensifyLimits = None, seed: int = 0,
                 rast: Rasterizer = None, masked: bool = True):
        self.g3 = {k: g3[k].contiguous() for k in G3_KEYS}
        self.g4 = {k: g4[k].contiguous() for k in g4_keys(g4)}
        self.extent = float(extent)
        self.schedule = schedule or Schedule()
        self.lr3, self.lr4 = dict(lr3 or LR3), dict(lr4 or LR4)
        self.limits3, self.limits4 = limits3 or DensifyLimits(), limits4 or DensifyLimits()
        self.rast = rast or Rasterizer(batched=True)
        self.masked = masked
        self.gen = torch.Generator(device="cuda")
        self.gen.manual_seed(seed)
        self.it = 0
        self.stages = []
        self._alloc_state(zero_moments=True)

    # -- buffers -------------------------------------------------------------------
    @property
    def n3(self) -> int:
        return int(self.g3["opacity"].numel())

    @property
    def n4(self) -> int:
        return int(self.g4["opacity"].numel())

    def _alloc_state(self, zero_moments: bool):
        self.gr3 = {k: torch.empty_like(v) for k, v in self.g3.items()}
        self.gr4 = {k: torch.empty_like(v) for k, v in self.g4.items()}
        if zero_moments:
            self.m3 = {k: torch.zeros_like(v) for k, v in self.g3.items()}
            self.v3 = {k: torch.zeros_like(v) for k, v in self.g3.items()}
            self.m4 = {k: torch.zeros_like(v) for k, v in self.g4.items()}
            self.v4 = {k: torch.zeros_like(v) for k, v in self.g4.items()}
        self.st3, self.st4 = new_stats(self.n3, self.n4)

    def _groups(self):
        """Per parameter array: (param, grad, m, v, lr, visibility mask)."""
        out = []
        for g, gr, m, v, lr, st in ((self.g3, self.gr3, self.m3, self.v3, self.lr3, self.st3),
                                    (self.g4, self.gr4, self.m4, self.v4, self.lr4, self.st4)):
            for k in g:
                if g[k].numel():
                    # the colour's time coefficients train at the SH rate
                    rate = lr.get(k, lr["sh"])
                    out.append((g[k], gr[k], m[k], v[k], rate, st["step_visible"] if self.masked else None))
        return out

    # -- one iteration ---------------------------------------------------------------
    def step(self, views, targets) -> torch.Tensor:
        """Render `views`, L1 loss against `targets`, backward, Adam; then a
        densification stage when the schedule says so.  Returns the loss
        (a 1-element CUDA tensor; not synchronised)."""
        self.it += 1
        rast = self.rast
        h = rast.forward(self.g3, self.g4, views)
        dls = [torch.empty_like(t) for t in targets]
        loss = torch.zeros(1, device="cuda")
        l1_loss_grad(rast, h.images, targets, views, dls, loss)
        rast.backward(h, self.g3, self.g4, dls, out=(self.gr3, self.gr4), stats=(self.st3, self.st4))
        grp = self._groups()
        if grp:
            adam_step(rast, [x[0] for x in grp], [x[1] for x in grp], [x[2] for x in grp], [x[3] for x in grp],
                      [x[4] for x in grp], self.it, masks=[x[5] for x in grp] if self.masked else None)
        if self.schedule.stage_at(self.it):
            self.stage()
        return loss

    def stage(self) -> StageReport:
        """Densify and prune each set, then move the static 4D Gaussians to
        the 3D set; the moments follow their rows (zero for new rows and new
        quaternions) and the statistics restart."""
        n3_in, n4_in = self.n3, self.n4
        ns = (self.limits3.split_n, 3, n3_in)
        nf = (self.limits4.split_n, 4, n4_in)
        noise3 = torch.randn(ns, generator=self.gen, device="cuda")
        noise4 = torch.randn(nf, generator=self.gen, device="cuda")
        g3, g4, _, _, moved = densify(self.rast, self.g3, self.g4, self.st3, self.st4, noise3, noise4,
                                      self.limits3.params(self.extent), self.limits4.params(self.extent),
                                      moments=[(self.m3, self.m4), (self.v3, self.v4)])
        (m3, m4), (v3, v4) = moved
        n3_d, n4_d = int(g3["opacity"].numel()), int(g4["opacity"].numel())
        g3, g4, _, moved = convert_static(self.rast, g3, g4, self.schedule.tau, moments=[(m3, m4), (v3, v4)])
        (self.m3, self.m4), (self.v3, self.v4) = moved
        self.g3, self.g4 = g3, g4
        self._alloc_state(zero_moments=False)
        rep = StageReport(self.it, n3_in, n4_in, n3_d, n4_d, self.n3, self.n4)
        self.stages.append(rep)
        return rep
