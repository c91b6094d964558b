"""Launch-configuration autotuner: picks the tile edge and the number of list
entries staged in LDS per round (the chunk) for a workload, by timing its
training step (forward, L1 loss gradient, adjoint) under every supported pair.

Images do not depend on either knob (a pixel's contributors are fixed by its
own pixel square and alpha tests, not by the tiling), so the choice changes
speed only.  Picks are cached per workload key: device architecture, the
multiset of image sizes, the 3D and 4D Gaussian counts rounded up to powers
of two, the view count and the batched flag; the cache can be kept in a JSON
file between runs.
"""
from __future__ import annotations

import json
import os

import torch

from ._lib import H4D_ERR_CAPACITY, H4DError
from .render import Rasterizer, l1_loss_grad

# every (tile, chunk) pair the blending kernels are built for
CANDIDATES = tuple((t, c) for t in (8, 16, 32) for c in (64, 128, 256, 512))


def _pow2_bucket(n: int) -> int:
    return 0 if n <= 0 else 1 << (int(n) - 1).bit_length()


def workload_key(arch: str, n3: int, n4: int, sizes, batched: bool) -> str:
    """Cache key of a workload: architecture, Gaussian-count buckets, sorted
    image sizes (with multiplicity), view count, batched flag."""
    dims = ",".join(f"{w}x{h}" for w, h in sorted((int(w), int(h)) for w, h in sizes))
    return f"{arch}|n3<={_pow2_bucket(n3)}|n4<={_pow2_bucket(n4)}|views={len(sizes)}|{dims}|batched={int(bool(batched))}"


def _arch() -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return str(getattr(props, "gcnArchName", props.name)).split(":")[0]


class Autotuner:
    """``pick(g3, g4, views, batched)`` returns the fastest (tile, chunk) for
    the workload, timing each candidate once per key (a candidate the library
    rejects for the workload, e.g. for its tile-list capacity, is skipped).
    ``candidates`` restricts the pairs tried.  ``timer`` (for tests) replaces
    the measurement: ``timer(tile, chunk) -> ms``."""

    def __init__(self, cache_file: str | None = None, steps: int = 3, warmup: int = 1,
                 candidates=CANDIDATES, timer=None):
        self.cache_file = cache_file
        self.steps, self.warmup = int(steps), int(warmup)
        self.candidates = tuple(candidates)
        self.timer = timer
        self.cache: dict = {}
        self.last_timings: dict = {}
        if cache_file and os.path.exists(cache_file):
            with open(cache_file) as fh:
                self.cache = {k: tuple(v) for k, v in json.load(fh).items()}

    def key(self, g3: dict, g4: dict, views, batched: bool, arch: str | None = None) -> str:
        n3 = int(g3["opacity"].shape[0])
        n4 = int(g4["opacity"].shape[0])
        return workload_key(arch if arch is not None else _arch(), n3, n4,
                            [(v.width, v.height) for v in views], batched)

    def pick(self, g3: dict, g4: dict, views, batched: bool = True, arch: str | None = None) -> tuple:
        k = self.key(g3, g4, views, batched, arch)
        if k in self.cache:
            return self.cache[k]
        timings = {}
        for tile, chunk in self.candidates:
            try:
                if self.timer is not None:
                    timings[(tile, chunk)] = float(self.timer(tile, chunk))
                else:
                    timings[(tile, chunk)] = self.measure(tile, chunk, g3, g4, views, batched)
            except H4DError:
                # a configuration the library rejects for this workload (its
                # tile-list slots beyond the capacity limit)
                timings[(tile, chunk)] = float("inf")
                if self.timer is None:
                    torch.cuda.empty_cache()
        feasible = {tc: ms for tc, ms in timings.items() if ms != float("inf")}
        if not feasible:
            raise H4DError(H4D_ERR_CAPACITY, "no launch configuration fits this workload")
        best = min(feasible, key=lambda tc: (feasible[tc], tc))
        self.last_timings = timings
        self.cache[k] = best
        if self.cache_file:
            tmp = self.cache_file + ".tmp"
            with open(tmp, "w") as fh:
                json.dump({kk: list(v) for kk, v in self.cache.items()}, fh, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_file)
        return best

    def measure(self, tile: int, chunk: int, g3: dict, g4: dict, views, batched: bool) -> float:
        """Milliseconds per training step of the workload under (tile, chunk):
        warm-up steps with eager capacity checks (they size the workspace), then
        ``steps`` timed steps with the check deferred to their end."""
        views = list(views)
        rast = Rasterizer(tile=tile, chunk=chunk, batched=batched)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(0)
        targets = [torch.rand((3, v.height, v.width), generator=gen, device="cuda") for v in views]
        dls = [torch.empty_like(t) for t in targets]
        gr3 = {k: torch.empty_like(v) for k, v in g3.items()}
        gr4 = {k: torch.empty_like(v) for k, v in g4.items()}

        def step():
            h = rast.forward(g3, g4, views)
            l1_loss_grad(rast, h.images, targets, views, dls, None)
            rast.backward(h, g3, g4, dls, out=(gr3, gr4))

        for _ in range(max(1, self.warmup)):
            step()
        torch.cuda.synchronize()
        rast.check_mode = "deferred"
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(self.steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        rast.verify()
        ms = e0.elapsed_time(e1) / self.steps
        del rast, targets, dls, gr3, gr4
        torch.cuda.empty_cache()
        return ms
