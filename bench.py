"""Training-step throughput of the hybrid 3D/4D rasterizer on one MI355X.

A step is one pass of the whole hot path over one synthetic view: slice the 4D
Gaussians at the view's time, merge with the 3D set, project, bin, sort, blend,
L1 loss gradient, the full backward to every raw parameter and an Adam update
of every parameter.  Workload: 250k Gaussians (70 % static 3D, 30 % dynamic
4D) in a 4 m box, 20 cameras on a 1 m arc, 300 frame times, 1352x1014 images,
one (camera, time) view per step drawn by seed.

Prints ONE JSON line (rank 0).  Usage:
    python bench.py [--gpus 1] [--steps 50] [--warmup 10] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd training-step Mpix/s at 250k–1M Gaussians; batched vs single-view, % HBM peak"

# Algorithmic FP32 operations per (pixel, splat) evaluation of the blending
# kernels (an FMA counts 2): see the design notes for the itemisation.
FLOPS_EVAL = 15          # offset, quadratic form, exp, opacity product, clamp, threshold
FLOPS_BLEND_FWD = 10     # transmittance step, stop test, colour accumulation
FLOPS_BLEND_BWD = 49     # prefix, colour behind, dalpha, nine gradients, transmittance
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector, published
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E, published

# Learning rates per parameter array (the paper does not list its own; the
# 3DGS-lineage magnitudes are used).
LR3 = dict(mean=1.6e-4, log_scale=5e-3, quat=1e-3, opacity=5e-2, sh=2.5e-3)
LR4 = dict(mean=1.6e-4, mean_t=1.6e-4, log_scale=5e-3, quat_l=1e-3, quat_r=1e-3, opacity=5e-2, sh=2.5e-3)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_train_step_250k_1352x1014.md")
# the blending kernels as built: their sources and the compile flags
KERNEL_SOURCES = ("paper_2505_13215_amd/csrc/composite.hip", "paper_2505_13215_amd/csrc/walk.hpp",
                  "paper_2505_13215_amd/csrc/common.hpp",
                  "paper_2505_13215_amd/build.py")


def recorded_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated on a copy of known size), or None when
    the blending sources changed since the counters were taken."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = [ln.split() for ln in fh if ln.strip().startswith("traffic ")]
    except OSError:
        return None
    for parts in lines:
        if len(parts) >= 5 and parts[1] == kernel:
            kv = dict(p.split("=", 1) for p in parts[2:])
            if kv.get("source_sha256") == h.hexdigest():
                return int(kv["fetch_bytes"]) + int(kv["write_bytes"])
    return None


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(scene, views, adam_scalars: int, reps: int = 3) -> dict:
    """The FP64 oracle, as it stands, on a bounded sample of the timed step:
    ``reps`` runs over the given views, each timing the forward and the
    backward of every view and one Adam step over the step's scalars; the
    medians over the runs give the per-step rate (one view, its forward, its
    backward and one Adam step per step)."""
    import oracle
    oracle.build()
    fwd, bwd, adam = [], [], []
    z = np.zeros(adam_scalars, np.float32)
    for _ in range(reps):
        tf = tb = 0.0
        for v in views:
            t0 = time.perf_counter()
            ref = oracle.render(scene, v)
            t1 = time.perf_counter()
            dl = np.sign(ref["img"] - 0.5).astype(np.float32) / (3 * v.width * v.height)
            t2 = time.perf_counter()
            oracle.render_bwd(scene, [v], [dl])
            t3 = time.perf_counter()
            tf += t1 - t0
            tb += t3 - t2
        t0 = time.perf_counter()
        oracle.adam(z, z, z, z, 1e-3, 0.9, 0.999, 1e-8, 1)
        adam.append(time.perf_counter() - t0)
        fwd.append(tf)
        bwd.append(tb)
    f, b, a = float(np.median(fwd)), float(np.median(bwd)), float(np.median(adam))
    nv = len(views)
    pix = sum(v.width * v.height for v in views)
    step = f + b + nv * a
    return {"value": pix / step / 1e6, "unit": "Mpix/s", "cores": oracle.num_threads(), "kind": "oracle",
            "fwd_s_per_view": round(f / nv, 3), "bwd_s_per_view": round(b / nv, 3), "adam_s": round(a, 3),
            "fwd_mpix_s": round(pix / f / 1e6, 4), "bwd_mpix_s": round(pix / b / 1e6, 4),
            "sample": f"{nv} view(s) of 1352x1014 of the 250k-Gaussian scene, median of {reps} runs: FP64 "
                      f"forward, backward and one Adam step over {adam_scalars} scalars per view"}


# Algorithmic HBM bytes of a step (the fixed yardstick: what the method must
# move, not what this implementation moves).
B_PARAM3, B_PARAM4 = 236, 260  # parameter row of a 3D / 4D Gaussian
B_ONSCREEN = 48 + 48 + 36 + 36  # screen record written + read back, 2D gradient accumulator written + read
B_PAIR = 16                     # list entry: emission write (depth + id) and one ordering read
B_TRAVERSED = 40 + 40 + 36      # entry read by the forward, by the adjoint, gradient written
B_PIXEL = 64                    # colour, T, n_contrib written; target, dL/dC, adjoint state read
B_ADAM = 28                     # per scalar: p, g, m, v read; p, m, v written


def alg_bytes(n3: int, n4: int, param_passes: int, cnt: dict, pixels: int) -> dict:
    """param_passes: times the parameter rows are read for the rendering of
    one step (once per view when views are rendered one after another, once
    per step when batched); each step then reads them again in the adjoint and
    writes an equal gradient."""
    params = (B_PARAM3 * n3 + B_PARAM4 * n4) * (param_passes + 2)
    parts = {"params": params, "onscreen": B_ONSCREEN * cnt["onscreen"], "pairs": B_PAIR * cnt["list_entries"],
             "traversed": B_TRAVERSED * cnt["traversed"], "pixels": B_PIXEL * pixels}
    parts["total"] = sum(parts.values())
    return parts


def hbm_entry(bytes_alg: float, seconds: float) -> dict:
    gbs = bytes_alg / seconds / 1e9
    return {"bytes_alg": int(bytes_alg), "achieved_gbs": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4)}


def copy_bandwidth(torch, mib: int = 2048, reps: int = 5) -> float:
    """GB/s (read + write) of a plain device copy on this GPU, median of reps."""
    src = torch.ones((mib << 20) // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) * 1e-3)
    del src, dst
    return round(2 * (mib << 20) / float(np.median(ts)) / 1e9, 1)


def count_step(rast, fn) -> dict:
    """Workload counts of one call of fn (counting variants of the kernels,
    outside any timed region)."""
    rast.stats(True)
    mode = rast.check_mode
    rast.check_mode = "eager"
    fn()
    c = rast.stats_read()
    rast.stats(False)
    rast.check_mode = mode
    return c


def convert_leg(h4d, torch, rast, g3, g4, reps: int = 5) -> dict:
    """Median wall time of convert_static(0.5) (mask, compaction, Eq. 9 on the
    converted rows, copies), which ends in a host read of the two counts."""
    for _ in range(2):
        h4d.convert_static(rast, g3, g4, 0.5)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        o3, o4, _ = h4d.convert_static(rast, g3, g4, 0.5)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return {"ms": round(1e3 * float(np.median(ts)), 4), "n4_in": int(g4["opacity"].numel()),
            "n3_in": int(g3["opacity"].numel()), "n4_out": int(o4["opacity"].numel()),
            "n3_out": int(o3["opacity"].numel())}


def _time_steps(torch, fn, steps: int, warmup: int) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def hybrid_leg(h4d, torch, sg, steps: int, warmup: int) -> dict:
    """The paper's central comparison (Sec. 4): 500k Gaussians generated all-4D
    with a static fraction f of long temporal scales; fwd + L1 + bwd per view
    (1352x1014, one view per step) on the all-4D scene, then after
    convert_static(0.5) on the hybrid 3D/4D scene, same views."""
    out = {"workload": "hybrid_ratio_500k_1352x1014"}
    for f in (0.0, 0.5, 0.9):
        scene = sg.hybrid_ratio_scene(f)
        sched = [v[0] for v in sg.view_schedule(scene, steps + warmup, 1, seed=2)]
        W, H = scene.views[0].width, scene.views[0].height
        rast = h4d.Rasterizer()
        gen = torch.Generator(device="cuda")
        gen.manual_seed(1)
        target = torch.rand((3, H, W), generator=gen, device="cuda")
        dl = torch.empty_like(target)
        row = {}
        g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
        t0 = time.perf_counter()
        o3, o4, _ = h4d.convert_static(rast, g3, g4, 0.5)
        torch.cuda.synchronize()
        row["convert_ms"] = round(1e3 * (time.perf_counter() - t0), 3)
        for name, (a3, a4) in (("all4d", (g3, g4)), ("hybrid", (o3, o4))):
            it = {"i": 0}
            gr = ({k: torch.empty_like(v) for k, v in a3.items()}, {k: torch.empty_like(v) for k, v in a4.items()})
            rast.check_mode = "eager"
            rast.forward(a3, a4, [sched[0]])
            torch.cuda.synchronize()
            rast.capacity = int(rast.last_pairs * 1.5) + 4096
            rast.check_mode = "deferred"

            def step():
                v = sched[it["i"] % len(sched)]
                it["i"] += 1
                h = rast.forward(a3, a4, [v])
                h4d.l1_loss_grad(rast, h.images, [target], [v], [dl], None)
                rast.backward(h, a3, a4, [dl], out=gr)

            dt = _time_steps(torch, step, steps, warmup)
            rast.verify()
            row[name] = {"ms_per_step": round(dt * 1e3, 4), "mpix_s": round(W * H / dt / 1e6, 2),
                         "n3": int(a3["opacity"].numel()), "n4": int(a4["opacity"].numel())}
        row["speedup"] = round(row["all4d"]["ms_per_step"] / row["hybrid"]["ms_per_step"], 3)
        out[f"static_fraction_{f}"] = row
        del g3, g4, o3, o4, rast
        torch.cuda.empty_cache()
    return out


def training_leg(h4d, torch, sg, steps: int, warmup: int) -> dict:
    """2M Gaussians (85 % static), 2704x2028, 4 views per step drawn from 20
    cameras x 300 frame times, all views in one launch per stage (batched):
    fwd + L1 + bwd + Adam over all parameters."""
    scene = sg.training_scene()
    sched = sg.view_schedule(scene, steps + warmup, 4, seed=2)
    W, H = scene.views[0].width, scene.views[0].height
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    n_gauss = scene.n3 + scene.n4
    del scene
    gr3 = {k: torch.empty_like(v) for k, v in g3.items()}
    gr4 = {k: torch.empty_like(v) for k, v in g4.items()}
    keys = [("3", k) for k in h4d.G3_KEYS] + [("4", k) for k in h4d.G4_KEYS]
    params = [(g3 if w == "3" else g4)[k] for w, k in keys]
    grads = [(gr3 if w == "3" else gr4)[k] for w, k in keys]
    ms = [torch.zeros_like(p) for p in params]
    vs = [torch.zeros_like(p) for p in params]
    lrs = [(LR3 if w == "3" else LR4)[k] for w, k in keys]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    targets = [torch.rand((3, H, W), generator=gen, device="cuda") for _ in range(4)]
    dls = [torch.empty_like(t) for t in targets]
    rast = h4d.Rasterizer(batched=True)
    rast.forward(g3, g4, sched[0])
    torch.cuda.synchronize()
    rast.capacity = int(rast.last_pairs * 1.3) + 4096
    rast.check_mode = "deferred"
    it = {"i": 0, "step": 0}

    def step():
        views = sched[it["i"] % len(sched)]
        it["i"] += 1
        h = rast.forward(g3, g4, views)
        h4d.l1_loss_grad(rast, h.images, targets, views, dls, None)
        rast.backward(h, g3, g4, dls, out=(gr3, gr4))
        it["step"] += 1
        h4d.adam_step(rast, params, grads, ms, vs, lrs, it["step"])

    dt = _time_steps(torch, step, steps, warmup)
    rast.verify()
    mpix = 4 * W * H / 1e6

    def counted():
        views = sched[0]
        h = rast.forward(g3, g4, views)
        h4d.l1_loss_grad(rast, h.images, targets, views, dls, None)
        rast.backward(h, g3, g4, dls, out=(gr3, gr4))

    cnt = count_step(rast, counted)
    n3, n4 = int(g3["opacity"].numel()), int(g4["opacity"].numel())
    n_scalars = sum(p.numel() for p in params)
    alg = alg_bytes(n3, n4, 1, cnt, 4 * W * H)
    # the static identification every 500 steps: convert_static(0.5) with the
    # Adam moments moved along, timed on the step's sets and spread over 500 steps
    m3 = {k: ms[i] for i, (w, k) in enumerate(keys) if w == "3"}
    m4 = {k: ms[i] for i, (w, k) in enumerate(keys) if w == "4"}
    v3 = {k: vs[i] for i, (w, k) in enumerate(keys) if w == "3"}
    v4 = {k: vs[i] for i, (w, k) in enumerate(keys) if w == "4"}
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o3, o4, _, moved = h4d.convert_static(rast, g3, g4, 0.5, moments=[(m3, m4), (v3, v4)])
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        del o3, o4, moved
    conv_ms = 1e3 * float(np.median(ts))
    per = dt * 1e3 + conv_ms / 500.0
    return {"workload": "training_2M_2704x2028_4_views", "gaussians": n_gauss, "ms_per_step": round(dt * 1e3, 3),
            "mpix_s": round(mpix / dt, 2), "views_per_step": 4, "step": "fwd+L1+bwd+Adam, batched",
            "pairs_per_step": rast.last_pairs, "counts": {k: int(v) for k, v in cnt.items()},
            "hbm": hbm_entry(alg["total"] + B_ADAM * n_scalars, dt),
            "convert_every_500": {"convert_with_moments_ms": round(conv_ms, 3),
                                  "ms_per_step_amortized": round(per, 4), "mpix_s_amortized": round(mpix / per * 1e3, 2)}}


def batched_leg(h4d, torch, sg, steps: int, warmup: int, forms: str = "both") -> dict:
    """fwd + L1 + bwd over 32 views per call (1M Gaussians, 80 % static; 8 arc
    cameras, four at 1352x1014 and four at 2704x2028, times 0.125 ... 0.875):
    views one after another (eager launches), against all views in one launch
    per stage replayed from a HIP graph.  Adam is not part of this step."""
    scene = sg.batched_scene()
    views = sg.batched_views(scene)
    g3, g4 = h4d.to_device(scene.g3), h4d.to_device(scene.g4)
    del scene
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    targets = [torch.rand((3, v.height, v.width), generator=gen, device="cuda") for v in views]
    gr3 = {k: torch.empty_like(v) for k, v in g3.items()}
    gr4 = {k: torch.empty_like(v) for k, v in g4.items()}
    mpix = sum(v.width * v.height for v in views) / 1e6
    out = {"workload": "batched_1M_32views", "views": len(views), "mpix_per_step": round(mpix, 3),
           "gaussians": int(g3["opacity"].numel() + g4["opacity"].numel())}

    if forms != "batched":
        out["single_view"] = _single_view_form(h4d, torch, g3, g4, views, targets, gr3, gr4, mpix, steps, warmup, out)
    if forms != "single":
        out["batched_graph"] = _batched_form(h4d, torch, g3, g4, views, targets, gr3, gr4, mpix, steps, warmup)
    if forms == "both":
        # the launch configuration the autotuner picks for this call (tiles of
        # 16 and 32 pixels: 8-pixel tiles split the call into two binning
        # passes, which gives up the shared static binning), replayed the same
        # way
        tuner = h4d.Autotuner(candidates=[(t, c) for t in (16, 32) for c in (64, 128, 256, 512)])
        tile, chunk = tuner.pick(g3, g4, views, batched=True)
        tuned = {"pick": {"tile": tile, "chunk": chunk},
                 "eager_ms": {f"{t}x{c}": round(ms, 3) for (t, c), ms in sorted(tuner.last_timings.items())}}
        if (tile, chunk) == (h4d.DEFAULT_TILE, h4d.DEFAULT_CHUNK):
            tuned.update(out["batched_graph"])
        else:
            tuned.update(_batched_form(h4d, torch, g3, g4, views, targets, gr3, gr4, mpix, steps, warmup,
                                       tile=tile, chunk=chunk))
        out["batched_graph_autotuned"] = tuned
    if forms != "both":
        return out
    out["speedup"] = round(out["single_view"]["ms_per_step"] / out["batched_graph"]["ms_per_step"], 3)
    out["speedup_autotuned"] = round(out["single_view"]["ms_per_step"] /
                                     out["batched_graph_autotuned"]["ms_per_step"], 3)
    # workload counts of the call (the same lists either way) and the share of
    # the HBM roofline of each form: the batched form reads the parameters once
    # per call, the views one after another once per view
    crast = h4d.Rasterizer(batched=True)
    dls = [torch.empty_like(t) for t in targets]

    def counted():
        h = crast.forward(g3, g4, views)
        h4d.l1_loss_grad(crast, h.images, targets, views, dls, None)
        crast.backward(h, g3, g4, dls, out=(gr3, gr4))

    cnt = count_step(crast, counted)
    n3, n4 = int(g3["opacity"].numel()), int(g4["opacity"].numel())
    pix = int(round(mpix * 1e6))
    a_single = alg_bytes(n3, n4, len(views), cnt, pix)
    a_batched = alg_bytes(n3, n4, 1, cnt, pix)
    out["counts"] = {k: int(v) for k, v in cnt.items()}
    out["hbm"] = {"single_view": hbm_entry(a_single["total"], out["single_view"]["ms_per_step"] * 1e-3),
                  "batched_graph": hbm_entry(a_batched["total"], out["batched_graph"]["ms_per_step"] * 1e-3)}
    return out


def _single_view_form(h4d, torch, g3, g4, views, targets, gr3, gr4, mpix, steps, warmup, out) -> dict:
    """The views one after another, eager launches."""
    rast = h4d.Rasterizer()
    dls = [torch.empty_like(t) for t in targets]
    loss = torch.zeros(1, device="cuda")

    def eager_step():
        h = rast.forward(g3, g4, views)
        h4d.l1_loss_grad(rast, h.images, targets, views, dls, loss)
        rast.backward(h, g3, g4, dls, out=(gr3, gr4))

    rast.check_mode = "eager"
    eager_step()
    torch.cuda.synchronize()
    out["pairs_per_step"] = rast.last_pairs
    rast.check_mode = "deferred"
    for _ in range(warmup):
        eager_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        eager_step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    rast.verify()
    del rast, dls
    torch.cuda.empty_cache()
    return {"ms_per_step": round(dt * 1e3, 3), "mpix_s": round(mpix / dt, 2)}


def _batched_form(h4d, torch, g3, g4, views, targets, gr3, gr4, mpix, steps, warmup, tile=None,
                  chunk=None) -> dict:
    """All views in one launch per stage, captured once and replayed."""
    rast = h4d.Rasterizer(tile=tile or h4d.DEFAULT_TILE, chunk=chunk or h4d.DEFAULT_CHUNK, batched=True)
    step = h4d.CapturedStep(rast, g3, g4, views, targets, (gr3, gr4))
    for _ in range(warmup):
        step.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    step.verify()
    del step, rast
    torch.cuda.empty_cache()
    return {"ms_per_step": round(dt * 1e3, 3), "mpix_s": round(mpix / dt, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tile", type=int, default=None)
    ap.add_argument("--chunk", type=int, default=None)
    ap.add_argument("--gaussians", type=int, default=250_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=4)
    ap.add_argument("--stats-views", type=int, default=8)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched vs single-view leg")
    ap.add_argument("--no-extra", action="store_true", help="skip the hybrid-ratio and 2M training legs")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--batched-only", choices=("both", "single", "batched"),
                    help="profiling aid: run only the batched-call leg (one or both forms) and print its result")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, run one plain device copy of MIB MiB (a known-size reference for counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only (--gpus 1); multi-GPU runs are not part of it",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import scenegen as sg
    import paper_2505_13215_amd as h4d

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    args.tile = args.tile or h4d.DEFAULT_TILE
    args.chunk = args.chunk or h4d.DEFAULT_CHUNK
    torch.cuda.set_device(0)
    if args.batched_only:
        res = batched_leg(h4d, torch, sg, args.batched_steps, 1, forms=args.batched_only)
        print(json.dumps({"batched_vs_single": res}), flush=True)
        return
    log("building the synthetic scene")
    scene = sg.multiview_scene(n_total=args.gaussians)
    sched = sg.view_schedule(scene, args.warmup + args.steps, 1, seed=2)
    W, H = scene.views[0].width, scene.views[0].height
    g3 = h4d.to_device(scene.g3)
    g4 = h4d.to_device(scene.g4)
    gr3 = {k: torch.empty_like(v) for k, v in g3.items()}
    gr4 = {k: torch.empty_like(v) for k, v in g4.items()}
    keys = [("3", k) for k in h4d.G3_KEYS] + [("4", k) for k in h4d.G4_KEYS]
    params = [(g3 if w == "3" else g4)[k] for w, k in keys]
    grads = [(gr3 if w == "3" else gr4)[k] for w, k in keys]
    ms = [torch.zeros_like(p) for p in params]
    vs = [torch.zeros_like(p) for p in params]
    lrs = [(LR3 if w == "3" else LR4)[k] for w, k in keys]
    n_scalars = sum(p.numel() for p in params)
    rng = np.random.default_rng(1)
    targets = [torch.as_tensor(rng.uniform(0, 1, size=(3, H, W)).astype(np.float32), device="cuda") for _ in range(4)]
    dl = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    rast = h4d.Rasterizer(tile=args.tile, chunk=args.chunk, pair_capacity=1 << 24, check="eager")
    state = {"step": 0}

    def step(i):
        v = sched[i][0]
        h = rast.forward(g3, g4, [v])
        h4d.l1_loss_grad(rast, h.images, [targets[i % len(targets)]], [v], [dl], loss)
        rast.backward(h, g3, g4, [dl], out=(gr3, gr4))
        state["step"] += 1
        h4d.adam_step(rast, params, grads, ms, vs, lrs, state["step"])

    log(f"warmup {args.warmup} steps (eager capacity checks)")
    peak_pairs = 0
    for i in range(args.warmup):
        step(i)
        peak_pairs = max(peak_pairs, rast.last_pairs)
    torch.cuda.synchronize()

    # stage breakdown over the views of the timed steps (untimed: event pairs
    # between stages add idle time); it also sizes the pair buffer for them
    rast.profile(1)
    rast.profile_read()
    for i in range(args.warmup, args.warmup + args.steps):
        step(i)
        peak_pairs = max(peak_pairs, rast.last_pairs)
    torch.cuda.synchronize()
    sprof = rast.profile_read()
    rast.profile(0)
    stages = {k: (v[0] / max(v[1], 1)) for k, v in sprof.items() if v[1] > 0}
    log("stage ms per launch: " + ", ".join(f"{k} {v:.3f}" for k, v in stages.items()))
    dom = max(("blend_fwd", "blend_bwd"), key=lambda k: stages.get(k, 0.0))

    rast.capacity = int(max(peak_pairs, 1) * 1.5) + 4096
    rast.check_mode = "deferred"
    log(f"timing {args.steps} steps (pairs per view up to {peak_pairs})")
    for attempt in range(2):
        # the dominant blending kernel timed from its own dispatch: nothing is
        # added to the stream
        rast.profile(3 if dom == "blend_fwd" else 4)
        rast.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.warmup, args.warmup + args.steps):
            step(i)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = rast.profile_read()
        rast.profile(False)
        try:
            rast.verify()
            break
        except h4d.H4DError:
            log("pair capacity exceeded during timing; retrying with more capacity")
            rast.check_mode = "eager"
            step(args.warmup)
            rast.capacity = int(rast.last_pairs * 1.5) + 4096
            rast.check_mode = "deferred"
    else:
        raise RuntimeError("could not size the pair buffer")
    dt = t1 - t0
    ms_step = dt * 1e3 / args.steps
    mpix = args.steps * W * H / dt / 1e6
    kernel_ms = {k: (v[0] / max(v[1], 1)) for k, v in prof.items() if v[1] > 0}
    log("blend kernels, ms per launch in the timed region: " +
        ", ".join(f"{k} {v:.4f}" for k, v in kernel_ms.items()))

    # the same steps without the optimiser (render_fwd + loss gradient +
    # render_bwd, the fwd+bwd step the Mpix/s metric is defined on), reported beside
    def step_fb(i):
        v = sched[i][0]
        h = rast.forward(g3, g4, [v])
        h4d.l1_loss_grad(rast, h.images, [targets[i % len(targets)]], [v], [dl], loss)
        rast.backward(h, g3, g4, [dl], out=(gr3, gr4))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        step_fb(i)
    torch.cuda.synchronize()
    dt_fb = time.perf_counter() - t0
    rast.verify()
    fwd_bwd = {"step": "fwd+L1+bwd (no optimiser)", "ms_per_step": round(dt_fb * 1e3 / args.steps, 4),
               "mpix_s": round(args.steps * W * H / dt_fb / 1e6, 2)}
    log(f"without the optimiser: {fwd_bwd}")

    # inference render (no adjoint state) over the same views, beside
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        rast.infer(g3, g4, [sched[i][0]])
    torch.cuda.synchronize()
    dt_inf = time.perf_counter() - t0
    rast.verify()
    inference = {"render": "render_infer, one view per frame", "ms_per_frame": round(dt_inf * 1e3 / args.steps, 4),
                 "frames_per_s": round(args.steps / dt_inf, 1)}
    log(f"inference: {inference}")

    # evaluation counts of the blending kernels (counting instantiation, outside the timed region)
    log(f"counting blend evaluations on {args.stats_views} views")
    rast.stats(True)
    rast.check_mode = "eager"
    cnt = dict(fwd_eval=0, fwd_blend=0, bwd_eval=0, bwd_blend=0, list_entries=0, traversed=0, onscreen=0)
    nst = max(1, min(args.stats_views, args.steps))
    for i in range(args.warmup, args.warmup + nst):
        v = sched[i][0]
        h = rast.forward(g3, g4, [v])
        h4d.l1_loss_grad(rast, h.images, [targets[i % len(targets)]], [v], [dl], None)
        rast.backward(h, g3, g4, [dl], out=(gr3, gr4))
        c = rast.stats_read()
        for k in cnt:
            cnt[k] += c[k]
    rast.stats(False)
    for k in cnt:
        cnt[k] /= nst
    flops_fwd = FLOPS_EVAL * cnt["fwd_eval"] + FLOPS_BLEND_FWD * cnt["fwd_blend"]
    flops_bwd = FLOPS_EVAL * cnt["bwd_eval"] + FLOPS_BLEND_BWD * cnt["bwd_blend"]
    dom_ms = kernel_ms[dom]
    dom_flops = flops_bwd if dom == "blend_bwd" else flops_fwd
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    kname = f"k_composite_{dom[6:]}"
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": recorded_traffic(kname), "kernel": kname,
                "kernel_ms": round(dom_ms, 4), "flops_per_launch": dom_flops}

    # share of the HBM roofline: algorithmic bytes of a step (counted per view
    # above) over its measured time, against the published 8 TB/s
    alg = alg_bytes(scene.n3, scene.n4, 1, cnt, W * H)
    copy_gbs = copy_bandwidth(torch)
    hbm = {"yardstick_bytes_per_step": {k: int(v) for k, v in alg.items()},
           "fwd_bwd_step": hbm_entry(alg["total"], dt_fb / args.steps),
           "train_step_with_adam": hbm_entry(alg["total"] + B_ADAM * n_scalars, dt / args.steps),
           "peak_gbs": PEAK_HBM_GBS, "copy_kernel_gbs": copy_gbs}
    log(f"HBM: {hbm}")

    # static conversion (Sec. 4.1-4.2): on the workload's sets, and on 500k all-4D
    # Gaussians of which half are static
    log("timing convert_static")
    conv = {"workload": convert_leg(h4d, torch, rast, g3, g4)}
    rng4 = np.random.default_rng(5)
    half = h4d.to_device(sg.draw_4d(rng4, 500_000, 2.0, static_fraction=0.5, tau=0.5))
    conv["all4d_500k_half_static"] = convert_leg(h4d, torch, rast, h4d.to_device(sg.empty_3d()), half)
    del half

    batched = None
    if not args.no_batched:
        log("batched vs single-view: 1M Gaussians, 32 views per step")
        del rast
        torch.cuda.empty_cache()
        batched = batched_leg(h4d, torch, sg, args.batched_steps, 1)
        log(f"batched vs single-view: {batched}")

    hybrid = training = None
    if not args.no_extra:
        log("hybrid-ratio leg: 500k all-4D vs converted, f = 0, 0.5, 0.9")
        hybrid = hybrid_leg(h4d, torch, sg, 10, 3)
        log(f"hybrid: {hybrid}")
        torch.cuda.empty_cache()
        log("training leg: 2M Gaussians, 2704x2028, 4 views per step")
        training = training_leg(h4d, torch, sg, 5, 2)
        log(f"training: {training}")
        torch.cuda.empty_cache()

    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nbytes} bytes read, {nbytes} written")
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        log(f"CPU baseline: FP64 oracle on {args.cpu_views} view(s)")
        cpu = cpu_baseline(scene, [sched[args.warmup + i][0] for i in range(args.cpu_views)], n_scalars)

    out = {
        "metric": METRIC, "value": round(mpix, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "multiview_250k_1352x1014_single_view_train_step", "gaussians": args.gaussians,
                   "static_3d": scene.n3, "dynamic_4d": scene.n4, "image": [W, H], "views_per_step": 1,
                   "tile": args.tile, "chunk": args.chunk, "step": "fwd+L1+bwd+Adam",
                   "parallelism": "single_gpu"},
        "roofline": roofline,
        "hbm": hbm,
        "cpu_baseline": cpu,
        "fwd_bwd_only": fwd_bwd,
        "inference": inference,
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "blend_evals_per_view": {k: int(v) for k, v in cnt.items()},
        "pairs_per_view_max": peak_pairs,
        "convert_static": conv,
        "batched_vs_single": batched,
        "hybrid_ratio": hybrid,
        "training_2m": training,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
