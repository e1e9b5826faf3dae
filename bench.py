"""Benchmark: one DGR fwd+bwd optimisation iteration on one MI355X.

Workload: 256^3 volume, 100,000 anisotropic Gaussians (scales log-uniform in
[0.004, 0.03]), cone beam 360 views over 360 degrees onto 512 x 512 pixels at
0.8 mm, DSO 1000 mm, DSD 1500 mm, march step 0.5 voxel, L1 projection loss
against the noisy analytic projections of a seeded ellipsoid phantom.  A step
is voxelize -> project + L1 -> backproject -> voxelize backward -> Adam, with
all inputs resident in HBM.

Prints ONE JSON line (see the repository's benchmark contract).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np
import torch

METRIC = "fwd+bwd ms/iter @256^3,100k Gaussians,360 views; s to 35 dB PSNR vs plain"

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3  # published binary32 vector peak
# Single-issue VALU rate derived from the chip: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
# lane-instructions per second (one wave64 instruction per SIMD every 4 cycles)
VALU_LANE_INSTR_PER_S = 256 * 4 * 16 * 2.4e9

# Algorithmic work per ray sample: position, weights, seven lerps and the sum
# (forward); position, weights, eight products (backward)
FLOP_PER_SAMPLE = {"project_l1": 31.0, "backproject": 34.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def count_samples(prob) -> int:
    """Exact number of ray samples of the geometry (same k-range rule as the
    projector: every sample with -1 <= u <= D on all axes), in binary64."""
    from paper_2411_04844_amd import inputs
    g, geom = prob.grid, prob.geom
    dev = prob.target.device
    total = 0
    for j0 in range(0, geom.n_views, 8):
        idx = np.arange(j0, min(j0 + 8, geom.n_views))
        o, d = inputs._ray_dirs(geom, idx, dev, torch)
        c = o - (o * d).sum(-1, keepdim=True) * d
        lo = torch.tensor(g.lo, dtype=torch.float64, device=dev)
        ih = torch.tensor(g.inv_h, dtype=torch.float64, device=dev)
        dims = torch.tensor(g.dims, dtype=torch.float64, device=dev)
        cu = (c - lo) * ih - 0.5
        du = d * ih * geom.step
        with torch.no_grad():
            t0 = (-1.0 - cu) / du
            t1 = (dims - cu) / du
            tmin = torch.minimum(t0, t1).amax(-1)
            tmax = torch.maximum(t0, t1).amin(-1)
            k0, k1 = torch.ceil(tmin), torch.floor(tmax)
            total += int(torch.clamp(k1 - k0 + 1, min=0).sum().item())
    return total


REPO = os.path.dirname(os.path.abspath(__file__))
COUNTER_FILE = os.path.join(REPO, "profiles", "counters_cone256.txt")
KERNEL_SOURCE = {"backproject": "backproject_bricks<true,false>", "project_l1": "project_bundles<1,2>"}
# the source file each profiled kernel is built from (with internal.h)
# kernels (and launches per stage) of the HBM-stage lines
STAGE_KERNELS = {"voxelize": [("voxelize_tiles", 1)], "voxelize_backward": [("voxelize_grad", 1)],
                 "adam": [("adam_kernel", 4)], "projection_loss": [("ssim_fwd", 1), ("ssim_bwd", 1)],
                 "tv": [("tv_kernel", 1)]}
KERNEL_FILE = {"backproject_bricks<true,false>": "project.hip", "project_bundles<1,2>": "project.hip",
               "voxelize_tiles": "voxelize.hip", "voxelize_grad": "voxelize_bwd.hip",
               "ssim_fwd": "objective.hip", "ssim_bwd": "objective.hip", "tv_kernel": "objective.hip",
               "adam_kernel": "adam.hip"}


def source_digest(name: str) -> str:
    """sha256 (first 16 hex) of a kernel's source file and internal.h, to tell
    whether committed counters still apply to the kernel."""
    h = hashlib.sha256()
    cdir = os.path.join(REPO, "paper_2411_04844_amd", "csrc")
    for fn in (name, "internal.h"):
        with open(os.path.join(cdir, fn), "rb") as f:
            h.update(fn.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def committed_counters(kernel: str):
    """Per-launch counters of `kernel` from the committed rocprofv3 --pmc
    summary, with HBM bytes (FETCH_SIZE and WRITE_SIZE, each scaled by the
    ratio of known bytes to counter reading for a plain copy kernel), or None
    when the summary is missing or was taken on other sources."""
    if not os.path.exists(COUNTER_FILE):
        return None
    rows = {}
    for line in open(COUNTER_FILE):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows[f[0]] = dict(zip(f[1::2], f[2::2]))
    cal, k = rows.get("copy_calibration"), rows.get(kernel)
    if not cal or not k or k.get("source") != source_digest(KERNEL_FILE[kernel]):
        return None
    fetch_factor = float(cal["read_bytes"]) / (float(cal["fetch_kib"]) * 1024.0)
    write_factor = float(cal["write_bytes"]) / (float(cal["write_kib"]) * 1024.0)
    out = {c: float(v) for c, v in k.items() if c != "source"}
    out["hbm_bytes"] = (float(k["fetch_kib"]) * 1024.0 * fetch_factor +
                        float(k["write_kib"]) * 1024.0 * write_factor)
    return out


def copy_calibration(mib: int = 1024, reps: int = 3):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": 4 * n, "bytes_written": 4 * n,
                                           "dispatches": reps}}), flush=True)


def recon_leg(max_iters: int):
    """Sparse-view loop (256^3, 25 views, 1 % noise): time from resident
    projections to the first PSNR >= 35 dB for the plain FDK-sampled
    initialisation (50,000 Gaussians of 1.5 voxels, the loop's
    specification; the same with 3-voxel Gaussians; 150,000, the paper's own
    initial count) and for the learned initialisation (50,000 Gaussians
    proposed by the U-Net), with the L1 objective and with the paper's full
    objective (0.6 L1 + 0.2 SSIM + 1 TV).  Every run is capped at max_iters
    iterations; the PSNR is measured after every iteration, so the step that
    first reaches 35 dB is exact."""
    from paper_2411_04844_amd import learned, recon
    prob, gt = recon.sparse_view_problem(device="cuda")
    params = learned.load() if os.path.exists(learned.WEIGHTS) else None
    out = []
    for kind, n, sv, obj in (("plain", 50_000, 1.5, "l1"), ("plain", 50_000, 3.0, "l1"),
                             ("plain", 150_000, 1.5, "l1"), ("learned", 50_000, None, "l1"),
                             ("plain", 50_000, 1.5, "full"), ("plain", 50_000, 3.0, "full"),
                             ("learned", 50_000, None, "full")):
        if kind == "learned" and params is None:
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob.params = (recon.fdk_init(prob, n=n, scale_vox=sv) if kind == "plain"
                       else learned.learned_init(prob, params, n=n))
        res = recon.reconstruct(prob, gt, max_iters=max_iters, t_start=t0, objective=obj, check_every=100,
                                log=lambda m: log(f"recon {kind} n={n} sv={sv} {obj}:", m))
        h = res["history"]
        out.append({"init": kind, "gaussians": n, "scale_voxels": sv, "objective": obj,
                    "target_psnr_db": 35.0, "max_iters": max_iters,
                    "iterations_to_target": res["iterations"],
                    "seconds_to_target": None if res["seconds"] is None else round(res["seconds"], 3),
                    "psnr_after_init_db": round(h[0][2], 3),
                    "best_psnr_db": round(res["best_psnr"], 3), "best_iter": res["best_iter"],
                    "final_psnr_db": round(res["final_psnr"], 3), "iterations_run": h[-1][0],
                    "seconds_total": round(h[-1][1], 2)})
    return out


def fan_leg(max_iters: int, steps: int = 10):
    """The fan-beam settings of the paper's Tabs. 2-4 (a stack of fan-beam
    slices, one detector row per slice, 384 columns, 256^3 cube):
    * fwd+bwd+Adam iteration at 100,000 Gaussians and 60 views, ms;
    * the same with the full objective, 150,000 isotropic Gaussians and the
      fixed boxes 13^3 .. 19^3 of the box-size sweep (Tab. 4), ms;
    * 60-view sparse-view loop from 50,000 FBP-sampled Gaussians (3 voxels)
      with the full objective;
    * 90-degree limited-angle loop (90 views, 1 degree apart) from 50,000
      random Gaussians (the paper's random initialisation for this setting)
      with the full objective.
    Both run max_iters iterations and report the best PSNR and the first
    iteration and time at which 30, 33 and 35 dB were reached."""
    import math
    from paper_2411_04844_amd import inputs, recon
    prob = recon.cone_problem(geom=inputs.fan_workload(256, 60, 384), device="cuda")
    it = recon.Iteration(prob)
    for _ in range(3):
        it.step()
    torch.cuda.synchronize()
    ev = {}
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        it.step(events=ev)
    b.record()
    torch.cuda.synchronize()
    it.check()
    out = {"iteration_256^3_100k_60x384x256": {
        "ms_per_iter": round(a.elapsed_time(b) / steps, 3),
        "stage_ms": {k: round(float(np.mean([x.elapsed_time(y) for x, y in v])), 3) for k, v in ev.items()}}}
    del it, prob
    # The box-size sweep of the paper's Tab. 4 (60-view fan beam, full
    # objective, fixed cuboid boxes 13^3 .. 19^3) with 150,000 isotropic
    # Gaussians: fwd+bwd+Adam ms per iteration, each box from the same
    # initial parameters.  The paper's times per iteration (its 1K-iteration
    # runs on its GPU) also include densification, which is not in these.
    prob = recon.cone_problem(n=150_000, geom=inputs.fan_workload(256, 60, 384), device="cuda")
    prob.params["scale"][:, 1] = prob.params["scale"][:, 0]
    prob.params["scale"][:, 2] = prob.params["scale"][:, 0]
    init = {k: v.clone() for k, v in prob.params.items()}
    sweep = []
    for bh in (6, 7, 8, 9):
        for k in init:
            prob.params[k].copy_(init[k])
        prob.k_sigma, prob.box_half = 0.0, bh
        it = recon.Iteration(prob, objective="full")
        for _ in range(3):
            it.step()
        torch.cuda.synchronize()
        a.record()
        for _ in range(steps):
            it.step()
        b.record()
        torch.cuda.synchronize()
        it.check()
        sweep.append({"box": 2 * bh + 1, "ms_per_iter": round(a.elapsed_time(b) / steps, 3)})
        del it
    out["box_sweep_60view_full_objective_150k_isotropic"] = sweep
    del prob, init
    loops = []
    for name, n_views, arc, init in (("sparse_view_60", 60, 2 * math.pi, "fbp"),
                                     ("limited_angle_90deg", 90, math.pi / 2, "random")):
        if max_iters <= 0:
            break
        prob, gt = recon.fan_problem(n_views=n_views, arc=arc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob.params = (recon.fdk_init(prob, n=50_000, scale_vox=3.0) if init == "fbp"
                       else recon.random_init(prob, n=50_000))
        res = recon.reconstruct(prob, gt, max_iters=max_iters, t_start=t0, objective="full",
                                target_psnr=float("inf"), log=lambda m: log(f"fan {name}:", m))
        reached = {}
        for level in (30.0, 33.0, 35.0):
            hit = next((h for h in res["history"] if h[2] >= level), None)
            reached[f"{level:g}"] = None if hit is None else {"iteration": hit[0], "seconds": round(hit[1], 3)}
        loops.append({"setting": name, "views": n_views, "arc_deg": round(math.degrees(arc)), "init": init,
                      "gaussians": 50_000, "objective": "full", "max_iters": max_iters,
                      "reached_db": reached, "best_psnr_db": round(res["best_psnr"], 3),
                      "best_iter": res["best_iter"], "seconds_total": round(res["history"][-1][1], 2)})
        del prob, gt
    out["loops"] = loops
    return out


def fvr_leg(reps: int = 5):
    """The paper's own voxelization setting (sec. 4.2; box-size sweep of
    Tab. 4, timing of Tab. 5): 256^3, 150,000 isotropic Gaussians (scales
    log-uniform in [0.004, 0.03]), fixed cuboid box floor(u) +- b for box
    edges 13..19: voxelize and voxelize backward, ms per call."""
    from paper_2411_04844_amd import inputs, native
    grid = inputs.cube_grid(256)
    G = inputs.gaussians(150_000, 2001, 0.004, 0.03)
    G["scale"][:, 1] = G["scale"][:, 0]
    G["scale"][:, 2] = G["scale"][:, 0]
    P = {k: torch.as_tensor(v).cuda().contiguous() for k, v in G.items()}
    gen = torch.Generator(device="cuda").manual_seed(7)
    dV = torch.randn(grid.shape, generator=gen, device="cuda")
    out = []
    for bh in (6, 7, 8, 9):
        ws, bws = native.Workspace(), native.Workspace()
        pairs = native.dgr_voxelize_plan(P["mu"], P["scale"], P["quat"], grid, 0.0, bh, ws)
        V = torch.empty(grid.shape, device="cuda")
        grads = tuple(torch.empty_like(P[k]) for k in ("mu", "scale", "quat", "density"))
        f = lambda: native.dgr_voxelize(P["mu"], P["scale"], P["quat"], P["density"], grid, 0.0, bh, out=V,
                                        ws=ws, max_pairs=pairs)
        b = lambda: native.dgr_voxelize_backward(P["mu"], P["scale"], P["quat"], P["density"], dV, grid,
                                                 0.0, bh, ws=bws, outs=grads)
        res = {"box": 2 * bh + 1, "tile_pairs": pairs}
        for name, fn in (("voxelize_ms", f), ("voxelize_backward_ms", b)):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            res[name] = round(e0.elapsed_time(e1) / reps, 3)
        native.dgr_check(ws)
        out.append(res)
    return out


def cpu_baseline(prob, n_views_sample: int, n_views_single: int = 2):
    """Time the binary64 oracle on a bounded sample of the same workload, on
    all host cores and on one."""
    import oracle
    g = prob.grid
    P = {k: v.cpu().numpy() for k, v in prob.params.items()}
    nthreads = oracle.num_threads()

    def run(nv):
        t = time.perf_counter()
        box = oracle.bbox(P["mu"], P["scale"], P["quat"], g.dims, g.lo, g.inv_h)
        V = oracle.voxelize(P["mu"], P["scale"], P["quat"], P["density"], g.dims, g.lo, g.inv_h, box)
        t_vox = time.perf_counter() - t
        sel = np.linspace(0, prob.geom.n_views - 1, nv).round().astype(int)
        views = prob.geom.views[sel]
        y = prob.target[sel].cpu().numpy()
        t = time.perf_counter()
        Ph = oracle.project(V, g.dims, g.lo, g.inv_h, prob.geom.kind, views, prob.geom.nu, prob.geom.nv,
                            prob.geom.step, prob.geom.length_scale)
        _, gr = oracle.l1(Ph, y)
        t_proj = time.perf_counter() - t
        t = time.perf_counter()
        dV = oracle.backproject(gr, g.dims, g.lo, g.inv_h, prob.geom.kind, views, prob.geom.nu,
                                prob.geom.nv, prob.geom.step, prob.geom.length_scale)
        t_bp = time.perf_counter() - t
        t = time.perf_counter()
        oracle.voxelize_grad(P["mu"], P["scale"], P["quat"], P["density"], g.dims, g.lo, g.inv_h, box, dV)
        t_grad = time.perf_counter() - t
        scale = prob.geom.n_views / nv
        return 1e3 * (t_vox + t_grad + (t_proj + t_bp) * scale), t_vox + t_proj + t_bp + t_grad, scale

    ms, wall, scale = run(n_views_sample)
    out = {"value": round(ms, 1), "unit": "ms/iter", "cores": nthreads, "kind": "oracle",
           "sample": (f"binary64 oracle: full voxelization and voxelization gradient "
                      f"(100k Gaussians, 256^3), projection+L1 and backprojection over "
                      f"{n_views_sample} of 360 views scaled x{scale:.1f}; {wall:.1f} s wall")}
    oracle.set_num_threads(1)
    try:
        ms1, wall1, scale1 = run(n_views_single)
    finally:
        oracle.set_num_threads(nthreads)
    out["single_thread"] = {"value": round(ms1, 1), "unit": "ms/iter", "cores": 1,
                            "sample": (f"the same on one thread, projection+L1 and backprojection over "
                                       f"{n_views_single} of 360 views scaled x{scale1:.0f}; {wall1:.1f} s wall")}
    return out


def large_leg(steps: int = 2):
    """The 512^3 workload: 500,000 anisotropic Gaussians (scale ratio up to
    10:1), cone beam 720 views x 1024^2 at 0.4 mm; fwd+bwd+Adam ms per
    iteration and the peak device memory of the run (the volume is recomputed
    for the backward pass, never stored)."""
    from paper_2411_04844_amd import recon
    torch.cuda.reset_peak_memory_stats()
    prob = recon.cone_problem(D=512, n=500_000, n_views=720, n_det=1024, pitch_mm=0.4,
                              seeds=(4001, 4002, 4003), ratio_max=10.0, device="cuda")
    it = recon.Iteration(prob)
    it.step()
    torch.cuda.synchronize()
    ev = {}
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(steps):
        it.step(events=ev)
        log(f"512^3 step {i + 1}/{steps} enqueued")
    b.record()
    torch.cuda.synchronize()
    it.check()
    out = {"ms_per_iter": round(a.elapsed_time(b) / steps, 2),
           "stage_ms": {k: round(float(np.mean([x.elapsed_time(y) for x, y in v])), 2) for k, v in ev.items()},
           "peak_device_gib": round(torch.cuda.max_memory_allocated() / 2 ** 30, 2),
           "projection_workspace_gib": round(it.proj_ws.buf.numel() / 2 ** 30, 2),
           "gaussians": 500_000, "views": 720, "detector": 1024, "volume": 512}
    del it, prob
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-views", type=int, default=40, help="views in the oracle's timed sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--recon", type=int, default=5000, metavar="MAX_ITERS",
                    help="iteration cap of the 25-view sparse loops to 35 dB (0: skip them)")
    ap.add_argument("--large-steps", type=int, default=2,
                    help="timed iterations of the 512^3 / 720 x 1024^2 workload (0: skip it)")
    ap.add_argument("--fan-iters", type=int, default=300,
                    help="iterations of the fan-beam loops (0: skip them)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--iteration-only", action="store_true",
                    help="time the iteration and skip every other leg (for profiler runs)")
    ap.add_argument("--objective", choices=("l1", "full", "both"), default="l1",
                    help="with --iteration-only: the L1 iteration, the full-objective one, or both")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(the path would shard by views, one all-reduce of the parameter gradient)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    from paper_2411_04844_amd import native, recon
    native.lib()  # fail loudly if the HIP library is missing
    torch.cuda.init()
    log("building workload (256^3, 100k Gaussians, 360 x 512^2 cone)")
    prob = recon.cone_problem(device="cuda")
    it = recon.Iteration(prob)
    samples = count_samples(prob)
    log(f"pairs capacity {it.max_pairs}, ray samples per projection {samples:.4g}")

    for _ in range(args.warmup):
        it.step()
    torch.cuda.synchronize()
    it.check()

    events = {}
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for i in range(args.steps):
        it.step(events=events)
        log(f"step {i + 1}/{args.steps} enqueued")
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    it.check()
    ms = start.elapsed_time(stop) / args.steps
    stage_ms = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in events.items()}
    log("stage ms:", json.dumps({k: round(v, 3) for k, v in stage_ms.items()}),
        f"wall {wall:.2f}s loss {float(it.loss):.6g}")

    dom = max(FLOP_PER_SAMPLE, key=lambda k: stage_ms[k])
    kname = KERNEL_SOURCE[dom]
    achieved = FLOP_PER_SAMPLE[dom] * samples / (stage_ms[dom] * 1e-3) / 1e12
    ctr = committed_counters(kname)
    roofline = {"kernel": kname, "stage": dom, "bound": "alu",
                "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": None if ctr is None else round(ctr["hbm_bytes"]),
                "flop_per_sample": FLOP_PER_SAMPLE[dom], "samples": samples}
    if ctr is not None and "valu" in ctr:
        # VALU wave-instructions of one launch (SQ_INSTS_VALU) at the stage's
        # measured duration, against the single-issue lane rate of the chip
        lane = ctr["valu"] * 64.0
        roofline["valu"] = {"lane_instr_per_sample": round(lane / samples, 2),
                            "lane_instr_per_s": lane / (stage_ms[dom] * 1e-3),
                            "single_issue_peak": VALU_LANE_INSTR_PER_S,
                            "frac": round(lane / (stage_ms[dom] * 1e-3) / VALU_LANE_INSTR_PER_S, 4)}
    # HBM-bound stages: algorithmic bytes over the measured stage time
    n = prob.params["mu"].shape[0]
    nvox = int(np.prod(prob.grid.dims))
    stage_bytes = {"voxelize": 44 * n + 4 * nvox, "voxelize_backward": 44 * n + 4 * nvox + 44 * n,
                   "adam": 28 * 11 * n}
    hbm = {k: {"bytes": b, "ms": round(stage_ms[k], 4),
               "GB/s": round(b / (stage_ms[k] * 1e-3) / 1e9, 1),
               "frac": round(b / (stage_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)} for k, b in stage_bytes.items()}

    if args.iteration_only:
        line = {"metric": METRIC, "value": round(ms, 3), "unit": "ms/iter",
                "stage_ms": {k: round(v, 3) for k, v in stage_ms.items()}}
        if args.objective in ("full", "both"):
            itf = recon.Iteration(prob, objective="full")
            ev_f = {}
            for i in range(args.warmup + args.steps):
                itf.step(events=ev_f if i >= args.warmup else None)
                log(f"full-objective step {i + 1}/{args.warmup + args.steps} enqueued")
            torch.cuda.synchronize()
            itf.check()
            line["full_objective_stage_ms"] = {k: round(float(np.mean([a.elapsed_time(b) for a, b in v])), 3)
                                               for k, v in ev_f.items()}
        print(json.dumps(line), flush=True)
        return

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a sample of the workload")
        cpu = cpu_baseline(prob, args.cpu_views)

    log("full-objective iteration (L1 + SSIM + TV)")
    itf = recon.Iteration(prob, objective="full")
    for _ in range(2):
        itf.step()
    torch.cuda.synchronize()
    ev_f = {}
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record()
    for _ in range(5):
        itf.step(events=ev_f)
    f1.record()
    torch.cuda.synchronize()
    itf.check()
    full = {"ms_per_iter": round(f0.elapsed_time(f1) / 5, 3),
            "stage_ms": {k: round(float(np.mean([a.elapsed_time(b) for a, b in v])), 3) for k, v in ev_f.items()},
            "weights": list(itf.weights)}
    # projection loss: P_hat and y read, dL/dP_hat written; TV: V read, dL/dV
    # read and written
    npix = prob.target.numel()
    for k, b in (("projection_loss", 12 * npix), ("tv", 12 * nvox)):
        t = full["stage_ms"][k]
        hbm[k] = {"bytes": b, "ms": t, "GB/s": round(b / (t * 1e-3) / 1e9, 1),
                  "frac": round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del itf
    # the same stages against the VALU issue rate (committed counters of
    # their kernels, while the sources are unchanged): the voxelization pair
    # is bound by its exp2 evaluations, not by HBM
    for k, kernels in STAGE_KERNELS.items():
        rows = [(committed_counters(kn), calls) for kn, calls in kernels]
        if k not in hbm or any(c is None for c, _ in rows):
            continue
        lane = sum(c["valu"] * calls for c, calls in rows) * 64.0
        rate = lane / (hbm[k]["ms"] * 1e-3)
        hbm[k]["valu_issue_frac"] = round(rate / VALU_LANE_INSTR_PER_S, 4)
        hbm[k]["bound"] = "alu" if hbm[k]["valu_issue_frac"] > hbm[k]["frac"] else "hbm"
    log("fixed-box voxelization sweep")
    fvr = fvr_leg()
    rec = None
    if args.recon > 0:
        log("sparse-view loop to 35 dB")
        rec = recon_leg(args.recon)
    log("fan-beam settings")
    fan = fan_leg(args.fan_iters)
    large = None
    if args.large_steps > 0:
        log("512^3 / 500k / 720 x 1024^2 iteration")
        large = large_leg(args.large_steps)

    out = {
        "metric": METRIC, "value": round(ms, 3), "unit": "ms/iter", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dgr_cone_fwd_bwd_256^3_100k_gauss_360x512^2",
                   "volume": 256, "gaussians": 100000, "views": 360, "detector": 512,
                   "ray_samples": samples, "pair_capacity": it.max_pairs},
        "stage_ms": {k: round(v, 3) for k, v in stage_ms.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "hbm_stages": hbm,
    }
    out["full_objective_iteration"] = full
    out["fvr_fixed_box_256^3_150k_isotropic"] = fvr
    if rec is not None:
        out["recon"] = rec
    out["fan_beam"] = fan
    if large is not None:
        out["large_512^3_500k_720x1024^2"] = large
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
