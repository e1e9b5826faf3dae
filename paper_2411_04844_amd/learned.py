"""Learned initialisation (driver): training data made by the plain method,
training of the U-Net on the GPU kernels, and Gaussians proposed from its
output.  Every numerical step runs in libdgr.so; this module sequences the
calls and holds the tensors.

Data.  For a seeded ellipsoid phantom at 128^3 (2 mm voxels), 25-view cone
beam onto 256^2 pixels at 1.6 mm: the FDK volume is the network input, and a
plain DGR run (20,000 FDK-sampled Gaussians, 200 fwd+bwd+Adam iterations of
the full objective with the rate decayed tenfold) gives the Gaussian set
near its plateau whose fields are the targets (dgr_unet_targets).
Input and density targets are divided by INPUT_SCALE (the largest
attenuation of the phantom family, mm^-1).

Use at any resolution D: the D^3 FDK volume is pooled to (D/2)^3 when D is
twice the training resolution, the network runs there, and the Gaussians are
drawn on that grid (dgr_init_from_unet); their densities are then scaled by
the least-squares fit to the projections, as in the plain initialisation.
"""
from __future__ import annotations

import math
import os
import time

import numpy as np
import torch

from . import inputs, native, recon

INPUT_SCALE = 0.05
TRAIN_D = 128
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_b32_d128.npy")


# ---- data made by the plain method ---------------------------------------------------
def training_problem(seed: int, D=TRAIN_D, n_views=25, n_det=256, pitch_mm=1.6, noise_frac=0.01):
    grid = inputs.cube_grid(D)
    geom = inputs.cone_workload(D, n_views, n_det, pitch_mm)
    ph = inputs.ellipsoid_phantom(seed)
    y = inputs.add_noise(inputs.phantom_projections(ph, geom, device="cuda"), seed + 1_000_000,
                         noise_frac).contiguous()
    views = torch.as_tensor(geom.views).cuda().contiguous()
    return recon.Problem(grid, geom, views, y, {})


def make_pair(seed: int, n_gauss=20_000, iters=200, D=TRAIN_D, objective="full"):
    """(input [D,D,D], target [D,D,D,3]) from one plain DGR run (rate decayed
    tenfold over the run; with the full objective 200 iterations bring a
    128^3 run within about 0.4 dB of where 300 leave it)."""
    prob = training_problem(seed, D)
    f = native.dgr_fdk(prob.target, prob.grid, prob.geom, prob.views)
    prob.params = recon.fdk_init(prob, n=n_gauss, seed=seed + 2_000_000)
    it = recon.Iteration(prob, objective=objective)
    for i in range(iters):
        it.lr_factor = 0.1 ** (i / iters)
        it.step()
    it.voxelize()
    it.check()
    P = prob.params
    tgt = native.dgr_unet_targets(P["mu"], P["scale"], prob.grid, it.V, INPUT_SCALE)
    x = (f * (1.0 / INPUT_SCALE)).contiguous()
    return x, tgt


def make_dataset(seeds, log=None, **kw):
    data = []
    t0 = time.perf_counter()
    for k, s in enumerate(seeds):
        data.append(make_pair(int(s), **kw))
        if log and (k + 1) % 10 == 0:
            torch.cuda.synchronize()
            log(f"data {k + 1}/{len(seeds)}: {time.perf_counter() - t0:.1f}s")
    return data


# ---- training ---------------------------------------------------------------------------
def init_params(seed=0):
    """He-normal conv weights, zero biases; head bias starts the occupancy
    logit at log(1/99) (about 1 % of voxels hold a Gaussian mean)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = native.dgr_unet_param_count()
    flat = torch.empty(n, dtype=torch.float32)
    B = native.UNET_BASE
    shapes = [(1, B), (B, 2 * B), (2 * B, 4 * B), (4 * B, 8 * B), (12 * B, 4 * B), (6 * B, 2 * B),
              (3 * B, B), (B, 3)]
    off = 0
    for k, (ci, co) in enumerate(shapes):
        taps = 1 if k == 7 else 27
        nw = taps * ci * co
        flat[off:off + nw] = torch.randn(nw, generator=g) * math.sqrt(2.0 / (taps * ci))
        flat[off + nw:off + nw + co] = 0.0
        if k == 7:
            flat[off:off + nw] *= 0.1
            flat[off + nw + 2] = math.log(1.0 / 99.0)
        off += nw + co
    assert off == n
    return flat.cuda()


def train(data, epochs=10, lr=1e-3, lr_final=1e-4, seed=0, log=None, params=None):
    """Adam on the mean per-voxel loss, one volume per step, shuffled
    epochs, exponential rate decay.  Returns (params, loss history)."""
    p = init_params(seed) if params is None else params
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    ws, lws = native.Workspace(), native.Workspace()
    rng = np.random.default_rng(seed)
    hist = []
    steps = epochs * len(data)
    t = 0
    t0 = time.perf_counter()
    for e in range(epochs):
        order = rng.permutation(len(data))
        acc = torch.zeros((), dtype=torch.float64, device="cuda")
        for i in order:
            x, tgt = data[i]
            t += 1
            rate = lr * (lr_final / lr) ** ((t - 1) / max(1, steps - 1))
            out = native.dgr_unet_forward(p, x, ws=ws)
            L, d = native.dgr_unet_loss(out, tgt, ws=lws)
            g = native.dgr_unet_backward(p, x, d, ws)
            native.dgr_adam(p, g, m, v, rate, t)
            acc += L.double()
        hist.append(float(acc) / len(data))
        if log:
            log(f"epoch {e + 1}/{epochs}: loss {hist[-1]:.5f}, {time.perf_counter() - t0:.1f}s")
    return p, hist


def save(params, path=WEIGHTS):
    """Weights as bfloat16 bit patterns (uint16 .npy): what the matrix cores use."""
    os.makedirs(os.path.dirname(path), exist_ok=True)
    bits = params.detach().to(torch.bfloat16).view(torch.int16).cpu().numpy().view(np.uint16)
    np.save(path, bits)


def load(path=WEIGHTS, device="cuda"):
    bits = np.load(path)  # no pickle
    t = torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16).to(torch.float32)
    return t.to(device).contiguous()


# ---- use -------------------------------------------------------------------------------
def learned_init(prob: recon.Problem, params, n=50_000, seed=3004, fdk=None):
    """Gaussians proposed by the network for prob (grid D = TRAIN_D or 2 TRAIN_D)."""
    f = native.dgr_fdk(prob.target, prob.grid, prob.geom, prob.views) if fdk is None else fdk
    D = prob.grid.dims[0]
    if D == 2 * TRAIN_D:
        f = native.dgr_pool2_f32(f)
        cgrid = inputs.cube_grid(D // 2)
    elif D == TRAIN_D:
        cgrid = prob.grid
    else:
        raise ValueError(f"learned initialisation supports {TRAIN_D}^3 and {2 * TRAIN_D}^3 grids")
    x = (f * (1.0 / INPUT_SCALE)).contiguous()
    out = native.dgr_unet_forward(params, x)
    g = torch.Generator(device="cpu").manual_seed(seed)
    uni = torch.rand((n, 4), generator=g, dtype=torch.float32).cuda()
    mu, sc, q, rho = native.dgr_init_from_unet(out, cgrid, n, uni, INPUT_SCALE)
    V1 = native.dgr_voxelize(mu, sc, q, rho, prob.grid, prob.k_sigma, prob.box_half)
    P1 = native.dgr_project(V1, prob.grid, prob.geom, prob.views)
    native.dgr_fit_density_scale(P1, prob.target, rho)
    return {"mu": mu, "scale": sc, "quat": q, "density": rho}


# ---- evaluation against the plain initialisation ------------------------------------
def time_to(history, level):
    """(iteration, seconds) of the first PSNR check at or above level, or None."""
    for i, s, p, _ in history:
        if p >= level:
            return i, s
    return None


def evaluate(params, seeds=(3002, 59000, 59001), D=256, n=50_000, iters=600, check_every=20,
             levels=(30.0, 31.0, 32.0, 33.0, 35.0), log=None):
    """Plain FDK-sampled vs learned initialisation on 25-view cone problems:
    PSNR after initialisation and iterations / seconds to each PSNR level.
    The clock starts with the projections resident on the GPU and includes
    FDK, the network and the density fit."""
    res = []
    for seed in seeds:
        prob, gt = recon.sparse_view_problem(D=D, seeds=(seed, seed + 1))
        row = {"phantom_seed": seed}
        for kind in ("plain", "learned"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            prob.params = (recon.fdk_init(prob, n=n) if kind == "plain" else learned_init(prob, params, n=n))
            V0 = native.dgr_voxelize(*(prob.params[k] for k in recon.Iteration.ORDER), prob.grid,
                                     prob.k_sigma, prob.box_half)
            p0 = float(native.dgr_psnr(V0, gt)[0])
            r = recon.reconstruct(prob, gt, max_iters=iters, check_every=check_every, t_start=t0,
                                  target_psnr=1e9)
            h = r["history"]
            row[kind] = {"psnr_init": round(p0, 3), "best_psnr": round(r["best_psnr"], 3),
                         "best_iter": r["best_iter"], "final_psnr": round(r["final_psnr"], 3),
                         "seconds": round(h[-1][1], 2),
                         "to_level": {f"{lv:g}": time_to(h, lv) for lv in levels}}
            if log:
                log(f"seed {seed} {kind}: init {p0:.2f} dB, best {r['best_psnr']:.2f} dB @ {r['best_iter']}, "
                    f"levels {row[kind]['to_level']}")
        res.append(row)
    return res


def quick_eval(params, seeds=(59100, 59110), n=50_000, iters=40, plain_scale=None):
    """Held-out 256^3 sparse-view phantoms, L1 loop, PSNR after every step:
    PSNR after the initialisation and after 10 / 20 / 40 steps, steps to
    35 dB, and the proposed scales in 256^3 voxels (quartiles).  With
    plain_scale the plain FDK-sampled initialisation at that scale instead."""
    out = []
    for seed in seeds:
        prob, gt = recon.sparse_view_problem(D=256, seeds=(seed, seed + 1))
        prob.params = (recon.fdk_init(prob, n=n, scale_vox=plain_scale) if plain_scale is not None
                       else learned_init(prob, params, n=n))
        sc = prob.params["scale"][:, 0].float() * prob.grid.inv_h[0]
        q = torch.quantile(sc, torch.tensor([0.25, 0.5, 0.75], device=sc.device)).tolist()
        r = recon.reconstruct(prob, gt, max_iters=iters, check_every=20, target_psnr=1e9)
        h = [x[2] for x in r["history"]]
        out.append({"seed": seed, "psnr": {k: round(h[k], 2) for k in (0, 10, 20, iters)},
                    "steps_to_35": next((x[0] for x in r["history"] if x[2] >= 35.0), None),
                    "scale_vox_quartiles": [round(v, 2) for v in q]})
    return out


def learning_curve(sizes, first_seed=50_000, epochs=8, objective="full", iters=200, out_dir=None, log=None,
                   compare=None):
    """Models trained (same recipe) on nested subsets of one set of pairs,
    each scored by quick_eval, beside the plain initialisation at 3 voxels
    (and the weights at path `compare`)."""
    t0 = time.perf_counter()
    data = make_dataset(range(first_seed, first_seed + max(sizes)), log=log, objective=objective,
                        iters=iters)
    res = {"objective": objective, "iters": iters, "epochs": epochs,
           "data_s": round(time.perf_counter() - t0, 1), "plain3": quick_eval(None, plain_scale=3.0)}
    if log:
        log(f"plain3: {res['plain3']}")
    if compare:
        res["compare"] = {"weights": os.path.basename(compare), "eval": quick_eval(load(compare))}
        if log:
            log(f"compare: {res['compare']}")
    for n in sizes:
        t0 = time.perf_counter()
        params, hist = train(data[:n], epochs=epochs)
        ev = quick_eval(params)
        res[str(n)] = {"final_loss": round(hist[-1], 5), "train_s": round(time.perf_counter() - t0, 1),
                       "eval": ev}
        if log:
            log(f"{n} pairs: {res[str(n)]}")
        if out_dir:
            save(params, os.path.join(out_dir, f"unet_b32_d128_{n}.npy"))
    return res


def conv_flops(D=TRAIN_D, B=None):
    """Multiply-add flops (x2) of one forward pass on a D^3 volume."""
    B = B or native.UNET_BASE
    V = [D ** 3 // 8 ** l for l in range(4)]
    layers = [(1, B, 0), (B, 2 * B, 1), (2 * B, 4 * B, 2), (4 * B, 8 * B, 3), (12 * B, 4 * B, 2),
              (6 * B, 2 * B, 1), (3 * B, B, 0)]
    f = sum(2 * 27 * ci * co * V[l] for ci, co, l in layers)
    return f + 2 * B * 3 * V[0]


def step_bench(steps=20, D=TRAIN_D, log=None):
    """Time training steps (forward, loss, backward, Adam) on a random D^3
    volume; returns ms per step and achieved bf16 TFLOP/s (forward + data
    gradient + weight gradient ~ 3x the forward's flops, less the first
    layer's data gradient)."""
    p = init_params(1)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    g = torch.Generator(device="cuda").manual_seed(2)
    x = torch.randn((D, D, D), generator=g, device="cuda")
    tgt = torch.rand((D, D, D, 3), generator=g, device="cuda")
    ws, lws = native.Workspace(), native.Workspace()

    def one(t):
        out = native.dgr_unet_forward(p, x, ws=ws)
        L, d = native.dgr_unet_loss(out, tgt, ws=lws)
        gr = native.dgr_unet_backward(p, x, d, ws)
        native.dgr_adam(p, gr, m, v, 1e-4, t)

    one(1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for t in range(steps):
        one(t + 2)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    fw = conv_flops(D)
    flops = 3 * fw - 2 * 27 * native.UNET_BASE * D ** 3
    res = {"volume": D, "ms_per_step": round(ms, 3), "tflops_per_step": round(flops / 1e12, 3),
           "achieved_tflops": round(flops / (ms * 1e-3) / 1e12, 1), "bf16_peak_tflops": 2500.0}
    if log:
        log(str(res))
    return res


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="learned initialisation: train or evaluate the U-Net")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--pairs", type=int, default=1600)
    t.add_argument("--first-seed", type=int, default=50_000)
    t.add_argument("--epochs", type=int, default=8)
    t.add_argument("--gaussians", type=int, default=20_000)
    t.add_argument("--iters", type=int, default=200)
    t.add_argument("--objective", default="full", choices=("l1", "full"))
    t.add_argument("--out", default=WEIGHTS)
    c = sub.add_parser("curve")
    c.add_argument("--sizes", default="125,250,500,1000")
    c.add_argument("--first-seed", type=int, default=50_000)
    c.add_argument("--epochs", type=int, default=8)
    c.add_argument("--iters", type=int, default=200)
    c.add_argument("--objective", default="full", choices=("l1", "full"))
    c.add_argument("--out-dir", default=None)
    c.add_argument("--json", default=None)
    c.add_argument("--compare", default=None)
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--seeds", default="3002,59000,59001")
    e.add_argument("--iters", type=int, default=600)
    e.add_argument("--json", default=None)
    sb = sub.add_parser("step-bench")
    sb.add_argument("--steps", type=int, default=20)
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)  # noqa: E731
    if a.cmd == "train":
        data = make_dataset(range(a.first_seed, a.first_seed + a.pairs), log=log, n_gauss=a.gaussians,
                            iters=a.iters, objective=a.objective)
        params, hist = train(data, epochs=a.epochs, log=log)
        save(params, a.out)
        log(json.dumps({"pairs": a.pairs, "epochs": a.epochs, "loss": hist}))
    elif a.cmd == "curve":
        if a.out_dir:
            os.makedirs(a.out_dir, exist_ok=True)
        res = learning_curve([int(x) for x in a.sizes.split(",")], first_seed=a.first_seed, epochs=a.epochs,
                             objective=a.objective, iters=a.iters, out_dir=a.out_dir, log=log,
                             compare=a.compare)
        txt = json.dumps(res)
        if a.json:
            with open(a.json, "w") as f:
                f.write(txt + "\n")
        print(txt, flush=True)
    elif a.cmd == "step-bench":
        print(json.dumps(step_bench(a.steps)), flush=True)
    else:
        params = load(a.weights)
        res = evaluate(params, seeds=[int(s) for s in a.seeds.split(",")], iters=a.iters, log=log)
        txt = json.dumps(res)
        if a.json:
            with open(a.json, "w") as f:
                f.write(txt + "\n")
        print(txt, flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
