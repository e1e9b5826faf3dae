"""One DGR optimisation iteration on the GPU, driven through the C ABI.

    voxelize (Alg. 1)  ->  project + L1 (sec. 4.3)  ->  backproject (adjoint)
    ->  voxelize backward  ->  Adam (sec. 5.1)

The volume is not kept for the backward pass: the projector is linear, so the
backward needs only dL/dP (written by the fused L1 kernel), and the voxelizer
backward needs only the parameters and dL/dV.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from . import inputs, native


@dataclass
class LearningRates:
    # density 1e-3; scale and mean 5e-4; quaternion 1e-3 (not fixed by the
    # workload description; chosen equal to the density rate)
    mu: float = 5e-4
    scale: float = 5e-4
    quat: float = 1e-3
    density: float = 1e-3


@dataclass
class Problem:
    grid: inputs.GridSpec
    geom: inputs.Geometry
    views: torch.Tensor          # device [n_views, 12]
    target: torch.Tensor         # device [n_views, nv, nu]
    params: dict                 # mu, scale, quat, density (device, float32)
    k_sigma: float = 3.0
    box_half: int = 8
    lr: LearningRates = field(default_factory=LearningRates)


class Iteration:
    """Buffers and workspaces for repeated fwd+bwd+Adam steps.

    objective "l1": mean |P_hat - P| (the fused projector + L1 kernel);
    "full": the paper's w1 L1 + w2 L_SSIM + w3 L_TV (sec. 4.3), with the
    projection terms on P_hat and TV on the kept volume."""

    ORDER = ("mu", "scale", "quat", "density")

    def __init__(self, prob: Problem, pair_headroom: float = 1.5, objective: str = "l1",
                 weights=(0.6, 0.2, 1.0)):
        if objective not in ("l1", "full"):
            raise ValueError(f"unknown objective {objective!r}")
        self.objective = objective
        self.weights = tuple(float(w) for w in weights)
        self.p = prob
        dev = prob.target.device
        self.vox_ws = native.Workspace(dev)
        self.bwd_ws = native.Workspace(dev)
        self.proj_ws = native.Workspace(dev)
        P = prob.params
        pairs = native.dgr_voxelize_plan(P["mu"], P["scale"], P["quat"], prob.grid, prob.k_sigma,
                                         prob.box_half, self.vox_ws)
        self.max_pairs = int(pairs * pair_headroom) + 1024
        self.V = torch.empty(prob.grid.shape, dtype=torch.float32, device=dev)
        self.dV = torch.empty_like(self.V)
        self.dproj = torch.empty_like(prob.target)
        self.loss = torch.zeros((), dtype=torch.float32, device=dev)
        self.grads = {k: torch.empty_like(P[k]) for k in self.ORDER}
        self.m = {k: torch.zeros_like(P[k]) for k in self.ORDER}
        self.v = {k: torch.zeros_like(P[k]) for k in self.ORDER}
        self.t = 0
        self.lr_factor = 1.0  # multiplies every group's rate (schedules)
        # projected steps: scales stay above 1/20 voxel, densities non-negative
        h = 1.0 / max(prob.grid.inv_h)
        self.lower = {"mu": float("-inf"), "scale": 0.05 * h, "quat": float("-inf"), "density": 0.0}
        # allocate the workspaces once, outside any timed region
        self.vox_ws.get(native.dgr_voxelize_workspace(P["mu"].shape[0], self.max_pairs, prob.grid))
        self.proj_ws.get(native.dgr_project_workspace(prob.grid, prob.geom, prob.views))
        if objective == "full":
            self.P = torch.empty_like(prob.target)
            self.loss = torch.zeros(3, dtype=torch.float32, device=dev)
            self.tv_value = torch.zeros(1, dtype=torch.float32, device=dev)
            self.obj_ws, self.tv_ws = native.Workspace(dev), native.Workspace(dev)
            g = prob.geom
            self.obj_ws.get(int(native.lib().dgr_projection_loss_workspace(g.n_views, g.nv, g.nu)))
            self.tv_ws.get(int(native.lib().dgr_tv_workspace()))
            self.STAGES = ("voxelize", "project", "projection_loss", "backproject", "tv",
                           "voxelize_backward", "adam")

    # individual stages (each one C-ABI call or a few)
    def voxelize(self):
        P, pr = self.p.params, self.p
        native.dgr_voxelize(P["mu"], P["scale"], P["quat"], P["density"], pr.grid, pr.k_sigma,
                            pr.box_half, out=self.V, ws=self.vox_ws, max_pairs=self.max_pairs)

    def project_l1(self):
        pr = self.p
        native.dgr_project_l1(self.V, pr.target, pr.grid, pr.geom, pr.views, loss=self.loss,
                              dproj=self.dproj, ws=self.proj_ws)

    def project(self):
        pr = self.p
        native.dgr_project(self.V, pr.grid, pr.geom, pr.views, out=self.P, ws=self.proj_ws)

    def projection_loss(self):
        native.dgr_projection_loss(self.P, self.p.target, self.weights[0], self.weights[1], loss=self.loss,
                                   dproj=self.dproj, ws=self.obj_ws)

    def tv(self):
        native.dgr_tv(self.V, self.p.grid, self.dV, self.weights[2], loss=self.tv_value, ws=self.tv_ws)

    def total_loss(self) -> float:
        """The objective's value (synchronises)."""
        if self.objective == "l1":
            return float(self.loss)
        return float(self.loss[0]) + self.weights[2] * float(self.tv_value[0])

    def backproject(self):
        pr = self.p
        native.dgr_backproject(self.dproj, pr.grid, pr.geom, pr.views, out=self.dV, ws=self.proj_ws)

    def voxelize_backward(self):
        P, pr = self.p.params, self.p
        native.dgr_voxelize_backward(P["mu"], P["scale"], P["quat"], P["density"], self.dV, pr.grid,
                                     pr.k_sigma, pr.box_half, ws=self.bwd_ws,
                                     outs=tuple(self.grads[k] for k in self.ORDER))

    def adam(self):
        self.t += 1
        for k in self.ORDER:
            native.dgr_adam(self.p.params[k], self.grads[k], self.m[k], self.v[k],
                            getattr(self.p.lr, k) * self.lr_factor, self.t, lower=self.lower[k])

    STAGES = ("voxelize", "project_l1", "backproject", "voxelize_backward", "adam")

    def set_gaussians(self, P, m, v, headroom: float = 1.5):
        """Install a new Gaussian set with its Adam moments (after density
        control): fresh gradient buffers and a re-planned pair capacity."""
        pr = self.p
        pr.params, self.m, self.v = P, m, v
        self.grads = {k: torch.empty_like(P[k]) for k in self.ORDER}
        pairs = native.dgr_voxelize_plan(P["mu"], P["scale"], P["quat"], pr.grid, pr.k_sigma, pr.box_half,
                                         self.vox_ws)
        self.max_pairs = int(pairs * headroom) + 1024
        self.vox_ws.get(native.dgr_voxelize_workspace(P["mu"].shape[0], self.max_pairs, pr.grid))

    def step(self, events=None):
        """One iteration; with `events` (dict stage -> list), HIP events
        bracket each stage on the current stream."""
        for name in self.STAGES:
            if events is not None:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                getattr(self, name)()
                b.record()
                events.setdefault(name, []).append((a, b))
            else:
                getattr(self, name)()

    def check(self):
        """Raise if a voxelization overflowed its pair capacity."""
        native.dgr_check(self.vox_ws)

    def replan(self, headroom: float = 1.25):
        """Synchronising: grow the pair capacity if the boxes now need more."""
        P, pr = self.p.params, self.p
        pairs = native.dgr_voxelize_plan(P["mu"], P["scale"], P["quat"], pr.grid, pr.k_sigma,
                                         pr.box_half, self.vox_ws)
        if pairs * headroom > self.max_pairs:
            self.max_pairs = int(pairs * 1.5) + 1024
            self.vox_ws.get(native.dgr_voxelize_workspace(P["mu"].shape[0], self.max_pairs,
                                                          pr.grid))
        return pairs


class DensityControl:
    """Alg. 2 on the GPU: ||dL/dmu|| accumulated every iteration, a clone /
    split / prune pass (dgr_densify) every `every` iterations, n capped at
    n_max.  theta defaults to 0.005 of the grid's body diagonal.  Split draws
    are standard normals from a seeded generator."""

    def __init__(self, prob: Problem, n_max=500_000, every=100, tau=2e-5, tau_prune=1e-9, theta=None,
                 size_vox=17.0, seed=3006):
        g = prob.grid
        diag = sum((g.dims[a] / g.inv_h[a]) ** 2 for a in range(3)) ** 0.5
        self.theta = 0.005 * diag if theta is None else theta
        self.n_max, self.every, self.tau, self.tau_prune, self.size_vox = n_max, every, tau, tau_prune, size_vox
        dev = prob.target.device
        self.bufs = []
        for _ in range(2):
            trio = []
            for _ in range(3):
                trio.append({k: torch.empty((n_max,) + (() if k == "density" else (native.WIDTH[k],)),
                                            dtype=torch.float32, device=dev) for k in Iteration.ORDER})
            self.bufs.append(tuple(trio))
        self.cur = None  # which buffer holds the current set (None: the problem's own tensors)
        self.acc = torch.zeros(prob.params["mu"].shape[0], dtype=torch.float32, device=dev)
        self.gen = torch.Generator(device=dev).manual_seed(seed)
        self.ws = native.Workspace(dev)
        self.log = []

    def accumulate(self, it: "Iteration"):
        native.dgr_accumulate_grad_norm(it.grads["mu"], self.acc)

    def densify(self, it: "Iteration", iteration: int):
        P = it.p.params
        n = P["mu"].shape[0]
        dst_i = 0 if self.cur != 0 else 1
        dst = self.bufs[dst_i]
        normals = torch.randn((n, 2, 3), generator=self.gen, device=self.acc.device)
        n_new, counts = native.dgr_densify(P, it.m, it.v, self.acc, normals, it.p.grid, dst, self.every,
                                           self.tau, self.tau_prune, self.theta, self.size_vox, self.n_max,
                                           ws=self.ws)
        it.set_gaussians({k: dst[0][k][:n_new] for k in Iteration.ORDER},
                         {k: dst[1][k][:n_new] for k in Iteration.ORDER},
                         {k: dst[2][k][:n_new] for k in Iteration.ORDER})
        self.cur = dst_i
        self.acc = torch.zeros(n_new, dtype=torch.float32, device=self.acc.device)
        self.log.append((iteration, n, n_new) + counts)
        return n_new, counts


# --------------------------------------------------------------------------
# workload builders
# --------------------------------------------------------------------------
def cone_problem(D=256, n=100_000, n_views=360, n_det=512, pitch_mm=0.8, s_lo=0.004, s_hi=0.03,
                 seeds=(2001, 2002, 2003), device="cuda", ratio_max=None, geom=None) -> Problem:
    """Synthetic cone-beam workload: seeded Gaussians, ellipsoid phantom with
    analytic projections plus 1 % Gaussian noise as the target.  `geom`
    replaces the cone geometry (e.g. a fan-beam slice stack)."""
    grid = inputs.cube_grid(D)
    geom = geom if geom is not None else inputs.cone_workload(D, n_views, n_det, pitch_mm)
    G = inputs.gaussians(n, seeds[0], s_lo, s_hi, ratio_max=ratio_max)
    ph = inputs.ellipsoid_phantom(seeds[1])
    y = inputs.phantom_projections(ph, geom, device=device)
    y = inputs.add_noise(y, seeds[2]).contiguous()
    params = {k: torch.as_tensor(G[k]).to(device).contiguous() for k in Iteration.ORDER}
    views = torch.as_tensor(geom.views).to(device).contiguous()
    return Problem(grid, geom, views, y, params)


# --------------------------------------------------------------------------
# sparse-view reconstruction loop
# --------------------------------------------------------------------------
def sparse_view_problem(D=256, n_views=25, n_det=512, pitch_mm=0.8, seeds=(3002, 3003),
                        device="cuda", noise_frac=0.01):
    """Cone-beam sparse-view workload and its ground-truth volume (the phantom
    averaged over 4^3 points per voxel); the target carries Gaussian noise of
    noise_frac * max(y).  Parameters are filled in by an initialisation."""
    grid = inputs.cube_grid(D)
    geom = inputs.cone_workload(D, n_views, n_det, pitch_mm)
    ph = inputs.ellipsoid_phantom(seeds[0])
    y = inputs.add_noise(inputs.phantom_projections(ph, geom, device=device), seeds[1],
                         noise_frac).contiguous()
    gt = inputs.phantom_volume(ph, grid, device=device).to(torch.float32).contiguous()
    views = torch.as_tensor(geom.views).to(device).contiguous()
    return Problem(grid, geom, views, y, {}), gt


def fan_problem(D=256, n_views=60, n_det=384, arc=2 * math.pi, start=0.0, seeds=(3002, 3003),
                device="cuda", noise_frac=0.01):
    """Fan-beam workload: a stack of D fan-beam slices (one detector row per
    slice), n_views over `arc` radians from `start`; with arc = pi/2 it is the
    90-degree limited-angle setting.  The same phantom recipe and noise as the
    cone-beam workloads; returns (Problem, ground-truth volume)."""
    grid = inputs.cube_grid(D)
    geom = inputs.fan_workload(D, n_views, n_det, arc=arc, start=start)
    ph = inputs.ellipsoid_phantom(seeds[0])
    y = inputs.add_noise(inputs.phantom_projections(ph, geom, device=device), seeds[1],
                         noise_frac).contiguous()
    gt = inputs.phantom_volume(ph, grid, device=device).to(torch.float32).contiguous()
    views = torch.as_tensor(geom.views).to(device).contiguous()
    return Problem(grid, geom, views, y, {}), gt


def fdk_init(prob: Problem, n=50_000, seed=3004, scale_vox=1.5, thresh=0.1, arc=2 * math.pi):
    """FDK volume (fan-beam FBP for a fan-beam problem) -> n Gaussians drawn
    where it exceeds thresh * max, isotropic scale of scale_vox voxels,
    density = FDK value times the least-squares scale that best fits the
    projections.  Returns the parameter dict."""
    dev = prob.target.device
    f = native.dgr_fdk(prob.target, prob.grid, prob.geom, prob.views, arc=arc)
    g = torch.Generator(device="cpu").manual_seed(seed)
    uni = torch.rand((n, 4), generator=g, dtype=torch.float32).to(dev)
    h = 1.0 / prob.grid.inv_h[0]
    mu, sc, q, rho = native.dgr_init_from_volume(f, prob.grid, n, uni, scale_vox * h, thresh)
    V1 = native.dgr_voxelize(mu, sc, q, rho, prob.grid, prob.k_sigma, prob.box_half)
    P1 = native.dgr_project(V1, prob.grid, prob.geom, prob.views)
    native.dgr_fit_density_scale(P1, prob.target, rho)
    return {"mu": mu, "scale": sc, "quat": q, "density": rho}


def random_init(prob: Problem, n=50_000, seed=3005, s_lo=0.004, s_hi=0.03):
    """Random Gaussians (the fallback initialisation), densities fitted to the
    projections by the same least-squares scale."""
    dev = prob.target.device
    G = inputs.gaussians(n, seed, s_lo, s_hi)
    P = {k: torch.as_tensor(G[k]).to(dev).contiguous() for k in Iteration.ORDER}
    V1 = native.dgr_voxelize(P["mu"], P["scale"], P["quat"], P["density"], prob.grid,
                             prob.k_sigma, prob.box_half)
    P1 = native.dgr_project(V1, prob.grid, prob.geom, prob.views)
    native.dgr_fit_density_scale(P1, prob.target, P["density"])
    return P


def reconstruct(prob: Problem, gt, max_iters=5000, target_psnr=35.0, check_every=10, log=None,
                t_start=None, lr_final_frac=1.0, decay_iters=None, objective="l1", density_control=None):
    """Run fwd+bwd+Adam iterations until the volume PSNR against gt reaches
    target_psnr or max_iters.

    The PSNR is measured after every step, on the device: each iteration's own
    voxelization is the volume of the parameters after the previous step, so
    the extra work is one PSNR reduction per iteration and the first step at
    or above target_psnr is found exactly.  The host reads the values (and
    the loss) every check_every iterations.  The time of step i is taken from
    a HIP event recorded after its Adam update, measured from t_start (the
    caller's perf_counter() before its initialisation; default: entry).

    lr_final_frac < 1 decays every rate exponentially to that fraction over
    decay_iters iterations (default max_iters) and holds it there; the paper
    decays its rate tenfold over training (sec. 5.1).  Returns a dict with
    the step count at which the target was reached (0: the initialisation
    itself), its seconds, and the history [(steps, seconds, psnr, loss or
    None)] with one entry per step.

    density_control: None, or a dict of DensityControl arguments (Alg. 2
    every `every` iterations)."""
    import time
    t0 = time.perf_counter() if t_start is None else t_start
    it = Iteration(prob, objective=objective)
    dc = DensityControl(prob, **density_control) if density_control is not None else None
    decay_iters = decay_iters or max_iters
    dev = prob.target.device
    rows = torch.empty((check_every, 3), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t_before = time.perf_counter() - t0  # initialisation, before the first step
    ev0 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    hist, pending = [], []
    reached = None
    done, last_ev = 0, ev0
    while True:
        it.voxelize()  # the volume of the parameters after `done` steps
        native.dgr_psnr(it.V, gt, out=rows[len(pending)])
        pending.append((done, last_ev))
        if len(pending) == check_every or done == max_iters:
            torch.cuda.synchronize()
            vals = rows[:len(pending), 0].cpu().tolist()
            for (steps, ev), val in zip(pending, vals):
                sec = t_before + (ev0.elapsed_time(ev) / 1e3 if steps > 0 else 0.0)
                hist.append((steps, sec, val, None))
                if reached is None and val >= target_psnr:
                    reached = steps
            pending.clear()
            it.check()
            loss = it.total_loss() if done > 0 else None
            hist[-1] = hist[-1][:3] + (loss,)
            if log:
                log(f"iter {done}: PSNR {hist[-1][2]:.2f} dB, loss {loss if loss is None else f'{loss:.5g}'}, "
                    f"{hist[-1][1]:.1f}s")
            if reached is not None or done == max_iters:
                break
            it.replan()
        # the rest of step done + 1
        it.lr_factor = lr_final_frac ** (min(done, decay_iters) / decay_iters)
        for name in it.STAGES[1:]:
            getattr(it, name)()
        done += 1
        if dc is not None:
            dc.accumulate(it)
            if done % dc.every == 0 and done < max_iters:
                n_new, counts = dc.densify(it, done)
                if log:
                    log(f"iter {done}: density control -> {n_new} Gaussians (cloned {counts[0]}, split "
                        f"{counts[1]}, pruned {counts[2]})")
        last_ev = torch.cuda.Event(enable_timing=True)
        last_ev.record()
    best = max(hist, key=lambda h: h[2])
    extra = {"density_control": dc.log} if dc is not None else {}
    at = next((h for h in hist if h[0] == reached), None)
    return {**extra, "iterations": reached, "seconds": at[1] if at else None,
            "final_psnr": hist[-1][2], "best_psnr": best[2], "best_iter": best[0],
            "history": hist}
