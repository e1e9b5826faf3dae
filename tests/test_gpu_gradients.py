"""Gradients through the autograd wrappers and the binary64 finite-difference
path, checked against the oracle.

* The autograd chain (DGRVoxelize -> DGRProject -> loss) gives the oracle's
  gradient (voxelize -> project -> dL/dP -> backproject -> voxelize_grad).
  An L2 loss is used here: L1 takes the sign of residuals, and residuals near
  zero flip sign between binary32 and binary64.
* The GPU binary64 finite-difference kernel reproduces finite differences the
  oracle computes with its own voxelizer, projector and L1 loss.
* Central differences of the L1 loss agree with the analytic binary32 gradient.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2411_04844_amd import autograd, inputs, native

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


GRID = inputs.GridSpec((40, 36, 32), (-1.0, -0.9, -0.8), (20.0, 20.0, 20.0))
GEOM = inputs.cone_geometry(8, 48, 40, 0.045, 7.8125, 11.71875, 0.025, arc=2 * math.pi)
NAMES = ("mu", "scale", "quat", "density")


def _gauss(n, seed, lo, hi):
    G = inputs.gaussians(n, seed, lo, hi, mean_lim=0.55)
    return G, {k: torch.as_tensor(G[k]).cuda() for k in NAMES}


def test_autograd_chain_matches_oracle_l2():
    say("autograd L2")
    G, d = _gauss(250, 301, 0.03, 0.09)
    views = torch.as_tensor(GEOM.views).cuda()
    rng = np.random.default_rng(1)
    y = rng.uniform(0.0, 2.0, size=(GEOM.n_views, GEOM.nv, GEOM.nu)).astype(np.float32)
    params = {k: d[k].clone().requires_grad_(True) for k in NAMES}
    V = autograd.voxelize(params["mu"], params["scale"], params["quat"], params["density"], GRID)
    P = autograd.project(V, GRID, GEOM, views)
    L = ((P - torch.as_tensor(y).cuda()) ** 2).mean()
    L.backward()
    # oracle chain
    box = oracle.bbox(G["mu"], G["scale"], G["quat"], GRID.dims, GRID.lo, GRID.inv_h)
    Vo = oracle.voxelize(G["mu"], G["scale"], G["quat"], G["density"], GRID.dims, GRID.lo, GRID.inv_h, box)
    Po = oracle.project(Vo, GRID.dims, GRID.lo, GRID.inv_h, GEOM.kind, GEOM.views, GEOM.nu, GEOM.nv,
                        GEOM.step, GEOM.length_scale)
    dP = 2.0 * (Po - y.astype(np.float64)) / Po.size
    dV = oracle.backproject(dP, GRID.dims, GRID.lo, GRID.inv_h, GEOM.kind, GEOM.views, GEOM.nu, GEOM.nv,
                            GEOM.step, GEOM.length_scale)
    want = oracle.voxelize_grad(G["mu"], G["scale"], G["quat"], G["density"], GRID.dims, GRID.lo,
                                GRID.inv_h, box, dV)
    for k, w in zip(NAMES, want):
        err = rel_l2(params[k].grad.cpu().numpy(), w)
        say("autograd", k, err)
        assert err < 1e-5, (k, err)


def test_voxelize_f64_matches_oracle():
    say("voxelize f64")
    G, d = _gauss(400, 302, 0.02, 0.08)
    V = native.dgr_voxelize_f64(d["mu"], d["scale"], d["quat"], d["density"], GRID).cpu().numpy()
    box = oracle.bbox(G["mu"], G["scale"], G["quat"], GRID.dims, GRID.lo, GRID.inv_h)
    want = oracle.voxelize(G["mu"], G["scale"], G["quat"], G["density"], GRID.dims, GRID.lo, GRID.inv_h, box)
    err = rel_l2(V, want)
    say("voxelize f64 rel_l2", err)
    assert err < 1e-13


def _fd_setup(seed):
    G, d = _gauss(120, seed, 0.09, 0.14)  # sigma 1.8 - 2.8 voxels
    views = torch.as_tensor(GEOM.views).cuda()
    box = oracle.bbox(G["mu"], G["scale"], G["quat"], GRID.dims, GRID.lo, GRID.inv_h)
    Vo = oracle.voxelize(G["mu"], G["scale"], G["quat"], G["density"], GRID.dims, GRID.lo, GRID.inv_h, box)
    Po = oracle.project(Vo, GRID.dims, GRID.lo, GRID.inv_h, GEOM.kind, GEOM.views, GEOM.nu, GEOM.nv,
                        GEOM.step, GEOM.length_scale)
    # residuals bounded away from zero, so that +-h never crosses a kink of |r|
    rng = np.random.default_rng(seed)
    off = Po.std()
    y = (Po + off * (1.0 + 0.2 * rng.uniform(size=Po.shape))).astype(np.float32)
    return G, d, views, box, y


def _perturbed(G, gid, comp, h):
    P = {k: G[k].astype(np.float64).copy() for k in NAMES}
    if comp < 3:
        P["mu"][gid, comp] += h
    elif comp < 6:
        P["scale"][gid, comp - 3] += h
    elif comp < 10:
        P["quat"][gid, comp - 6] += h
    else:
        P["density"][gid] += h
    return P


def test_fd_kernel_matches_oracle_finite_differences():
    say("fd kernel vs oracle")
    G, d, views, box, y = _fd_setup(303)
    jobs = [(3, 0, 1e-4), (7, 4, 1e-4), (11, 7, 1e-4), (20, 10, 1e-4), (33, 2, 1e-4), (40, 9, 1e-4)]
    V64 = native.dgr_voxelize_f64(d["mu"], d["scale"], d["quat"], d["density"], GRID)
    got = native.dgr_fd_l1_f64(V64, torch.as_tensor(y).cuda(), d["mu"], d["scale"], d["quat"],
                               d["density"], GRID, GEOM, views, jobs).cpu().numpy()

    def loss(P):
        V = oracle.voxelize(P["mu"], P["scale"], P["quat"], P["density"], GRID.dims, GRID.lo,
                            GRID.inv_h, box)
        Pr = oracle.project(V, GRID.dims, GRID.lo, GRID.inv_h, GEOM.kind, GEOM.views, GEOM.nu,
                            GEOM.nv, GEOM.step, GEOM.length_scale)
        return oracle.l1(Pr, y)[0]

    L0 = loss({k: G[k].astype(np.float64) for k in NAMES})
    for i, (gid, comp, h) in enumerate(jobs):
        dp = loss(_perturbed(G, gid, comp, h)) - L0
        dm = loss(_perturbed(G, gid, comp, -h)) - L0
        say("fd job", (gid, comp), got[i], (dp, dm))
        # the oracle differences full losses, so they carry the binary64
        # rounding of L0 (a sum over every ray): allow 1e-12 |L0| besides 1e-6
        tol = 1e-6 * max(abs(dp), abs(dm)) + 1e-12 * abs(L0)
        assert abs(got[i, 0] - dp) <= tol
        assert abs(got[i, 1] - dm) <= tol


def test_fd_agrees_with_analytic_gradient():
    say("fd vs analytic")
    G, d, views, box, y = _fd_setup(304)
    yt = torch.as_tensor(y).cuda()
    V = native.dgr_voxelize(d["mu"], d["scale"], d["quat"], d["density"], GRID)
    loss, dproj = native.dgr_project_l1(V, yt, GRID, GEOM, views)
    dV = native.dgr_backproject(dproj, GRID, GEOM, views)
    grads = native.dgr_voxelize_backward(d["mu"], d["scale"], d["quat"], d["density"], dV, GRID)
    flat = [g.cpu().numpy().astype(np.float64) for g in grads]
    rng = np.random.default_rng(5)
    gids = rng.choice(len(G["density"]), size=16, replace=False)
    comps = rng.integers(0, 11, size=16)
    h = 1e-4
    jobs = [(int(g), int(c), h) for g, c in zip(gids, comps)]
    V64 = native.dgr_voxelize_f64(d["mu"], d["scale"], d["quat"], d["density"], GRID)
    fd = native.dgr_fd_l1_f64(V64, yt, d["mu"], d["scale"], d["quat"], d["density"], GRID, GEOM,
                              views, jobs).cpu().numpy()
    errs = []
    for i, (g, c, _) in enumerate(jobs):
        num = (fd[i, 0] - fd[i, 1]) / (2 * h)
        if c < 3:
            ana = flat[0][g, c]
        elif c < 6:
            ana = flat[1][g, c - 3]
        elif c < 10:
            ana = flat[2][g, c - 6]
        else:
            ana = flat[3][g]
        errs.append(abs(num - ana) / max(abs(ana), 1e-3 * np.abs(np.concatenate([f.ravel() for f in flat])).max()))
        say("fd", (g, c), num, ana)
    say("fd vs analytic max rel err", max(errs))
    assert max(errs) < 1e-3
