"""Large-volume gradient check: 512^3, 500,000 anisotropic Gaussians (scale
ratio up to 10:1), cone beam 720 views x 1024^2 at 0.4 mm.

The binary32 gradient of the mean-L1 loss (project + L1 -> backproject ->
voxelize backward; the volume is never kept for the backward pass) is checked
against binary64 central differences on 64 randomly chosen (Gaussian,
parameter) pairs: 32 from Gaussians with a scale ratio of 5:1 to 10:1 and 32
from the rest.  The step is h = 1e-4 (world units for means and scales, raw
components for quaternions and densities), shrunk in proportion for means and
scales of Gaussians whose smallest scale is below 0.004 (about one voxel), so that
the central difference's own error, about (h / scale)^2 / 6, stays below
1e-4.  The boxes are held fixed on both sides.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2411_04844_amd import inputs, native, recon

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_large_volume_gradient_vs_finite_differences():
    say("large: building 512^3 / 500k / 720 x 1024^2")
    prob = recon.cone_problem(D=512, n=500_000, n_views=720, n_det=1024, pitch_mm=0.4,
                              seeds=(4001, 4002, 4003), ratio_max=10.0)
    it = recon.Iteration(prob)
    it.voxelize()
    it.project_l1()
    it.backproject()
    it.voxelize_backward()
    torch.cuda.synchronize()
    it.check()
    say("large: binary32 gradient done, loss", float(it.loss))
    P = {k: v.cpu().numpy() for k, v in prob.params.items()}
    smin, smax = P["scale"].min(axis=1), P["scale"].max(axis=1)
    ratio = smax / smin
    rng = np.random.default_rng(4004)
    aniso = np.nonzero(ratio >= 5.0)[0]
    rest = np.nonzero(ratio < 5.0)[0]
    gids = np.concatenate([rng.choice(aniso, size=32, replace=False), rng.choice(rest, size=32, replace=False)])
    comps = rng.integers(0, 11, size=64)
    hs = [1e-4 * (min(1.0, smin[g] / 0.004) if c < 6 else 1.0) for g, c in zip(gids, comps)]
    jobs = [(int(g), int(c), float(h)) for g, c, h in zip(gids, comps, hs)]
    V64 = native.dgr_voxelize_f64(*(prob.params[k] for k in recon.Iteration.ORDER), prob.grid)
    fd = native.dgr_fd_l1_f64(V64, prob.target, *(prob.params[k] for k in recon.Iteration.ORDER),
                              prob.grid, prob.geom, prob.views, jobs, box_cap=1 << 17).cpu().numpy()
    assert np.all(np.isfinite(fd))
    grads = [it.grads[k].cpu().numpy().astype(np.float64) for k in recon.Iteration.ORDER]

    def ana(g, c):
        if c < 3:
            return grads[0][g, c]
        if c < 6:
            return grads[1][g, c - 3]
        if c < 10:
            return grads[2][g, c - 6]
        return grads[3][g]

    hv = np.array(hs)
    num = (fd[:, 0] - fd[:, 1]) / (2 * hv)
    a = np.array([ana(g, c) for g, c, _ in jobs])
    floor = 1e-3 * np.abs(a).max()
    err = np.abs(num - a) / np.maximum(np.abs(a), floor)
    for (g, c, h), e, x, y in zip(jobs, err, num, a):
        say(f"large: gid {g} comp {c} ratio {ratio[g]:.2f} smin/vox {smin[g] * prob.grid.inv_h[0]:.3f} "
            f"h {h:.2e} fd {x:.6e} analytic {y:.6e} err {e:.2e}")
    say("large: FD rel err median", float(np.median(err)), "p90", float(np.quantile(err, 0.9)),
        "max", float(err.max()), "| ratio >= 5 max", float(err[:32].max()), "| rest max", float(err[32:].max()))
    assert ratio[gids[:32]].max() > 8.0  # the 10:1 end of the range is covered
    assert np.quantile(err, 0.9) < 1e-4
    assert err.max() < 1e-3


def test_large_backproject_across_view_batches():
    """720 views of 1024^2 need six batches of the ray table (6 GiB each at
    most): data on two views of different batches backprojects, through the
    packed tile whose sums each batch adds to the previous batches', to the
    oracle's volume voxel by voxel.  (Two views of random data and two of
    constant data, so both the rounding and the largest sums are tested.)"""
    import oracle
    grid = inputs.cube_grid(512)
    geom = inputs.cone_workload(512, 720, 1024, 0.4)
    views = torch.as_tensor(geom.views).cuda()
    rng = np.random.default_rng(4005)
    for name, sel in (("random", [7, 371]), ("constant", [250, 611])):
        say("large backproject across batches", name, sel)
        g = np.zeros((geom.n_views, geom.nv, geom.nu), np.float32)
        g[sel] = rng.normal(size=(len(sel), geom.nv, geom.nu)) if name == "random" else 1.0
        got = native.dgr_backproject(torch.as_tensor(g).cuda(), grid, geom, views).cpu().numpy()
        want = oracle.backproject(g[sel].astype(np.float64), grid.dims, grid.lo, grid.inv_h, geom.kind,
                                  geom.views[sel], geom.nu, geom.nv, geom.step, geom.length_scale)
        err = float(np.linalg.norm(got.astype(np.float64) - want) / np.linalg.norm(want))
        worst = float(np.abs(got.astype(np.float64) - want).max() / np.abs(want).max())
        say("large backproject", name, "rel_l2", err, "worst voxel / max", worst)
        assert err < 1e-5 and worst < 1e-5
