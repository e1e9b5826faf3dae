"""Parity of the kernels around the learned-initialisation network (pooling,
training targets, Gaussians drawn from the output fields) with the oracle,
and the gain of the trained network over the plain initialisation."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import unet as U
from paper_2411_04844_amd import inputs, learned, native

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_pool2_f32():
    r = np.random.default_rng(31)
    x = r.normal(size=(6, 4, 10)).astype(np.float32)
    got = native.dgr_pool2_f32(torch.as_tensor(x).cuda()).cpu().numpy()
    want = x.astype(np.float64).reshape(3, 2, 2, 2, 5, 2).mean(axis=(1, 3, 5))
    assert np.max(np.abs(got - want)) < 1e-6


def test_unet_targets_parity():
    grid = inputs.cube_grid(16)
    G = inputs.gaussians(3000, 32, 0.01, 0.2, mean_lim=1.05)
    vol = np.random.default_rng(33).uniform(size=grid.shape).astype(np.float32)
    got = native.dgr_unet_targets(torch.as_tensor(G["mu"]).cuda(), torch.as_tensor(G["scale"]).cuda(), grid,
                                  torch.as_tensor(vol).cuda(), 0.05).cpu().numpy()
    want = U.targets(G["mu"], G["scale"], grid.dims, grid.lo, grid.inv_h, vol, 0.05)
    say("targets occupied", int(want[..., 2].sum()), "max diff", float(np.abs(got - want).max()))
    assert np.array_equal(got[..., 2], want[..., 2])
    assert np.max(np.abs(got[..., 1] - want[..., 1])) < 1e-6
    assert np.max(np.abs(got[..., 0] - want[..., 0]) / np.maximum(np.abs(want[..., 0]), 1e-6)) < 1e-6


def test_init_from_unet_parity():
    grid = inputs.cube_grid(8)
    r = np.random.default_rng(34)
    out = np.stack([r.normal(size=grid.shape), r.normal(scale=0.7, size=grid.shape),
                    r.normal(scale=2.0, size=grid.shape)], axis=-1).astype(np.float32)
    n = 20000
    uni = r.uniform(size=(n, 4)).astype(np.float32)
    mu, sc, q, rho = native.dgr_init_from_unet(torch.as_tensor(out).cuda(), grid, n,
                                               torch.as_tensor(uni).cuda(), 0.05)
    mu_r, sc_r, rho_r, v_r = U.draw_from_fields(out, grid.dims, grid.lo, grid.inv_h, uni, 0.05)
    mu, sc, rho = mu.cpu().numpy(), sc.cpu().numpy(), rho.cpu().numpy()
    # the voxel choice may differ only where u W falls within rounding of a
    # cumulative-weight boundary (binary32 weights summed in another order)
    same = np.all(np.abs(mu - mu_r) < 1e-5, axis=1)
    say("init_from_unet mismatched draws", int((~same).sum()), "of", n)
    assert (~same).sum() <= 2
    assert np.max(np.abs(sc[same] - sc_r[same]) / sc_r[same]) < 1e-5
    assert np.max(np.abs(rho[same] - rho_r[same])) < 1e-7
    assert np.all(q.cpu().numpy() == np.array([1.0, 0.0, 0.0, 0.0], np.float32))


@pytest.mark.skipif(not os.path.exists(learned.WEIGHTS), reason="trained weights not present")
def test_learned_init_against_plain_inits():
    """Held-out phantom, 256^3, 25 views, 50,000 Gaussians, L1 loop with the
    PSNR measured after every step: the network's proposal is well ahead of
    the plain FDK-sampled initialisation as specified (1.5-voxel isotropic
    scale, which plateaus near 32 dB) after the same number of steps, and
    reaches 35 dB in no more steps than the plain initialisation with the
    tuned 3-voxel scale."""
    from paper_2411_04844_amd import recon
    params = learned.load()
    prob, gt = recon.sparse_view_problem(D=256, seeds=(59100, 59101))
    hist, steps = {}, {}
    for kind, sv in (("plain1.5", 1.5), ("plain3", 3.0), ("learned", None)):
        prob.params = (recon.fdk_init(prob, n=50_000, scale_vox=sv) if sv is not None
                       else learned.learned_init(prob, params, n=50_000))
        r = recon.reconstruct(prob, gt, max_iters=40, check_every=20, target_psnr=1e9)
        hist[kind] = [h[2] for h in r["history"]]
        steps[kind] = next((h[0] for h in r["history"] if h[2] >= 35.0), None)
        say(kind, "PSNR after 0/10/20/40 steps", [round(hist[kind][i], 2) for i in (0, 10, 20, 40)],
            "steps to 35 dB", steps[kind])
    assert hist["learned"][40] > hist["plain1.5"][40] + 2.0
    assert steps["learned"] is not None and steps["plain3"] is not None
    assert steps["learned"] <= steps["plain3"]
