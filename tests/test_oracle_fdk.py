"""Pins of the oracle's FDK and volume-driven initialisation."""
import math

import numpy as np

import oracle
from paper_2411_04844_amd import inputs


def _ball_phantom(radius, att):
    return inputs.Phantom(np.zeros((1, 3)), np.full((1, 3), radius), np.eye(3)[None], np.array([att]))


def test_fdk_reconstructs_uniform_ball():
    D = 48
    grid = inputs.cube_grid(D)
    geom = inputs.cone_geometry(180, 96, 96, 0.03, 7.8125, 11.71875, 1.0 / D)
    att = 0.02
    y = inputs.phantom_projections(_ball_phantom(0.5, att), geom).numpy()
    f = oracle.fdk(y, geom.views, geom.nu, geom.nv, 2 * math.pi, geom.length_scale, grid.dims,
                   grid.lo, grid.inv_h)
    c = -1 + (np.arange(D) + 0.5) / grid.inv_h[0]
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    inner = f[r < 0.35].mean()
    outer = np.abs(f[(r > 0.65) & (r < 0.9) & (np.abs(Z) < 0.3)]).mean()
    assert abs(inner / att - 1.0) < 0.03, inner / att
    assert outer / att < 0.03, outer / att


def test_init_sampling_matches_numpy_inverse_cdf():
    rng = np.random.default_rng(4)
    dims = (9, 7, 5)
    f = rng.uniform(size=(5, 7, 9)).astype(np.float32) ** 3
    u = rng.uniform(size=(500, 4))
    mu, sc, q, rho, vox, above = oracle.init_from_volume(f, dims, (-1, -1, -1), (4.0, 4.0, 4.0),
                                                         0.1, u, 0.3)
    w = f.ravel().astype(np.float64)
    w = np.where(w > 0.1 * w.max(), w, 0.0)
    cdf = np.cumsum(w)
    want = np.searchsorted(cdf, u[:, 0] * cdf[-1], side="right")
    assert np.array_equal(vox, want)
    assert above == np.count_nonzero(w)
    x, y, z = want % 9, (want // 9) % 7, want // 63
    assert np.allclose(mu[:, 0], -1 + (x + 0.5 + u[:, 1] - 0.5) / 4.0)
    assert np.allclose(mu[:, 2], -1 + (z + 0.5 + u[:, 3] - 0.5) / 4.0)
    assert np.all(sc == 0.3) and np.all(q[:, 0] == 1) and np.array_equal(rho, f.ravel()[want])


def test_init_sampling_frequencies():
    f = np.zeros((2, 2, 2), np.float32)
    f[0, 0, 1] = 1.0
    f[1, 1, 0] = 3.0
    u = np.random.default_rng(5).uniform(size=(40000, 4))
    *_, vox, above = oracle.init_from_volume(f, (2, 2, 2), (0, 0, 0), (1.0, 1.0, 1.0), 0.1, u, 0.5)
    assert above == 2
    frac = np.mean(vox == 6)
    assert abs(frac - 0.75) < 0.01 and np.all((vox == 6) | (vox == 1))
