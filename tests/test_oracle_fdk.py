"""Pins of the oracle's FDK and volume-driven initialisation."""
import math

import numpy as np
import pytest

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


def test_fdk_off_centre_ball_distance_weights():
    """A ball off the rotation axis, seen from a close source (DSO 3, DSD
    4.5 world units): over a full scan every voxel is near the source in
    some views and far in others, and only the right cosine and (R/U)^2
    weights make the two halves of the ball (nearer to and farther from the
    axis) come out equal.  Measured on planted mistakes: (R/U) instead of
    (R/U)^2 separates them by 1.1 %, (R/U)^3 by 1.9 %, a missing or squared
    cosine weight by 0.7 %; the oracle by 1e-4."""
    D = 64
    grid = inputs.cube_grid(D)
    dso, dsd, nu = 3.0, 4.5, 128
    geom = inputs.cone_geometry(180, nu, nu, 2.75 * dsd / dso / nu, dso, dsd, 1.0 / D)
    att, centre, rad = 0.02, (0.4, 0.0, 0.0), 0.3
    ph = inputs.Phantom(np.array([centre]), np.full((1, 3), rad), np.eye(3)[None], np.array([att]))
    y = inputs.phantom_projections(ph, geom).numpy()
    f = oracle.fdk(y, geom.views, geom.nu, geom.nv, 2 * math.pi, geom.length_scale, grid.dims,
                   grid.lo, grid.inv_h)
    c = -1 + (np.arange(D) + 0.5) / grid.inv_h[0]
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt((X - centre[0]) ** 2 + Y ** 2 + Z ** 2)
    inner = (r < 0.7 * rad) & (np.abs(Z) < 0.5 * rad)
    far_axis = f[inner & (X > centre[0])].mean() / att
    near_axis = f[inner & (X < centre[0])].mean() / att
    assert abs(far_axis - near_axis) < 3e-3, (far_axis, near_axis)
    assert abs(f[inner].mean() / att - 1.0) < 1e-2


def test_ramp_filter_impulse_response():
    """The filter of one impulse is the tap table of the discrete Ram-Lak
    filter (Kak & Slaney, ch. 3): 1/(4 tau) at 0, 0 at even offsets,
    -1/(k^2 pi^2 tau) at odd offsets k."""
    nu, tau, c = 41, 0.37, 20
    p = np.zeros(nu)
    p[c] = 1.0
    q = oracle.ramp_filter(p, tau)
    k = np.arange(nu) - c
    want = np.where(k == 0, 0.25, np.where(k % 2 == 0, 0.0, -1.0 / (np.pi ** 2 * k.astype(float) ** 2))) / tau
    np.testing.assert_allclose(q, want, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("omega", [0.05 * np.pi, 0.3 * np.pi, 0.77 * np.pi])
def test_ramp_filter_is_a_ramp(omega):
    """Far from the ends of a long row the filter scales cos(w i) by
    |w| / (2 pi tau): the Fourier series sum_{k odd} cos(k w) / k^2 =
    pi^2/8 - pi |w| / 4 on [-pi, pi] turns the taps into the ramp.  The
    tail beyond the row (|k| > 2000) contributes below 2e-4 / tau."""
    nu, tau = 8001, 0.5
    i = np.arange(nu)
    q = oracle.ramp_filter(np.cos(omega * i), tau)
    mid = slice(nu // 2 - 200, nu // 2 + 200)
    np.testing.assert_allclose(q[mid], abs(omega) / (2 * np.pi * tau) * np.cos(omega * i[mid]), atol=2e-4 / tau)


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
