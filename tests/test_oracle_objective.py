"""Pins of the full-objective oracle (CPU only)."""
import numpy as np

from oracle import objective as O


def test_ssim_map_matches_brute_force_window():
    r = np.random.default_rng(1)
    x = r.uniform(size=(9, 13))
    y = x + 0.1 * r.normal(size=x.shape)
    S, _ = O.ssim_terms(x[None], y[None], 1.0)
    np.testing.assert_allclose(S[0], O.ssim_map_brute(x, y, 1.0), rtol=1e-12, atol=1e-12)


def test_ssim_of_identical_views_is_one_with_zero_gradient():
    r = np.random.default_rng(2)
    x = r.uniform(size=(2, 12, 15))
    L, g = O.ssim_loss(x, x.copy(), 1.0)
    assert abs(L) < 1e-14
    assert np.max(np.abs(g)) < 1e-14


def test_ssim_of_constant_views_closed_form():
    # interior pixels of two constant images a, b see zero variances:
    # S = (2ab + C1) C2 / ((a^2 + b^2 + C1) C2) = (2ab + C1) / (a^2 + b^2 + C1)
    a, b, R = 0.3, 0.7, 1.0
    x, y = np.full((1, 31, 31), a), np.full((1, 31, 31), b)
    S, _ = O.ssim_terms(x, y, R)
    C1 = (0.01 * R) ** 2
    assert abs(S[0, 15, 15] - (2 * a * b + C1) / (a * a + b * b + C1)) < 1e-13


def test_ssim_gradient_central_differences():
    r = np.random.default_rng(3)
    x = r.uniform(0.2, 1.0, size=(2, 10, 12))
    y = r.uniform(0.2, 1.0, size=x.shape)
    _, g = O.ssim_loss(x, y, 1.0)
    h = 1e-6
    for k in range(12):
        i = tuple(int(r.integers(s)) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        num = (O.ssim_loss(xp, y, 1.0)[0] - O.ssim_loss(xm, y, 1.0)[0]) / (2 * h)
        assert abs(num - g[i]) < 1e-7 * max(1.0, abs(g[i])) + 1e-10, (i, num, g[i])


def test_tv_of_ramp_closed_form_and_gradient():
    # V = 0.5 x on a 6 x 5 x 4 grid: only x differences, each 0.5, (nx-1) of
    # them per row: L = 0.5 (nx - 1) ny nz / N = 0.5 (nx - 1) / nx
    nz, ny, nx = 6, 5, 4
    V = 0.5 * np.broadcast_to(np.arange(nx), (nz, ny, nx)).astype(np.float64)
    L, g = O.tv_loss(V)
    assert abs(L - 0.5 * (nx - 1) / nx) < 1e-15
    r = np.random.default_rng(4)
    W = r.normal(size=(5, 4, 6))
    _, g = O.tv_loss(W)
    h = 1e-7
    for k in range(12):
        i = tuple(int(r.integers(s)) for s in W.shape)
        wp, wm = W.copy(), W.copy()
        wp[i] += h
        wm[i] -= h
        num = (O.tv_loss(wp)[0] - O.tv_loss(wm)[0]) / (2 * h)
        assert abs(num - g[i]) < 1e-8, (i, num, g[i])


def test_objective_weights():
    r = np.random.default_rng(5)
    P = r.uniform(size=(2, 8, 8))
    Ph = P + 0.05 * r.normal(size=P.shape)
    V = r.normal(size=(4, 4, 4))
    tot, (l1, ls, lt), gP, gV = O.objective(Ph, P, V, 1.0)
    assert abs(tot - (0.6 * l1 + 0.2 * ls + 1.0 * lt)) < 1e-15
    np.testing.assert_allclose(gV, O.tv_loss(V)[1])
