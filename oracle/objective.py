"""Oracle for the paper's full objective (binary64 numpy).

TEST INFRASTRUCTURE.  Only ``tests/`` may import this module; it shares no
code with the HIP library.

The objective of sec. 4.3 (weights there and in App. D.1):

    L = l1 * L1(P_hat, P) + l2 * L_SSIM(P_hat, P) + l3 * L_TV(V),
    l1 = 0.6, l2 = 0.2, l3 = 1.

Readings (the paper names the terms and gives the SSIM formula of App. C.2,
not their discretisation):

* L1 = mean |P_hat - P| over all views and pixels.
* L_SSIM = 1 - mean over all views and pixels of the SSIM map of each 2-D
  view, with local statistics from an 11 x 11 Gaussian window (sigma 1.5,
  weights normalised to sum 1) applied with zero padding outside the
  detector; C1 = (0.01 R)^2, C2 = (0.03 R)^2 with R the range (max) of the
  target projections.
* L_TV = mean over voxels of sum over axes of |V[i + e_a] - V[i]| (forward
  differences inside the grid; the last plane of each axis has none).

Gradients: d|r|/dr = sign(r) with sign(0) = 0; the TV gradient likewise.

Pins (tests/test_oracle_objective.py): SSIM map against a brute-force window
sum; SSIM(x, x) = 1 with zero gradient; SSIM of two constant images against
its closed form; TV of a ramp against its closed form; the SSIM and TV
gradients against binary64 central differences.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

LAMBDA = (0.6, 0.2, 1.0)
WIN = 11
SIGMA = 1.5


def window_1d():
    t = np.arange(WIN) - WIN // 2
    g = np.exp(-(t * t) / (2.0 * SIGMA * SIGMA))
    return g / g.sum()


def blur(img):
    """Separable Gaussian window, zero padding, 'same' size, per view.
    img [..., nv, nu]."""
    g = window_1d()
    out = ndimage.correlate1d(img, g, axis=-1, mode="constant", cval=0.0)
    return ndimage.correlate1d(out, g, axis=-2, mode="constant", cval=0.0)


def ssim_terms(x, y, R):
    C1, C2 = (0.01 * R) ** 2, (0.03 * R) ** 2
    mx, my = blur(x), blur(y)
    exx, eyy, exy = blur(x * x), blur(y * y), blur(x * y)
    A = 2 * mx * my + C1
    Bt = 2 * (exy - mx * my) + C2
    C = mx * mx + my * my + C1
    D = (exx - mx * mx) + (eyy - my * my) + C2
    S = A * Bt / (C * D)
    return S, (mx, my, A, Bt, C, D)


def ssim_loss(x, y, R):
    """(L_SSIM, dL/dx) for x, y [views, nv, nu]."""
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    S, (mx, my, A, Bt, C, D) = ssim_terms(x, y, R)
    M = x.size
    # dS/d(first, second, cross moments of x) at every pixel
    a = S * (2 * my / A - 2 * my / Bt - 2 * mx / C + 2 * mx / D)
    b = -S / D
    c = 2 * S / Bt
    # the window is symmetric, so the adjoint of blur is blur
    grad = -(blur(a) + 2 * x * blur(b) + y * blur(c)) / M
    return 1.0 - S.mean(), grad


def l1_loss(x, y):
    r = np.asarray(x, np.float64) - np.asarray(y, np.float64)
    return np.abs(r).mean(), np.sign(r) / r.size


def tv_loss(V):
    """(L_TV, dL/dV) for V [nz, ny, nx]."""
    V = np.asarray(V, np.float64)
    N = V.size
    L = 0.0
    g = np.zeros_like(V)
    for ax in range(3):
        d = np.diff(V, axis=ax)
        L += np.abs(d).sum()
        s = np.sign(d)
        pad_lo = [(0, 0)] * 3
        pad_hi = [(0, 0)] * 3
        pad_lo[ax] = (1, 0)
        pad_hi[ax] = (0, 1)
        # d|V[i+1] - V[i]| / dV[i] = -s_i, / dV[i+1] = +s_i
        g += np.pad(s, pad_lo) - np.pad(s, pad_hi)
    return L / N, g / N


def objective(P_hat, P, V, R, lam=LAMBDA):
    """(total, (L1, L_SSIM, L_TV), dL/dP_hat, dL/dV)."""
    l1, g1 = l1_loss(P_hat, P)
    ls, gs = ssim_loss(P_hat, P, R)
    lt, gt = tv_loss(V)
    total = lam[0] * l1 + lam[1] * ls + lam[2] * lt
    return total, (l1, ls, lt), lam[0] * g1 + lam[1] * gs, lam[2] * gt


def ssim_map_brute(x, y, R):
    """SSIM map of one view by explicit window sums (tiny images only)."""
    g1 = window_1d()
    W = np.outer(g1, g1)
    nv, nu = x.shape
    h = WIN // 2
    C1, C2 = (0.01 * R) ** 2, (0.03 * R) ** 2
    S = np.zeros((nv, nu))
    for i in range(nv):
        for j in range(nu):
            s = {"x": 0.0, "y": 0.0, "xx": 0.0, "yy": 0.0, "xy": 0.0}
            for a in range(-h, h + 1):
                for b in range(-h, h + 1):
                    ii, jj = i + a, j + b
                    if 0 <= ii < nv and 0 <= jj < nu:
                        w = W[a + h, b + h]
                        xv, yv = x[ii, jj], y[ii, jj]
                        s["x"] += w * xv
                        s["y"] += w * yv
                        s["xx"] += w * xv * xv
                        s["yy"] += w * yv * yv
                        s["xy"] += w * xv * yv
            vx, vy = s["xx"] - s["x"] ** 2, s["yy"] - s["y"] ** 2
            cxy = s["xy"] - s["x"] * s["y"]
            S[i, j] = ((2 * s["x"] * s["y"] + C1) * (2 * cxy + C2)) / \
                ((s["x"] ** 2 + s["y"] ** 2 + C1) * (vx + vy + C2))
    return S
