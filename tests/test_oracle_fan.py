"""Pins of the oracle's fan-beam geometry (a stack of fan-beam slices, the
setting of the paper's fan-beam sparse-view and limited-angle experiments,
sec. 5.1, Tabs. 2-3) and its slice-by-slice FBP (CPU only)."""
import math

import numpy as np
from scipy.ndimage import map_coordinates

import oracle
from paper_2411_04844_amd import inputs


def _physical_rays(n_views, arc, start, nu, nv, pu, pv, dso, dsd):
    """Rays of a fan-beam slice stack built from the scanner description
    (angle, source and detector distances, column pitch, slice height), not
    from the view table: for view j at angle t the source of the slice at
    height z sits at (dso cos t, dso sin t, z) and column u of that slice's
    detector line at -(dsd - dso)(cos t, sin t) + u (-sin t, cos t), height z.
    Returns, per view, the point nearest the origin and the unit direction."""
    out = []
    for j in range(n_views):
        t = start + arc * j / n_views
        c, s = math.cos(t), math.sin(t)
        u = (np.arange(nu) - 0.5 * (nu - 1)) * pu
        z = (np.arange(nv) - 0.5 * (nv - 1)) * pv
        U, Z = np.meshgrid(u, z)  # [nv, nu]
        src = np.stack([np.full_like(U, dso * c), np.full_like(U, dso * s), Z], -1)
        pix = np.stack([-(dsd - dso) * c - U * s, -(dsd - dso) * s + U * c, Z], -1)
        d = pix - src
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        cpt = src - np.sum(src * d, -1, keepdims=True) * d
        out.append((cpt.reshape(-1, 3), d.reshape(-1, 3)))
    return out


def test_fan_projector_matches_scanner_rays():
    dims, lo, inv_h = (14, 12, 10), (-0.875, -0.75, -0.625), (8.0, 8.0, 8.0)
    V = np.random.default_rng(21).uniform(size=(dims[2], dims[1], dims[0]))
    step, arc, start = 0.05, 1.9, 0.3
    nu, nv, pu, pv, dso, dsd = 9, 7, 0.25, 0.1, 4.0, 6.0
    geom = inputs.fan_geometry(3, nu, nv, pu, pv, dso, dsd, step, arc=arc, start=start, length_scale=1.0)
    P = oracle.project(V, dims, lo, inv_h, 2, geom.views, nu, nv, step)
    k = np.arange(-200, 201)
    scale = 0.0
    for j, (c, d) in enumerate(_physical_rays(3, arc, start, nu, nv, pu, pv, dso, dsd)):
        pts = c[:, None, :] + (k * step)[None, :, None] * d[:, None, :]
        u = (pts - np.array(lo)) * np.array(inv_h) - 0.5
        coords = np.stack([u[..., 2].ravel(), u[..., 1].ravel(), u[..., 0].ravel()])
        vals = map_coordinates(V, coords, order=1, mode="grid-constant", cval=0.0)
        want = step * vals.reshape(len(c), len(k)).sum(1)
        scale = max(scale, np.abs(want).max())
        # the view table is binary32; the scanner rays are exact
        assert np.abs(P[j].ravel() - want).max() < 2e-5 * scale
        assert np.count_nonzero(want) > 0.8 * want.size


def test_fan_rows_of_an_extruded_volume_agree():
    """A volume constant along z has identical fan-beam rows on every slice
    height inside the grid (no vertical divergence), unlike a cone beam."""
    D = 16
    dims, lo, inv_h = (D, D, D), (-1.0, -1.0, -1.0), (D / 2.0,) * 3
    f = np.random.default_rng(22).uniform(size=(D, D))
    V = np.broadcast_to(f, (D, D, D)).copy()
    h = 2.0 / D
    fan = inputs.fan_geometry(4, 24, D, 2.0 * h, h, 3.0, 5.0, h / 2, length_scale=1.0)
    Pf = oracle.project(V, dims, lo, inv_h, 2, fan.views, 24, D, h / 2)
    assert np.abs(Pf - Pf[:, :1, :]).max() < 1e-12 * np.abs(Pf).max()
    cone = inputs.cone_geometry(4, 24, D, 2.0 * h, 3.0, 5.0, h / 2, length_scale=1.0)
    Pc = oracle.project(V, dims, lo, inv_h, 1, cone.views, 24, D, h / 2)
    assert np.abs(Pc - Pc[:, :1, :]).max() > 1e-2 * np.abs(Pc).max()


def test_fan_single_row_is_the_cone_central_row():
    dims, lo, inv_h = (12, 12, 12), (-0.75, -0.75, -0.75), (8.0, 8.0, 8.0)
    V = np.random.default_rng(23).uniform(size=(12, 12, 12))
    fan = inputs.fan_geometry(5, 17, 1, 0.2, 0.1, 3.0, 4.5, 0.06, length_scale=1.0)
    cone = inputs.cone_geometry(5, 17, 1, 0.2, 3.0, 4.5, 0.06, length_scale=1.0)
    a = oracle.project(V, dims, lo, inv_h, 2, fan.views, 17, 1, 0.06)
    b = oracle.project(V, dims, lo, inv_h, 1, cone.views, 17, 1, 0.06)
    assert np.array_equal(a, b)


def test_fan_adjoint_identity():
    dims, lo, inv_h = (13, 11, 9), (-0.8125, -0.6875, -0.5625), (8.0, 8.0, 8.0)
    rng = np.random.default_rng(24)
    x = rng.normal(size=(9, 11, 13))
    geom = inputs.fan_geometry(5, 15, 9, 0.15, 0.125, 3.0, 4.5, 0.07, arc=math.pi / 2, length_scale=2.0)
    Ax = oracle.project(x, dims, lo, inv_h, 2, geom.views, 15, 9, 0.07, geom.length_scale)
    y = rng.normal(size=Ax.shape)
    ATy = oracle.backproject(y, dims, lo, inv_h, 2, geom.views, 15, 9, 0.07, geom.length_scale)
    lhs, rhs = np.sum(Ax * y), np.sum(x * ATy)
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum(Ax ** 2) * np.sum(y ** 2))
    assert np.count_nonzero(Ax) > 0.5 * Ax.size


def _ball(radius, att):
    return inputs.Phantom(np.zeros((1, 3)), np.full((1, 3), radius), np.eye(3)[None], np.array([att]))


def test_fbp_of_a_ball_slice_by_slice():
    """Analytic fan-beam data of a ball reconstructed by fan FBP: the cap
    slice at z = 0.4 (radius 0.3) is as accurate as the central one.  The
    cone reading of the same rows (one source for all rows) reads the cap
    from rows magnified to z = 0.6, outside the ball."""
    D = 48
    grid = inputs.cube_grid(D)
    h = 2.0 / D
    geom = inputs.fan_geometry(180, 96, D, 0.045, h, 4.0, 6.0, h / 2, length_scale=1.0)
    att = 0.02
    y = inputs.phantom_projections(_ball(0.5, att), geom).numpy() / inputs.MM_PER_UNIT
    c = -1 + (np.arange(D) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    rxy = np.sqrt(X ** 2 + Y ** 2)
    for kind in (2, 1):
        f = oracle.fdk(y, geom.views, geom.nu, geom.nv, 2 * math.pi, 1.0, grid.dims, grid.lo, grid.inv_h,
                       kind=kind)
        mid = f[(np.abs(Z) < 0.05) & (rxy < 0.35)].mean() / att
        cap = f[(np.abs(Z - 0.4) < 0.03) & (rxy < 0.15)].mean() / att
        out = np.abs(f[(rxy > 0.7) & (rxy < 0.9) & (np.abs(Z) < 0.3)]).mean() / att
        if kind == 2:
            assert abs(mid - 1.0) < 0.03, mid
            assert abs(cap - 1.0) < 0.03, cap
            assert out < 0.03, out
        else:
            assert abs(cap - 1.0) > 0.5, cap
