"""Pins of the CPU oracle against what the mathematics fixes.

Every check here is independent of the oracle's own code path: closed
forms, a library rotation (SciPy), SciPy's trilinear interpolation, brute
force, exact chord lengths and binary64 finite differences.  Grids are
non-cubic on purpose so that an axis transposition fails.
"""
import math

import numpy as np
import pytest
from scipy.ndimage import map_coordinates
from scipy.spatial.transform import Rotation
from scipy.special import erf

import oracle
from paper_2411_04844_amd import inputs


def _grid(dims, lo=(-1.0, -1.0, -1.0), h=None):
    h = h if h is not None else 2.0 / dims[0]
    return tuple(dims), tuple(lo), (1.0 / h,) * 3


def _sigma_world(scale, quat):
    """Covariance via SciPy's rotation (independent of the oracle)."""
    q = np.asarray(quat, np.float64)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    s = np.asarray(scale, np.float64)
    return R @ np.diag(s * s) @ R.T


def _centres(dims, lo, inv_h):
    xs = [lo[a] + (np.arange(dims[a]) + 0.5) / inv_h[a] for a in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return np.stack([X, Y, Z], -1)


# --------------------------------------------------------------------------
# O1 bbox and O2 tiles
# --------------------------------------------------------------------------
def test_bbox_is_the_k_sigma_slab_in_binary64():
    dims, lo, inv_h = (40, 36, 28), (-1.25, -1.0, -0.875), (16.0, 16.0, 16.0)
    rng = np.random.default_rng(7)
    n = 3000
    mu = rng.uniform(-1.6, 1.6, (n, 3)).astype(np.float32)
    scale = np.exp(rng.uniform(np.log(0.005), np.log(0.4), (n, 3))).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    box = oracle.bbox(mu, scale, q, dims, lo, inv_h, 3.0)
    checked = 0
    for g in range(n):
        S = _sigma_world(scale[g], q[g])
        for k in range(3):
            u = (float(mu[g, k]) - lo[k]) * inv_h[k] - 0.5
            r = 3.0 * math.sqrt(S[k, k]) * inv_h[k]
            # skip Gaussians whose bound lies within 1e-4 voxel of an integer
            if min(abs((u - r) - round(u - r)), abs((u + r) - round(u + r))) < 1e-4:
                break
        else:
            for k in range(3):
                u = (float(mu[g, k]) - lo[k]) * inv_h[k] - 0.5
                r = 3.0 * math.sqrt(S[k, k]) * inv_h[k]
                idx = np.arange(dims[k])
                inside = idx[np.abs(idx - u) <= r]
                if inside.size:
                    assert box[g, k] == inside.min() and box[g, 3 + k] == inside.max(), (g, k)
                else:
                    assert box[g, k] > box[g, 3 + k] or any(
                        box[g, a] > box[g, 3 + a] for a in range(3)), (g, k)
            checked += 1
    assert checked > 2900


def test_bbox_fixed_cuboid_is_alg1_validity():
    dims, lo, inv_h = _grid((20, 24, 16), h=0.1)
    rng = np.random.default_rng(3)
    mu = rng.uniform(-1.3, 1.5, (500, 3)).astype(np.float32)
    scale = np.full((500, 3), 0.05, np.float32)
    q = np.tile(np.float32([1, 0, 0, 0]), (500, 1))
    box = oracle.bbox(mu, scale, q, dims, lo, inv_h, 0.0, 4)
    u = (mu.astype(np.float64) - np.array(lo)) * np.array(inv_h) - 0.5
    f = np.floor(u)
    for k in range(3):
        want_lo = np.clip(f[:, k] - 4, 0, dims[k])
        want_hi = np.clip(f[:, k] + 4, -1, dims[k] - 1)
        assert np.array_equal(box[:, k], want_lo.astype(np.int32))
        assert np.array_equal(box[:, 3 + k], want_hi.astype(np.int32))


def test_bbox_binary32_sequence_matches_numpy_float32():
    """Consistency of the C binary32 sequence with numpy float32 arithmetic."""
    G = inputs.gaussians(4000, 11, 0.004, 0.05)
    dims, lo, inv_h = (64, 64, 64), (-1.0, -1.0, -1.0), (32.0, 32.0, 32.0)
    box = oracle.bbox(G["mu"], G["scale"], G["quat"], dims, lo, inv_h, 3.0)
    f = np.float32
    q = G["quat"]
    n2 = ((q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1]) + q[:, 2] * q[:, 2]) + q[:, 3] * q[:, 3]
    m = np.sqrt(n2)
    w, x, y, z = (q[:, i] / m for i in range(4))
    R = [[f(1) - f(2) * (y * y + z * z), f(2) * (x * y - w * z), f(2) * (x * z + w * y)],
         [f(2) * (x * y + w * z), f(1) - f(2) * (x * x + z * z), f(2) * (y * z - w * x)],
         [f(2) * (x * z - w * y), f(2) * (y * z + w * x), f(1) - f(2) * (x * x + y * y)]]
    s = G["scale"]
    for k in range(3):
        a = [R[k][j] * s[:, j] for j in range(3)]
        skk = (a[0] * a[0] + a[1] * a[1]) + a[2] * a[2]
        r = (f(3) * np.sqrt(skk)) * f(inv_h[k])
        u = (G["mu"][:, k] - f(lo[k])) * f(inv_h[k]) - f(0.5)
        lo_k = np.clip(np.ceil(u - r), 0, dims[k]).astype(np.int32)
        hi_k = np.clip(np.floor(u + r), -1, dims[k] - 1).astype(np.int32)
        assert np.array_equal(box[:, k], lo_k)
        assert np.array_equal(box[:, 3 + k], hi_k)


def test_tile_pairs_match_enumeration():
    dims = (40, 27, 19)  # ragged last tiles on every axis
    rng = np.random.default_rng(5)
    n = 400
    lo = np.stack([rng.integers(-3, d + 2, n) for d in dims], 1)
    ext = rng.integers(-2, 14, (n, 3))
    hi = lo + ext
    lo = np.clip(lo, 0, np.array(dims))
    hi = np.clip(hi, -1, np.array(dims) - 1)
    box = np.concatenate([lo, hi], 1).astype(np.int32)
    pairs, tb = oracle.tile_pairs(box, dims)
    T = [(d + 7) // 8 for d in dims]
    want = []
    for g in range(n):
        if np.any(box[g, :3] > box[g, 3:]):
            continue
        for tz in range(T[2]):
            for ty in range(T[1]):
                for tx in range(T[0]):
                    t0 = np.array([tx, ty, tz]) * 8
                    t1 = t0 + 7
                    if np.all(box[g, :3] <= t1) and np.all(box[g, 3:] >= t0):
                        want.append(((tz * T[1] + ty) * T[0] + tx, g))
    want = np.array(sorted(want), np.uint32)
    assert np.array_equal(pairs, want)
    assert np.array_equal(tb, np.searchsorted(want[:, 0], np.arange(np.prod(T) + 1), side="left"))


# --------------------------------------------------------------------------
# O3 voxelization
# --------------------------------------------------------------------------
def _full_box(n, dims):
    return np.tile(np.int32([0, 0, 0, dims[0] - 1, dims[1] - 1, dims[2] - 1]), (n, 1))


def test_voxelize_grid_sum_closed_form():
    """Poisson summation: a well-resolved Gaussian sums to rho (2pi)^1.5 sqrt(det S)/h^3."""
    dims, lo, inv_h = _grid((56, 52, 48), h=1.0 / 24)
    rng = np.random.default_rng(1)
    for t in range(6):
        s = rng.uniform(1.5, 3.0, 3) / inv_h[0]
        q = rng.normal(size=4)
        mu = rng.uniform(-0.15, 0.15, 3)
        rho = rng.uniform(0.2, 2.0)
        box = oracle.bbox(mu[None], s[None], q[None], dims, lo, inv_h, 8.0)
        V = oracle.voxelize(mu[None], s[None], q[None], [rho], dims, lo, inv_h, box)
        want = rho * (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(_sigma_world(s, q))) * inv_h[0] ** 3
        assert abs(V.sum() / want - 1.0) < 1e-7


def test_voxelize_matches_scipy_rotation_definition():
    dims, lo, inv_h = _grid((22, 18, 15), h=0.1)
    rng = np.random.default_rng(2)
    n = 7
    mu = rng.uniform(-0.5, 0.5, (n, 3))
    s = rng.uniform(0.08, 0.3, (n, 3))
    q = rng.normal(size=(n, 4))
    rho = rng.uniform(0.1, 1, n)
    V = oracle.voxelize(mu, s, q, rho, dims, lo, inv_h, _full_box(n, dims))
    X = _centres(dims, lo, inv_h)
    want = np.zeros(X.shape[:3])
    for g in range(n):
        Sinv = np.linalg.inv(_sigma_world(s[g], q[g]))
        d = X - mu[g]
        want += rho[g] * np.exp(-0.5 * np.einsum("...a,ab,...b->...", d, Sinv, d))
    assert np.max(np.abs(V - want)) <= 1e-13 * np.max(np.abs(want))


def test_voxelize_45deg_about_z_is_elongated_along_diagonal():
    dims, lo, inv_h = _grid((21, 21, 21), h=0.1)
    c = math.cos(math.pi / 8)
    q = np.array([[c, 0, 0, math.sin(math.pi / 8)]])
    s = np.array([[0.3, 0.1, 0.15]])
    mu = np.array([[0.05, 0.05, 0.05]])  # voxel 10's centre
    V = oracle.voxelize(mu, s, q, [1.0], dims, lo, inv_h, _full_box(1, dims))
    a0 = np.array([1, 1, 0]) / math.sqrt(2)
    a1 = np.array([-1, 1, 0]) / math.sqrt(2)
    a2 = np.array([0, 0, 1.0])
    S = 0.3 ** 2 * np.outer(a0, a0) + 0.1 ** 2 * np.outer(a1, a1) + 0.15 ** 2 * np.outer(a2, a2)
    Sinv = np.linalg.inv(S)
    for off in ([2, 2, 0], [2, -2, 0], [3, 1, -1]):
        d = np.array(off) * 0.1
        want = math.exp(-0.5 * d @ Sinv @ d)
        got = V[10 + off[2], 10 + off[1], 10 + off[0]]
        assert abs(got - want) < 1e-14
    assert V[10, 12, 12] > 20 * V[10, 8, 12]


def test_voxelize_axis_aligned_is_separable():
    dims, lo, inv_h = _grid((30, 26, 20), h=1.0 / 12)
    mu = np.array([[0.11, -0.07, 0.2]])
    s = np.array([[0.12, 0.2, 0.09]])
    for q, perm in (([1, 0, 0, 0], (0, 1, 2)),
                    ([math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)], (1, 0, 2))):
        box = oracle.bbox(mu, s, np.array([q]), dims, lo, inv_h, 3.0)
        V = oracle.voxelize(mu, s, np.array([q]), [0.7], dims, lo, inv_h, box)
        sw = s[0][list(perm)]
        g1 = []
        for a in range(3):
            x = lo[a] + (np.arange(dims[a]) + 0.5) / inv_h[a]
            v = np.exp(-0.5 * ((x - mu[0, a]) / sw[a]) ** 2)
            keep = (np.arange(dims[a]) >= box[0, a]) & (np.arange(dims[a]) <= box[0, 3 + a])
            g1.append(v * keep)
        want = 0.7 * g1[2][:, None, None] * g1[1][None, :, None] * g1[0][None, None, :]
        assert np.max(np.abs(V - want)) <= 1e-14


def test_voxelize_truncated_mass_bounds():
    """k_sigma = 3: the kept cells cover the 3-sigma slabs to within half a
    voxel, so the mass ratio lies between the union bound of the slabs
    shrunk by h/2 and the smallest single slab grown by h/2."""
    dims, lo, inv_h = _grid((64, 64, 64))
    rng = np.random.default_rng(9)
    for t in range(5):
        s = rng.uniform(2.0, 3.0, 3) / inv_h[0]
        q = rng.normal(size=4)
        mu = rng.uniform(-0.1, 0.1, 3)
        box = oracle.bbox(mu[None], s[None], q[None], dims, lo, inv_h, 3.0)
        V = oracle.voxelize(mu[None], s[None], q[None], [1.0], dims, lo, inv_h, box)
        S = _sigma_world(s, q)
        full = (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(S)) * inv_h[0] ** 3
        ratio = V.sum() / full
        sig = np.sqrt(np.diag(S)) * inv_h[0]  # marginal std, voxels
        lower = 1.0 - sum(1.0 - erf((3 * sk - 0.5) / (sk * math.sqrt(2))) for sk in sig)
        upper = min(erf((3 * sk + 0.5) / (sk * math.sqrt(2))) for sk in sig)
        assert lower < ratio < upper, (lower, ratio, upper)


def test_voxelize_quaternion_sign_and_scale_invariance_and_shift():
    dims, lo, inv_h = _grid((24, 20, 18), h=0.1)
    rng = np.random.default_rng(4)
    mu = rng.uniform(-0.3, 0.3, (5, 3))
    s = rng.uniform(0.05, 0.2, (5, 3))
    q = rng.normal(size=(5, 4))
    rho = rng.uniform(size=5)
    box = oracle.bbox(mu, s, q, dims, lo, inv_h, 3.0)
    V = oracle.voxelize(mu, s, q, rho, dims, lo, inv_h, box)
    for q2 in (-q, 2.5 * q):
        V2 = oracle.voxelize(mu, s, q2, rho, dims, lo, inv_h, box)
        assert np.max(np.abs(V2 - V)) <= 1e-14 * V.max()
    shift = np.array([0.1, 0.0, 0.0])
    box2 = box.copy()
    box2[:, 0] += 1
    box2[:, 3] += 1
    V3 = oracle.voxelize(mu + shift, s, q, rho, dims, lo, inv_h, box2)
    assert np.max(np.abs(V3[:, :, 1:] - V[:, :, :-1])) <= 1e-13


def test_voxelize_brute_equals_box_loops():
    G = inputs.gaussians(300, 12, 0.01, 0.05)
    dims, lo, inv_h = (32, 24, 20), (-1.0, -0.75, -0.625), (16.0, 16.0, 16.0)
    box = oracle.bbox(G["mu"], G["scale"], G["quat"], dims, lo, inv_h, 3.0)
    a = oracle.voxelize(G["mu"], G["scale"], G["quat"], G["density"], dims, lo, inv_h, box, brute=True)
    b = oracle.voxelize(G["mu"], G["scale"], G["quat"], G["density"], dims, lo, inv_h, box)
    assert np.linalg.norm(a - b) <= 1e-14 * np.linalg.norm(a)
    assert a.max() > 0


# --------------------------------------------------------------------------
# O4 projector, O5 Siddon, O7 adjoint
# --------------------------------------------------------------------------
def test_parallel_axis_identity():
    D = 16
    dims, lo, inv_h = _grid((D, D, D))
    h = 1.0 / inv_h[0]
    rng = np.random.default_rng(0)
    V = rng.uniform(size=(D, D, D))
    geom = inputs.parallel_geometry(2, D, D, h, h / 2)
    P = oracle.project(V, dims, lo, inv_h, 0, geom.views, D, D, h / 2)
    assert np.allclose(P[0], h * V.sum(axis=2), rtol=1e-12, atol=0)
    assert np.allclose(P[1], h * V.sum(axis=1)[:, ::-1], rtol=1e-12, atol=1e-15)


def _rays(geom, j):
    v = geom.views[j].astype(np.float64)
    iu = np.arange(geom.nu) - 0.5 * (geom.nu - 1)
    iv = np.arange(geom.nv) - 0.5 * (geom.nv - 1)
    pix = v[3:6] + iu[None, :, None] * v[6:9] + iv[:, None, None] * v[9:12]
    if geom.kind == 0:
        d = np.broadcast_to(v[0:3], pix.shape)
        o = pix
    elif geom.kind == 1:
        o = np.broadcast_to(v[0:3], pix.shape)
        d = pix - o
    else:  # fan: the source of row iv sits at a + iv e_v
        o = np.broadcast_to(v[0:3] + iv[:, None, None] * v[9:12], pix.shape)
        d = pix - o
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    c = o - np.sum(o * d, -1, keepdims=True) * d
    return c.reshape(-1, 3), d.reshape(-1, 3)


@pytest.mark.parametrize("kind", [0, 1])
def test_projector_matches_scipy_trilinear(kind):
    dims, lo, inv_h = (14, 12, 10), (-0.875, -0.75, -0.625), (8.0, 8.0, 8.0)
    rng = np.random.default_rng(8)
    V = rng.uniform(size=(dims[2], dims[1], dims[0]))
    step = 0.05
    if kind == 0:
        geom = inputs.parallel_geometry(3, 9, 7, 0.2, step)
    else:
        geom = inputs.cone_geometry(3, 9, 7, 0.25, 4.0, 6.0, step, length_scale=1.0)
    P = oracle.project(V, dims, lo, inv_h, kind, geom.views, geom.nu, geom.nv, step)
    k = np.arange(-200, 201)
    for j in range(3):
        c, d = _rays(geom, j)
        pts = c[:, None, :] + (k * step)[None, :, None] * d[:, None, :]
        u = (pts - np.array(lo)) * np.array(inv_h) - 0.5
        coords = np.stack([u[..., 2].ravel(), u[..., 1].ravel(), u[..., 0].ravel()])
        vals = map_coordinates(V, coords, order=1, mode="grid-constant", cval=0.0)
        want = step * vals.reshape(len(c), len(k)).sum(1)
        assert np.allclose(P[j].ravel(), want, rtol=1e-12, atol=1e-13)


def _gauss_line_integral(c, d, mu, Q):
    r = c - mu
    a = d @ Q @ d
    b = d @ Q @ r
    return math.sqrt(2 * math.pi / a) * math.exp(-0.5 * (r @ Q @ r - b * b / a))


@pytest.mark.parametrize("kind", [0, 1])
def test_projector_converges_to_gaussian_line_integral(kind):
    """Error of the discrete operator against the continuous line integral
    shrinks as h^2 / sigma^2 (ratio about 4 when sigma doubles in voxels)."""
    q = np.array([0.9, 0.2, -0.3, 0.25])
    errs = []
    for sig_vox in (2.0, 4.0):
        D = 48
        dims, lo, inv_h = _grid((D, D, D))
        h = 1.0 / inv_h[0]
        s = np.array([1.0, 1.3, 0.8]) * sig_vox * h
        mu = np.array([0.013, -0.021, 0.017])
        box = oracle.bbox(mu[None], s[None], q[None], dims, lo, inv_h, 7.0)
        V = oracle.voxelize(mu[None], s[None], q[None], [1.0], dims, lo, inv_h, box)
        if kind == 0:
            geom = inputs.parallel_geometry(4, 24, 24, 1.7 * h, h / 2, arc=math.pi * 0.9)
        else:
            geom = inputs.cone_geometry(4, 24, 24, 2.5 * h, 5.0, 7.5, h / 2, length_scale=1.0)
        P = oracle.project(V, dims, lo, inv_h, kind, geom.views, geom.nu, geom.nv, h / 2)
        Q = np.linalg.inv(_sigma_world(s, q))
        want = np.zeros_like(P)
        for j in range(4):
            c, d = _rays(geom, j)
            want[j] = np.array([_gauss_line_integral(c[i], d[i], mu, Q)
                                for i in range(len(c))]).reshape(geom.nv, geom.nu)
        errs.append(np.linalg.norm(P - want) / np.linalg.norm(want))
    assert errs[0] < 0.05
    assert 2.5 < errs[0] / errs[1] < 6.0, errs


def _slab_chord(c, d, lo, hi):
    t0, t1 = -np.inf, np.inf
    for a in range(3):
        if d[a] == 0:
            if not (lo[a] < c[a] < hi[a]):
                return 0.0
            continue
        ta, tb = sorted(((lo[a] - c[a]) / d[a], (hi[a] - c[a]) / d[a]))
        t0, t1 = max(t0, ta), min(t1, tb)
    return max(0.0, t1 - t0)


def test_siddon_single_voxel_chord():
    dims, lo, inv_h = (9, 8, 7), (-0.45, -0.4, -0.35), (10.0, 10.0, 10.0)
    V = np.zeros((7, 8, 9))
    vi = (4, 3, 2)  # x, y, z
    V[vi[2], vi[1], vi[0]] = 1.0
    geom = inputs.cone_geometry(5, 20, 16, 0.03, 2.0, 3.0, 0.01, arc=1.7, length_scale=1.0)  # no ray lies on a cell face
    P = oracle.project_siddon(V, dims, lo, inv_h, 1, geom.views, geom.nu, geom.nv)
    vlo = np.array(lo) + np.array(vi) * 0.1
    vhi = vlo + 0.1
    nz = 0
    for j in range(5):
        c, d = _rays(geom, j)
        want = np.array([_slab_chord(c[i], d[i], vlo, vhi) for i in range(len(c))])
        assert np.allclose(P[j].ravel(), want, atol=1e-12)
        nz += np.count_nonzero(want)
    assert nz > 20


def test_siddon_converges_to_ball_chords():
    errs = []
    R = 0.55
    for D in (24, 48):
        dims, lo, inv_h = _grid((D, D, D))
        sub = 6
        offs = (np.arange(sub) + 0.5) / sub
        x = -1 + (np.arange(D)[:, None] + offs[None]).ravel() / inv_h[0]
        occ = (x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2) <= R * R
        V = occ.reshape(D, sub, D, sub, D, sub).mean(axis=(1, 3, 5)).astype(np.float64)
        geom = inputs.cone_geometry(3, 31, 31, 0.045, 4.0, 6.0, 0.01, length_scale=1.0)
        P = oracle.project_siddon(V, dims, lo, inv_h, 1, geom.views, geom.nu, geom.nv)
        want = np.zeros_like(P)
        for j in range(3):
            c, d = _rays(geom, j)
            b2 = np.sum(c * c, -1)  # c is the point nearest the ball centre (origin)
            want[j] = (2 * np.sqrt(np.clip(R * R - b2, 0, None))).reshape(31, 31)
        errs.append(np.abs(P - want).mean() / want.mean())
    assert errs[1] < 0.02 and 1.6 < errs[0] / errs[1] < 2.6, errs  # first order in h


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_siddon_transpose(kind):
    """The exact-path transpose: adjoint identity with the forward, and one
    ray's backprojection sums to its chord through the grid box (slab
    clipping, computed independently)."""
    dims, lo, inv_h = (13, 11, 9), (-0.8125, -0.6875, -0.5625), (8.0, 8.0, 8.0)
    rng = np.random.default_rng(30 + kind)
    if kind == 0:
        geom = inputs.parallel_geometry(5, 15, 11, 0.11, 0.07)
    elif kind == 1:
        geom = inputs.cone_geometry(5, 15, 11, 0.15, 3.0, 4.5, 0.07, length_scale=2.0)
    else:
        geom = inputs.fan_geometry(5, 15, 11, 0.15, 0.125, 3.0, 4.5, 0.07, arc=2.0, length_scale=2.0)
    ell = geom.length_scale
    x = rng.normal(size=(9, 11, 13))
    Ax = oracle.project_siddon(x, dims, lo, inv_h, kind, geom.views, 15, 11, ell)
    y = rng.normal(size=Ax.shape)
    ATy = oracle.backproject_siddon(y, dims, lo, inv_h, kind, geom.views, 15, 11, ell)
    assert abs(np.sum(Ax * y) - np.sum(x * ATy)) <= 1e-12 * np.sqrt(np.sum(Ax ** 2) * np.sum(y ** 2))
    one = np.zeros_like(y)
    one[2, 5, 7] = 1.0
    B = oracle.backproject_siddon(one, dims, lo, inv_h, kind, geom.views, 15, 11, ell)
    c, d = _rays(geom, 2)
    hi = np.array(lo) + np.array(dims) / np.array(inv_h)
    chord = _slab_chord(c[5 * 15 + 7], d[5 * 15 + 7], np.array(lo), hi)
    assert chord > 0 and abs(B.sum() - ell * chord) < 1e-12 * ell * chord
    assert np.count_nonzero(B) > 5


def test_raymarch_and_siddon_agree_on_smooth_volume():
    D = 40
    dims, lo, inv_h = _grid((D, D, D))
    h = 1.0 / inv_h[0]
    mu = np.array([[0.02, -0.03, 0.01]])
    s = np.array([[6 * h, 5 * h, 7 * h]])
    q = np.array([[1.0, 0.3, 0.2, 0.1]])
    box = oracle.bbox(mu, s, q, dims, lo, inv_h, 6.0)
    V = oracle.voxelize(mu, s, q, [1.0], dims, lo, inv_h, box)
    geom = inputs.cone_geometry(3, 20, 20, 2 * h, 5.0, 7.5, h / 2, length_scale=1.0)
    a = oracle.project(V, dims, lo, inv_h, 1, geom.views, 20, 20, h / 2)
    b = oracle.project_siddon(V, dims, lo, inv_h, 1, geom.views, 20, 20)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-2


@pytest.mark.parametrize("kind", [0, 1])
def test_adjoint_identity(kind):
    dims, lo, inv_h = (13, 11, 9), (-0.8125, -0.6875, -0.5625), (8.0, 8.0, 8.0)
    rng = np.random.default_rng(10 + kind)
    x = rng.normal(size=(9, 11, 13))
    if kind == 0:
        geom = inputs.parallel_geometry(5, 15, 11, 0.11, 0.07)
    else:
        geom = inputs.cone_geometry(5, 15, 11, 0.15, 3.0, 4.5, 0.07, length_scale=2.0)
    Ax = oracle.project(x, dims, lo, inv_h, kind, geom.views, 15, 11, 0.07, geom.length_scale)
    y = rng.normal(size=Ax.shape)
    ATy = oracle.backproject(y, dims, lo, inv_h, kind, geom.views, 15, 11, 0.07, geom.length_scale)
    lhs, rhs = np.sum(Ax * y), np.sum(x * ATy)
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum(Ax ** 2) * np.sum(y ** 2))
    assert np.count_nonzero(Ax) > 0.5 * Ax.size


# --------------------------------------------------------------------------
# O8 gradient
# --------------------------------------------------------------------------
def test_voxelize_grad_matches_central_differences():
    dims, lo, inv_h = (18, 16, 14), (-0.5625, -0.5, -0.4375), (16.0, 16.0, 16.0)
    rng = np.random.default_rng(21)
    n = 10
    mu = rng.uniform(-0.2, 0.2, (n, 3))
    s = rng.uniform(1.5, 3.0, (n, 3)) / 16.0
    q = rng.normal(size=(n, 4))
    rho = rng.uniform(0.2, 1.0, n)
    q[3] = 0.0  # identity rotation, zero quaternion gradient
    box = oracle.bbox(mu, s, q, dims, lo, inv_h, 3.0)
    w = rng.normal(size=(dims[2], dims[1], dims[0]))
    dmu, ds, dq, dr = oracle.voxelize_grad(mu, s, q, rho, dims, lo, inv_h, box, w)

    def L(mu_, s_, q_, r_):
        return float(np.sum(w * oracle.voxelize(mu_, s_, q_, r_, dims, lo, inv_h, box)))

    for name, arr, grad, eps in (("mu", mu, dmu, 1e-6), ("scale", s, ds, 1e-7),
                                 ("quat", q, dq, 1e-6), ("rho", rho, dr, 1e-6)):
        fd = np.zeros_like(grad)
        for idx in np.ndindex(arr.shape):
            if name == "quat" and idx[0] == 3:
                continue
            args = [mu.copy(), s.copy(), q.copy(), rho.copy()]
            k = ("mu", "scale", "quat", "rho").index(name)
            args[k][idx] += eps
            lp = L(*args)
            args[k][idx] -= 2 * eps
            lm = L(*args)
            fd[idx] = (lp - lm) / (2 * eps)
        err = np.linalg.norm(fd - grad) / np.linalg.norm(fd)
        assert err < 1e-6, (name, err)
    assert np.all(dq[3] == 0.0)
    # d rho is the projection of dL/dV on the unit-density Gaussian
    V1 = oracle.voxelize(mu[:1], s[:1], q[:1], [1.0], dims, lo, inv_h, box[:1])
    assert abs(np.sum(w * V1) - dr[0]) < 1e-12 * np.sum(np.abs(w * V1))


# --------------------------------------------------------------------------
# L1, Adam, PSNR
# --------------------------------------------------------------------------
def test_l1_hand_values():
    p = np.array([1.0, 2.0, 3.0, 4.0])
    y = np.float32([1.5, 2.0, 2.0, 5.0])
    loss, g = oracle.l1(p, y)
    assert loss == pytest.approx((0.5 + 0 + 1 + 1) / 4, abs=1e-15)
    assert np.array_equal(g, np.array([-0.25, 0.0, 0.25, -0.25]))


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    p0 = rng.normal(size=50)
    grads = rng.normal(size=(4, 50))
    t = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for i in range(4):
        opt.zero_grad()
        t.grad = torch.tensor(grads[i])
        opt.step()
        oracle.adam(p, grads[i], m, v, 1e-3, i + 1)
    assert np.allclose(p, t.detach().numpy(), rtol=0, atol=1e-15)
    # first step moves every entry by lr * |g| / (|g| + eps)
    p1, m1, v1 = p0.copy(), np.zeros(50), np.zeros(50)
    oracle.adam(p1, grads[0], m1, v1, 1e-3, 1)
    assert np.allclose(p0 - p1, 1e-3 * grads[0] / (np.abs(grads[0]) + 1e-8), atol=1e-16)


@pytest.mark.parametrize("lower", [0.0, -0.5])
def test_projected_adam_matches_torch_then_clamp(lower):
    """The projected step equals torch.optim.Adam followed by clamp_ onto
    p >= lower (the moments are not touched by the projection); many entries
    start at or near the bound so that a good share is clamped."""
    import torch
    rng = np.random.default_rng(3)
    n = 400
    p0 = np.concatenate([np.full(100, lower), lower + rng.uniform(0, 2e-3, size=100), rng.normal(size=200)])
    p0 = np.maximum(p0, lower)
    grads = rng.normal(size=(6, n))
    grads[:, :150] = np.abs(grads[:, :150])  # pushes those entries down, into the bound
    t = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    clamped = 0
    for i in range(6):
        opt.zero_grad()
        t.grad = torch.tensor(grads[i])
        opt.step()
        with torch.no_grad():
            clamped += int((t < lower).sum())
            t.clamp_(min=lower)
        oracle.adam(p, grads[i], m, v, 1e-3, i + 1, lower=lower)
        np.testing.assert_allclose(p, t.detach().numpy(), rtol=0, atol=1e-15)
    assert clamped >= 150
    assert np.all(p >= lower) and np.sum(p == lower) >= 100
    np.testing.assert_allclose(m, opt.state[t]["exp_avg"].numpy(), rtol=0, atol=1e-15)


def test_psnr_hand_value():
    gt = np.zeros(1000)
    gt[0] = 2.0
    x = gt.copy()
    x[1:101] = 0.02  # MSE = 100 * 4e-4 / 1000 = 4e-5
    assert oracle.psnr(x, gt) == pytest.approx(10 * math.log10(4.0 / 4e-5), abs=1e-10)
