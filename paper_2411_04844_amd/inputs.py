"""Seeded synthetic inputs for the DGR hot path.

This module holds only random draws and acquisition set-up: Gaussian
parameter sets, view tables (source/detector vectors), ellipsoid phantoms
with their analytic line integrals, and noise.  It contains none of the
method's arithmetic (no voxelization, projection or gradient), so the HIP
library, its tests and the oracle can all be fed from it without sharing
compute.  Everything is deterministic given the seed (NumPy PCG64).

Units.  The reconstruction cube is [-1, 1]^3 in world units.  For the
cone-beam workloads one world unit is 128 mm, so the cube is 256 mm wide;
line integrals are multiplied by ``MM_PER_UNIT`` so that attenuation in
mm^-1 gives dimensionless projections.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

MM_PER_UNIT = 128.0


def _f32(x) -> float:
    return float(np.float32(x))


@dataclass(frozen=True)
class GridSpec:
    """Voxel grid.  lo and inv_h are stored rounded to binary32, the precision
    the C ABI takes them in, so every consumer sees the same numbers."""
    dims: tuple  # (nx, ny, nz)
    lo: tuple    # world coordinate of the lower faces
    inv_h: tuple  # 1 / voxel size per axis

    def __post_init__(self):
        object.__setattr__(self, "dims", tuple(int(d) for d in self.dims))
        object.__setattr__(self, "lo", tuple(_f32(x) for x in self.lo))
        object.__setattr__(self, "inv_h", tuple(_f32(x) for x in self.inv_h))

    @property
    def shape(self):  # numpy/torch shape [nz, ny, nx]
        return (self.dims[2], self.dims[1], self.dims[0])

    @property
    def h(self):
        return 1.0 / self.inv_h[0]


def cube_grid(D: int) -> GridSpec:
    """D^3 voxels over [-1, 1]^3; inv_h = D/2 is exact in binary32."""
    return GridSpec((D, D, D), (-1.0, -1.0, -1.0), (D / 2.0, D / 2.0, D / 2.0))


@dataclass(frozen=True)
class Geometry:
    """Acquisition geometry; step and length_scale are stored rounded to
    binary32 (the ABI's precision), views are binary32."""
    kind: int          # 0 parallel, 1 cone, 2 fan (a stack of fan-beam rows)
    views: np.ndarray  # float32 [n_views, 12]
    nu: int
    nv: int
    step: float        # march step, world units
    length_scale: float

    def __post_init__(self):
        object.__setattr__(self, "views", np.ascontiguousarray(self.views, np.float32))
        object.__setattr__(self, "step", _f32(self.step))
        object.__setattr__(self, "length_scale", _f32(self.length_scale))

    @property
    def n_views(self):
        return int(self.views.shape[0])

    @property
    def n_rays(self):
        return self.n_views * self.nu * self.nv


def gaussians(n: int, seed: int, s_lo: float, s_hi: float, mean_lim: float = 0.8,
              ratio_max: float | None = None):
    """Gaussian parameter set, float32.

    Draw order: means U[-mean_lim, mean_lim]^3; scales log-uniform in
    [s_lo, s_hi] per axis (or, with ``ratio_max``, a largest scale
    log-uniform in [s_lo, s_hi] and the other two divided by factors
    log-uniform in [1, ratio_max]); quaternions normalised N(0, I_4)
    (uniform rotations); densities U[0, 1].
    """
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-mean_lim, mean_lim, size=(n, 3))
    if ratio_max is None:
        scale = np.exp(rng.uniform(math.log(s_lo), math.log(s_hi), size=(n, 3)))
    else:
        smax = np.exp(rng.uniform(math.log(s_lo), math.log(s_hi), size=(n, 1)))
        fac = np.exp(rng.uniform(0.0, math.log(ratio_max), size=(n, 2)))
        scale = np.concatenate([smax, smax / fac], axis=1)
        perm = np.argsort(rng.uniform(size=(n, 3)), axis=1)
        scale = np.take_along_axis(scale, perm, axis=1)
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    rho = rng.uniform(0.0, 1.0, size=n)
    return dict(mu=mu.astype(np.float32), scale=scale.astype(np.float32),
                quat=q.astype(np.float32), density=rho.astype(np.float32))


def parallel_geometry(n_views: int, nu: int, nv: int, pitch: float, step: float,
                      arc: float = math.pi, length_scale: float = 1.0) -> Geometry:
    """Parallel beam rotating about z: view j at theta = arc * j / n_views.

    Ray direction (cos t, sin t, 0); detector plane through the origin with
    e_u = pitch (-sin t, cos t, 0), e_v = pitch (0, 0, 1).
    """
    v = np.zeros((n_views, 12), np.float64)
    for j in range(n_views):
        t = arc * j / n_views
        c, s = math.cos(t), math.sin(t)
        v[j, 0:3] = (c, s, 0.0)
        v[j, 3:6] = (0.0, 0.0, 0.0)
        v[j, 6:9] = (-s * pitch, c * pitch, 0.0)
        v[j, 9:12] = (0.0, 0.0, pitch)
    return Geometry(0, v.astype(np.float32), nu, nv, step, length_scale)


def cone_geometry(n_views: int, nu: int, nv: int, pitch: float, dso: float, dsd: float,
                  step: float, arc: float = 2 * math.pi,
                  length_scale: float = MM_PER_UNIT) -> Geometry:
    """Circular cone beam about z with a flat detector, world units.

    Source at dso (cos t, sin t, 0); detector centre at -(dsd - dso)(cos t,
    sin t, 0); e_u = pitch (-sin t, cos t, 0), e_v = pitch (0, 0, 1).
    """
    v = np.zeros((n_views, 12), np.float64)
    for j in range(n_views):
        t = arc * j / n_views
        c, s = math.cos(t), math.sin(t)
        v[j, 0:3] = (dso * c, dso * s, 0.0)
        v[j, 3:6] = (-(dsd - dso) * c, -(dsd - dso) * s, 0.0)
        v[j, 6:9] = (-s * pitch, c * pitch, 0.0)
        v[j, 9:12] = (0.0, 0.0, pitch)
    return Geometry(1, v.astype(np.float32), nu, nv, step, length_scale)


def fan_geometry(n_views: int, nu: int, nv: int, pitch_u: float, pitch_v: float, dso: float,
                 dsd: float, step: float, arc: float = 2 * math.pi, start: float = 0.0,
                 length_scale: float = MM_PER_UNIT) -> Geometry:
    """A stack of nv fan-beam slices about z with a flat (line) detector per
    slice, world units: view j at t = start + arc * j / n_views.

    Source of the central row at dso (cos t, sin t, 0), detector centre at
    -(dsd - dso)(cos t, sin t, 0); e_u = pitch_u (-sin t, cos t, 0) and
    e_v = pitch_v (0, 0, 1).  Row iv sits at height (iv - (nv-1)/2) pitch_v,
    its source at the same height.
    """
    v = np.zeros((n_views, 12), np.float64)
    for j in range(n_views):
        t = start + arc * j / n_views
        c, s = math.cos(t), math.sin(t)
        v[j, 0:3] = (dso * c, dso * s, 0.0)
        v[j, 3:6] = (-(dsd - dso) * c, -(dsd - dso) * s, 0.0)
        v[j, 6:9] = (-s * pitch_u, c * pitch_u, 0.0)
        v[j, 9:12] = (0.0, 0.0, pitch_v)
    return Geometry(2, v.astype(np.float32), nu, nv, step, length_scale)


def fan_workload(D: int, n_views: int, n_det: int, arc: float = 2 * math.pi, start: float = 0.0,
                 dso_mm: float = 595.0, dsd_mm: float = 1085.6) -> Geometry:
    """Fan beam over the 256 mm cube: one detector row per slice (pitch = the
    slice thickness, so rows sit on voxel centres in z), n_det columns that
    span 1.5 D voxels at the isocentre (the cube's diagonal is 1.41 D), march
    step 0.5 voxel.  Distances follow a clinical fan-beam scanner
    (source-isocentre 595 mm, source-detector 1085.6 mm)."""
    h = 2.0 / D
    mag = dsd_mm / dso_mm
    return fan_geometry(n_views, n_det, D, mag * h * 1.5 * D / n_det, h, dso_mm / MM_PER_UNIT,
                        dsd_mm / MM_PER_UNIT, 0.5 * h, arc, start)


def cone_workload(D: int, n_views: int, n_det: int, pitch_mm: float, arc=2 * math.pi,
                  dso_mm: float = 1000.0, dsd_mm: float = 1500.0) -> Geometry:
    """Cone geometry in world units for a 256 mm cube, march step 0.5 voxel."""
    h = 2.0 / D
    return cone_geometry(n_views, n_det, n_det, pitch_mm / MM_PER_UNIT, dso_mm / MM_PER_UNIT,
                         dsd_mm / MM_PER_UNIT, 0.5 * h, arc)


# --------------------------------------------------------------------------
# Ellipsoid phantoms (synthetic measurements and ground truth)
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Phantom:
    centers: np.ndarray   # [m, 3] world units
    axes: np.ndarray      # [m, 3] semi-axes, world units
    rot: np.ndarray       # [m, 3, 3] columns are the ellipsoid axes
    att: np.ndarray       # [m] attenuation, mm^-1


def _random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def ellipsoid_phantom(seed: int, count=(10, 20), axes=(0.05, 0.6), att=(0.0, 0.05),
                      r_xy: float = 0.9, z_lim: float = 0.85) -> Phantom:
    """10-20 random ellipsoids; attenuations add where they overlap.

    Centres are redrawn until the bounding sphere (radius = largest
    semi-axis) lies inside the cylinder r_xy, |z| <= z_lim.
    """
    rng = np.random.default_rng(seed)
    m = int(rng.integers(count[0], count[1] + 1))
    C, A, Rs, mu = [], [], [], []
    for _ in range(m):
        a = rng.uniform(axes[0], axes[1], size=3)
        R = _random_rotation(rng)
        rad = float(a.max())
        while True:
            c = rng.uniform(-1.0, 1.0, size=3)
            if math.hypot(c[0], c[1]) + rad <= r_xy and abs(c[2]) + rad <= z_lim:
                break
            # shrink the ellipsoid if it cannot fit at all
            if rad >= min(r_xy, z_lim):
                a *= 0.5 * min(r_xy, z_lim) / rad
                rad = float(a.max())
        C.append(c), A.append(a), Rs.append(R), mu.append(rng.uniform(att[0], att[1]))
    return Phantom(np.array(C), np.array(A), np.array(Rs), np.array(mu))


def _ray_dirs(geom: Geometry, views_idx, device, torch):
    """Origins and unit directions (float64) of all rays of the given views."""
    v = torch.as_tensor(geom.views[views_idx].astype(np.float64), device=device)
    iu = torch.arange(geom.nu, device=device, dtype=torch.float64) - 0.5 * (geom.nu - 1)
    iv = torch.arange(geom.nv, device=device, dtype=torch.float64) - 0.5 * (geom.nv - 1)
    pix = (v[:, None, None, 3:6] + iu[None, None, :, None] * v[:, None, None, 6:9]
           + iv[None, :, None, None] * v[:, None, None, 9:12])
    if geom.kind == 0:
        d = v[:, None, None, 0:3].expand_as(pix)
        o = pix
    elif geom.kind == 1:
        o = v[:, None, None, 0:3].expand_as(pix)
        d = pix - o
    else:  # fan: each row's source sits at the row's height
        o = v[:, None, None, 0:3] + iv[None, :, None, None] * v[:, None, None, 9:12]
        o = o.expand_as(pix)
        d = pix - o
    d = d / torch.linalg.norm(d, dim=-1, keepdim=True)
    return o, d


def phantom_projections(ph: Phantom, geom: Geometry, device="cpu", chunk: int = 8):
    """Analytic line integrals of the phantom, float32 [n_views, nv, nu].

    Each ellipsoid contributes attenuation x chord length (mm), the chord of
    the line o + t d through {x : (x-c)^T A (x-c) <= 1} being
    2 sqrt(b^2 - a (g - 1)) / a with a = d^T A d, b = d^T A (o - c),
    g = (o - c)^T A (o - c).
    """
    import torch
    out = torch.empty((geom.n_views, geom.nv, geom.nu), dtype=torch.float32, device=device)
    Amats = [R @ np.diag(1.0 / ax ** 2) @ R.T for R, ax in zip(ph.rot, ph.axes)]
    for j0 in range(0, geom.n_views, chunk):
        idx = np.arange(j0, min(j0 + chunk, geom.n_views))
        o, d = _ray_dirs(geom, idx, device, torch)
        acc = torch.zeros(o.shape[:-1], dtype=torch.float64, device=device)
        for c, A, mu in zip(ph.centers, Amats, ph.att):
            At = torch.as_tensor(A, device=device)
            oc = o - torch.as_tensor(c, device=device)
            Ad = d @ At
            a = (Ad * d).sum(-1)
            b = (Ad * oc).sum(-1)
            g = ((oc @ At) * oc).sum(-1)
            disc = torch.clamp(b * b - a * (g - 1.0), min=0.0)
            acc += float(mu) * 2.0 * torch.sqrt(disc) / a
        out[idx[0]:idx[-1] + 1] = (acc * MM_PER_UNIT).to(torch.float32)
    return out


def add_noise(y, seed: int, frac: float = 0.01):
    """y + N(0, (frac * max y)^2), seeded, same device and dtype as y."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    noise = torch.randn(y.shape, generator=g, dtype=torch.float32)
    return y + (frac * float(y.max())) * noise.to(y.device)


def phantom_volume(ph: Phantom, grid: GridSpec, sub: int = 4, device="cpu"):
    """Ground-truth attenuation (mm^-1), averaged over sub^3 points per voxel."""
    import torch
    nx, ny, nz = grid.dims
    out = torch.zeros(grid.shape, dtype=torch.float64, device=device)
    offs = (torch.arange(sub, dtype=torch.float64, device=device) + 0.5) / sub
    for zi in range(nz):
        z = grid.lo[2] + (zi + offs) / grid.inv_h[2]
        y = grid.lo[1] + (torch.arange(ny, device=device, dtype=torch.float64)[:, None] + offs) / grid.inv_h[1]
        x = grid.lo[0] + (torch.arange(nx, device=device, dtype=torch.float64)[:, None] + offs) / grid.inv_h[0]
        Z = z[:, None, None, None, None].expand(sub, ny, sub, nx, sub)
        Y = y[None, :, :, None, None].expand(sub, ny, sub, nx, sub)
        X = x[None, None, None, :, :].expand(sub, ny, sub, nx, sub)
        P = torch.stack([X, Y, Z], dim=-1)
        slab = torch.zeros((sub, ny, sub, nx, sub), dtype=torch.float64, device=device)
        for c, ax, R, mu in zip(ph.centers, ph.axes, ph.rot, ph.att):
            loc = (P - torch.as_tensor(c, device=device)) @ torch.as_tensor(R, device=device)
            inside = ((loc / torch.as_tensor(ax, device=device)) ** 2).sum(-1) <= 1.0
            slab += float(mu) * inside
        out[zi] = slab.mean(dim=(0, 2, 4))
    return out
