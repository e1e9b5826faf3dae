"""CPU oracle for the DGR hot path (binary64, plain C behind ctypes).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library in ``paper_2411_04844_amd`` and imports nothing from
it; the product path never calls into it.

Paper: Wu et al., "Discretized Gaussian Representation for Tomographic
Reconstruction", arXiv 2411.04844.

What pins each function (tests under ``tests/test_oracle_*.py``):

* ``bbox`` -- binary32 definition of the truncation box.  Pinned by a
  brute-force scan of voxel centres against the k-sigma slab in binary64
  (equal away from ties) and by the fixed-cuboid special case of Alg. 1.
* ``tile_pairs`` -- pinned by an independent enumeration (numpy) of
  tile/box overlaps and a library sort.
* ``voxelize_brute`` / ``voxelize_box`` -- pinned by: grid sum of a
  well-resolved untruncated Gaussian equals the closed form
  rho (2 pi)^{3/2} sqrt(det Sigma) / voxel volume (Poisson summation);
  an axis-aligned Gaussian equals the outer product of 1-D Gaussians;
  a 45-degree rotation about z is elongated along (1, 1, 0);
  q, -q and c q give the same volume; the truncated mass ratio lies in
  [erf(3/sqrt 2)^3, erf(3/sqrt 2)] for k_sigma = 3.
* ``project`` -- pinned by the axis identity (parallel beam along a grid
  axis through voxel centres gives voxel size x the column sum), by SciPy's
  ``map_coordinates(order=1, mode='grid-constant')`` at the same sample
  points, and by convergence to the closed-form line integral of a Gaussian
  for parallel and cone geometry.
* ``project_siddon`` -- pinned by exact chord lengths through a single voxel
  and by convergence to analytic chords of a ball.
* ``backproject`` -- pinned by the adjoint identity <Ax, y> = <x, A^T y>.
* ``voxelize_grad`` -- pinned by binary64 central differences of
  ``voxelize_box`` with frozen boxes, and by d rho = <dL/dV, G>.
* ``l1``, ``adam``, ``psnr`` -- pinned by hand-computed values and by
  ``torch.optim.Adam`` (followed by ``clamp_`` for the projected step).
* ``fdk`` -- pinned by reconstructing a uniform ball from its analytic
  projections (interior value and exterior zero within a few per cent), an
  off-centre ball whose halves nearer and farther from the rotation axis
  must agree (the distance weights), and by its ramp filter
  (``ramp_filter``): the impulse response is the textbook tap table, and a
  cosine row is scaled by |w| / (2 pi tau), the filter's Fourier series.
* ``init_from_volume`` -- pinned by brute-force inverse-CDF sampling in
  numpy and by the sampling frequencies of a two-voxel volume.
* ``oracle.unet`` (numpy, binary64) -- the learned-initialisation network:
  3x3x3 convolution against a seven-loop brute force and the impulse
  response, its backward against the adjoint identities, pooling/upsampling
  against theirs, the network and loss gradients against central
  differences (see that module's header).
* ``oracle.objective`` (numpy, binary64) -- the paper's full objective
  0.6 L1 + 0.2 L_SSIM + 1 L_TV: SSIM map against a brute-force window sum,
  SSIM(x, x) = 1, constant images against the closed form, TV of a ramp,
  both gradients against central differences.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dgr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fexcess-precision=standard", "-lm"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary64, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *_CFLAGS[:-1], _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_double
        L.orc_bbox.argtypes = [P, P, P, i64, P, P, P, f32, i32, P]
        L.orc_bbox.restype = None
        L.orc_tile_pairs.argtypes = [P, i64, P, P, P]
        L.orc_tile_pairs.restype = i64
        for name in ("orc_voxelize_brute", "orc_voxelize_box"):
            getattr(L, name).argtypes = [P, P, P, P, i64, P, P, P, P, P]
            getattr(L, name).restype = None
        L.orc_voxelize_grad.argtypes = [P, P, P, P, i64, P, P, P, P, P, P, P, P, P]
        L.orc_voxelize_grad.restype = None
        L.orc_project.argtypes = [P, P, P, P, i32, i32, i32, i32, P, f64, f64, P]
        L.orc_project.restype = None
        L.orc_backproject.argtypes = [P, P, P, P, i32, i32, i32, i32, P, f64, f64, P]
        L.orc_backproject.restype = None
        L.orc_project_siddon.argtypes = [P, P, P, P, i32, i32, i32, i32, P, f64, P]
        L.orc_project_siddon.restype = None
        L.orc_backproject_siddon.argtypes = [P, P, P, P, i32, i32, i32, i32, P, f64, P]
        L.orc_backproject_siddon.restype = None
        L.orc_l1.argtypes = [P, P, i64, P]
        L.orc_l1.restype = f64
        L.orc_adam.argtypes = [P, P, P, P, i64, f64, f64, f64, f64, i64, f64]
        L.orc_adam.restype = None
        L.orc_psnr.argtypes = [P, P, i64]
        L.orc_psnr.restype = f64
        L.orc_ramp_filter.argtypes = [P, i64, f64, P]
        L.orc_ramp_filter.restype = None
        L.orc_fdk.argtypes = [P, i32, i32, i32, i32, P, f64, f64, P, P, P, P]
        L.orc_fdk.restype = None
        L.orc_init_from_volume.argtypes = [P, P, P, P, f64, i64, P, f64, P, P, P, P, P]
        L.orc_init_from_volume.restype = i64
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [i32]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the following oracle calls (OpenMP)."""
    lib().orc_set_num_threads(int(n))


def _grid_args(dims, lo, inv_h, dtype):
    return _c(dims, np.int32), _c(lo, dtype), _c(inv_h, dtype)


def bbox(mu, scale, quat, dims, lo, inv_h, k_sigma=3.0, box_half=8):
    """Truncation boxes, int32 [n, 6] = (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z)."""
    mu, scale, quat = _c(mu, np.float32), _c(scale, np.float32), _c(quat, np.float32)
    n = mu.shape[0]
    d, l, h = _grid_args(dims, lo, inv_h, np.float32)
    box = np.zeros((n, 6), np.int32)
    lib().orc_bbox(_p(mu), _p(scale), _p(quat), n, _p(d), _p(l), _p(h),
                   float(k_sigma), int(box_half), _p(box))
    return box


def tile_pairs(box, dims):
    """Sorted (tile, gid) pairs uint32 [P, 2] and tile_begin int64 [T+1]."""
    box = _c(box, np.int32)
    d = _c(dims, np.int32)
    n = box.shape[0]
    P = lib().orc_tile_pairs(_p(box), n, _p(d), None, None)
    T = int(np.prod([(x + 7) // 8 for x in dims]))
    pairs = np.zeros((max(P, 1), 2), np.uint32)
    tb = np.zeros(T + 1, np.int64)
    lib().orc_tile_pairs(_p(box), n, _p(d), _p(pairs), _p(tb))
    return pairs[:P], tb


def _params64(mu, scale, quat, density):
    return (_c(mu, np.float64), _c(scale, np.float64), _c(quat, np.float64),
            _c(density, np.float64))


def voxelize(mu, scale, quat, density, dims, lo, inv_h, box, brute=False):
    """Volume float64 [nz, ny, nx]: sum of rho * G over each Gaussian's box."""
    mu, scale, quat, density = _params64(mu, scale, quat, density)
    box = _c(box, np.int32)
    d, l, h = _grid_args(dims, lo, inv_h, np.float64)
    V = np.zeros((dims[2], dims[1], dims[0]), np.float64)
    fn = lib().orc_voxelize_brute if brute else lib().orc_voxelize_box
    fn(_p(mu), _p(scale), _p(quat), _p(density), mu.shape[0], _p(d), _p(l), _p(h), _p(box), _p(V))
    return V


def voxelize_grad(mu, scale, quat, density, dims, lo, inv_h, box, dV):
    """Gradients (dmu, dscale, dquat, ddensity) in float64 given dL/dV."""
    mu, scale, quat, density = _params64(mu, scale, quat, density)
    box = _c(box, np.int32)
    dV = _c(dV, np.float64)
    d, l, h = _grid_args(dims, lo, inv_h, np.float64)
    n = mu.shape[0]
    dmu, ds, dq, dr = (np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 4)), np.zeros(n))
    lib().orc_voxelize_grad(_p(mu), _p(scale), _p(quat), _p(density), n, _p(d), _p(l), _p(h),
                            _p(box), _p(dV), _p(dmu), _p(ds), _p(dq), _p(dr))
    return dmu, ds, dq, dr


def project(V, dims, lo, inv_h, kind, views, nu, nv, step, length_scale=1.0):
    """Trilinear ray-march projection float64 [n_views, nv, nu]."""
    V = _c(V, np.float64)
    views = _c(views, np.float32)
    nviews = views.shape[0]
    d, l, h = _grid_args(dims, lo, inv_h, np.float64)
    out = np.zeros((nviews, nv, nu), np.float64)
    lib().orc_project(_p(V), _p(d), _p(l), _p(h), int(kind), nviews, int(nu), int(nv), _p(views),
                      float(step), float(length_scale), _p(out))
    return out


def backproject(proj, dims, lo, inv_h, kind, views, nu, nv, step, length_scale=1.0):
    """Adjoint of ``project``: float64 volume [nz, ny, nx]."""
    proj = _c(proj, np.float64)
    views = _c(views, np.float32)
    nviews = views.shape[0]
    d, l, h = _grid_args(dims, lo, inv_h, np.float64)
    V = np.zeros((dims[2], dims[1], dims[0]), np.float64)
    lib().orc_backproject(_p(proj), _p(d), _p(l), _p(h), int(kind), nviews, int(nu), int(nv),
                          _p(views), float(step), float(length_scale), _p(V))
    return V


def backproject_siddon(proj, dims, lo, inv_h, kind, views, nu, nv, length_scale=1.0):
    """Transpose of project_siddon: float64 volume [nz, ny, nx]."""
    proj = _c(proj, np.float64)
    views = _c(views, np.float32)
    nviews = views.shape[0]
    d, l, h = _grid_args(dims, lo, inv_h, np.float64)
    V = np.zeros((dims[2], dims[1], dims[0]), np.float64)
    lib().orc_backproject_siddon(_p(proj), _p(d), _p(l), _p(h), int(kind), nviews, int(nu), int(nv),
                                 _p(views), float(length_scale), _p(V))
    return V


def project_siddon(V, dims, lo, inv_h, kind, views, nu, nv, length_scale=1.0):
    """Exact-path (Siddon) projection float64 [n_views, nv, nu]."""
    V = _c(V, np.float64)
    views = _c(views, np.float32)
    nviews = views.shape[0]
    d, l, h = _grid_args(dims, lo, inv_h, np.float64)
    out = np.zeros((nviews, nv, nu), np.float64)
    lib().orc_project_siddon(_p(V), _p(d), _p(l), _p(h), int(kind), nviews, int(nu), int(nv),
                             _p(views), float(length_scale), _p(out))
    return out


def l1(proj, target):
    """Mean absolute residual and its gradient sign(r)/M (float64)."""
    proj = _c(proj, np.float64)
    target = _c(target, np.float32)
    g = np.zeros(proj.shape, np.float64)
    loss = lib().orc_l1(_p(proj), _p(target), proj.size, _p(g))
    return float(loss), g


def adam(p, g, m, v, lr, t, b1=0.9, b2=0.999, eps=1e-8, lower=-np.inf):
    """One Adam step in place on float64 arrays p, m, v, projected onto
    p >= lower (-inf: the plain step)."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _c(g, np.float64)
    lib().orc_adam(_p(p), _p(g), _p(m), _p(v), p.size, float(lr), float(b1), float(b2),
                   float(eps), int(t), float(lower))


def ramp_filter(p, tau):
    """The FDK step's discrete Ram-Lak filter of one row (float64)."""
    p = _c(p, np.float64)
    q = np.zeros_like(p)
    lib().orc_ramp_filter(_p(p), p.size, float(tau), _p(q))
    return q


def fdk(proj, views, nu, nv, arc, length_scale, dims, lo, inv_h, kind=1):
    """FDK volume float64 [nz, ny, nx] from cone-beam projections (kind 1),
    or slice-by-slice fan-beam FBP (kind 2)."""
    proj = _c(proj, np.float32)
    views = _c(views, np.float32)
    d, l, h = _grid_args(dims, lo, inv_h, np.float64)
    V = np.zeros((dims[2], dims[1], dims[0]), np.float64)
    lib().orc_fdk(_p(proj), int(kind), views.shape[0], int(nu), int(nv), _p(views), float(arc),
                  float(length_scale), _p(d), _p(l), _p(h), _p(V))
    return V


def init_from_volume(f, dims, lo, inv_h, thresh_frac, uniforms, scale):
    """Initial Gaussians drawn from a volume; returns (mu, scale, quat, rho,
    voxel index, count of voxels above the threshold)."""
    f = _c(f, np.float32)
    u = _c(uniforms, np.float64)
    n = u.shape[0]
    d, l, h = _grid_args(dims, lo, inv_h, np.float64)
    mu, sc, q, rho = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 4)), np.zeros(n)
    vox = np.zeros(n, np.int64)
    above = lib().orc_init_from_volume(_p(f), _p(d), _p(l), _p(h), float(thresh_frac), n, _p(u),
                                       float(scale), _p(mu), _p(sc), _p(q), _p(rho), _p(vox))
    return mu, sc, q, rho, vox, int(above)


def psnr(x, gt):
    x, gt = _c(x, np.float64), _c(gt, np.float64)
    return float(lib().orc_psnr(_p(x), _p(gt), x.size))
