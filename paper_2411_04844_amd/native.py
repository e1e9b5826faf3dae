"""ctypes binding of libdgr.so (argument marshalling only).

Every function here has the name of the C entry point it calls and takes
torch tensors on the GPU; all computation happens in the HIP kernels.  The
library must have been built (``python -m paper_2411_04844_amd.build``);
loading fails loudly otherwise -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

from .inputs import Geometry, GridSpec

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdgr.so")

DGR_OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "workspace", 3: "capacity", 4: "hip"}


class DgrError(RuntimeError):
    def __init__(self, fn, status, detail):
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {detail}")
        self.status = status


class DgrGrid(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3), ("lo", ctypes.c_float * 3),
                ("inv_h", ctypes.c_float * 3)]


class DgrTrunc(ctypes.Structure):
    _fields_ = [("k_sigma", ctypes.c_float), ("box_half", ctypes.c_int32)]


class DgrGeometry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_views", ctypes.c_int32), ("nu", ctypes.c_int32),
                ("nv", ctypes.c_int32), ("views", ctypes.c_void_p), ("step", ctypes.c_float),
                ("length_scale", ctypes.c_float)]


class DgrGaussians(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("mu", "scale", "quat", "density", "m_mu", "m_scale", "m_quat",
                                               "m_density", "v_mu", "v_scale", "v_quat", "v_density")]


class DgrDensifyParams(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("tau", ctypes.c_float), ("tau_prune", ctypes.c_float),
                ("theta", ctypes.c_float), ("size_vox", ctypes.c_float), ("n_max", ctypes.c_int64)]


_lib = None
_SIGS = {
    "dgr_voxelize_workspace": (ctypes.c_size_t, ["i64", "i64", "grid"]),
    "dgr_voxelize_plan": ("st", ["p", "p", "p", "i64", "grid", "trunc", "p", "p", "sz", "p"]),
    "dgr_voxelize": ("st", ["p", "p", "p", "p", "i64", "grid", "trunc", "p", "p", "sz", "p"]),
    "dgr_voxelize_backward_workspace": (ctypes.c_size_t, ["i64"]),
    "dgr_voxelize_backward": ("st", ["p", "p", "p", "p", "i64", "grid", "trunc", "p", "p", "p",
                                     "p", "p", "p", "sz", "p"]),
    "dgr_voxelize_backward_noalloc_max": (ctypes.c_int64, []),
    "dgr_voxelize_backward_noalloc": ("st", ["p", "p", "p", "p", "i64", "grid", "trunc", "p", "p", "p",
                                             "p", "p", "p"]),
    "dgr_project_workspace": (ctypes.c_size_t, ["grid", "geom"]),
    "dgr_project": ("st", ["p", "grid", "geom", "p", "p", "sz", "p"]),
    "dgr_project_l1": ("st", ["p", "grid", "geom", "p", "p", "p", "p", "sz", "p"]),
    "dgr_backproject": ("st", ["p", "grid", "geom", "p", "p", "sz", "p"]),
    "dgr_backproject_weight_bound": ("st", ["grid", "geom", "p", "p"]),
    "dgr_project_siddon": ("st", ["p", "grid", "geom", "p", "p"]),
    "dgr_backproject_siddon_workspace": (ctypes.c_size_t, ["grid"]),
    "dgr_backproject_siddon": ("st", ["p", "grid", "geom", "p", "p", "sz", "p"]),
    "dgr_adam": ("st", ["p", "p", "p", "p", "i64", "f32", "f32", "f32", "f32", "i64", "f32", "p"]),
    "dgr_bbox": ("st", ["p", "p", "p", "i64", "grid", "trunc", "p", "p"]),
    "dgr_bin": ("st", ["p", "p", "p", "i64", "grid", "trunc", "p", "p", "p", "sz", "p"]),
    "dgr_check": ("st", ["p", "p"]),
    "dgr_voxelize_f64_workspace": (ctypes.c_size_t, ["i64", "i64", "grid"]),
    "dgr_voxelize_f64": ("st", ["p", "p", "p", "p", "i64", "grid", "trunc", "p", "p", "sz", "p"]),
    "dgr_fd_l1_f64_workspace": (ctypes.c_size_t, ["i64", "i32", "i64", "geom"]),
    "dgr_fd_l1_f64": ("st", ["p", "grid", "geom", "p", "p", "p", "p", "p", "i64", "trunc", "p", "p",
                             "p", "i32", "i64", "p", "p", "sz", "p"]),
    "dgr_fdk_workspace": (ctypes.c_size_t, ["grid", "geom"]),
    "dgr_fdk": ("st", ["p", "grid", "geom", "f32", "p", "p", "sz", "p"]),
    "dgr_reduce_workspace": (ctypes.c_size_t, []),
    "dgr_psnr": ("st", ["p", "p", "i64", "p", "p", "sz", "p"]),
    "dgr_init_workspace": (ctypes.c_size_t, ["grid"]),
    "dgr_init_from_volume": ("st", ["p", "grid", "f32", "i64", "p", "f32", "p", "p", "p", "p", "p",
                                    "sz", "p"]),
    "dgr_fit_density_scale": ("st", ["p", "p", "i64", "p", "i64", "p", "p", "sz", "p"]),
    "dgr_unet_param_count": (ctypes.c_int64, ["i32"]),
    "dgr_unet_workspace": (ctypes.c_size_t, ["dims", "i32"]),
    "dgr_unet_forward": ("st", ["p", "p", "dims", "i32", "p", "p", "sz", "p"]),
    "dgr_unet_backward": ("st", ["p", "p", "dims", "i32", "p", "p", "p", "sz", "p"]),
    "dgr_unet_loss_workspace": (ctypes.c_size_t, []),
    "dgr_unet_loss": ("st", ["p", "p", "i64", "p", "p", "p", "sz", "p"]),
    "dgr_conv3_forward": ("st", ["p", "i32", "dims", "i32", "p", "p", "i32", "i32", "p", "i32", "p"]),
    "dgr_conv3_grad_workspace": (ctypes.c_size_t, ["dims", "i32", "i32"]),
    "dgr_conv3_backward": ("st", ["p", "i32", "dims", "i32", "p", "p", "i32", "p", "p", "p", "p", "sz",
                                  "p"]),
    "dgr_accumulate_grad_norm": ("st", ["p", "i64", "p", "p"]),
    "dgr_densify_workspace": (ctypes.c_size_t, ["i64"]),
    "dgr_densify": ("st", ["gs", "i64", "p", "p", "grid", "dens", "gs", "p", "p", "p", "sz", "p"]),
    "dgr_projection_loss_workspace": (ctypes.c_size_t, ["i32", "i32", "i32"]),
    "dgr_projection_loss": ("st", ["p", "p", "i32", "i32", "i32", "f32", "f32", "f32", "p", "p", "p", "sz",
                                   "p"]),
    "dgr_tv_workspace": (ctypes.c_size_t, []),
    "dgr_tv": ("st", ["p", "grid", "f32", "p", "p", "p", "sz", "p"]),
    "dgr_pool2_f32": ("st", ["p", "dims", "p", "p"]),
    "dgr_unet_targets_workspace": (ctypes.c_size_t, ["grid"]),
    "dgr_unet_targets": ("st", ["p", "p", "i64", "grid", "p", "f32", "p", "p", "sz", "p"]),
    "dgr_init_from_unet_workspace": (ctypes.c_size_t, ["grid"]),
    "dgr_init_from_unet": ("st", ["p", "grid", "i64", "p", "f32", "p", "p", "p", "p", "p", "sz", "p"]),
    "dgr_status_string": (ctypes.c_char_p, ["i32"]),
    "dgr_last_error": (ctypes.c_char_p, []),
    "dgr_version": (ctypes.c_int32, []),
}
_CT = {"p": ctypes.c_void_p, "i64": ctypes.c_int64, "i32": ctypes.c_int32, "f32": ctypes.c_float,
       "sz": ctypes.c_size_t, "grid": ctypes.POINTER(DgrGrid), "trunc": ctypes.POINTER(DgrTrunc),
       "geom": ctypes.POINTER(DgrGeometry), "st": ctypes.c_int,
       "dims": ctypes.POINTER(ctypes.c_int32), "gs": ctypes.POINTER(DgrGaussians),
       "dens": ctypes.POINTER(DgrDensifyParams)}


def lib():
    """Load libdgr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                               "`python -m paper_2411_04844_amd.build` (no fallback exists)")
        L = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = _CT[res] if isinstance(res, str) else res
            f.argtypes = [_CT[a] for a in args]
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(fn, st):
    if st != DGR_OK:
        raise DgrError(fn, st, lib().dgr_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, shape=None, name="tensor"):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} GPU tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def c_grid(grid: GridSpec) -> DgrGrid:
    g = DgrGrid()
    for a in range(3):
        g.dims[a], g.lo[a], g.inv_h[a] = grid.dims[a], grid.lo[a], grid.inv_h[a]
    return g


def c_trunc(k_sigma=3.0, box_half=8) -> DgrTrunc:
    return DgrTrunc(float(k_sigma), int(box_half))


def c_geom(geom: Geometry, views_dev: torch.Tensor) -> DgrGeometry:
    _need(views_dev, torch.float32, (geom.n_views, 12), "views")
    return DgrGeometry(geom.kind, geom.n_views, geom.nu, geom.nv, views_dev.data_ptr(),
                       float(geom.step), float(geom.length_scale))


class Workspace:
    """A zero-initialised, 256-byte-aligned device buffer that grows on demand."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.zeros(nbytes + 256, dtype=torch.uint8, device=self.device)
        return self.buf

    def ptr_size(self, nbytes):
        b = self.get(nbytes)
        base = b.data_ptr()
        off = (-base) % 256
        return ctypes.c_void_p(base + off), b.numel() - off


# --------------------------------------------------------------------------
# entry points
# --------------------------------------------------------------------------
def dgr_voxelize_workspace(n, max_pairs, grid: GridSpec) -> int:
    g = c_grid(grid)
    return int(lib().dgr_voxelize_workspace(int(n), int(max_pairs), ctypes.byref(g)))


def dgr_voxelize_plan(mu, scale, quat, grid: GridSpec, k_sigma=3.0, box_half=8, ws=None) -> int:
    n = mu.shape[0]
    ws = ws or Workspace(mu.device)
    p, sz = ws.ptr_size(dgr_voxelize_workspace(n, 0, grid))
    out = ctypes.c_int64(0)
    g, t = c_grid(grid), c_trunc(k_sigma, box_half)
    _check("dgr_voxelize_plan", lib().dgr_voxelize_plan(
        _ptr(mu), _ptr(scale), _ptr(quat), n, ctypes.byref(g), ctypes.byref(t), ctypes.byref(out),
        p, sz, _stream()))
    return int(out.value)


def dgr_voxelize(mu, scale, quat, density, grid: GridSpec, k_sigma=3.0, box_half=8, out=None,
                 ws: Workspace | None = None, max_pairs: int | None = None):
    n = mu.shape[0]
    for name, t, c in (("mu", mu, 3), ("scale", scale, 3), ("quat", quat, 4)):
        _need(t, torch.float32, (n, c), name)
    _need(density, torch.float32, (n,), "density")
    if out is None:
        out = torch.empty(grid.shape, dtype=torch.float32, device=mu.device)
    _need(out, torch.float32, grid.shape, "out")
    ws = ws or Workspace(mu.device)
    if max_pairs is None:
        max_pairs = dgr_voxelize_plan(mu, scale, quat, grid, k_sigma, box_half, ws)
    p, sz = ws.ptr_size(dgr_voxelize_workspace(n, max_pairs, grid))
    g, t = c_grid(grid), c_trunc(k_sigma, box_half)
    _check("dgr_voxelize", lib().dgr_voxelize(
        _ptr(mu), _ptr(scale), _ptr(quat), _ptr(density), n, ctypes.byref(g), ctypes.byref(t),
        _ptr(out), p, sz, _stream()))
    return out


def dgr_voxelize_backward(mu, scale, quat, density, dvolume, grid: GridSpec, k_sigma=3.0,
                          box_half=8, ws: Workspace | None = None, outs=None):
    n = mu.shape[0]
    _need(dvolume, torch.float32, grid.shape, "dvolume")
    if outs is None:
        outs = (torch.empty_like(mu), torch.empty_like(scale), torch.empty_like(quat),
                torch.empty_like(density))
    ws = ws or Workspace(mu.device)
    p, sz = ws.ptr_size(int(lib().dgr_voxelize_backward_workspace(n)))
    g, t = c_grid(grid), c_trunc(k_sigma, box_half)
    _check("dgr_voxelize_backward", lib().dgr_voxelize_backward(
        _ptr(mu), _ptr(scale), _ptr(quat), _ptr(density), n, ctypes.byref(g), ctypes.byref(t),
        _ptr(dvolume), *(_ptr(o) for o in outs), p, sz, _stream()))
    return outs


def dgr_voxelize_backward_noalloc(mu, scale, quat, density, dvolume, grid: GridSpec, k_sigma=3.0,
                                  box_half=8, outs=None):
    """dgr_voxelize_backward with the per-Gaussian records in the library's
    fixed device array (no workspace)."""
    n = mu.shape[0]
    _need(dvolume, torch.float32, grid.shape, "dvolume")
    if outs is None:
        outs = (torch.empty_like(mu), torch.empty_like(scale), torch.empty_like(quat),
                torch.empty_like(density))
    g, t = c_grid(grid), c_trunc(k_sigma, box_half)
    _check("dgr_voxelize_backward_noalloc", lib().dgr_voxelize_backward_noalloc(
        _ptr(mu), _ptr(scale), _ptr(quat), _ptr(density), n, ctypes.byref(g), ctypes.byref(t),
        _ptr(dvolume), *(_ptr(o) for o in outs), _stream()))
    return outs


def dgr_project_workspace(grid: GridSpec, geom: Geometry, views_dev) -> int:
    g, G = c_grid(grid), c_geom(geom, views_dev)
    return int(lib().dgr_project_workspace(ctypes.byref(g), ctypes.byref(G)))


def dgr_project(volume, grid: GridSpec, geom: Geometry, views_dev, out=None,
                ws: Workspace | None = None):
    _need(volume, torch.float32, grid.shape, "volume")
    if out is None:
        out = torch.empty((geom.n_views, geom.nv, geom.nu), dtype=torch.float32, device=volume.device)
    _need(out, torch.float32, (geom.n_views, geom.nv, geom.nu), "out")
    ws = ws or Workspace(volume.device)
    g, G = c_grid(grid), c_geom(geom, views_dev)
    p, sz = ws.ptr_size(lib().dgr_project_workspace(ctypes.byref(g), ctypes.byref(G)))
    _check("dgr_project", lib().dgr_project(_ptr(volume), ctypes.byref(g), ctypes.byref(G),
                                            _ptr(out), p, sz, _stream()))
    return out


def dgr_project_l1(volume, target, grid: GridSpec, geom: Geometry, views_dev, loss=None,
                   dproj=None, ws: Workspace | None = None):
    shape = (geom.n_views, geom.nv, geom.nu)
    _need(volume, torch.float32, grid.shape, "volume")
    _need(target, torch.float32, shape, "target")
    if loss is None:
        loss = torch.empty((), dtype=torch.float32, device=volume.device)
    if dproj is None:
        dproj = torch.empty(shape, dtype=torch.float32, device=volume.device)
    ws = ws or Workspace(volume.device)
    g, G = c_grid(grid), c_geom(geom, views_dev)
    p, sz = ws.ptr_size(lib().dgr_project_workspace(ctypes.byref(g), ctypes.byref(G)))
    _check("dgr_project_l1", lib().dgr_project_l1(
        _ptr(volume), ctypes.byref(g), ctypes.byref(G), _ptr(target), _ptr(loss), _ptr(dproj), p, sz,
        _stream()))
    return loss, dproj


def dgr_backproject(proj, grid: GridSpec, geom: Geometry, views_dev, out=None,
                    ws: Workspace | None = None):
    _need(proj, torch.float32, (geom.n_views, geom.nv, geom.nu), "proj")
    if out is None:
        out = torch.empty(grid.shape, dtype=torch.float32, device=proj.device)
    _need(out, torch.float32, grid.shape, "out")
    ws = ws or Workspace(proj.device)
    g, G = c_grid(grid), c_geom(geom, views_dev)
    p, sz = ws.ptr_size(lib().dgr_project_workspace(ctypes.byref(g), ctypes.byref(G)))
    _check("dgr_backproject", lib().dgr_backproject(_ptr(proj), ctypes.byref(g), ctypes.byref(G),
                                                    _ptr(out), p, sz, _stream()))
    return out


def dgr_backproject_weight_bound(grid: GridSpec, geom: Geometry, views_dev):
    """Per-view weight bound of the backprojection's fixed-point tile, float32 [n_views]."""
    out = torch.empty(geom.n_views, dtype=torch.float32, device=views_dev.device)
    g, G = c_grid(grid), c_geom(geom, views_dev)
    _check("dgr_backproject_weight_bound",
           lib().dgr_backproject_weight_bound(ctypes.byref(g), ctypes.byref(G), _ptr(out), _stream()))
    return out


def dgr_project_siddon(volume, grid: GridSpec, geom: Geometry, views_dev, out=None):
    """Exact-path (Siddon) projection, float32 [n_views, nv, nu]."""
    _need(volume, torch.float32, grid.shape, "volume")
    if out is None:
        out = torch.empty((geom.n_views, geom.nv, geom.nu), dtype=torch.float32, device=volume.device)
    _need(out, torch.float32, (geom.n_views, geom.nv, geom.nu), "out")
    g, G = c_grid(grid), c_geom(geom, views_dev)
    _check("dgr_project_siddon", lib().dgr_project_siddon(_ptr(volume), ctypes.byref(g), ctypes.byref(G),
                                                          _ptr(out), _stream()))
    return out


def dgr_backproject_siddon(proj, grid: GridSpec, geom: Geometry, views_dev, out=None,
                           ws: Workspace | None = None):
    """Transpose of dgr_project_siddon, float32 volume [nz, ny, nx]."""
    _need(proj, torch.float32, (geom.n_views, geom.nv, geom.nu), "proj")
    if out is None:
        out = torch.empty(grid.shape, dtype=torch.float32, device=proj.device)
    _need(out, torch.float32, grid.shape, "out")
    ws = ws or Workspace(proj.device)
    g, G = c_grid(grid), c_geom(geom, views_dev)
    p, sz = ws.ptr_size(lib().dgr_backproject_siddon_workspace(ctypes.byref(g)))
    _check("dgr_backproject_siddon", lib().dgr_backproject_siddon(_ptr(proj), ctypes.byref(g), ctypes.byref(G),
                                                                  _ptr(out), p, sz, _stream()))
    return out


def dgr_adam(param, grad, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8, lower=float("-inf")):
    for name, t in (("param", param), ("grad", grad), ("m", m), ("v", v)):
        _need(t, torch.float32, param.shape, name)
    _check("dgr_adam", lib().dgr_adam(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(),
                                       float(lr), float(b1), float(b2), float(eps), int(step),
                                       float(lower), _stream()))


def dgr_bbox(mu, scale, quat, grid: GridSpec, k_sigma=3.0, box_half=8):
    n = mu.shape[0]
    box = torch.empty((n, 6), dtype=torch.int32, device=mu.device)
    g, t = c_grid(grid), c_trunc(k_sigma, box_half)
    _check("dgr_bbox", lib().dgr_bbox(_ptr(mu), _ptr(scale), _ptr(quat), n, ctypes.byref(g),
                                      ctypes.byref(t), _ptr(box), _stream()))
    return box


def dgr_bin(mu, scale, quat, grid: GridSpec, k_sigma=3.0, box_half=8):
    n = mu.shape[0]
    ws = Workspace(mu.device)
    P = dgr_voxelize_plan(mu, scale, quat, grid, k_sigma, box_half, ws)
    T = 1
    for d in grid.dims:
        T *= (d + 7) // 8
    pairs = torch.empty((max(P, 1), 2), dtype=torch.int32, device=mu.device)
    tb = torch.empty(T + 1, dtype=torch.int32, device=mu.device)
    p, sz = ws.ptr_size(dgr_voxelize_workspace(n, P, grid))
    g, t = c_grid(grid), c_trunc(k_sigma, box_half)
    _check("dgr_bin", lib().dgr_bin(_ptr(mu), _ptr(scale), _ptr(quat), n, ctypes.byref(g),
                                    ctypes.byref(t), _ptr(pairs), _ptr(tb), p, sz, _stream()))
    return pairs[:P], tb


def dgr_check(ws: Workspace):
    p, _ = ws.ptr_size(256)
    _check("dgr_check", lib().dgr_check(p, _stream()))


def dgr_voxelize_f64(mu, scale, quat, density, grid: GridSpec, k_sigma=3.0, box_half=8,
                     ws: Workspace | None = None):
    n = mu.shape[0]
    out = torch.empty(grid.shape, dtype=torch.float64, device=mu.device)
    ws = ws or Workspace(mu.device)
    P = dgr_voxelize_plan(mu, scale, quat, grid, k_sigma, box_half, ws)
    g, t = c_grid(grid), c_trunc(k_sigma, box_half)
    p, sz = ws.ptr_size(int(lib().dgr_voxelize_f64_workspace(n, P, ctypes.byref(g))))
    _check("dgr_voxelize_f64", lib().dgr_voxelize_f64(
        _ptr(mu), _ptr(scale), _ptr(quat), _ptr(density), n, ctypes.byref(g), ctypes.byref(t),
        _ptr(out), p, sz, _stream()))
    return out


def dgr_fd_l1_f64(volume64, target, mu, scale, quat, density, grid: GridSpec, geom: Geometry,
                  views_dev, jobs, box_cap=1 << 16, k_sigma=3.0, box_half=8):
    """jobs: list of (gid, component, h).  Returns float64 [n_jobs, 2] of loss
    changes (L(+h) - L, L(-h) - L)."""
    import numpy as np
    n = mu.shape[0]
    nj = len(jobs)
    gid = np.ascontiguousarray([j[0] for j in jobs], np.int32)
    comp = np.ascontiguousarray([j[1] for j in jobs], np.int32)
    hh = np.ascontiguousarray([j[2] for j in jobs], np.float64)
    out = torch.empty((nj, 2), dtype=torch.float64, device=mu.device)
    g, t, G = c_grid(grid), c_trunc(k_sigma, box_half), c_geom(geom, views_dev)
    ws = Workspace(mu.device)
    p, sz = ws.ptr_size(int(lib().dgr_fd_l1_f64_workspace(n, nj, int(box_cap), ctypes.byref(G))))
    _check("dgr_fd_l1_f64", lib().dgr_fd_l1_f64(
        _ptr(volume64), ctypes.byref(g), ctypes.byref(G), _ptr(target), _ptr(mu), _ptr(scale),
        _ptr(quat), _ptr(density), n, ctypes.byref(t), gid.ctypes.data_as(ctypes.c_void_p),
        comp.ctypes.data_as(ctypes.c_void_p), hh.ctypes.data_as(ctypes.c_void_p), nj, int(box_cap),
        _ptr(out), p, sz, _stream()))
    return out


def dgr_fdk(proj, grid: GridSpec, geom: Geometry, views_dev, arc=2 * 3.141592653589793, out=None,
            ws: Workspace | None = None):
    _need(proj, torch.float32, (geom.n_views, geom.nv, geom.nu), "proj")
    if out is None:
        out = torch.empty(grid.shape, dtype=torch.float32, device=proj.device)
    g, G = c_grid(grid), c_geom(geom, views_dev)
    ws = ws or Workspace(proj.device)
    p, sz = ws.ptr_size(int(lib().dgr_fdk_workspace(ctypes.byref(g), ctypes.byref(G))))
    _check("dgr_fdk", lib().dgr_fdk(_ptr(proj), ctypes.byref(g), ctypes.byref(G), float(arc),
                                    _ptr(out), p, sz, _stream()))
    return out


def dgr_psnr(x, gt, out=None, ws: Workspace | None = None):
    """Device tensor float64 [3] = (psnr, mse, max)."""
    _need(x, torch.float32, None, "x")
    _need(gt, torch.float32, tuple(x.shape), "gt")
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=x.device)
    ws = ws or Workspace(x.device)
    p, sz = ws.ptr_size(int(lib().dgr_reduce_workspace()))
    _check("dgr_psnr", lib().dgr_psnr(_ptr(x), _ptr(gt), x.numel(), _ptr(out), p, sz, _stream()))
    return out


def dgr_init_from_volume(volume, grid: GridSpec, n, uniforms, scale, thresh_frac=0.1,
                         ws: Workspace | None = None):
    _need(volume, torch.float32, grid.shape, "volume")
    _need(uniforms, torch.float32, (n, 4), "uniforms")
    dev = volume.device
    mu = torch.empty((n, 3), dtype=torch.float32, device=dev)
    sc = torch.empty((n, 3), dtype=torch.float32, device=dev)
    q = torch.empty((n, 4), dtype=torch.float32, device=dev)
    rho = torch.empty(n, dtype=torch.float32, device=dev)
    g = c_grid(grid)
    ws = ws or Workspace(dev)
    p, sz = ws.ptr_size(int(lib().dgr_init_workspace(ctypes.byref(g))))
    _check("dgr_init_from_volume", lib().dgr_init_from_volume(
        _ptr(volume), ctypes.byref(g), float(thresh_frac), int(n), _ptr(uniforms), float(scale),
        _ptr(mu), _ptr(sc), _ptr(q), _ptr(rho), p, sz, _stream()))
    return mu, sc, q, rho


def dgr_fit_density_scale(p1, target, density, kappa=None, ws: Workspace | None = None):
    _need(p1, torch.float32, None, "p1")
    _need(target, torch.float32, tuple(p1.shape), "target")
    ws = ws or Workspace(p1.device)
    if kappa is None:
        kappa = torch.empty(1, dtype=torch.float64, device=p1.device)
    p, sz = ws.ptr_size(int(lib().dgr_reduce_workspace()))
    _check("dgr_fit_density_scale", lib().dgr_fit_density_scale(
        _ptr(p1), _ptr(target), p1.numel(), _ptr(density), density.numel(), _ptr(kappa), p, sz,
        _stream()))
    return kappa


# ---- learned initialisation (U-Net) -----------------------------------------------
UNET_BASE = 32


def _dims(shape3):
    """Volume shape (nz, ny, nx) -> C dims {nx, ny, nz}."""
    nz, ny, nx = (int(v) for v in shape3)
    return (ctypes.c_int32 * 3)(nx, ny, nz)


def dgr_unet_param_count(base=UNET_BASE) -> int:
    n = int(lib().dgr_unet_param_count(base))
    if n < 0:
        raise ValueError(f"unsupported U-Net base width {base}")
    return n


def dgr_unet_forward(params, x, out=None, ws: Workspace | None = None, base=UNET_BASE):
    """x float32 [nz, ny, nx] -> out float32 [nz, ny, nx, 3]; ws keeps the
    activations for dgr_unet_backward."""
    _need(params, torch.float32, (dgr_unet_param_count(base),), "params")
    _need(x, torch.float32, None, "x")
    if out is None:
        out = torch.empty(tuple(x.shape) + (3,), dtype=torch.float32, device=x.device)
    _need(out, torch.float32, tuple(x.shape) + (3,), "out")
    dims = _dims(x.shape)
    need = int(lib().dgr_unet_workspace(dims, base))
    if need == 0:
        raise ValueError(f"unsupported U-Net volume shape {tuple(x.shape)}")
    ws = ws or Workspace(x.device)
    p, sz = ws.ptr_size(need)
    _check("dgr_unet_forward", lib().dgr_unet_forward(_ptr(params), _ptr(x), dims, base, _ptr(out), p,
                                                      sz, _stream()))
    return out


def dgr_unet_backward(params, x, dout, ws: Workspace, grad=None, base=UNET_BASE):
    _need(dout, torch.float32, tuple(x.shape) + (3,), "dout")
    if grad is None:
        grad = torch.empty_like(params)
    _need(grad, torch.float32, tuple(params.shape), "grad")
    dims = _dims(x.shape)
    p, sz = ws.ptr_size(int(lib().dgr_unet_workspace(dims, base)))
    _check("dgr_unet_backward", lib().dgr_unet_backward(_ptr(params), _ptr(x), dims, base, _ptr(dout),
                                                        _ptr(grad), p, sz, _stream()))
    return grad


def dgr_unet_loss(out, target, loss=None, dout=None, ws: Workspace | None = None):
    _need(out, torch.float32, None, "out")
    _need(target, torch.float32, tuple(out.shape), "target")
    if loss is None:
        loss = torch.empty((), dtype=torch.float32, device=out.device)
    if dout is None:
        dout = torch.empty_like(out)
    ws = ws or Workspace(out.device)
    p, sz = ws.ptr_size(int(lib().dgr_unet_loss_workspace()))
    _check("dgr_unet_loss", lib().dgr_unet_loss(_ptr(out), _ptr(target), out.numel() // 3, _ptr(loss),
                                                _ptr(dout), p, sz, _stream()))
    return loss, dout


def dgr_conv3_forward(x, cin, w, bias, cout, relu=True, y=None, y_stride=None):
    """x bfloat16 [nz, ny, nx, x_stride]; w bfloat16 [27, cout, cin]."""
    _need(x, torch.bfloat16, None, "x")
    _need(w, torch.bfloat16, (27, cout, cin), "w")
    if bias is not None:
        _need(bias, torch.float32, (cout,), "bias")
    ys = y_stride or cout
    if y is None:
        y = torch.zeros(tuple(x.shape[:3]) + (ys,), dtype=torch.bfloat16, device=x.device)
    _check("dgr_conv3_forward", lib().dgr_conv3_forward(_ptr(x), x.shape[3], _dims(x.shape[:3]), cin,
                                                        _ptr(w), _ptr(bias), cout, int(relu), _ptr(y),
                                                        y.shape[3], _stream()))
    return y


def dgr_conv3_backward(x, cin, w, dy, ws: Workspace | None = None):
    """-> (dw float32 [27, cout, cin], db float32 [cout], dx bfloat16 [..., cin])."""
    _need(x, torch.bfloat16, None, "x")
    cout = w.shape[1]
    _need(w, torch.float32, (27, cout, cin), "w")
    _need(dy, torch.bfloat16, tuple(x.shape[:3]) + (cout,), "dy")
    dev = x.device
    dw = torch.empty((27, cout, cin), dtype=torch.float32, device=dev)
    db = torch.empty(cout, dtype=torch.float32, device=dev)
    dx = torch.empty(tuple(x.shape[:3]) + (cin,), dtype=torch.bfloat16, device=dev)
    dims = _dims(x.shape[:3])
    ws = ws or Workspace(dev)
    p, sz = ws.ptr_size(int(lib().dgr_conv3_grad_workspace(dims, cin, cout)))
    _check("dgr_conv3_backward", lib().dgr_conv3_backward(_ptr(x), x.shape[3], dims, cin, _ptr(w), _ptr(dy),
                                                          cout, _ptr(dw), _ptr(db), _ptr(dx), p, sz,
                                                          _stream()))
    return dw, db, dx


def dgr_pool2_f32(x, out=None):
    """x float32 [nz, ny, nx] (even) -> [nz/2, ny/2, nx/2] block means."""
    _need(x, torch.float32, None, "x")
    shp = tuple(v // 2 for v in x.shape)
    if out is None:
        out = torch.empty(shp, dtype=torch.float32, device=x.device)
    _need(out, torch.float32, shp, "out")
    _check("dgr_pool2_f32", lib().dgr_pool2_f32(_ptr(x), _dims(x.shape), _ptr(out), _stream()))
    return out


def dgr_unet_targets(mu, scale, grid: GridSpec, volume, input_scale, target=None, ws=None):
    _need(volume, torch.float32, grid.shape, "volume")
    if target is None:
        target = torch.empty(tuple(grid.shape) + (3,), dtype=torch.float32, device=volume.device)
    g = c_grid(grid)
    ws = ws or Workspace(volume.device)
    p, sz = ws.ptr_size(int(lib().dgr_unet_targets_workspace(ctypes.byref(g))))
    _check("dgr_unet_targets", lib().dgr_unet_targets(_ptr(mu), _ptr(scale), mu.shape[0], ctypes.byref(g),
                                                      _ptr(volume), float(input_scale), _ptr(target), p,
                                                      sz, _stream()))
    return target


def dgr_init_from_unet(out, grid: GridSpec, n, uniforms, input_scale, ws=None):
    _need(out, torch.float32, tuple(grid.shape) + (3,), "out")
    _need(uniforms, torch.float32, (n, 4), "uniforms")
    dev = out.device
    mu = torch.empty((n, 3), dtype=torch.float32, device=dev)
    sc = torch.empty((n, 3), dtype=torch.float32, device=dev)
    q = torch.empty((n, 4), dtype=torch.float32, device=dev)
    rho = torch.empty(n, dtype=torch.float32, device=dev)
    g = c_grid(grid)
    ws = ws or Workspace(dev)
    p, sz = ws.ptr_size(int(lib().dgr_init_from_unet_workspace(ctypes.byref(g))))
    _check("dgr_init_from_unet", lib().dgr_init_from_unet(_ptr(out), ctypes.byref(g), n, _ptr(uniforms),
                                                          float(input_scale), _ptr(mu), _ptr(sc), _ptr(q),
                                                          _ptr(rho), p, sz, _stream()))
    return mu, sc, q, rho


# ---- the paper's full objective ------------------------------------------------------
def dgr_projection_loss(proj, target, w_l1=0.6, w_ssim=0.2, range_=0.0, loss=None, dproj=None,
                        ws: Workspace | None = None):
    """-> (loss float32 [3] = (w1 L1 + w2 L_SSIM, L1, L_SSIM), dproj)."""
    _need(proj, torch.float32, None, "proj")
    _need(target, torch.float32, tuple(proj.shape), "target")
    V, nv, nu = (int(v) for v in proj.shape)
    if loss is None:
        loss = torch.empty(3, dtype=torch.float32, device=proj.device)
    if dproj is None:
        dproj = torch.empty_like(proj)
    ws = ws or Workspace(proj.device)
    p, sz = ws.ptr_size(int(lib().dgr_projection_loss_workspace(V, nv, nu)))
    _check("dgr_projection_loss", lib().dgr_projection_loss(_ptr(proj), _ptr(target), V, nv, nu, float(w_l1),
                                                            float(w_ssim), float(range_), _ptr(loss),
                                                            _ptr(dproj), p, sz, _stream()))
    return loss, dproj


def dgr_tv(volume, grid: GridSpec, dvolume, w_tv=1.0, loss=None, ws: Workspace | None = None):
    """loss float32 [1] = L_TV; dvolume += w_tv dL_TV/dV (in place)."""
    _need(volume, torch.float32, grid.shape, "volume")
    _need(dvolume, torch.float32, grid.shape, "dvolume")
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=volume.device)
    g = c_grid(grid)
    ws = ws or Workspace(volume.device)
    p, sz = ws.ptr_size(int(lib().dgr_tv_workspace()))
    _check("dgr_tv", lib().dgr_tv(_ptr(volume), ctypes.byref(g), float(w_tv), _ptr(loss), _ptr(dvolume), p, sz,
                                  _stream()))
    return loss


# ---- adaptive density control ----------------------------------------------------------
GROUPS = ("mu", "scale", "quat", "density")
WIDTH = {"mu": 3, "scale": 3, "quat": 4, "density": 1}


def dgr_accumulate_grad_norm(dmu, acc):
    _need(dmu, torch.float32, None, "dmu")
    _need(acc, torch.float32, (dmu.shape[0],), "acc")
    _check("dgr_accumulate_grad_norm", lib().dgr_accumulate_grad_norm(_ptr(dmu), dmu.shape[0], _ptr(acc),
                                                                      _stream()))


def _gauss_struct(P, m, v):
    g = DgrGaussians()
    for k in GROUPS:
        setattr(g, k, P[k].data_ptr())
        setattr(g, "m_" + k, m[k].data_ptr())
        setattr(g, "v_" + k, v[k].data_ptr())
    return g


def dgr_densify(P, m, v, acc, normals, grid: GridSpec, dst, iters, tau, tau_prune, theta, size_vox, n_max,
                ws: Workspace | None = None):
    """One pass of Alg. 2.  P, m, v: dicts of the current Gaussians and Adam
    moments (n rows); dst: (P', m', v') dicts with at least n_max rows.
    Returns (new n, (cloned, split, pruned)) (synchronising)."""
    n = P["mu"].shape[0]
    for k in GROUPS:
        shp = (n,) if k == "density" else (n, WIDTH[k])
        for name, t in (("P", P[k]), ("m", m[k]), ("v", v[k])):
            _need(t, torch.float32, shp, f"{name}[{k}]")
        for t in dst:
            if not (t[k].is_cuda and t[k].is_contiguous() and t[k].shape[0] >= n_max):
                raise ValueError(f"destination {k} must hold n_max rows")
    _need(acc, torch.float32, (n,), "acc")
    _need(normals, torch.float32, (n, 2, 3), "normals")
    src = _gauss_struct(P, m, v)
    d = _gauss_struct(*dst)
    prm = DgrDensifyParams(int(iters), float(tau), float(tau_prune), float(theta), float(size_vox), int(n_max))
    g = c_grid(grid)
    n_out = ctypes.c_int64(0)
    counts = (ctypes.c_int64 * 3)()
    ws = ws or Workspace(acc.device)
    p, sz = ws.ptr_size(int(lib().dgr_densify_workspace(n)))
    _check("dgr_densify", lib().dgr_densify(ctypes.byref(src), n, _ptr(acc), _ptr(normals), ctypes.byref(g),
                                            ctypes.byref(prm), ctypes.byref(d), ctypes.byref(n_out), counts, p,
                                            sz, _stream()))
    return int(n_out.value), (int(counts[0]), int(counts[1]), int(counts[2]))
