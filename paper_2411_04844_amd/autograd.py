"""torch.autograd.Function wrappers around the C ABI.

``DGRVoxelize``: forward ``dgr_voxelize``, backward ``dgr_voxelize_backward``
(the hand-written chain rule for mean, scale, quaternion and density; boxes
held fixed).  ``DGRProject``: forward ``dgr_project``, backward
``dgr_backproject`` (its exact transpose).  Neither keeps the volume alive for
the backward pass: the projector is linear and the voxelizer backward needs
only the parameters and dL/dV, so a 512^3 volume is never stored between the
two passes.
"""
from __future__ import annotations

import torch

from . import native
from .inputs import Geometry, GridSpec


class DGRVoxelize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu, scale, quat, density, grid: GridSpec, k_sigma: float = 3.0,
                box_half: int = 8, ws: native.Workspace | None = None):
        mu, scale, quat, density = (t.contiguous() for t in (mu, scale, quat, density))
        V = native.dgr_voxelize(mu, scale, quat, density, grid, k_sigma, box_half, ws=ws)
        ctx.save_for_backward(mu, scale, quat, density)
        ctx.cfg = (grid, k_sigma, box_half)
        return V

    @staticmethod
    def backward(ctx, dV):
        mu, scale, quat, density = ctx.saved_tensors
        grid, k_sigma, box_half = ctx.cfg
        dmu, ds, dq, dr = native.dgr_voxelize_backward(mu, scale, quat, density, dV.contiguous(),
                                                       grid, k_sigma, box_half)
        return dmu, ds, dq, dr, None, None, None, None


class DGRProject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, volume, grid: GridSpec, geom: Geometry, views: torch.Tensor,
                ws: native.Workspace | None = None):
        ctx.cfg = (grid, geom, views)
        return native.dgr_project(volume.contiguous(), grid, geom, views, ws=ws)

    @staticmethod
    def backward(ctx, dP):
        grid, geom, views = ctx.cfg
        return native.dgr_backproject(dP.contiguous(), grid, geom, views), None, None, None, None


def voxelize(mu, scale, quat, density, grid, k_sigma=3.0, box_half=8, ws=None):
    return DGRVoxelize.apply(mu, scale, quat, density, grid, k_sigma, box_half, ws)


def project(volume, grid, geom, views, ws=None):
    return DGRProject.apply(volume, grid, geom, views, ws)
