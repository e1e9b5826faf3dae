"""Parity of the exact-path (Siddon) projector and its transpose with the
binary64 oracle, through the C ABI: parallel, cone and fan beams on a ragged
grid, rays lying on cell planes, the adjoint identity, and the 256^3 cone
workload on sampled views."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2411_04844_amd import inputs, native

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(got, want):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300))


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dtype)


GRID = inputs.GridSpec((37, 29, 21), (-1.15625, -0.90625, -0.65625), (16.0, 16.0, 16.0))


def _geom(kind):
    if kind == "parallel":
        return inputs.parallel_geometry(7, 41, 27, 0.06, 0.05)
    if kind == "cone":
        return inputs.cone_geometry(6, 45, 31, 0.07, 4.0, 6.0, 0.05, arc=2.0, length_scale=3.0)
    return inputs.fan_geometry(6, 45, 21, 0.07, 1.0 / 16, 4.0, 6.0, 0.05, arc=math.pi / 2, length_scale=3.0)


@pytest.mark.parametrize("kind", ["parallel", "cone", "fan"])
def test_siddon_project_and_transpose_parity(kind):
    geom = _geom(kind)
    say("siddon", kind)
    rng = np.random.default_rng(400)
    V = rng.uniform(size=GRID.shape).astype(np.float32)
    views = dev(geom.views)
    got = native.dgr_project_siddon(dev(V), GRID, geom, views).cpu().numpy()
    want = oracle.project_siddon(V.astype(np.float64), GRID.dims, GRID.lo, GRID.inv_h, geom.kind,
                                 geom.views, geom.nu, geom.nv, geom.length_scale)
    assert np.count_nonzero(want) > 0.5 * want.size and np.count_nonzero(want) < want.size
    err = rel_l2(got, want)
    say("siddon project", kind, "rel_l2", err)
    assert err < TOL
    assert np.all(got[want == 0] == 0.0)
    g = rng.normal(size=want.shape).astype(np.float32)
    gotb = native.dgr_backproject_siddon(dev(g), GRID, geom, views).cpu().numpy()
    wantb = oracle.backproject_siddon(g.astype(np.float64), GRID.dims, GRID.lo, GRID.inv_h, geom.kind,
                                      geom.views, geom.nu, geom.nv, geom.length_scale)
    errb = rel_l2(gotb, wantb)
    say("siddon backproject", kind, "rel_l2", errb)
    assert errb < TOL
    lhs = float(np.sum(got.astype(np.float64) * g))
    rhs = float(np.sum(V.astype(np.float64) * gotb))
    assert abs(lhs - rhs) <= TOL * np.linalg.norm(got) * np.linalg.norm(g)


def test_siddon_rays_on_cell_planes():
    """Parallel rays along x lying exactly on y and z cell planes (odd
    detector, pitch = voxel size): both sides give each segment to the cell
    above the plane."""
    say("siddon planes")
    grid = inputs.GridSpec((12, 8, 8), (-0.75, -0.5, -0.5), (8.0, 8.0, 8.0))
    geom = inputs.parallel_geometry(1, 9, 9, 0.125, 0.05)
    V = np.random.default_rng(401).uniform(size=grid.shape).astype(np.float32)
    got = native.dgr_project_siddon(dev(V), grid, geom, dev(geom.views)).cpu().numpy()
    want = oracle.project_siddon(V.astype(np.float64), grid.dims, grid.lo, grid.inv_h, geom.kind,
                                 geom.views, geom.nu, geom.nv, geom.length_scale)
    assert rel_l2(got, want) < TOL
    # interior rays on planes: the sum of the cells above the planes in y and z
    h = 0.125
    for iv in range(1, 8):
        for iu in range(1, 8):
            k = (iv - 4) + 4  # z cell index above the plane at z = (iv - 4) h
            jy = (iu - 4) + 4
            assert abs(float(got[0, iv, iu]) - h * float(V[k, jy, :].astype(np.float64).sum())) < 1e-5


def test_siddon_full_size_sampled_views():
    say("siddon full")
    grid = inputs.cube_grid(256)
    geom = inputs.cone_workload(256, 360, 512, 0.8)
    G = inputs.gaussians(100_000, 2001, 0.004, 0.03)
    d = {k: torch.as_tensor(v).cuda() for k, v in G.items()}
    V = native.dgr_voxelize(d["mu"], d["scale"], d["quat"], d["density"], grid)
    views = torch.as_tensor(geom.views).cuda()
    P = native.dgr_project_siddon(V, grid, geom, views).cpu().numpy()
    sel = [0, 137, 271]
    want = oracle.project_siddon(V.cpu().numpy().astype(np.float64), grid.dims, grid.lo, grid.inv_h,
                                 geom.kind, geom.views[sel], geom.nu, geom.nv, geom.length_scale)
    err = rel_l2(P[sel], want)
    say("siddon full project rel_l2 (3 views)", err)
    assert err < TOL


def test_siddon_full_size_transpose_sampled_views():
    say("siddon full transpose")
    grid = inputs.cube_grid(256)
    geom = inputs.cone_workload(256, 360, 512, 0.8)
    sel = [11, 190, 333]
    g = np.zeros((geom.n_views, geom.nv, geom.nu), np.float32)
    g[sel] = np.random.default_rng(402).normal(size=(len(sel), geom.nv, geom.nu))
    views = torch.as_tensor(geom.views).cuda()
    got = native.dgr_backproject_siddon(torch.as_tensor(g).cuda(), grid, geom, views).cpu().numpy()
    want = oracle.backproject_siddon(g[sel].astype(np.float64), grid.dims, grid.lo, grid.inv_h, geom.kind,
                                     geom.views[sel], geom.nu, geom.nv, geom.length_scale)
    err = rel_l2(got, want)
    say("siddon full transpose rel_l2 (3 views)", err)
    assert err < TOL
