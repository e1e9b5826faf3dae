"""Parity of the HIP path (through the C ABI) with the binary64 oracle.

Integer outputs (boxes, tile pairs) must match bit for bit; binary32
volumes, projections and gradients must lie within 1e-5 relative L2 of the
oracle given the same inputs (each operator is fed the same upstream data,
promoted exactly to binary64 on the oracle side).
"""
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


def gauss_dev(G):
    return dev(G["mu"]), dev(G["scale"]), dev(G["quat"]), dev(G["density"])


GRIDS = {
    "64cube": inputs.cube_grid(64),
    "ragged": inputs.GridSpec((37, 29, 21), (-1.15625, -0.90625, -0.65625), (16.0, 16.0, 16.0)),
}


def small_gaussians(n=2000, seed=1001):
    return inputs.gaussians(n, seed, 0.01, 0.05)


# --------------------------------------------------------------------------
# boxes and tile pairs: bit-exact
# --------------------------------------------------------------------------
@pytest.mark.parametrize("gname", list(GRIDS))
def test_bbox_bit_exact(gname):
    grid = GRIDS[gname]
    say("bbox", gname)
    G = inputs.gaussians(20000, 77, 0.002, 0.3, mean_lim=1.3)
    G["quat"][:10] = 0.0  # identity rotation
    for k_sigma, bh in ((3.0, 8), (0.0, 8), (0.0, 0), (5.5, 8)):
        got = native.dgr_bbox(*gauss_dev(G)[:3], grid, k_sigma, bh).cpu().numpy()
        want = oracle.bbox(G["mu"], G["scale"], G["quat"], grid.dims, grid.lo, grid.inv_h, k_sigma, bh)
        assert np.array_equal(got, want), (k_sigma, np.argwhere(got != want)[:5])


@pytest.mark.parametrize("gname", list(GRIDS))
def test_tile_pairs_bit_exact(gname):
    grid = GRIDS[gname]
    say("bin", gname)
    G = inputs.gaussians(3000, 78, 0.005, 0.12, mean_lim=1.1)
    pairs, tb = native.dgr_bin(*gauss_dev(G)[:3], grid)
    box = oracle.bbox(G["mu"], G["scale"], G["quat"], grid.dims, grid.lo, grid.inv_h)
    wp, wtb = oracle.tile_pairs(box, grid.dims)
    assert np.array_equal(pairs.cpu().numpy().astype(np.uint32), wp)
    assert np.array_equal(tb.cpu().numpy().astype(np.int64), wtb)


def test_tile_pairs_many_sort_passes():
    """A grid with more than 2^16 tiles needs three radix passes."""
    grid = inputs.GridSpec((2080, 2080, 8), (-1.0, -1.0, -4.0 / 1040), (1040.0, 1040.0, 1040.0))
    say("bin 3-pass")
    G = inputs.gaussians(6000, 79, 0.002, 0.004, mean_lim=0.95)
    G["mu"][:, 2] *= 0.003
    pairs, tb = native.dgr_bin(*gauss_dev(G)[:3], grid)
    box = oracle.bbox(G["mu"], G["scale"], G["quat"], grid.dims, grid.lo, grid.inv_h)
    wp, wtb = oracle.tile_pairs(box, grid.dims)
    assert wp[:, 0].max() >= 65536
    assert np.array_equal(pairs.cpu().numpy().astype(np.uint32), wp)
    assert np.array_equal(tb.cpu().numpy().astype(np.int64), wtb)


# --------------------------------------------------------------------------
# voxelization
# --------------------------------------------------------------------------
def _vox_pair(G, grid, k_sigma=3.0, bh=8):
    got = native.dgr_voxelize(*gauss_dev(G), grid, k_sigma, bh).cpu().numpy()
    box = oracle.bbox(G["mu"], G["scale"], G["quat"], grid.dims, grid.lo, grid.inv_h, k_sigma, bh)
    want = oracle.voxelize(G["mu"], G["scale"], G["quat"], G["density"], grid.dims, grid.lo,
                           grid.inv_h, box)
    return got, want


def test_voxelize_64cube_2000_brute_force():
    grid = inputs.cube_grid(64)
    say("voxelize 64^3 / 2000")
    G = small_gaussians()
    got = native.dgr_voxelize(*gauss_dev(G), grid).cpu().numpy()
    box = oracle.bbox(G["mu"], G["scale"], G["quat"], grid.dims, grid.lo, grid.inv_h)
    want = oracle.voxelize(G["mu"], G["scale"], G["quat"], G["density"], grid.dims, grid.lo,
                           grid.inv_h, box, brute=True)
    say("voxelize 64^3 / 2000 rel_l2", rel_l2(got, want))
    assert rel_l2(got, want) < TOL


@pytest.mark.parametrize("case", ["ragged", "fixed_box", "large_sigma", "outside"])
def test_voxelize_cases(case):
    say("voxelize", case)
    grid = GRIDS["ragged"]
    k_sigma, bh = 3.0, 8
    if case == "ragged":
        G = inputs.gaussians(1500, 80, 0.01, 0.08, mean_lim=1.0)
    elif case == "fixed_box":
        G = inputs.gaussians(800, 81, 0.02, 0.1)
        k_sigma, bh = 0.0, 4
    elif case == "large_sigma":  # boxes spanning many tiles, more than 256 per tile
        G = inputs.gaussians(700, 82, 0.1, 0.4)
    else:  # everything outside the grid: an all-zero volume
        G = inputs.gaussians(100, 83, 0.01, 0.02)
        G["mu"] += 5.0
    got, want = _vox_pair(G, grid, k_sigma, bh)
    if case == "outside":
        assert np.all(got == 0.0)
    else:
        assert rel_l2(got, want) < TOL


def test_voxelize_empty_and_single():
    grid = GRIDS["ragged"]
    say("voxelize empty/single")
    G = inputs.gaussians(0, 84, 0.01, 0.02)
    got = native.dgr_voxelize(*gauss_dev(G), grid).cpu().numpy()
    assert got.shape == grid.shape and np.all(got == 0.0)
    G = inputs.gaussians(1, 85, 0.05, 0.06, mean_lim=0.1)
    got, want = _vox_pair(G, grid)
    assert rel_l2(got, want) < TOL


def test_voxelize_deterministic_and_capacity_error():
    grid = inputs.cube_grid(64)
    say("voxelize determinism")
    G = small_gaussians()
    a = native.dgr_voxelize(*gauss_dev(G), grid)
    b = native.dgr_voxelize(*gauss_dev(G), grid)
    assert torch.equal(a, b)
    ws = native.Workspace()
    P = native.dgr_voxelize_plan(*gauss_dev(G)[:3], grid, ws=ws)
    out = native.dgr_voxelize(*gauss_dev(G), grid, ws=ws, max_pairs=P // 2)
    with pytest.raises(native.DgrError) as e:
        native.dgr_check(ws)
    assert e.value.status == 3
    assert torch.isnan(out).all()
    native.dgr_check(ws)  # flag cleared


# --------------------------------------------------------------------------
# projection, L1, backprojection
# --------------------------------------------------------------------------
def small_parallel_geometry():
    h = 2.0 / 64
    return inputs.parallel_geometry(50, 64, 64, h, h / 2)


def _rand_volume(grid, seed):
    G = inputs.gaussians(600, seed, 0.03, 0.12)
    return oracle.voxelize(G["mu"], G["scale"], G["quat"], G["density"], grid.dims, grid.lo,
                           grid.inv_h, oracle.bbox(G["mu"], G["scale"], G["quat"], grid.dims,
                                                   grid.lo, grid.inv_h)).astype(np.float32)


def _geoms():
    grid_p = inputs.cube_grid(64)
    grid_c = inputs.GridSpec((48, 44, 40), (-1.0, -1.0 * 44 / 48, -1.0 * 40 / 48), (24.0, 24.0, 24.0))
    cone = inputs.cone_geometry(10, 70, 45, 0.02, 7.8125, 11.71875, 1.0 / 48, arc=2 * math.pi)
    cone_coarse = inputs.cone_geometry(10, 40, 30, 0.04, 7.8125, 11.71875, 1.0 / 48, arc=2 * math.pi)
    # parallel rays 35 degrees out of the detector's normal (a tilted beam)
    par = small_parallel_geometry()
    v = par.views.astype(np.float64).copy()
    b = math.radians(35.0)
    v[:, 0:3] = np.stack([v[:, 0] * math.cos(b), v[:, 1] * math.cos(b), np.full(len(v), math.sin(b))], axis=1)
    oblique = inputs.Geometry(0, v.astype(np.float32), par.nu, par.nv, par.step, par.length_scale)
    return {"parallel": (grid_p, small_parallel_geometry()), "cone": (grid_c, cone),
            "cone_coarse": (grid_c, cone_coarse), "parallel_oblique": (grid_p, oblique)}


# Tile format of the brickwise backprojection per geometry: the per-view weight
# bound (rays through the eight cells around a tile point times one ray's
# largest weight sum there) is about 71 for "parallel", 112 for
# "parallel_oblique" (the rays' 1/cos widens their footprint) and 219 for
# "cone_coarse" (packed 32-bit halves), 875 for "cone" (pixels twice as fine:
# the exact 64-bit tile; the packed format needs a bound of at most 512).
BACKPROJECT_KINDS = ["parallel", "parallel_oblique", "cone", "cone_coarse"]


@pytest.mark.parametrize("kind", ["parallel", "cone"])
def test_project_parity(kind):
    grid, geom = _geoms()[kind]
    say("project", kind)
    V = _rand_volume(grid, 90)
    views = dev(geom.views)
    got = native.dgr_project(dev(V), grid, geom, views).cpu().numpy()
    want = oracle.project(V.astype(np.float64), grid.dims, grid.lo, grid.inv_h, geom.kind, geom.views,
                          geom.nu, geom.nv, geom.step, geom.length_scale)
    assert np.count_nonzero(want) > 0.2 * want.size
    say("project", kind, "rel_l2", rel_l2(got, want))
    assert rel_l2(got, want) < TOL


@pytest.mark.parametrize("kind", ["parallel", "cone"])
def test_project_l1_parity(kind):
    grid, geom = _geoms()[kind]
    say("project_l1", kind)
    V = _rand_volume(grid, 91)
    want_p = oracle.project(V.astype(np.float64), grid.dims, grid.lo, grid.inv_h, geom.kind,
                            geom.views, geom.nu, geom.nv, geom.step, geom.length_scale)
    rng = np.random.default_rng(5)
    y = (want_p + rng.normal(scale=0.05 * want_p.max(), size=want_p.shape)).astype(np.float32)
    y.ravel()[:50] = want_p.ravel()[:50].astype(np.float32)  # near-zero residuals
    loss, g = native.dgr_project_l1(dev(V), dev(y), grid, geom, dev(geom.views))
    wl, wg = oracle.l1(want_p, y)
    assert abs(float(loss) - wl) / wl < TOL
    g = g.cpu().numpy()
    M = want_p.size
    assert set(np.unique(np.abs(g))) <= {np.float32(0.0), np.float32(1.0 / M)}
    r = np.abs(want_p - y.astype(np.float64))
    # signs may differ only where the residual is within the projection's error
    tol_r = 1e-5 * np.abs(want_p).max()
    mism = np.sign(g) != np.sign(wg)
    say("project_l1", kind, "loss rel err", abs(float(loss) - wl) / wl, "sign flips", int(mism.sum()))
    assert np.all(r[mism] < tol_r)
    assert mism.mean() < 2e-3


def _coarse_geoms():
    """Detectors whose pixels are about four voxels wide at the isocentre, so
    that a forward work-group's rays (16 x 16 pixels, 32 x 16 for cone beams)
    cover about 64 x 64 voxels: every chunk's box of cells (at least 10 x 66 x
    66) exceeds the LDS box and the taps come from the padded copy in HBM.
    Both detectors leave ragged tiles (24 = 16 + 8 columns, 40 = 32 + 8)."""
    grid_p = inputs.cube_grid(64)
    h = 2.0 / 64
    par = inputs.parallel_geometry(12, 24, 24, 4 * h, h / 2)
    grid_c = inputs.GridSpec((48, 44, 40), (-1.0, -1.0 * 44 / 48, -1.0 * 40 / 48), (24.0, 24.0, 24.0))
    cone = inputs.cone_geometry(8, 40, 20, 0.25, 7.8125, 11.71875, 1.0 / 48, arc=2 * math.pi)
    return {"parallel": (grid_p, par), "cone": (grid_c, cone)}


@pytest.mark.parametrize("kind", ["parallel", "cone"])
def test_project_parity_box_overflow(kind):
    grid, geom = _coarse_geoms()[kind]
    say("project box overflow", kind)
    V = _rand_volume(grid, 92)
    want = oracle.project(V.astype(np.float64), grid.dims, grid.lo, grid.inv_h, geom.kind, geom.views,
                          geom.nu, geom.nv, geom.step, geom.length_scale)
    assert np.count_nonzero(want) > 0.2 * want.size
    views = dev(geom.views)
    got = native.dgr_project(dev(V), grid, geom, views).cpu().numpy()
    say("project box overflow", kind, "rel_l2", rel_l2(got, want))
    assert rel_l2(got, want) < TOL
    y = np.random.default_rng(8).uniform(0, want.max(), size=want.shape).astype(np.float32)
    loss, g = native.dgr_project_l1(dev(V), dev(y), grid, geom, views)
    wl, wg = oracle.l1(want, y)
    assert abs(float(loss) - wl) / wl < TOL
    mism = np.sign(g.cpu().numpy()) != np.sign(wg)
    assert np.all(np.abs(want - y.astype(np.float64))[mism] < 1e-5 * np.abs(want).max())


@pytest.mark.parametrize("kind", BACKPROJECT_KINDS)
def test_backproject_parity_and_adjoint(kind):
    grid, geom = _geoms()[kind]
    say("backproject", kind)
    rng = np.random.default_rng(6)
    g = rng.normal(size=(geom.n_views, geom.nv, geom.nu)).astype(np.float32)
    views = dev(geom.views)
    got = native.dgr_backproject(dev(g), grid, geom, views).cpu().numpy()
    want = oracle.backproject(g.astype(np.float64), grid.dims, grid.lo, grid.inv_h, geom.kind,
                              geom.views, geom.nu, geom.nv, geom.step, geom.length_scale)
    worst = float(np.abs(got.astype(np.float64) - want).max() / np.abs(want).max())
    say("backproject", kind, "rel_l2", rel_l2(got, want), "worst voxel / max", worst)
    assert rel_l2(got, want) < TOL and worst < 1e-5
    x = rng.normal(size=grid.shape).astype(np.float32)
    Ax = native.dgr_project(dev(x), grid, geom, views).cpu().numpy().astype(np.float64)
    lhs = float(np.sum(Ax * g))
    rhs = float(np.sum(x.astype(np.float64) * got))
    assert abs(lhs - rhs) <= TOL * np.linalg.norm(Ax) * np.linalg.norm(g)


def test_backproject_brick_rectangle_beyond_2_22_candidates():
    """A 4096 x 1100 detector lying inside the shadow of a brick: the brick's
    detector rectangle holds 4.5 M candidate pixels, more than the 2^22 up to
    which the set-up takes pixel rows from a binary32 reciprocal; the rows
    beyond take the integer path."""
    say("backproject large rectangle")
    grid = inputs.GridSpec((20, 20, 10), (-10 / 64, -10 / 64, -5 / 64), (64.0, 64.0, 64.0))
    geom = inputs.cone_geometry(1, 4096, 1100, 1e-4, 4.0, 6.0, 0.5 / 64, length_scale=1.0)
    assert geom.nu * geom.nv > 2 ** 22
    g = np.random.default_rng(97).normal(size=(1, geom.nv, geom.nu)).astype(np.float32)
    got = native.dgr_backproject(dev(g), grid, geom, dev(geom.views)).cpu().numpy()
    want = oracle.backproject(g.astype(np.float64), grid.dims, grid.lo, grid.inv_h, geom.kind, geom.views,
                              geom.nu, geom.nv, geom.step, geom.length_scale)
    err = rel_l2(got, want)
    worst = float(np.abs(got.astype(np.float64) - want).max() / np.abs(want).max())
    say("backproject large rectangle rel_l2", err, "worst voxel / max", worst)
    assert np.count_nonzero(want) > 0.5 * want.size
    assert err < TOL and worst < 1e-5


@pytest.mark.parametrize("kind", ["cone", "cone_coarse"])
def test_backproject_tiny_and_huge_values(kind):
    """The fixed-point scale follows max |g| and ranges beyond binary32
    (2^-128 ... 2^180): data scaled by 2^-120 or 2^100 backprojects to the
    same numbers scaled alike, and matches the oracle (64-bit tile: a power of
    two; packed tile: the weight bound's quotient)."""
    grid, geom = _geoms()[kind]
    say("backproject tiny and huge values", kind)
    g = np.random.default_rng(96).normal(size=(geom.n_views, geom.nv, geom.nu)).astype(np.float32)
    views = dev(geom.views)
    base = native.dgr_backproject(dev(g), grid, geom, views).cpu().numpy().astype(np.float64)
    for e in (-120, 100):
        gs = (g.astype(np.float64) * 2.0 ** e).astype(np.float32)
        got = native.dgr_backproject(dev(gs), grid, geom, views).cpu().numpy().astype(np.float64)
        want = oracle.backproject(gs.astype(np.float64), grid.dims, grid.lo, grid.inv_h, geom.kind, geom.views,
                                  geom.nu, geom.nv, geom.step, geom.length_scale)
        say("backproject scaled 2^%d" % e, "rel_l2", rel_l2(got, want))
        assert np.all(np.isfinite(got)) and np.abs(got).max() > 0
        assert rel_l2(got, want) < TOL
        assert rel_l2(got * 2.0 ** -e, base) < 1e-6


@pytest.mark.parametrize("kind", BACKPROJECT_KINDS)
def test_backproject_constant_data(kind):
    """g = 1 on every pixel: every tile point receives its largest possible
    sum (all values of one sign at the largest magnitude), the case that
    presses the packed tile's 32-bit halves hardest; the result still matches
    the oracle voxel by voxel."""
    grid, geom = _geoms()[kind]
    say("backproject constant data", kind)
    g = np.ones((geom.n_views, geom.nv, geom.nu), np.float32)
    got = native.dgr_backproject(dev(g), grid, geom, dev(geom.views)).cpu().numpy()
    want = oracle.backproject(g.astype(np.float64), grid.dims, grid.lo, grid.inv_h, geom.kind, geom.views,
                              geom.nu, geom.nv, geom.step, geom.length_scale)
    worst = float(np.abs(got.astype(np.float64) - want).max() / np.abs(want).max())
    say("backproject constant data", kind, "rel_l2", rel_l2(got, want), "worst voxel / max", worst)
    assert rel_l2(got, want) < TOL and worst < 1e-5


@pytest.mark.parametrize("kind", ["cone", "cone_coarse"])
def test_backproject_zero_data(kind):
    """All-zero data (max |g| = 0: no fixed-point scale can be formed; every
    ray is skipped) backprojects to exact zeros on both tile formats."""
    grid, geom = _geoms()[kind]
    say("backproject zero data", kind)
    g = np.zeros((geom.n_views, geom.nv, geom.nu), np.float32)
    out = native.dgr_backproject(dev(g), grid, geom, dev(geom.views))
    assert not bool(torch.any(out != 0.0))


def _weight_bound_cases():
    """(name, grid, geometry, views to check against the oracle, packed?)"""
    cases = [(k, grid, geom, [0, geom.n_views // 3], k != "cone") for k, (grid, geom) in _geoms().items()]
    gf = inputs.GridSpec((48, 44, 40), (-1.0, -1.0 * 44 / 48, -1.0 * 40 / 48), (24.0, 24.0, 24.0))
    fan = inputs.fan_geometry(8, 70, 40, 0.04, 1.0 / 24, 7.8125, 11.71875, 1.0 / 48)
    v = fan.views.astype(np.float64).copy()
    src = v[:, 0:3] / np.linalg.norm(v[:, 0:3], axis=1, keepdims=True)
    v[:, 9:12] += 0.05 * np.linalg.norm(v[:, 9:12], axis=1, keepdims=True) * src
    tilted = inputs.Geometry(2, v.astype(np.float32), fan.nu, fan.nv, fan.step, fan.length_scale)
    cases += [("fan", gf, fan, [0, 3], True), ("fan_tilted", gf, tilted, [1, 5], True),
              ("cone_dense", inputs.cube_grid(32), inputs.cone_workload(32, 8, 128, 0.8), [0, 3], False)]
    return cases


@pytest.mark.parametrize("case", [c[0] for c in _weight_bound_cases()])
def test_backproject_weight_bound_holds(case):
    """The per-view weight bound the backprojection computes on the device
    (which sets the packed tile's scale) is at least the largest weight any
    tile point receives from that view: the oracle's backprojection of ones
    for that view alone, on the grid widened by one voxel per side (the
    tiles' border points), divided by length_scale * step.  The largest bound
    also picks the tile format expected for the geometry."""
    name, grid, geom, sel, packed = next(c for c in _weight_bound_cases() if c[0] == case)
    B = native.dgr_backproject_weight_bound(grid, geom, dev(geom.views)).cpu().numpy().astype(np.float64)
    say("weight bound", name, "max", float(B.max()), "min", float(B.min()))
    assert np.all(np.isfinite(B)) and np.all(B > 0)
    assert (B.max() <= 512.0) == packed
    h = 1.0 / np.asarray(grid.inv_h, np.float64)
    dims = tuple(d + 2 for d in grid.dims)
    lo = tuple(np.asarray(grid.lo, np.float64) - h)
    for j in sel:
        g = np.ones((1, geom.nv, geom.nu))
        W = oracle.backproject(g, dims, lo, grid.inv_h, geom.kind, geom.views[j:j + 1], geom.nu, geom.nv,
                               geom.step, geom.length_scale)
        peak = float(W.max()) / (float(geom.length_scale) * float(geom.step))
        say("weight bound", name, "view", j, "largest weight", round(peak, 3), "bound", float(B[j]))
        assert peak <= B[j]


def test_project_rays_with_disjoint_sample_ranges():
    """Two rays of one pixel bundle whose sample ranges are far apart
    ([-149, -50] and [50, 149]): the chunks between them hold no sample of
    any ray of the bundle and must be skipped."""
    say("project disjoint ranges")
    grid = inputs.GridSpec((160, 4, 4), (-5.0, -0.125, -0.125), (16.0, 16.0, 16.0))
    a, h = 0.1, 1.0 / 16
    v = np.zeros((1, 12), np.float64)
    v[0, 0:3] = (math.cos(a), math.sin(a), 0.0)
    v[0, 6:9] = (-math.sin(a) * 10 * h, math.cos(a) * 10 * h, 0.0)
    v[0, 9:12] = (0.0, 0.0, h)
    geom = inputs.Geometry(0, v.astype(np.float32), 2, 1, h / 2, 1.0)
    V = np.random.default_rng(93).uniform(size=grid.shape).astype(np.float32)
    views = dev(geom.views)
    got = native.dgr_project(dev(V), grid, geom, views).cpu().numpy()
    want = oracle.project(V.astype(np.float64), grid.dims, grid.lo, grid.inv_h, geom.kind, geom.views,
                          geom.nu, geom.nv, geom.step, geom.length_scale)
    assert np.all(want > 0)
    say("project disjoint ranges rel_l2", rel_l2(got, want))
    assert rel_l2(got, want) < TOL
    g = np.array([[[1.0, -2.0]]], np.float32)
    gotb = native.dgr_backproject(dev(g), grid, geom, views).cpu().numpy()
    wantb = oracle.backproject(g.astype(np.float64), grid.dims, grid.lo, grid.inv_h, geom.kind, geom.views,
                               geom.nu, geom.nv, geom.step, geom.length_scale)
    assert rel_l2(gotb, wantb) < TOL


def test_projector_degenerate_cases():
    """Rays that all miss the grid give exact zeros both ways; a one-pixel
    detector matches the oracle; a zero gradient (max |g| = 0, the
    fixed-point scale's degenerate case) backprojects to exact zeros."""
    say("project degenerate")
    grid = GRIDS["ragged"]
    V = np.random.default_rng(94).uniform(size=grid.shape).astype(np.float32)
    v = np.zeros((2, 12), np.float32)
    v[:, 0:3] = (1.0, 0.0, 0.0)            # along x
    v[:, 3:6] = (0.0, 5.0, 0.0)            # detector far beside the grid
    v[:, 6:9] = (0.0, 0.05, 0.0)
    v[:, 9:12] = (0.0, 0.0, 0.05)
    miss = inputs.Geometry(0, v, 7, 5, 0.03, 1.0)
    views = dev(miss.views)
    P = native.dgr_project(dev(V), grid, miss, views).cpu().numpy()
    assert np.all(P == 0.0)
    g = np.random.default_rng(95).normal(size=(2, 5, 7)).astype(np.float32)
    B = native.dgr_backproject(dev(g), grid, miss, views).cpu().numpy()
    assert np.all(B == 0.0)
    one = inputs.cone_geometry(3, 1, 1, 0.05, 3.0, 4.5, 0.03, arc=2.0, length_scale=1.0)
    got = native.dgr_project(dev(V), grid, one, dev(one.views)).cpu().numpy()
    want = oracle.project(V.astype(np.float64), grid.dims, grid.lo, grid.inv_h, one.kind, one.views,
                          one.nu, one.nv, one.step, one.length_scale)
    assert np.all(want > 0) and rel_l2(got, want) < TOL
    gone = np.array([[[0.7]], [[-1.3]], [[2.1]]], np.float32)
    gotb = native.dgr_backproject(dev(gone), grid, one, dev(one.views)).cpu().numpy()
    wantb = oracle.backproject(gone.astype(np.float64), grid.dims, grid.lo, grid.inv_h, one.kind, one.views,
                               one.nu, one.nv, one.step, one.length_scale)
    assert rel_l2(gotb, wantb) < TOL
    cone = inputs.cone_geometry(4, 9, 7, 0.1, 3.0, 4.5, 0.03, length_scale=1.0)
    Z = native.dgr_backproject(torch.zeros((4, 7, 9), device="cuda"), grid, cone,
                               dev(cone.views)).cpu().numpy()
    assert np.all(Z == 0.0)


# --------------------------------------------------------------------------
# voxelization backward and Adam
# --------------------------------------------------------------------------
@pytest.mark.parametrize("gname", list(GRIDS))
def test_voxelize_backward_parity(gname):
    grid = GRIDS[gname]
    say("voxelize_backward", gname)
    G = inputs.gaussians(1200, 92, 0.01, 0.08, mean_lim=0.95)
    G["quat"][0] = 0.0
    rng = np.random.default_rng(7)
    w = rng.normal(size=grid.shape).astype(np.float32)
    got = native.dgr_voxelize_backward(*gauss_dev(G), dev(w), grid)
    box = oracle.bbox(G["mu"], G["scale"], G["quat"], grid.dims, grid.lo, grid.inv_h)
    want = oracle.voxelize_grad(G["mu"], G["scale"], G["quat"], G["density"], grid.dims, grid.lo,
                                grid.inv_h, box, w)
    for name, a, b in zip(("dmu", "dscale", "dquat", "ddensity"), got, want):
        err = rel_l2(a.cpu().numpy(), b)
        say("voxelize_backward", gname, name, "rel_l2", err)
        assert err < TOL, (name, err)
    assert np.all(got[2][0].cpu().numpy() == 0.0)


@pytest.mark.parametrize("lower", [-np.inf, 0.0, -0.25])
def test_adam_parity(lower):
    """The (projected) Adam step against the oracle.  With a finite bound a
    good share of the entries start at or just above it and get gradients
    that push them into it, so the clamp is exercised every step."""
    say("adam", "lower", lower)
    rng = np.random.default_rng(8)
    n = 5000
    p0 = rng.normal(size=n).astype(np.float32)
    if np.isfinite(lower):
        p0[:1500] = np.float32(lower) + rng.uniform(0, 2e-3, size=1500).astype(np.float32)
        p0[:500] = np.float32(lower)
        p0 = np.maximum(p0, np.float32(lower))
    p, m, v = dev(p0), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    P, M, Vv = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    steps = 5
    f = lambda x: float(np.float32(x))  # the ABI takes binary32 hyper-parameters
    for t in range(1, steps + 1):
        g = rng.normal(size=n).astype(np.float32)
        if np.isfinite(lower):
            g[:1500] = np.abs(g[:1500])
        native.dgr_adam(p, dev(g), m, v, 1e-3, t, lower=lower)
        oracle.adam(P, g, M, Vv, f(1e-3), t, b1=f(0.9), b2=f(0.999), eps=f(1e-8), lower=f(lower))
    # moments agree to binary32 rounding; the parameter differs from the
    # binary64 oracle only by one rounding of the stored value per step
    assert rel_l2(m.cpu().numpy(), M) < 1e-6 and rel_l2(v.cpu().numpy(), Vv) < 1e-6
    pg = p.cpu().numpy().astype(np.float64)
    # one rounding per step at the largest magnitude the entry passed through
    ulp = np.spacing((np.maximum(np.abs(P), np.abs(p0)) + steps * 1e-3).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(pg - P) <= steps * ulp)
    assert rel_l2(pg - p0, P - p0) < 1e-4
    if np.isfinite(lower):
        at = P == f(lower)
        assert at.sum() >= 1000, at.sum()
        # the same entries sit on the bound, up to a binary32 rounding that
        # lands a step exactly on it (the ulp bound above covers their values)
        assert int(np.sum((pg == f(lower)) != at)) <= 5
        assert np.all(pg >= f(lower))
