"""The allocation-free voxelization backward (records in the library's fixed
device array) against dgr_voxelize_backward with a caller workspace: two
calls in a row through the C ABI, the second with fewer Gaussians, each
bit-identical (same kernels, deterministic wave reductions)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2411_04844_amd import inputs, native

pytestmark = pytest.mark.gpu


def _case(n, seed, dims, s_lo, s_hi):
    grid = inputs.GridSpec(dims, (-1.0, -1.0, -1.0), tuple(d / 2.0 for d in dims))
    G = inputs.gaussians(n, seed, s_lo, s_hi)
    d = {k: torch.as_tensor(v).cuda().contiguous() for k, v in G.items()}
    gen = torch.Generator(device="cuda").manual_seed(seed)
    dV = torch.randn(grid.shape, generator=gen, device="cuda")
    return grid, d, dV


def test_noalloc_backward_matches_workspace_backward_twice():
    assert native.lib().dgr_voxelize_backward_noalloc_max() == 1 << 19
    for n, seed, dims, s_lo, s_hi in ((3000, 11, (64, 64, 64), 0.01, 0.05),
                                      (1200, 12, (48, 40, 56), 0.02, 0.08)):
        print(f"noalloc backward n={n} dims={dims} seed={seed}", flush=True)
        grid, d, dV = _case(n, seed, dims, s_lo, s_hi)
        ref = native.dgr_voxelize_backward(d["mu"], d["scale"], d["quat"], d["density"], dV, grid)
        # poison the outputs: every element must be written
        outs = tuple(torch.full_like(d[k], float("nan")) for k in ("mu", "scale", "quat", "density"))
        got = native.dgr_voxelize_backward_noalloc(d["mu"], d["scale"], d["quat"], d["density"], dV, grid,
                                                   outs=outs)
        torch.cuda.synchronize()
        for name, a, b in zip(("dmu", "dscale", "dquat", "ddensity"), got, ref):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.all(np.isfinite(a)), name
            assert np.array_equal(a, b), f"{name} differs (n={n})"
            assert np.abs(b).max() > 0, name


def test_noalloc_backward_rejects_more_than_its_capacity():
    L = native.lib()
    cap = int(L.dgr_voxelize_backward_noalloc_max())
    g = native.c_grid(inputs.GridSpec((32, 32, 32), (-1.0, -1.0, -1.0), (16.0, 16.0, 16.0)))
    t = native.c_trunc()
    fake = ctypes.c_void_p(0x10000)
    st = L.dgr_voxelize_backward_noalloc(fake, fake, fake, fake, cap + 1, ctypes.byref(g), ctypes.byref(t),
                                         fake, fake, fake, fake, fake, None)
    assert st == 1 and b"exceeds" in L.dgr_last_error()
