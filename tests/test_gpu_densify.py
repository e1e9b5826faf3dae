"""Parity of adaptive density control (Alg. 2) with the oracle."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import densify as Dn
from paper_2411_04844_amd import inputs, native

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _case(n, seed):
    r = np.random.default_rng(seed)
    P = {"mu": r.uniform(-0.5, 0.5, size=(n, 3)).astype(np.float32),
         "scale": np.exp(r.uniform(np.log(0.004), np.log(0.05), size=(n, 3))).astype(np.float32),
         "quat": r.normal(size=(n, 4)).astype(np.float32),
         "density": r.uniform(0.0, 1.0, size=n).astype(np.float32)}
    P["density"][:5] = 0.0
    state = {k: (r.normal(size=v.shape).astype(np.float32), r.uniform(size=v.shape).astype(np.float32))
             for k, v in P.items()}
    acc = (r.exponential(size=n) * 1e-3).astype(np.float32)
    acc[10:20] = 0.0
    acc[30:40] = acc[29]          # ties
    normals = r.normal(size=(n, 2, 3)).astype(np.float32)
    return P, state, acc, normals


@pytest.mark.parametrize("n,room", [(3000, 100000), (3000, 37), (3000, 700), (257, 0)])
def test_densify_parity(n, room):
    say("densify", n, room)
    P, state, acc, normals = _case(n, 51)
    grid = inputs.cube_grid(256)
    args = dict(iters=100, tau=2e-6, tau_prune=2e-9, theta=0.0173, size_vox=17.0)
    P2, S2, info = Dn.densify(P, state, acc, normals=normals, n_max=n + room, inv_h=grid.inv_h, **args)
    cu = lambda a: torch.as_tensor(a).cuda().contiguous()  # noqa: E731
    Pd = {k: cu(v) for k, v in P.items()}
    md = {k: cu(state[k][0]) for k in P}
    vd = {k: cu(state[k][1]) for k in P}
    cap = n + room
    dst = tuple({k: torch.full((cap,) + v.shape[1:], 7.0, device="cuda") for k, v in P.items()} for _ in range(3))
    n_new, counts = native.dgr_densify(Pd, md, vd, cu(acc), cu(normals), grid, dst, n_max=cap, **args)
    say("new n", n_new, info["new_n"], "counts", counts, (info["cloned"], info["split"], info["pruned"]))
    assert n_new == info["new_n"]
    assert counts == (info["cloned"], info["split"], info["pruned"])
    split_rows = np.zeros(n_new, bool)
    o = 0
    for g in range(n):
        if info["prune"][g]:
            continue
        if info["split_mask"][g]:
            split_rows[o:o + 2] = True
        o += 2 if (info["split_mask"][g] or info["clone"][g]) else 1
    for k in P:
        got = dst[0][k][:n_new].cpu().numpy()
        want = P2[k]
        np.testing.assert_array_equal(got[~split_rows], want[~split_rows])
        if split_rows.any():
            assert np.max(np.abs(got[split_rows] - want[split_rows])) < 1e-6
        for j in (1, 2):
            np.testing.assert_array_equal(dst[j][k][:n_new].cpu().numpy(), S2[k][j - 1])
