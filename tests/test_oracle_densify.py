"""Pins of the adaptive density control oracle (CPU only)."""
import numpy as np

from oracle import densify as Dn


def _case(n=400, seed=0):
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
    normals = r.normal(size=(n, 2, 3)).astype(np.float32)
    return P, state, acc, normals


ARGS = dict(iters=100, tau=2e-6, tau_prune=2e-9, theta=0.0173, size_vox=17, inv_h=(128.0, 128.0, 128.0))


def test_counts_and_mass():
    P, state, acc, normals = _case()
    P2, S2, info = Dn.densify(P, state, acc, normals=normals, n_max=10_000, **ARGS)
    assert info["new_n"] == info["n"] + info["cloned"] + info["split"] - info["pruned"]
    assert info["cloned"] > 0 and info["split"] > 0
    assert np.all(info["prune"][10:20])           # zero gradient: pruned
    assert not np.any(info["prune"] & (info["clone"] | info["split_mask"]))
    # clones keep the density mass; splits keep density x volume
    def mass(Q):
        return float(np.sum(Q["density"].astype(np.float64) * np.prod(Q["scale"].astype(np.float64), axis=1)))
    keep = ~info["prune"]
    kept = {k: v[keep] for k, v in P.items()}
    assert abs(mass(P2) - mass(kept)) < 1e-6 * mass(kept)
    for k in P:
        assert S2[k][0].shape[0] == info["new_n"]


def test_cap_and_top_k_against_brute_force():
    P, state, acc, normals = _case(seed=1)
    n = P["mu"].shape[0]
    room = 7
    P2, _, info = Dn.densify(P, state, acc, normals=normals, n_max=n + room, **ARGS)
    avg = acc / np.float32(100)
    sigma = P["scale"].max(axis=1)
    cand = np.nonzero((avg >= np.float32(2e-6)) & (sigma <= np.float32(0.0173)))[0]
    best = sorted(cand, key=lambda g: (-float(avg[g]), g))[:room]
    assert set(np.nonzero(info["clone"])[0]) == set(best)
    assert info["split"] == 0                     # the clones used all the room
    assert info["new_n"] <= n + room


def test_split_draws_have_the_gaussian_moments():
    r = np.random.default_rng(2)
    n = 20000
    q = np.tile(np.array([[0.9, 0.3, -0.2, 0.25]], np.float32), (n, 1))
    s = np.tile(np.array([[0.05, 0.02, 0.01]], np.float32), (n, 1))
    P = {"mu": np.zeros((n, 3), np.float32), "scale": s, "quat": q, "density": np.ones(n, np.float32)}
    state = {k: (np.zeros_like(v), np.zeros_like(v)) for k, v in P.items()}
    acc = np.full(n, 1.0, np.float32)
    normals = r.normal(size=(n, 2, 3)).astype(np.float32)
    P2, _, info = Dn.densify(P, state, acc, normals=normals, n_max=3 * n, iters=100, tau=1e-3, tau_prune=0.0,
                             theta=0.01, size_vox=17, inv_h=(128.0,) * 3)
    assert info["split"] == n
    X = P2["mu"].astype(np.float64)
    R = Dn.quat_to_rot(q[:1])[0]
    Sigma = R @ np.diag(s[0].astype(np.float64) ** 2) @ R.T
    C = X.T @ X / X.shape[0]
    assert np.max(np.abs(X.mean(axis=0))) < 5 * 0.05 / np.sqrt(2 * n)
    assert np.max(np.abs(C - Sigma)) < 0.05 * np.max(Sigma)
    np.testing.assert_allclose(P2["scale"][0], s[0] / 2 ** (1 / 3), rtol=1e-6)


def test_prune_of_oversized_gaussians():
    """Alg. 2's prune of Gaussians larger than 3 x size (read as box edges in
    voxels): at size 17 and 128 voxels per unit the bound is 51/128 = 0.3984.
    Hand cases just below and above it, and the other two prune reasons
    (near-zero gradient, non-positive density) left out."""
    n = 6
    bound = np.float32(3 * 17) / np.float32(128.0)
    s = np.full((n, 3), 0.01, np.float32)
    s[0, 2] = np.nextafter(bound, np.float32(0))  # just below: kept
    s[1, 0] = bound                               # equal: kept (strictly larger prunes)
    s[2, 1] = np.nextafter(bound, np.float32(1))  # just above: pruned
    s[3, :] = 0.5                                  # far above: pruned
    P = {"mu": np.zeros((n, 3), np.float32), "scale": s,
         "quat": np.tile(np.array([[1, 0, 0, 0]], np.float32), (n, 1)), "density": np.ones(n, np.float32)}
    state = {k: (np.zeros_like(v), np.zeros_like(v)) for k, v in P.items()}
    acc = np.full(n, 1e-6, np.float32)  # avg 1e-8: neither near zero nor enough to clone or split
    P2, _, info = Dn.densify(P, state, acc, iters=100, normals=np.zeros((n, 2, 3), np.float32), n_max=100,
                             tau=1e-3, tau_prune=1e-9, theta=0.0173, size_vox=17, inv_h=(128.0,) * 3)
    assert info["cloned"] == 0 and info["split"] == 0
    assert list(info["prune"]) == [False, False, True, True, False, False]
    np.testing.assert_array_equal(P2["scale"], s[[0, 1, 4, 5]])
