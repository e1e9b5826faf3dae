"""Oracle for adaptive density control (Alg. 2), numpy.

TEST INFRASTRUCTURE.  Only ``tests/`` may import this module; it shares no
code with the HIP library.

Readings of Alg. 2 (clone, split, prune every 100 iterations):

* avg_grad of Gaussian g = (sum over the iterations since the last pass of
  ||dL/dmu_g||_2) / (number of those iterations).
* sigma_g = largest of the three scales; theta = 0.005 x the body diagonal
  of the grid; size = the box edge in voxels (17).
* clone: avg_grad >= tau and sigma <= theta.  If more than the free room
  n_max - n qualify, the largest avg_grad win (ties: lower index).  A cloned
  Gaussian and its copy both carry half the density; the original keeps its
  Adam moments, the copy starts at zero.
* split (after cloning, with the room left): avg_grad >= tau and sigma > theta,
  same selection rule.  The original is replaced by two Gaussians with means
  mu + R diag(s) z_k (z_k standard normal, k = 1, 2; a draw from the
  Gaussian itself), scales s / 2^(1/3) (the pair keeps the total volume),
  the same density and rotation, and zero Adam moments.
* prune (among the Gaussians neither cloned nor split): avg_grad <= tau_prune
  (the paper's "near-zero gradient"; the literal avg_grad <= tau would remove
  every converged Gaussian), density <= 0, or sigma > 3 x size voxels.
* Output order: old Gaussians in index order, each emitting 0 (pruned),
  1 (kept), or 2 (cloned: original then copy; split: the two new ones).

Decisions are taken in binary32, like the kernels: avg = float32(acc) /
float32(iters), sigma, theta and the thresholds are binary32.

Pins (tests/test_oracle_densify.py): count identity, density mass
conservation for clones and volume-weighted mass for splits, the cap and the
top-k choice against a brute-force sort, and the first two moments of many
split draws against the Gaussian's mean and covariance.
"""
from __future__ import annotations

import numpy as np


def quat_to_rot(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def select_top(mask, key, room):
    """Boolean mask of the (at most room) entries of mask with the largest
    key, ties broken by lower index."""
    idx = np.nonzero(mask)[0]
    if len(idx) <= room:
        return mask.copy()
    order = np.lexsort((idx, -key[idx].astype(np.float64)))  # by key desc, then index
    keep = idx[order[:room]]
    out = np.zeros_like(mask)
    out[keep] = True
    return out


def densify(P, state, acc, iters, normals, n_max, tau, tau_prune, theta, size_vox, inv_h):
    """P: dict mu [n,3], scale [n,3], quat [n,4], density [n] (float32);
    state: dict of Adam moments with the same keys, each (m, v);
    acc [n] float32; normals [n, 2, 3] float32.  Returns (P', state', info)."""
    n = P["mu"].shape[0]
    f32 = np.float32
    avg = acc.astype(f32) / f32(iters)
    sigma = P["scale"].astype(f32).max(axis=1)
    big = sigma > f32(3 * size_vox) / f32(np.min(inv_h))
    clone = (avg >= f32(tau)) & (sigma <= f32(theta))
    clone = select_top(clone, avg, max(0, n_max - n))
    n1 = n + int(clone.sum())
    split = (avg >= f32(tau)) & (sigma > f32(theta))
    split = select_top(split, avg, max(0, n_max - n1))
    prune = ~clone & ~split & ((avg <= f32(tau_prune)) | (P["density"] <= 0) | big)
    R = quat_to_rot(P["quat"])
    rows = {k: [] for k in P}
    srows = {k: ([], []) for k in P}

    def zero_state(k):
        return np.zeros_like(state[k][0][0])

    for g in range(n):
        if prune[g]:
            continue
        if split[g]:
            for j in range(2):
                z = normals[g, j].astype(np.float64)
                mu = P["mu"][g].astype(np.float64) + R[g] @ (P["scale"][g].astype(np.float64) * z)
                vals = {"mu": mu.astype(f32), "scale": (P["scale"][g].astype(np.float64) / 2 ** (1 / 3)).astype(f32),
                        "quat": P["quat"][g], "density": P["density"][g]}
                for k in P:
                    rows[k].append(vals[k])
                    srows[k][0].append(zero_state(k))
                    srows[k][1].append(zero_state(k))
            continue
        copies = 2 if clone[g] else 1
        for c in range(copies):
            for k in P:
                v = P[k][g]
                if k == "density" and clone[g]:
                    v = f32(v * f32(0.5))
                rows[k].append(v)
                if c == 0:
                    srows[k][0].append(state[k][0][g])
                    srows[k][1].append(state[k][1][g])
                else:
                    srows[k][0].append(zero_state(k))
                    srows[k][1].append(zero_state(k))
    P2 = {k: np.array(rows[k], dtype=f32).reshape((-1,) + P[k].shape[1:]) for k in P}
    S2 = {k: (np.array(srows[k][0], dtype=f32).reshape((-1,) + P[k].shape[1:]),
              np.array(srows[k][1], dtype=f32).reshape((-1,) + P[k].shape[1:])) for k in P}
    info = {"n": n, "cloned": int(clone.sum()), "split": int(split.sum()), "pruned": int(prune.sum()),
            "new_n": P2["mu"].shape[0], "clone": clone, "split_mask": split, "prune": prune}
    return P2, S2, info
