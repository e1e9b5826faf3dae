"""Oracle for the learned-initialisation network (binary64 numpy).

TEST INFRASTRUCTURE.  Only ``tests/`` may import this module; it shares no
code with the HIP library.

The network is not part of DGR itself (the paper initialises Gaussians from
an FBP/FDK volume, Fig. 4 caption, or at random).  It maps a one-channel
volume to three per-voxel fields from which an initial Gaussian set is drawn:
density, log-scale and occupancy (a logit).  Architecture, with base width B:

    enc1 = relu(conv3(x; 1 -> B))                       at D
    enc2 = relu(conv3(pool(enc1); B -> 2B))             at D/2
    enc3 = relu(conv3(pool(enc2); 2B -> 4B))            at D/4
    bott = relu(conv3(pool(enc3); 4B -> 8B))            at D/8
    dec3 = relu(conv3([up(bott), enc3]; 12B -> 4B))     at D/4
    dec2 = relu(conv3([up(dec3), enc2]; 6B -> 2B))      at D/2
    dec1 = relu(conv3([up(dec2), enc1]; 3B -> B))       at D
    out  = head(dec1; B -> 3)                           1x1x1 convolution

conv3 is a 3x3x3 cross-correlation with zero padding 1:
    y[z,y,x,o] = b[o] + sum_{t, i} W[t, o, i] x[z+dz, y+dy, x+dx, i],
    t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1).
pool is the mean of each 2x2x2 block; up repeats each voxel into a 2x2x2
block; [a, b] concatenates channels (a first).  Arrays are channels-last
[Z, Y, X, C].

Flat parameter layout (the C ABI's): for each of the seven conv3 layers in
the order above, W[27][Cout][Cin] then b[Cout]; then the head W[3][B], b[3].

Loss over the V voxels, with targets (t_d, t_s, t_o), t_o in [0, 1]:
    L = mean (o_d - t_d)^2 + mean t_o (o_s - t_s)^2
        + mean [softplus(o_o) - t_o o_o]            (binary cross-entropy)

Pins (tests/test_oracle_unet.py): conv3 against a seven-loop brute force and
against the closed-form response to a unit impulse; the backward functions
against the adjoint identities of their forward functions; pool/up against
their adjoint identity and constant preservation; the whole network's
gradient and the loss gradient against binary64 central differences.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def layer_shapes(B: int):
    """(name, Cin, Cout) of the seven conv3 layers, then the head."""
    return [("enc1", 1, B), ("enc2", B, 2 * B), ("enc3", 2 * B, 4 * B), ("bott", 4 * B, 8 * B),
            ("dec3", 12 * B, 4 * B), ("dec2", 6 * B, 2 * B), ("dec1", 3 * B, B), ("head", B, 3)]


def param_count(B: int) -> int:
    n = 0
    for name, ci, co in layer_shapes(B):
        n += (1 if name == "head" else 27) * co * ci + co
    return n


def unpack(flat, B: int):
    """Flat vector -> {name: (W, b)} (views into flat)."""
    out, off = {}, 0
    for name, ci, co in layer_shapes(B):
        taps = 1 if name == "head" else 27
        nw = taps * co * ci
        W = flat[off:off + nw].reshape((co, ci) if name == "head" else (27, co, ci))
        off += nw
        b = flat[off:off + co]
        off += co
        out[name] = (W, b)
    assert off == flat.size
    return out


# ---- layers -------------------------------------------------------------------
def shifted(x, dz, dy, dx):
    """s[z, y, x] = x[z + dz, y + dy, x + dx], zero outside."""
    Z, Y, X = x.shape[:3]
    p = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    return p[1 + dz:1 + dz + Z, 1 + dy:1 + dy + Y, 1 + dx:1 + dx + X]


def conv3(x, W, b):
    y = np.zeros(x.shape[:3] + (W.shape[1],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += shifted(x, dz, dy, dx) @ W[t].T
    return y + b


def conv3_dgrad(dy, W):
    """dL/dx of conv3 given dL/dy: the adjoint of x -> conv3(x, W, 0)."""
    dx_ = np.zeros(dy.shape[:3] + (W.shape[2],))
    for t, (dz, dy_, dx) in enumerate(TAPS):
        dx_ += shifted(dy, -dz, -dy_, -dx) @ W[t]
    return dx_


def conv3_wgrad(x, dy):
    """(dL/dW [27, Cout, Cin], dL/db [Cout])."""
    co, ci = dy.shape[3], x.shape[3]
    dyf = dy.reshape(-1, co)
    dW = np.empty((27, co, ci))
    for t, (dz, dy_, dx) in enumerate(TAPS):
        dW[t] = dyf.T @ shifted(x, dz, dy_, dx).reshape(-1, ci)
    return dW, dyf.sum(axis=0)


def pool2(x):
    Z, Y, X, C = x.shape
    return x.reshape(Z // 2, 2, Y // 2, 2, X // 2, 2, C).mean(axis=(1, 3, 5))


def pool2_bwd(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, 0), 2, 1), 2, 2) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up2_bwd(dy):
    Z, Y, X, C = dy.shape
    return dy.reshape(Z // 2, 2, Y // 2, 2, X // 2, 2, C).sum(axis=(1, 3, 5))


def relu(x):
    return np.maximum(x, 0.0)


# ---- network ------------------------------------------------------------------
def forward(flat, x, B: int):
    """x [Z, Y, X] (Z, Y, X divisible by 8) -> out [Z, Y, X, 3] and a cache."""
    P = unpack(np.asarray(flat, np.float64), B)
    c = {"x": np.asarray(x, np.float64)[..., None]}
    c["enc1"] = relu(conv3(c["x"], *P["enc1"]))
    c["enc2"] = relu(conv3(pool2(c["enc1"]), *P["enc2"]))
    c["enc3"] = relu(conv3(pool2(c["enc2"]), *P["enc3"]))
    c["bott"] = relu(conv3(pool2(c["enc3"]), *P["bott"]))
    c["cat3"] = np.concatenate([up2(c["bott"]), c["enc3"]], axis=3)
    c["dec3"] = relu(conv3(c["cat3"], *P["dec3"]))
    c["cat2"] = np.concatenate([up2(c["dec3"]), c["enc2"]], axis=3)
    c["dec2"] = relu(conv3(c["cat2"], *P["dec2"]))
    c["cat1"] = np.concatenate([up2(c["dec2"]), c["enc1"]], axis=3)
    c["dec1"] = relu(conv3(c["cat1"], *P["dec1"]))
    Wh, bh = P["head"]
    out = c["dec1"] @ Wh.T + bh
    return out, c


def backward(flat, cache, dout, B: int):
    """Gradient of sum(dout * out) with respect to the flat parameters."""
    P = unpack(np.asarray(flat, np.float64), B)
    G = {}
    c = cache
    Wh, bh = P["head"]
    G["head"] = (dout.reshape(-1, 3).T @ c["dec1"].reshape(-1, B), dout.reshape(-1, 3).sum(0))
    d = (dout @ Wh) * (c["dec1"] > 0)                       # d pre-activation of dec1
    G["dec1"] = conv3_wgrad(c["cat1"], d)
    dcat = conv3_dgrad(d, P["dec1"][0])
    d_up, d_enc1 = dcat[..., :2 * B], dcat[..., 2 * B:]
    d = up2_bwd(d_up) * (c["dec2"] > 0)
    G["dec2"] = conv3_wgrad(c["cat2"], d)
    dcat = conv3_dgrad(d, P["dec2"][0])
    d_up, d_enc2 = dcat[..., :4 * B], dcat[..., 4 * B:]
    d = up2_bwd(d_up) * (c["dec3"] > 0)
    G["dec3"] = conv3_wgrad(c["cat3"], d)
    dcat = conv3_dgrad(d, P["dec3"][0])
    d_up, d_enc3 = dcat[..., :8 * B], dcat[..., 8 * B:]
    d = up2_bwd(d_up) * (c["bott"] > 0)
    G["bott"] = conv3_wgrad(pool2(c["enc3"]), d)
    d_enc3 = d_enc3 + pool2_bwd(conv3_dgrad(d, P["bott"][0]))
    d = d_enc3 * (c["enc3"] > 0)
    G["enc3"] = conv3_wgrad(pool2(c["enc2"]), d)
    d_enc2 = d_enc2 + pool2_bwd(conv3_dgrad(d, P["enc3"][0]))
    d = d_enc2 * (c["enc2"] > 0)
    G["enc2"] = conv3_wgrad(pool2(c["enc1"]), d)
    d_enc1 = d_enc1 + pool2_bwd(conv3_dgrad(d, P["enc2"][0]))
    d = d_enc1 * (c["enc1"] > 0)
    G["enc1"] = conv3_wgrad(c["x"], d)
    flat_g = []
    for name, _, _ in layer_shapes(B):
        flat_g += [G[name][0].ravel(), G[name][1].ravel()]
    return np.concatenate(flat_g)


def loss(out, t_d, t_s, t_o):
    """(L, dL/dout) for out [..., 3] and targets of shape out.shape[:-1]."""
    o_d, o_s, o_o = out[..., 0], out[..., 1], out[..., 2]
    V = o_d.size
    sp = np.logaddexp(0.0, o_o)
    L = (np.sum((o_d - t_d) ** 2) + np.sum(t_o * (o_s - t_s) ** 2) + np.sum(sp - t_o * o_o)) / V
    g = np.empty_like(out)
    g[..., 0] = 2.0 * (o_d - t_d) / V
    g[..., 1] = 2.0 * t_o * (o_s - t_s) / V
    g[..., 2] = (1.0 / (1.0 + np.exp(-o_o)) - t_o) / V
    return L, g


def conv3_brute(x, W, b):
    """Seven nested loops, for pinning conv3 on tiny inputs."""
    Z, Y, X, Ci = x.shape
    Co = W.shape[1]
    y = np.zeros((Z, Y, X, Co))
    for z in range(Z):
        for yy in range(Y):
            for xx in range(X):
                for o in range(Co):
                    acc = b[o]
                    for t, (dz, dy, dx) in enumerate(TAPS):
                        zz, y2, x2 = z + dz, yy + dy, xx + dx
                        if 0 <= zz < Z and 0 <= y2 < Y and 0 <= x2 < X:
                            for i in range(Ci):
                                acc += W[t, o, i] * x[zz, y2, x2, i]
                    y[z, yy, xx, o] = acc
    return y


# ---- around the network: training targets and the proposed Gaussians -----------------
def targets(mu, scale, dims, lo, inv_h, volume, input_scale):
    """target [nz, ny, nx, 3] = (volume / input_scale, mean log geometric-mean
    scale in voxels of the Gaussians whose mean lies in the voxel (else 0),
    1 if there is one else 0).  dims = (nx, ny, nz)."""
    nx, ny, nz = dims
    cnt = np.zeros(nz * ny * nx)
    lsum = np.zeros(nz * ny * nx)
    for m, s in zip(np.asarray(mu, np.float64), np.asarray(scale, np.float64)):
        u = (m - np.asarray(lo, np.float64)) * np.asarray(inv_h, np.float64)
        if np.all(u >= 0) and u[0] < nx and u[1] < ny and u[2] < nz:
            i = np.floor(u).astype(int)
            v = (i[2] * ny + i[1]) * nx + i[0]
            cnt[v] += 1
            lsum[v] += np.mean(np.log(s * np.asarray(inv_h, np.float64)))
    t = np.zeros((nz * ny * nx, 3))
    t[:, 0] = np.asarray(volume, np.float64).ravel() / input_scale
    has = cnt > 0
    t[has, 1] = lsum[has] / cnt[has]
    t[:, 2] = has
    return t.reshape(nz, ny, nx, 3)


def draw_from_fields(out, dims, lo, inv_h, uniforms, input_scale):
    """Gaussians drawn from network output out [nz, ny, nx, 3]: voxel v with
    probability sigmoid(o_o[v]) / sum (inverse CDF of uniforms[:, 0], first v
    whose cumulative weight exceeds u W), mean = centre + (u_1..3 - 1/2) voxel,
    isotropic scale clip(exp(o_s), 1/4, 8) voxels, density max(o_d, 0) s_in."""
    nx, ny, nz = dims
    o = np.asarray(out, np.float64).reshape(-1, 3)
    w = 1.0 / (1.0 + np.exp(-o[:, 2]))
    cdf = np.cumsum(w)
    U = np.asarray(uniforms, np.float64)
    v = np.searchsorted(cdf, U[:, 0] * cdf[-1], side="right")
    idx = np.stack([v % nx, (v // nx) % ny, v // (nx * ny)], axis=1)
    lo, ih = np.asarray(lo, np.float64), np.asarray(inv_h, np.float64)
    mu = lo + (idx + 0.5 + (U[:, 1:4] - 0.5)) / ih
    s_vox = np.clip(np.exp(o[v, 1]), 0.25, 8.0)
    sc = s_vox[:, None] / ih
    rho = np.maximum(o[v, 0], 0.0) * input_scale
    return mu, sc, rho, v
