"""Pins of the learned-initialisation network oracle (CPU only)."""
import numpy as np
import pytest

from oracle import unet as U


def rng(s=0):
    return np.random.default_rng(s)


def test_conv3_matches_brute_force():
    r = rng(1)
    x = r.normal(size=(4, 5, 3, 2))
    W = r.normal(size=(27, 3, 2))
    b = r.normal(size=3)
    np.testing.assert_allclose(U.conv3(x, W, b), U.conv3_brute(x, W, b), rtol=1e-12, atol=1e-12)


def test_conv3_impulse_response_is_flipped_kernel():
    # a unit impulse at c gives y[c - offset(t)] = W[t] for every tap t
    r = rng(2)
    W = r.normal(size=(27, 1, 1))
    x = np.zeros((5, 5, 5, 1))
    x[2, 2, 2, 0] = 1.0
    y = U.conv3(x, W, np.zeros(1))
    for t, (dz, dy, dx) in enumerate(U.TAPS):
        assert y[2 - dz, 2 - dy, 2 - dx, 0] == W[t, 0, 0]
    # and nothing outside the 3x3x3 neighbourhood
    mask = np.ones((5, 5, 5), bool)
    mask[1:4, 1:4, 1:4] = False
    assert np.all(y[mask, 0] == 0.0)


def test_conv3_backward_adjoint_identities():
    r = rng(3)
    x = r.normal(size=(4, 6, 5, 3))
    W = r.normal(size=(27, 4, 3))
    dy = r.normal(size=(4, 6, 5, 4))
    lhs = np.sum(U.conv3(x, W, np.zeros(4)) * dy)
    assert abs(lhs - np.sum(x * U.conv3_dgrad(dy, W))) < 1e-10 * abs(lhs) + 1e-10
    dW, db = U.conv3_wgrad(x, dy)
    assert abs(lhs - np.sum(W * dW)) < 1e-10 * abs(lhs) + 1e-10
    np.testing.assert_allclose(db, dy.sum(axis=(0, 1, 2)), rtol=1e-12)


def test_pool_and_up_adjoint_and_constants():
    r = rng(4)
    x = r.normal(size=(2, 3, 2, 3))
    y = r.normal(size=(4, 6, 4, 3))
    assert abs(np.sum(U.up2(x) * y) - np.sum(x * U.up2_bwd(y))) < 1e-12
    assert abs(np.sum(U.pool2(y) * x) - np.sum(y * U.pool2_bwd(x))) < 1e-12
    c = np.full((4, 4, 4, 2), 0.375)
    np.testing.assert_allclose(U.pool2(c), 0.375, rtol=0, atol=0)
    np.testing.assert_allclose(U.pool2(U.up2(x)), x, rtol=1e-15)


def test_param_count_matches_architecture():
    # B = 32: 27 * (32 + 2048 + 8192 + 32768 + 49152 + 12288 + 3072) weights,
    # 704 conv biases, 96 + 3 head parameters
    assert U.param_count(32) == 27 * 107552 + 704 + 99 == 2904707


def _net(B=2, D=8, seed=5):
    r = rng(seed)
    n = U.param_count(B)
    flat = r.normal(scale=0.6, size=n)
    x = r.normal(size=(D, D, D))
    return flat, x


def test_network_gradient_matches_central_differences():
    B = 2
    flat, x = _net(B)
    r = rng(6)
    w = r.normal(size=(8, 8, 8, 3))
    out, cache = U.forward(flat, x, B)
    g = U.backward(flat, cache, w, B)
    # check coordinates from every layer
    idx, off = [], 0
    for name, ci, co in U.layer_shapes(B):
        taps = 1 if name == "head" else 27
        nw = taps * co * ci
        idx += [off + int(r.integers(nw)), off + nw + int(r.integers(co))]
        off += nw + co
    h = 1e-6
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        num = (np.sum(U.forward(fp, x, B)[0] * w) - np.sum(U.forward(fm, x, B)[0] * w)) / (2 * h)
        # 1e-5: a ReLU kink within h of a pre-activation perturbs the difference
        assert abs(num - g[i]) <= 1e-5 * max(1.0, abs(g[i])), (i, num, g[i])


def test_loss_value_and_gradient():
    r = rng(7)
    out = r.normal(size=(3, 4, 2, 3))
    t_d, t_s = r.normal(size=(3, 4, 2)), r.normal(size=(3, 4, 2))
    t_o = r.uniform(size=(3, 4, 2))
    L, g = U.loss(out, t_d, t_s, t_o)
    h = 1e-6
    for k in range(10):
        i = tuple(int(r.integers(s)) for s in out.shape)
        op, om = out.copy(), out.copy()
        op[i] += h
        om[i] -= h
        num = (U.loss(op, t_d, t_s, t_o)[0] - U.loss(om, t_d, t_s, t_o)[0]) / (2 * h)
        assert abs(num - g[i]) < 1e-8
    # closed form: all-zero outputs and targets give log 2 (cross-entropy at p = 1/2)
    z = np.zeros((2, 2, 2))
    assert abs(U.loss(np.zeros((2, 2, 2, 3)), z, z, z)[0] - np.log(2.0)) < 1e-15


def test_targets_hand_example():
    # 2 x 2 x 2 grid on [0, 2]^3 (unit voxels); two Gaussians in voxel (1, 0, 0),
    # one in voxel (0, 1, 1), one outside
    dims, lo, ih = (2, 2, 2), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    mu = np.array([[1.2, 0.5, 0.1], [1.9, 0.2, 0.7], [0.5, 1.5, 1.5], [2.5, 0.5, 0.5]])
    sc = np.array([[1.0, 1.0, 1.0], [2.0, 2.0, 2.0], [1.0, 2.0, 4.0], [1.0, 1.0, 1.0]])
    vol = np.arange(8.0).reshape(2, 2, 2)
    t = U.targets(mu, sc, dims, lo, ih, vol, 0.5)
    np.testing.assert_allclose(t[..., 0], vol / 0.5)
    assert t[0, 0, 1, 2] == 1 and t[1, 1, 0, 2] == 1 and t[..., 2].sum() == 2
    assert abs(t[0, 0, 1, 1] - 0.5 * np.log(2.0)) < 1e-15     # mean of log 1 and log 2
    assert abs(t[1, 1, 0, 1] - np.log(2.0)) < 1e-15           # log of (1 * 2 * 4)^(1/3)


def test_draw_from_fields_frequencies_and_values():
    # two voxels with occupancy logits giving weights 1/4 and 3/4
    out = np.zeros((1, 1, 2, 3))
    out[0, 0, 0] = (0.3, np.log(2.0), -np.log(3.0))   # sigmoid = 1/4
    out[0, 0, 1] = (-1.0, 10.0, np.log(3.0))          # sigmoid = 3/4, scale clipped to 8
    r = rng(8)
    n = 200000
    uni = r.uniform(size=(n, 4))
    mu, sc, rho, v = U.draw_from_fields(out, (2, 1, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), uni, 0.05)
    frac = np.mean(v == 0)
    assert abs(frac - 0.25) < 4 * np.sqrt(0.25 * 0.75 / n)
    assert np.all(sc[v == 0] == 2.0) and np.all(sc[v == 1] == 8.0)
    assert np.allclose(rho[v == 0], 0.3 * 0.05) and np.all(rho[v == 1] == 0.0)
    assert np.all(np.floor(mu[:, 0]) == v) and np.all((mu[:, 1:] >= 0) & (mu[:, 1:] < 1))
