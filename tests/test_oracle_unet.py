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
