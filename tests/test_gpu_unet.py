"""Parity of the learned-initialisation network (bfloat16 matrix-core kernels)
with the binary64 oracle.

Tolerances.  A bfloat16 result rounded to nearest even is within 2^-9
relative of the binary32 accumulator, and the binary32 accumulation of exact
bfloat16 products adds ~sqrt(K) 2^-24, so single layers are held to 2^-8
relative per element (plus a floor of 1e-6 of the largest magnitude).  The
whole network rounds every activation to bfloat16 (7 layers deep), so its
output is held to 3e-2 relative L2 against a binary64 forward on the same
bfloat16-rounded weights.  Its parameter gradients pass through 7 ReLU masks
taken from those slightly different activations: a unit whose pre-activation
lies within the rounding difference of zero switches its mask, and a
fraction p of switched units changes the gradient by ~sqrt(p) in relative L2
(p ~ 3e-3 here gives ~5e-2).  Gradients are therefore held to 1e-1 relative
L2 and a cosine above 0.99 per layer; a wiring mistake (a wrong slice, tap or
mask) gives errors of order one.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import unet as U
from paper_2411_04844_amd import native

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def bf(a):
    """binary64 values of the bfloat16 rounding of a."""
    return torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def elementwise_ok(got, want, rel=2.0 ** -8, floor=1e-6):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    tol = rel * np.abs(want) + floor * np.abs(want).max()
    bad = np.abs(got - want) > tol
    return int(bad.sum()), float(np.max(np.abs(got - want) / (np.abs(want) + 1e-30)))


@pytest.mark.parametrize("shape,cin,cout,xs,off,relu", [
    ((6, 10, 12), 64, 96, 64, 0, True),      # 720 voxels (ragged), 2 x 16-channel tiles
    ((4, 8, 8), 32, 64, 96, 32, False),      # input is a channel slice, 4 x 16-channel tiles
    ((3, 5, 7), 96, 32, 96, 0, True),        # 105 voxels, less than one work-group
])
def test_conv3_forward_parity(shape, cin, cout, xs, off, relu):
    say("conv3 forward", shape, cin, cout, xs, off, relu)
    r = np.random.default_rng(11)
    xfull = bf(r.normal(size=shape + (xs,)))
    W = bf(r.normal(scale=0.1, size=(27, cout, cin)))
    b = r.normal(scale=0.1, size=cout).astype(np.float32)
    xt = torch.as_tensor(xfull).to(torch.bfloat16).cuda()
    x_slice = xt[..., off:] if off else xt
    # the kernel reads channels 0..cin-1 at stride xs from the slice start
    y = torch.zeros(shape + (cout,), dtype=torch.bfloat16, device="cuda")
    wt = torch.as_tensor(W).to(torch.bfloat16).cuda().contiguous()
    bt = torch.as_tensor(b).cuda()
    native._check("dgr_conv3_forward", native.lib().dgr_conv3_forward(
        native.ctypes.c_void_p(x_slice.data_ptr()), xs, native._dims(shape), cin, native._ptr(wt),
        native._ptr(bt), cout, int(relu), native._ptr(y), cout, native._stream()))
    want = U.conv3(xfull[..., off:off + cin], W, b.astype(np.float64))
    if relu:
        want = np.maximum(want, 0.0)
    got = y.float().cpu().numpy()
    nbad, worst = elementwise_ok(got, want)
    say("conv3 forward rel_l2", rel_l2(got, want), "bad", nbad, "worst rel", worst)
    assert nbad == 0


# 26 x 32 x 32 voxels: 13 weight-gradient chunks of voxel tiles, padded to 16
# so that each XCD takes whole chunks (three of the padded chunks exit at once)
@pytest.mark.parametrize("shape,cin,cout", [((6, 10, 12), 64, 96), ((4, 6, 8), 96, 32), ((26, 32, 32), 32, 64)])
def test_conv3_backward_parity(shape, cin, cout):
    say("conv3 backward", shape, cin, cout)
    r = np.random.default_rng(12)
    x = bf(r.normal(size=shape + (cin,)))
    W = r.normal(scale=0.1, size=(27, cout, cin)).astype(np.float32)
    dy = bf(r.normal(size=shape + (cout,)))
    dw, db, dx = native.dgr_conv3_backward(torch.as_tensor(x).to(torch.bfloat16).cuda(), cin,
                                           torch.as_tensor(W).cuda(),
                                           torch.as_tensor(dy).to(torch.bfloat16).cuda())
    dW_ref, db_ref = U.conv3_wgrad(x, dy)
    dx_ref = U.conv3_dgrad(dy, bf(W))
    e_w, e_b = rel_l2(dw.cpu().numpy(), dW_ref), rel_l2(db.cpu().numpy(), db_ref)
    nbad, worst = elementwise_ok(dx.float().cpu().numpy(), dx_ref)
    say("conv3 backward dW", e_w, "db", e_b, "dx bad", nbad, "worst", worst)
    assert e_w < 1e-5 and e_b < 1e-5
    assert nbad == 0


def _net_inputs(D=(16, 16, 16), seed=21):
    r = np.random.default_rng(seed)
    n = U.param_count(32)
    assert native.dgr_unet_param_count() == n
    flat = np.empty(n)
    off = 0
    for name, ci, co in U.layer_shapes(32):
        taps = 1 if name == "head" else 27
        nw = taps * co * ci
        flat[off:off + nw] = r.normal(scale=np.sqrt(2.0 / (taps * ci)), size=nw)  # He initialisation
        flat[off + nw:off + nw + co] = r.normal(scale=0.05, size=co)
        off += nw + co
    flat = flat.astype(np.float32)
    x = r.normal(size=D).astype(np.float32)
    return flat, x


def _oracle_params(flat):
    """The oracle runs on the weights the matrix cores see: conv weights of
    enc2 .. dec1 rounded to bfloat16 (enc1 and the head run in binary32)."""
    f = flat.astype(np.float64).copy()
    P = U.unpack(f, 32)
    for name in ("enc2", "enc3", "bott", "dec3", "dec2", "dec1"):
        P[name][0][...] = bf(P[name][0])
    return f


def test_unet_forward_backward_parity():
    say("unet forward/backward 16^3")
    flat, x = _net_inputs()
    r = np.random.default_rng(22)
    dout = r.normal(size=x.shape + (3,)).astype(np.float32)
    pt, xt = torch.as_tensor(flat).cuda(), torch.as_tensor(x).cuda()
    ws = native.Workspace()
    out = native.dgr_unet_forward(pt, xt, ws=ws)
    grad = native.dgr_unet_backward(pt, xt, torch.as_tensor(dout).cuda(), ws)
    torch.cuda.synchronize()
    fo = _oracle_params(flat)
    want, cache = U.forward(fo, x, 32)
    e_out = rel_l2(out.cpu().numpy(), want)
    g_ref = U.backward(fo, cache, dout.astype(np.float64), 32)
    g = grad.cpu().numpy()
    errs, off = {}, 0
    for name, ci, co in U.layer_shapes(32):
        taps = 1 if name == "head" else 27
        nw = taps * co * ci
        a, b = g[off:off + nw + co], g_ref[off:off + nw + co]
        errs[name] = (rel_l2(g[off:off + nw], g_ref[off:off + nw]),
                      rel_l2(g[off + nw:off + nw + co], g_ref[off + nw:off + nw + co]),
                      float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b))))
        off += nw + co
    say("unet out rel_l2", e_out)
    for k, v in errs.items():
        say(f"unet grad {k}: W {v[0]:.3e} b {v[1]:.3e} cos {v[2]:.6f}")
    assert e_out < 3e-2
    for k, (ew, eb, cos) in errs.items():
        assert ew < 1e-1 and eb < 1e-1 and cos > 0.99, k


def test_unet_loss_parity():
    say("unet loss")
    r = np.random.default_rng(23)
    out = r.normal(size=(8, 8, 16, 3)).astype(np.float32)
    tgt = np.stack([r.normal(size=(8, 8, 16)), r.normal(size=(8, 8, 16)), r.uniform(size=(8, 8, 16))],
                   axis=-1).astype(np.float32)
    L, d = native.dgr_unet_loss(torch.as_tensor(out).cuda(), torch.as_tensor(tgt).cuda())
    Lr, dr = U.loss(out.astype(np.float64), tgt[..., 0].astype(np.float64), tgt[..., 1].astype(np.float64),
                    tgt[..., 2].astype(np.float64))
    say("loss", float(L), Lr, "grad rel_l2", rel_l2(d.cpu().numpy(), dr))
    assert abs(float(L) - Lr) < 1e-5 * abs(Lr)
    assert rel_l2(d.cpu().numpy(), dr) < 1e-6


def test_unet_training_reduces_loss():
    """A few Adam steps on one fixed 16^3 example lower the loss (the network's
    gradient points downhill through the matrix-core backward pass)."""
    say("unet training sanity")
    flat, x = _net_inputs(seed=24)
    r = np.random.default_rng(25)
    tgt = np.stack([np.tanh(x), 0.5 * np.ones_like(x), (x > 0).astype(np.float32)], axis=-1).astype(np.float32)
    pt, xt, tt = (torch.as_tensor(a).cuda() for a in (flat, x, tgt))
    m, v = torch.zeros_like(pt), torch.zeros_like(pt)
    ws, lws = native.Workspace(), native.Workspace()
    losses = []
    for step in range(1, 41):
        out = native.dgr_unet_forward(pt, xt, ws=ws)
        L, d = native.dgr_unet_loss(out, tt, ws=lws)
        g = native.dgr_unet_backward(pt, xt, d, ws)
        native.dgr_adam(pt, g, m, v, 1e-3, step)
        losses.append(float(L))
    say("unet training losses", losses[0], losses[9], losses[-1])
    assert losses[-1] < 0.5 * losses[0]
