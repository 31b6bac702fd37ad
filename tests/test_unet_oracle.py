"""Pins of the FP64 U-Net oracle (learned compounding) on the CPU.

The convolution is checked against direct loops and an independent library
routine (scipy's N-d correlation); every backward formula and the whole
network's gradient are checked by central finite differences; pooling and
upsampling against their adjoint identities.
"""

import numpy as np
import pytest
from scipy import signal

from oracle import unet_oracle as U


def _direct_conv(x, w, b):
    D, H, W, _ = x.shape
    y = np.zeros((D, H, W, w.shape[0]))
    for d in range(D):
        for h in range(H):
            for ww in range(W):
                for k, (dz, dy, dx) in enumerate(U.TAPS):
                    z, yy, xx = d + dz, h + dy, ww + dx
                    if 0 <= z < D and 0 <= yy < H and 0 <= xx < W:
                        y[d, h, ww] += w[:, k, :] @ x[z, yy, xx]
    return y + b


def test_conv3d_matches_direct_loops():
    r = np.random.default_rng(0)
    x = r.standard_normal((4, 3, 5, 3))
    w = r.standard_normal((2, 27, 3))
    b = r.standard_normal(2)
    np.testing.assert_allclose(U.conv3d(x, w, b), _direct_conv(x, w, b), rtol=1e-12, atol=1e-12)


def test_conv3d_matches_scipy_correlate():
    r = np.random.default_rng(1)
    x = r.standard_normal((6, 5, 7, 1))
    k = r.standard_normal((3, 3, 3))
    w = k.reshape(1, 27, 1)  # tap order (dz, dy, dx) row-major == kernel[dz+1, dy+1, dx+1]
    ref = signal.correlate(x[..., 0], k, mode="same")
    np.testing.assert_allclose(U.conv3d(x, w, np.zeros(1))[..., 0], ref, rtol=1e-12, atol=1e-12)


def _fd(f, x, idx, h=1e-6):
    xp = x.copy()
    xm = x.copy()
    xp[idx] += h
    xm[idx] -= h
    return (f(xp) - f(xm)) / (2 * h)


def test_conv3d_backward_by_finite_differences():
    r = np.random.default_rng(2)
    x = r.standard_normal((3, 4, 3, 2))
    w = r.standard_normal((3, 27, 2))
    b = r.standard_normal(3)
    gy = r.standard_normal((3, 4, 3, 3))
    dx, dw, db = U.conv3d_backward(x, w, gy)
    L = lambda xx, ww, bb: float((U.conv3d(xx, ww, bb) * gy).sum())  # noqa: E731
    for idx in [(0, 0, 0, 0), (2, 3, 2, 1), (1, 2, 1, 0)]:
        assert dx[idx] == pytest.approx(_fd(lambda t: L(t, w, b), x, idx), rel=1e-6, abs=1e-8)
    for idx in [(0, 0, 0), (2, 26, 1), (1, 13, 0)]:
        assert dw[idx] == pytest.approx(_fd(lambda t: L(x, t, b), w, idx), rel=1e-6, abs=1e-8)
    for i in range(3):
        assert db[i] == pytest.approx(_fd(lambda t: L(x, w, t), b, (i,)), rel=1e-6, abs=1e-8)


def test_pool_and_upsample_adjoints():
    r = np.random.default_rng(3)
    x = r.standard_normal((4, 6, 2, 3))
    y = r.standard_normal((2, 3, 1, 3))
    assert np.isclose((U.avgpool2(x) * y).sum(), (x * U.avgpool2_backward(y)).sum())
    assert np.isclose((U.upsample2(y) * x).sum(), (y * U.upsample2_backward(x)).sum())
    np.testing.assert_allclose(U.avgpool2(U.upsample2(y)), y)


def _stable_fd(f, x, idx):
    """Central difference at two step sizes; None when they disagree (a ReLU kink inside the step)."""
    a, b = _fd(f, x, idx, h=1e-5), _fd(f, x, idx, h=1e-6)
    return a if abs(a - b) <= 1e-6 * max(abs(a), 1e-3) + 1e-9 else None


def test_unet_gradient_by_finite_differences():
    r = np.random.default_rng(4)
    chans = (8, 8, 16, 16)
    params = U.init_params(r, cin=8, chans=chans, cout=16, out_scale=1.0)
    params = {k: (w, r.standard_normal(b.shape) * 0.1) for k, (w, b) in params.items()}
    x = r.standard_normal((8, 8, 8, 8))
    base = r.standard_normal((8, 8, 8, 2))
    target = r.standard_normal((8, 8, 8, 2))

    def loss(p):
        net, _ = U.forward(p, x)
        return U.loss_and_grad_net(net, base, target)[0]

    net, cache = U.forward(params, x)
    _, gnet = U.loss_and_grad_net(net, base, target)
    grads = U.backward(params, cache, gnet)
    assert set(grads) == set(params)
    checked = nonzero = 0
    for name in [n for n, _, _ in U.layer_shapes(8, chans, 16)]:
        w, b = params[name]
        co = 2 if name == "out" else w.shape[0]  # only output channels 0, 1 enter the loss
        for _ in range(4):
            idx = (int(r.integers(0, co)), int(r.integers(0, 27)), int(r.integers(0, w.shape[2])))

            def lw(t, name=name):
                q = dict(params)
                q[name] = (t, params[name][1])
                return loss(q)
            num = _stable_fd(lw, w, idx)
            if num is None:
                continue
            assert grads[name][0][idx] == pytest.approx(num, rel=1e-5, abs=1e-9), (name, idx)
            checked += 1
            nonzero += abs(num) > 1e-7
        i = int(r.integers(0, co))

        def lb(t, name=name):
            q = dict(params)
            q[name] = (params[name][0], t)
            return loss(q)
        num = _stable_fd(lb, b, (i,))
        if num is not None:
            assert grads[name][1][i] == pytest.approx(num, rel=1e-5, abs=1e-9), (name, i)
    assert checked >= 45 and nonzero >= 25


def test_storage_hook_identity_and_bf16_sensitivity():
    """store=None is the plain network; storing every tensor in bfloat16 moves the gradients by a few per
    cent on a 16^3 volume but keeps cosine >= 0.99 per layer (the end-to-end bound the GPU test uses)."""
    import torch

    def bf16(a):
        return torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float32).numpy().astype(
            np.float64)
    r = np.random.default_rng(21)
    params = U.init_params(np.random.default_rng(5), out_scale=1.0)
    params = {k: (bf16(w), r.standard_normal(b.shape) * 0.05) for k, (w, b) in params.items()}
    x = bf16(r.standard_normal((16, 16, 16, 8)))
    base, tgt = r.standard_normal((16, 16, 16, 2)), r.standard_normal((16, 16, 16, 2))
    n0, c0 = U.forward(params, x)
    n1, _ = U.forward(params, x, store=lambda a: a)
    np.testing.assert_array_equal(n0, n1)
    g0 = U.backward(params, c0, U.loss_and_grad_net(n0, base, tgt)[1])
    nb, cb = U.forward(params, x, store=bf16)
    gb = U.backward(params, cb, U.loss_and_grad_net(nb, base, tgt)[1], store=bf16)
    assert np.linalg.norm(nb - n0) / np.linalg.norm(n0) < 1e-2
    worst = 1.0
    for name in g0:
        a, b = gb[name][0].ravel(), g0[name][0].ravel()
        worst = min(worst, float(a @ b / np.linalg.norm(a) / np.linalg.norm(b)))
    assert 0.99 <= worst < 0.9999  # visibly moved, still aligned
