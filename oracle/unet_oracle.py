"""FP64 oracle of the learned-compounding U-Net.  TEST INFRASTRUCTURE ONLY.

Not an operation of the paper (see the header of ``das_learn.h``): a 3D U-Net
that maps delay-and-sum volumes from 3 plane waves (6 real channels) to the
residual between the many-angle compound and (11/3) x the 3-angle sum.

Layers, channels-last [D, H, W, C] volumes in float64:
  conv3d   3x3x3, stride 1, zero padding; weights [Cout, 27, Cin] with
           tap = (dz+1)*9 + (dy+1)*3 + (dx+1); y[v] = sum_tap x[v+off] W[tap]^T + b
  relu, 2x average pooling, 2x nearest upsampling, channel concatenation
Architecture (channel counts c0..c3 = 16, 32, 48, 64 by default):
  enc l = 0..2: a_l = relu(conv(in_l)), s_l = relu(conv(a_l)), in_{l+1} = pool(s_l)
  bottom:       a_3 = relu(conv(in_3)), b_3 = relu(conv(a_3))
  dec l = 2..0: u = up(prev), c_la = relu(conv([s_l | u])), c_lb = relu(conv(c_la))
  out:          net = conv(c_0b)   (no activation; channels 0 and 1 are used)
  prediction = base + net[..., :2];  loss = mean((prediction - target)^2)
The gradients are the analytic backward pass of these definitions; they are
pinned by finite differences in the tests.

``store`` (default: none) is applied to every tensor at the points where an
implementation keeps it in memory: each activation and pooled tensor in the
forward pass, the loss gradient, and each propagated gradient in the backward
pass (after its ReLU mask).  Passing bfloat16 rounding there gives the exact
values of a network that stores its tensors in bfloat16 and computes in high
precision; ``store=None`` is the plain float64 network.
"""

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(x, dz, dy, dx):
    """s[v] = x[v + (dz, dy, dx)] with zeros outside the volume."""
    D, H, W = x.shape[:3]
    p = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    return p[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W]


def conv3d(x, w, b):
    """x [D,H,W,Cin], w [Cout,27,Cin], b [Cout] -> [D,H,W,Cout] (im2col + matmul)."""
    cols = np.stack([_shift(x, *t) for t in TAPS], axis=3)  # [D,H,W,27,Cin]
    D, H, W = x.shape[:3]
    y = cols.reshape(D * H * W, -1) @ w.reshape(w.shape[0], -1).T + b
    return y.reshape(D, H, W, -1)


def conv3d_backward(x, w, dy):
    """Gradients of conv3d: (dx, dw, db)."""
    D, H, W = x.shape[:3]
    g = dy.reshape(D * H * W, -1)
    cols = np.stack([_shift(x, *t) for t in TAPS], axis=3).reshape(D * H * W, -1)
    dw = (g.T @ cols).reshape(w.shape)
    db = g.sum(axis=0)
    dx = np.zeros_like(x)
    for k, (dz, dyy, dxx) in enumerate(TAPS):
        # y[v] gets x[v + off] W_k^T, so x[u] receives dy[u - off] W_k
        dx += _shift((g @ w[:, k, :]).reshape(D, H, W, -1), -dz, -dyy, -dxx)
    return dx, dw, db


def avgpool2(x):
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def avgpool2_backward(g):
    return np.repeat(np.repeat(np.repeat(g, 2, axis=0), 2, axis=1), 2, axis=2) / 8.0


def upsample2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=0), 2, axis=1), 2, axis=2)


def upsample2_backward(g):
    D, H, W, C = g.shape
    return g.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def layer_shapes(cin=8, chans=(16, 32, 48, 64), cout=16):
    """(name, Cin, Cout) of every convolution, in forward order."""
    c0, c1, c2, c3 = chans
    return [("e0a", cin, c0), ("e0b", c0, c0), ("e1a", c0, c1), ("e1b", c1, c1), ("e2a", c1, c2), ("e2b", c2, c2),
            ("e3a", c2, c3), ("e3b", c3, c3), ("d2a", c2 + c3, c2), ("d2b", c2, c2), ("d1a", c1 + c2, c1),
            ("d1b", c1, c1), ("d0a", c0 + c1, c0), ("d0b", c0, c0), ("out", c0, cout)]


def _identity(a):
    return a


def forward(params, x, store=None):
    """params: {name: (w, b)}; x [D,H,W,Cin].  Returns (net [D,H,W,Cout], cache)."""
    st = store or _identity
    relu = lambda a: np.maximum(a, 0.0)  # noqa: E731
    c = {"x": x}
    h = x
    for l in range(3):
        c["ea%d" % l] = st(relu(conv3d(h, *params["e%da" % l])))
        c["s%d" % l] = st(relu(conv3d(c["ea%d" % l], *params["e%db" % l])))
        c["p%d" % l] = st(avgpool2(c["s%d" % l]))
        h = c["p%d" % l]
    c["ea3"] = st(relu(conv3d(h, *params["e3a"])))
    c["b3"] = st(relu(conv3d(c["ea3"], *params["e3b"])))
    prev = c["b3"]
    for l in (2, 1, 0):
        c["cat%d" % l] = np.concatenate([c["s%d" % l], upsample2(prev)], axis=3)
        c["da%d" % l] = st(relu(conv3d(c["cat%d" % l], *params["d%da" % l])))
        c["db%d" % l] = st(relu(conv3d(c["da%d" % l], *params["d%db" % l])))
        prev = c["db%d" % l]
    net = conv3d(prev, *params["out"])
    return net, c


def loss_and_grad_net(net, base, target):
    """MSE of base + net[..., :2] against target; returns (loss, d loss / d net)."""
    e = base + net[..., :2] - target
    n = e.size
    g = np.zeros_like(net)
    g[..., :2] = 2.0 * e / n
    return float((e ** 2).sum() / n), g


def backward(params, cache, gnet, store=None):
    """Analytic gradients {name: (dw, db)} of the network for d loss / d net = gnet.

    A propagated gradient is stored after the ReLU mask of the tensor it
    belongs to; rounding commutes with a 0/1 mask, so store() may be applied
    before the mask multiplies it."""
    st = store or _identity
    grads = {}
    relu_mask = lambda a: (a > 0).astype(np.float64)  # noqa: E731
    g, grads["out"] = _conv_grads(cache["db0"], params["out"], st(gnet))
    skip_g = {}
    for l in (0, 1, 2):
        g = st(g) * relu_mask(cache["db%d" % l])
        g, grads["d%db" % l] = _conv_grads(cache["da%d" % l], params["d%db" % l], g)
        g = st(g) * relu_mask(cache["da%d" % l])
        g, grads["d%da" % l] = _conv_grads(cache["cat%d" % l], params["d%da" % l], g)
        g = st(g * relu_mask(cache["cat%d" % l]))
        cs = cache["s%d" % l].shape[3]
        skip_g[l] = g[..., :cs]
        g = upsample2_backward(g[..., cs:])
    g = st(g) * relu_mask(cache["b3"])
    g, grads["e3b"] = _conv_grads(cache["ea3"], params["e3b"], g)
    g = st(g) * relu_mask(cache["ea3"])
    g, grads["e3a"] = _conv_grads(cache["p2"], params["e3a"], g)
    for l in (2, 1, 0):
        g = st((skip_g[l] + st(avgpool2_backward(st(g)))) * relu_mask(cache["s%d" % l]))
        g, grads["e%db" % l] = _conv_grads(cache["ea%d" % l], params["e%db" % l], g)
        g = st(g) * relu_mask(cache["ea%d" % l])
        src = cache["p%d" % (l - 1)] if l > 0 else cache["x"]
        g, grads["e%da" % l] = _conv_grads(src, params["e%da" % l], g)
    return grads


def _conv_grads(x, wb, gy):
    dx, dw, db = conv3d_backward(x, wb[0], gy)
    return dx, (dw, db)


def init_params(rng, cin=8, chans=(16, 32, 48, 64), cout=16, out_scale=0.1):
    """He-normal weights, zero biases; the output layer is scaled down so the residual starts small."""
    p = {}
    for name, ci, co in layer_shapes(cin, chans, cout):
        std = np.sqrt(2.0 / (27 * ci)) * (out_scale if name == "out" else 1.0)
        p[name] = (rng.standard_normal((co, 27, ci)) * std, np.zeros(co))
    return p
