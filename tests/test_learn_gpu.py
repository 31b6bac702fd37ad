"""GPU parity of the learned-compounding kernels (das_learn.h) against the FP64 U-Net oracle.

Inputs are rounded to bfloat16 first and the oracle runs in float64 on those
rounded values, so the comparisons measure the kernels' own arithmetic:
FP32-accumulated convolutions (relative error ~1e-6 before the output
rounding), bfloat16 activations and gradients (2^-9 relative per rounding).
The whole network's gradients must reach cosine >= 0.999 and relative L2
<= 1e-2 per layer against the float64 backward pass taken at the same stored
forward tensors.
"""

import numpy as np
import pytest
import torch

from oracle import unet_oracle as U

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _learn():
    from paper_2604_06257_amd import learn
    return learn


def bf16_round(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float32).numpy().astype(
        np.float64)


def to_dev_bf16(a):
    """[D,H,W,C] or [V,C] numpy -> contiguous bfloat16 [V, C] on the GPU."""
    a = np.asarray(a)
    return torch.as_tensor(a.reshape(-1, a.shape[-1]).astype(np.float32)).to(torch.bfloat16).to(DEV).contiguous()


def host(t):
    return t.float().cpu().numpy().astype(np.float64)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def cosine(a, b):
    a, b = a.ravel(), b.ravel()
    return float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))


CONV_CASES = [  # (D, H, W, Cin, Cout, relu)
    (4, 4, 4, 8, 16, False),
    (5, 7, 9, 16, 32, True),     # ragged: V = 315 is not a multiple of 16
    (3, 6, 5, 48, 16, True),
    (6, 4, 6, 112, 48, False),
    (4, 4, 4, 64, 128, True),
    (1, 1, 3, 8, 16, False),     # fewer voxels than one wave tile
]


@pytest.mark.parametrize("D,H,W,cin,cout,relu", CONV_CASES)
def test_conv3d_forward_matches_oracle(D, H, W, cin, cout, relu):
    L = _learn()
    r = np.random.default_rng(100 + cin + cout + D)
    x = bf16_round(r.standard_normal((D, H, W, cin)))
    w = bf16_round(r.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin))
    b = r.standard_normal(cout).astype(np.float32).astype(np.float64)
    ref = U.conv3d(x, w, b)
    if relu:
        ref = np.maximum(ref, 0.0)
    out = torch.full((D * H * W, cout), 7.0, dtype=torch.float32, device=DEV)
    L.conv3d(to_dev_bf16(x), to_dev_bf16(w.reshape(cout, -1)).reshape(-1),
             torch.as_tensor(b, dtype=torch.float32, device=DEV), out, (D, H, W), relu=relu)
    got = host(out).reshape(ref.shape)
    np.testing.assert_allclose(got, ref, rtol=2e-5, atol=2e-5 * np.abs(ref).max())
    # bfloat16 output: the same values rounded to nearest even
    outb = torch.zeros((D * H * W, cout), dtype=torch.bfloat16, device=DEV)
    L.conv3d(to_dev_bf16(x), to_dev_bf16(w.reshape(cout, -1)).reshape(-1),
             torch.as_tensor(b, dtype=torch.float32, device=DEV), outb, (D, H, W), relu=relu)
    np.testing.assert_allclose(host(outb).reshape(ref.shape), bf16_round(got.reshape(ref.shape)), rtol=1e-2,
                               atol=1e-6 * np.abs(ref).max())
    assert np.mean(host(outb).reshape(ref.shape) == bf16_round(got.reshape(ref.shape))) > 0.99


def test_conv3d_slices_mask_and_flip_match_oracle():
    """Input and output as channel slices of wider buffers, a ReLU mask, and the flipped (input-gradient) form."""
    L = _learn()
    D, H, W, cin, cout = 4, 5, 6, 16, 32
    r = np.random.default_rng(7)
    wide = bf16_round(r.standard_normal((D, H, W, 40)))
    x = wide[..., 8:24]
    w = bf16_round(r.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin))
    maskv = bf16_round(np.maximum(r.standard_normal((D, H, W, 48)), 0.0))
    # forward with mask on a slice of a wider output buffer
    out = torch.full((D * H * W, 64), -3.0, dtype=torch.float32, device=DEV)
    L.conv3d(L.Slice(to_dev_bf16(wide), 8, cin), to_dev_bf16(w.reshape(cout, -1)).reshape(-1), None,
             L.Slice(out, 16, cout), (D, H, W), mask=L.Slice(to_dev_bf16(maskv), 16, cout))
    ref = U.conv3d(x, w, np.zeros(cout)) * (maskv[..., 16:48] > 0)
    got = host(out).reshape(D, H, W, 64)
    np.testing.assert_allclose(got[..., 16:48], ref, rtol=2e-5, atol=2e-5 * np.abs(ref).max())
    assert np.all(got[..., :16] == -3.0) and np.all(got[..., 48:] == -3.0)
    # flipped convolution with transposed weights == the oracle's input gradient
    gy = bf16_round(r.standard_normal((D, H, W, cout)))
    wt = torch.zeros(cout * 27 * cin, dtype=torch.bfloat16, device=DEV)
    L.transpose_weights(to_dev_bf16(w.reshape(cout, -1)).reshape(-1), wt, cin, cout)
    np.testing.assert_array_equal(host(wt).reshape(cin, 27, cout), w.transpose(2, 1, 0))
    dx = torch.zeros((D * H * W, cin), dtype=torch.float32, device=DEV)
    L.conv3d(to_dev_bf16(gy), wt, None, dx, (D, H, W), flip=True)
    ref_dx = U.conv3d_backward(x, w, gy)[0]
    np.testing.assert_allclose(host(dx).reshape(ref_dx.shape), ref_dx, rtol=2e-5, atol=2e-5 * np.abs(ref_dx).max())


def test_conv3d_unaligned_output_and_mask_slices():
    """Output and mask slices whose channel offset or row stride is not a multiple of 16 bytes take the
    epilogue's element-by-element stores: the same values as the oracle (float32 and bfloat16 output)."""
    L = _learn()
    D, H, W, cin, cout = 3, 9, 10, 16, 16
    r = np.random.default_rng(11)
    x = bf16_round(r.standard_normal((D, H, W, cin)))
    w = bf16_round(r.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin))
    b = r.standard_normal(cout).astype(np.float32).astype(np.float64)
    maskv = bf16_round(np.maximum(r.standard_normal((D, H, W, 21)), 0.0))  # stride 21, offset 3
    ref = np.maximum(U.conv3d(x, w, b), 0.0) * (maskv[..., 3:19] > 0)
    wd, bd = to_dev_bf16(w.reshape(cout, -1)).reshape(-1), torch.as_tensor(b, dtype=torch.float32, device=DEV)
    out = torch.full((D * H * W, 19), -5.0, dtype=torch.float32, device=DEV)  # float32: stride 19, offset 2
    L.conv3d(to_dev_bf16(x), wd, bd, L.Slice(out, 2, cout), (D, H, W), relu=True,
             mask=L.Slice(to_dev_bf16(maskv), 3, cout))
    got = host(out).reshape(D, H, W, 19)
    np.testing.assert_allclose(got[..., 2:18], ref, rtol=2e-5, atol=2e-5 * np.abs(ref).max())
    assert np.all(got[..., :2] == -5.0) and np.all(got[..., 18:] == -5.0)
    outb = torch.zeros((D * H * W, 20), dtype=torch.bfloat16, device=DEV)  # bfloat16: offset 4 (8 bytes)
    L.conv3d(to_dev_bf16(x), wd, bd, L.Slice(outb, 4, cout), (D, H, W), relu=True,
             mask=L.Slice(to_dev_bf16(maskv), 3, cout))
    gb = host(outb).reshape(D, H, W, 20)
    np.testing.assert_allclose(gb[..., 4:20], bf16_round(got[..., 2:18]), rtol=1e-2, atol=1e-6 * np.abs(ref).max())
    assert np.all(gb[..., :4] == 0.0)


@pytest.mark.parametrize("D,H,W,cin,cout,chunk", [(4, 4, 4, 8, 16, 32), (5, 7, 9, 16, 32, 64),
                                                  (6, 6, 6, 48, 16, 32), (4, 4, 4, 112, 48, 96),
                                                  (8, 8, 8, 64, 64, 512)])
def test_conv3d_wgrad_matches_oracle(D, H, W, cin, cout, chunk):
    L = _learn()
    r = np.random.default_rng(200 + cin + cout)
    x = bf16_round(r.standard_normal((D, H, W, cin)))
    gy = bf16_round(r.standard_normal((D, H, W, cout)))
    _, dw_ref, db_ref = U.conv3d_backward(x, np.zeros((cout, 27, cin)), gy)
    dw = torch.zeros(cout * 27 * cin, dtype=torch.float32, device=DEV)
    db = torch.zeros(cout, dtype=torch.float32, device=DEV)
    work = torch.zeros(L.wgrad_work_floats((D, H, W), cin, cout, chunk), dtype=torch.float32, device=DEV)
    L.conv3d_wgrad(to_dev_bf16(x), to_dev_bf16(gy), dw, db, work, (D, H, W), chunk)
    np.testing.assert_allclose(host(dw).reshape(dw_ref.shape), dw_ref, rtol=1e-4, atol=1e-5 * np.abs(dw_ref).max())
    np.testing.assert_allclose(host(db), db_ref, rtol=1e-4, atol=1e-5 * np.abs(db_ref).max())
    # deterministic: a second call gives identical bits
    dw2 = torch.zeros_like(dw)
    L.conv3d_wgrad(to_dev_bf16(x), to_dev_bf16(gy), dw2, db, work, (D, H, W), chunk)
    assert torch.equal(dw, dw2)


@pytest.mark.parametrize("Di,Hi,Wi,c", [(6, 4, 8, 16), (6, 4, 8, 12), (10, 6, 14, 16), (10, 6, 14, 24)])
def test_pool_upsample_and_masks_match_oracle(Di, Hi, Wi, c):
    """Channel counts that are multiples of 8 take the 16-byte vector kernels, others the scalar ones; the
    10 x 6 x 14 volume leaves partial blocks along W and H."""
    L = _learn()
    r = np.random.default_rng(9 + c)
    x = bf16_round(r.standard_normal((Di, Hi, Wi, c)))
    g = bf16_round(r.standard_normal((Di // 2, Hi // 2, Wi // 2, c)))
    dims_o = (Di // 2, Hi // 2, Wi // 2)
    p = torch.zeros((Di * Hi * Wi // 8, c), dtype=torch.bfloat16, device=DEV)
    L.avgpool2(to_dev_bf16(x), p, dims_o)
    np.testing.assert_allclose(host(p).reshape(g.shape), bf16_round(U.avgpool2(x)), rtol=1e-2, atol=1e-6)
    gi = torch.zeros((Di * Hi * Wi, c), dtype=torch.bfloat16, device=DEV)
    L.avgpool2_bwd(to_dev_bf16(g), gi, (Di, Hi, Wi))
    np.testing.assert_array_equal(host(gi).reshape(x.shape), U.avgpool2_backward(g))  # exact: x / 8
    prev = host(gi).reshape(x.shape)
    L.avgpool2_bwd(to_dev_bf16(g), gi, (Di, Hi, Wi), accumulate=True)
    np.testing.assert_array_equal(host(gi).reshape(x.shape), bf16_round(2 * prev))
    # upsample into a channel slice, and its masked gradient
    u = torch.zeros((Di * Hi * Wi, c + 8), dtype=torch.bfloat16, device=DEV)
    L.upsample2(to_dev_bf16(g), L.Slice(u, 8, c), (Di, Hi, Wi))
    np.testing.assert_array_equal(host(u)[:, 8:].reshape(x.shape), U.upsample2(g))
    assert not host(u)[:, :8].any()
    mask = bf16_round(np.maximum(r.standard_normal(g.shape), 0))
    gu = torch.zeros((Di * Hi * Wi // 8, c), dtype=torch.bfloat16, device=DEV)
    L.upsample2_bwd(to_dev_bf16(x), gu, dims_o, mask=to_dev_bf16(mask))
    np.testing.assert_allclose(host(gu).reshape(g.shape), bf16_round(U.upsample2_backward(x) * (mask > 0)),
                               rtol=1e-2, atol=1e-2)
    # add_mask
    a, b2, m = (bf16_round(r.standard_normal((50, c))) for _ in range(3))
    out = torch.zeros((50, c), dtype=torch.bfloat16, device=DEV)
    L.add_mask(to_dev_bf16(a), to_dev_bf16(b2), to_dev_bf16(m), out)
    np.testing.assert_allclose(host(out), bf16_round((a + b2) * (m > 0)), rtol=0, atol=0)


def test_mse_and_adam_match_definitions():
    L = _learn()
    r = np.random.default_rng(11)
    V, C = 1000, 16
    net = r.standard_normal((V, C)).astype(np.float32)
    base = r.standard_normal((V, 2)).astype(np.float32)
    tgt = r.standard_normal((V, 2)).astype(np.float32)
    grad = torch.full((V, C), 5.0, dtype=torch.bfloat16, device=DEV)
    pred = torch.zeros((V, 2), dtype=torch.float32, device=DEV)
    parts = L.mse_residual(torch.as_tensor(net, device=DEV), torch.as_tensor(base, device=DEV),
                           torch.as_tensor(tgt, device=DEV), grad, pred)
    loss_ref, g_ref = U.loss_and_grad_net(net[None, None].astype(np.float64), base[None, None].astype(np.float64),
                                          tgt[None, None].astype(np.float64))
    assert float(host(parts).sum()) / (2 * V) == pytest.approx(loss_ref, rel=1e-5)
    np.testing.assert_allclose(host(grad), bf16_round(g_ref[0, 0]), rtol=1e-2, atol=1e-9)
    np.testing.assert_allclose(host(pred), base.astype(np.float64) + net[:, :2], rtol=1e-6)
    # Adam (Kingma & Ba, Algorithm 1) with bias correction, three steps, float64 reference
    n = 777
    w = r.standard_normal(n)
    m = np.zeros(n)
    v = np.zeros(n)
    wd = torch.as_tensor(w, dtype=torch.float32, device=DEV)
    md, vd = torch.zeros(n, device=DEV), torch.zeros(n, device=DEV)
    wb = torch.zeros(n, dtype=torch.bfloat16, device=DEV)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    w = wd.double().cpu().numpy()
    for t in range(1, 4):
        g = r.standard_normal(n).astype(np.float32)
        L.adam(wd, md, vd, torch.as_tensor(g, device=DEV), wb, lr, t, b1, b2, eps)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g.astype(np.float64) ** 2
        w = w - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    np.testing.assert_allclose(host(wd), w, rtol=1e-5, atol=1e-6)
    np.testing.assert_array_equal(host(wb), bf16_round(host(wd)))


def _oracle_params(net_obj):
    return {k: (w.astype(np.float64), b.astype(np.float64)) for k, (w, b) in net_obj.get_params().items()}


def _gpu_cache(net, x, dims):
    """The network's stored forward tensors (bfloat16 values) in the oracle's cache layout."""
    c = net.chans
    D, H, W = dims

    def sh(l, ch):
        return (D >> l, H >> l, W >> l, ch)
    cache = {"x": x}
    for l in range(3):
        cache["ea%d" % l] = host(net.ea[l]).reshape(sh(l, c[l]))
        cache["cat%d" % l] = host(net.cat[l]).reshape(sh(l, c[l] + c[l + 1]))
        cache["s%d" % l] = cache["cat%d" % l][..., :c[l]]
        cache["p%d" % l] = host(net.pool[l]).reshape(sh(l + 1, c[l]))
        cache["da%d" % l] = host(net.da[l]).reshape(sh(l, c[l]))
        cache["db%d" % l] = host(net.db[l]).reshape(sh(l, c[l]))
    cache["ea3"] = host(net.ea[3]).reshape(sh(3, c[3]))
    cache["b3"] = host(net.b3).reshape(sh(3, c[3]))
    return cache


# (layer, input tensor, output tensor) of every convolution but the last
_LOCAL = [("e0a", "x", "ea0"), ("e0b", "ea0", "s0"), ("e1a", "p0", "ea1"), ("e1b", "ea1", "s1"), ("e2a", "p1", "ea2"),
          ("e2b", "ea2", "s2"), ("e3a", "p2", "ea3"), ("e3b", "ea3", "b3"), ("d2a", "cat2", "da2"),
          ("d2b", "da2", "db2"), ("d1a", "cat1", "da1"), ("d1b", "da1", "db1"), ("d0a", "cat0", "da0"),
          ("d0b", "da0", "db0")]


@pytest.mark.parametrize("dims,chans", [((16, 16, 16), (16, 32, 48, 64)), ((8, 16, 24), (16, 16, 32, 32))])
def test_unet_forward_and_gradients_match_oracle(dims, chans):
    """Forward: every layer reproduces the oracle layer on the same stored input (bfloat16 rounding of
    the float64 result, identical in >= 99.9 % of the elements), pooling and upsampling exactly, and the
    network output is within 1e-2 of the plain float64 network.  Backward: with the same stored forward
    tensors, every weight and bias gradient has cosine >= 0.999 and relative L2 <= 1e-2 against the
    float64 backward pass.  End to end against the plain float64 oracle, the bfloat16 storage itself
    moves the deepest layers' gradients by a few per cent (an oracle that only rounds its stored
    tensors does the same), so there the bound is cosine >= 0.99."""
    L = _learn()
    D, H, W = dims
    r = np.random.default_rng(21)
    net = L.UNet(dims, cin=8, chans=chans, cout=16)
    net.init_params(seed=5, out_scale=1.0)
    # random biases so that ReLU masks are not trivially aligned with zero
    p = net.get_params()
    p = {k: (w, r.standard_normal(b.shape).astype(np.float32) * 0.05) for k, (w, b) in p.items()}
    net.set_params(p)
    # the kernels read bfloat16 weights: the oracle gets the same rounded values
    params = {k: (bf16_round(w), b.astype(np.float32).astype(np.float64)) for k, (w, b) in p.items()}
    x = bf16_round(r.standard_normal((D, H, W, 8)))
    base = r.standard_normal((D, H, W, 2)).astype(np.float32)
    tgt = r.standard_normal((D, H, W, 2)).astype(np.float32)
    b64, t64 = base.astype(np.float64), tgt.astype(np.float64)
    xd = to_dev_bf16(x)
    got = host(net.forward(xd)).reshape(D, H, W, 16)
    parts = net.loss(torch.as_tensor(base.reshape(-1, 2), device=DEV), torch.as_tensor(tgt.reshape(-1, 2), device=DEV))
    net.backward(xd)
    grads = net.get_grads()
    gc = _gpu_cache(net, x, dims)
    # forward, layer by layer on the GPU's own inputs
    for name, src, dst in _LOCAL:
        y = bf16_round(np.maximum(U.conv3d(gc[src], *params[name]), 0.0))
        assert np.mean(gc[dst] == y) >= 0.999 and rel_l2(gc[dst], y) <= 1e-3, name  # rare one-ulp ties
    for l in range(3):
        np.testing.assert_array_equal(gc["p%d" % l], bf16_round(U.avgpool2(gc["s%d" % l])))
        up = gc["db%d" % (l + 1)] if l < 2 else gc["b3"]
        np.testing.assert_array_equal(gc["cat%d" % l][..., chans[l]:], U.upsample2(up))
    y = U.conv3d(gc["db0"], *params["out"])
    assert rel_l2(got, y) <= 1e-5
    ref_net, cache = U.forward(params, x)
    assert cosine(got, ref_net) > 0.9999 and rel_l2(got, ref_net) < 1e-2
    # backward given the same forward tensors
    loss_g, gnet = U.loss_and_grad_net(got, b64, t64)
    assert float(host(parts).sum()) / (2 * net.V[0]) == pytest.approx(loss_g, rel=1e-5)
    ref = U.backward(params, gc, gnet)
    # end to end against the plain float64 network
    _, gnet0 = U.loss_and_grad_net(ref_net, b64, t64)
    ref0 = U.backward(params, cache, gnet0)
    for name in ref:
        for i, what in enumerate(("w", "b")):
            g = grads[name][i].astype(np.float64).reshape(ref[name][i].shape)
            c, e = cosine(g, ref[name][i]), rel_l2(g, ref[name][i])
            c0, e0 = cosine(g, ref0[name][i]), rel_l2(g, ref0[name][i])
            print("%s.%s same-state cos %.6f relL2 %.2e | end-to-end cos %.5f relL2 %.2e" % (name, what, c, e, c0, e0))
            assert c >= 0.999 and e <= 1e-2, (name, what, c, e)
            assert c0 >= 0.99, (name, what, c0)


@pytest.mark.parametrize("dims", [(48, 48, 48), (40, 48, 64)])
def test_unet_gradients_match_independent_bf16_oracle(dims):
    """The network's weight and bias gradients against the FP64 oracle network run from the inputs alone (no
    tensor taken from the GPU).  The oracle stores its activations and propagated gradients rounded to bfloat16
    at the points where the kernels store theirs, so both compute the same function.

    Bound: cosine >= 0.999 and relative L2 <= 2e-2 for every layer.  A network that stores bfloat16 tensors
    is sensitive to the accumulation precision: where an FP32 and an FP64 sum round to neighbouring bfloat16
    values the difference propagates, and a ReLU decision can change.  The same oracle run with FP32
    accumulation (the yardstick computed here) differs from the FP64 one by up to 1.9e-2 relL2 at 48^3 and
    3.3e-2 at 32^3 in the deepest layers, so relL2 <= 1e-2 end to end is below the floor that any FP32
    implementation of this network meets (measured on the GPU test inputs: GPU 1.16e-2 and yardstick 1.07e-2
    at 48^3, 8.9e-3 and 7.1e-3 at 40 x 48 x 64).  The GPU's worst layer must stay within twice the
    yardstick's worst layer (and 1e-2), and every layer within 2e-2.  Given the same stored forward tensors
    (the test above) the bound is relL2 <= 1e-2."""
    L = _learn()
    D, H, W = dims
    chans = (16, 32, 48, 64)
    r = np.random.default_rng(51)
    net = L.UNet(dims, cin=8, chans=chans, cout=16)
    net.init_params(seed=7, out_scale=1.0)
    p = {k: (w, r.standard_normal(b.shape).astype(np.float32) * 0.05) for k, (w, b) in net.get_params().items()}
    net.set_params(p)
    params = {k: (bf16_round(w), b.astype(np.float32).astype(np.float64)) for k, (w, b) in p.items()}
    x = bf16_round(r.standard_normal((D, H, W, 8)))
    base = r.standard_normal((D, H, W, 2)).astype(np.float32)
    tgt = r.standard_normal((D, H, W, 2)).astype(np.float32)
    got = host(net.forward(to_dev_bf16(x))).reshape(D, H, W, 16)
    net.loss(torch.as_tensor(base.reshape(-1, 2), device=DEV), torch.as_tensor(tgt.reshape(-1, 2), device=DEV))
    net.backward(to_dev_bf16(x))
    grads = net.get_grads()
    ref_net, cache = U.forward(params, x, store=bf16_round)
    assert cosine(got, ref_net) > 0.9999 and rel_l2(got, ref_net) < 1e-2
    _, gnet = U.loss_and_grad_net(ref_net, base.astype(np.float64), tgt.astype(np.float64))
    ref = U.backward(params, cache, gnet, store=bf16_round)
    # yardstick: the same definition accumulated in float32
    st32 = lambda a: bf16_round(a).astype(np.float32)  # noqa: E731
    p32 = {k: (w.astype(np.float32), b.astype(np.float32)) for k, (w, b) in params.items()}
    net32, cache32 = U.forward(p32, x.astype(np.float32), store=st32)
    _, gnet32 = U.loss_and_grad_net(net32.astype(np.float64), base.astype(np.float64), tgt.astype(np.float64))
    ref32 = U.backward(p32, cache32, gnet32.astype(np.float32), store=st32)
    worst, worst32 = (1.0, 0.0), 0.0
    for name in ref:
        for i, what in enumerate(("w", "b")):
            g = grads[name][i].astype(np.float64).reshape(ref[name][i].shape)
            c, e = cosine(g, ref[name][i]), rel_l2(g, ref[name][i])
            e32 = rel_l2(ref32[name][i].astype(np.float64), ref[name][i])
            worst, worst32 = (min(worst[0], c), max(worst[1], e)), max(worst32, e32)
            print("%s.%s vs independent bf16-store FP64 oracle: GPU cos %.6f relL2 %.2e | FP32 yardstick relL2 %.2e"
                  % (name, what, c, e, e32))
            assert c >= 0.999 and e <= 2e-2, (name, what, c, e)
    print("worst over layers: GPU cos %.6f relL2 %.2e | FP32 yardstick relL2 %.2e" % (worst + (worst32,)))
    assert worst[1] <= 2.0 * max(5e-3, worst32)


def test_unet_training_reduces_loss_deterministically():
    """Adam on one fixed batch: within 100 steps the loss falls below 0.6 of its first value, and two identical
    runs give identical weights."""
    L = _learn()
    dims = (16, 16, 16)
    r = np.random.default_rng(31)
    x = to_dev_bf16(r.standard_normal((16 ** 3, 8)))
    base = torch.as_tensor(r.standard_normal((16 ** 3, 2)).astype(np.float32), device=DEV)
    # a target the network can fit: a smooth function of the input channels
    xs = host(x).reshape(16, 16, 16, 8)
    tgt_np = base.cpu().numpy().reshape(16, 16, 16, 2) + 0.5 * np.tanh(xs[..., :2] + xs[..., 2:4])
    tgt = torch.as_tensor(tgt_np.reshape(-1, 2).astype(np.float32), device=DEV)
    finals = []
    for _ in range(2):
        net = L.UNet(dims)
        net.init_params(seed=3)
        losses = []
        for _ in range(100):
            parts = net.train_step(x, base, tgt, lr=2e-3)
            losses.append(float(parts.sum()) / (2 * net.V[0]))
        torch.cuda.synchronize()
        print("loss ratio after 60 / 100 steps: %.3f / %.3f" % (losses[59] / losses[0], losses[-1] / losses[0]))
        assert losses[-1] < 0.6 * losses[0], losses
        finals.append(net.master.clone())
    assert torch.equal(finals[0], finals[1])
