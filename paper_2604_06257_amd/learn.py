"""Learned compounding: a 3D U-Net on the gfx950 kernels of ``das_learn.h``.

Argument marshalling only: every layer, gradient, loss and optimiser step runs
in the library's HIP kernels; PyTorch provides device memory and the stream.

The network maps the delay-and-sum volumes of a few plane waves (real and
imaginary parts as channels, zero-padded to ``cin``) to a residual that is
added to a fixed baseline (the scaled few-angle compound):

    enc l = 0..2: a_l = relu(conv(in_l)), s_l = relu(conv(a_l)), in_{l+1} = pool(s_l)
    bottom:       a_3 = relu(conv(in_3)), b_3 = relu(conv(a_3))
    dec l = 2..0: c_la = relu(conv([s_l | up(prev)])), c_lb = relu(conv(c_la))
    out:          net = conv(c_0b)         prediction = base + net[:, 0:2]

Volumes are channels-last [D*H*W, C] bfloat16; the skip tensor s_l is written
straight into the first channels of the concatenation buffer, the upsampled
tensor into the rest.  Weights live in one flat float32 master buffer
(Adam state beside it) with a bfloat16 copy the convolutions read.
"""

import ctypes

import numpy as np
import torch

from . import _lib

BF16 = torch.bfloat16


def layer_shapes(cin=8, chans=(16, 32, 48, 64), cout=16):
    """(name, Cin, Cout) of every convolution, in forward order."""
    c0, c1, c2, c3 = chans
    return [("e0a", cin, c0), ("e0b", c0, c0), ("e1a", c0, c1), ("e1b", c1, c1), ("e2a", c1, c2), ("e2b", c2, c2),
            ("e3a", c2, c3), ("e3b", c3, c3), ("d2a", c2 + c3, c2), ("d2b", c2, c2), ("d1a", c1 + c2, c1),
            ("d1b", c1, c1), ("d0a", c0 + c1, c0), ("d0b", c0, c0), ("out", c0, cout)]


def _p(t):
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("the learned-compounding kernels take contiguous device tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    return ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


class Slice:
    """A channel slice [coff, coff + c) of a channels-last buffer [V, stride]."""

    def __init__(self, buf, coff=0, c=None):
        self.buf = buf
        self.stride = buf.shape[1]
        self.coff = coff
        self.c = self.stride - coff if c is None else c

    def args(self):
        return _p(self.buf), self.stride, self.coff

    def tensor(self):
        return self.buf[:, self.coff:self.coff + self.c]


def _whole(t):
    return t if isinstance(t, Slice) else Slice(t)


# ---------------------------------------------------------------- single ops
def conv3d(x, w, bias, out, dims, flip=False, relu=False, mask=None, stream=None):
    """out = act(conv(x)) * (mask > 0): see das_conv3d.  x, out, mask are tensors or Slices."""
    x, out = _whole(x), _whole(out)
    lib = _lib.load()
    D, H, W = dims
    cout = out.c
    if mask is not None:
        mask = _whole(mask)
        mp, ms, mc = mask.args()
    else:
        mp, ms, mc = ctypes.c_void_p(0), 0, 0
    _lib.check(lib.das_conv3d(*x.args(), _p(w), _p(bias), *out.args(), int(out.buf.dtype == torch.float32),
                              mp, ms, mc, D, H, W, x.c, cout, int(flip), int(relu), _stream(stream)), learn=True)
    return out.buf


def conv3d_wgrad(x, dy, dw, db, work, dims, chunk, stream=None):
    x, dy = _whole(x), _whole(dy)
    D, H, W = dims
    _lib.check(_lib.load().das_conv3d_wgrad(*x.args(), *dy.args(), _p(dw), _p(db), _p(work), work.numel(),
                                            D, H, W, x.c, dy.c, chunk, _stream(stream)), learn=True)


def wgrad_work_floats(dims, cin, cout, chunk):
    return int(_lib.load().das_conv3d_wgrad_work(*dims, cin, cout, chunk))


def transpose_weights(w, wt, cin, cout, stream=None):
    _lib.check(_lib.load().das_transpose_weights(_p(w), _p(wt), cin, cout, _stream(stream)), learn=True)


def avgpool2(x, out, out_dims, stream=None):
    x, out = _whole(x), _whole(out)
    _lib.check(_lib.load().das_avgpool2(*x.args(), *out.args(), *out_dims, x.c, _stream(stream)), learn=True)


def avgpool2_bwd(gout, gin, in_dims, accumulate=False, stream=None):
    gout, gin = _whole(gout), _whole(gin)
    _lib.check(_lib.load().das_avgpool2_bwd(*gout.args(), *gin.args(), *in_dims, gin.c, int(accumulate),
                                            _stream(stream)), learn=True)


def upsample2(x, out, out_dims, stream=None):
    x, out = _whole(x), _whole(out)
    _lib.check(_lib.load().das_upsample2(*x.args(), *out.args(), *out_dims, x.c, _stream(stream)), learn=True)


def upsample2_bwd(gout, gin, in_dims, mask=None, stream=None):
    gout, gin = _whole(gout), _whole(gin)
    if mask is not None:
        mask = _whole(mask)
        margs = mask.args()
    else:
        margs = (ctypes.c_void_p(0), 0, 0)
    _lib.check(_lib.load().das_upsample2_bwd(*gout.args(), *gin.args(), *margs, *in_dims, gin.c,
                                             _stream(stream)), learn=True)


def add_mask(a, b, mask, g, stream=None):
    a, b, g = _whole(a), _whole(b), _whole(g)
    margs = _whole(mask).args() if mask is not None else (ctypes.c_void_p(0), 0, 0)
    _lib.check(_lib.load().das_add_mask(*a.args(), *b.args(), *margs, *g.args(), g.buf.shape[0], g.c,
                                        _stream(stream)), learn=True)


def mse_residual(net, base, target, grad=None, pred=None, loss_parts=None, stream=None):
    """Returns the loss-part buffer (sum / (2 V) is the mean squared error)."""
    V = base.shape[0]
    if loss_parts is None:
        loss_parts = torch.empty((V + 255) // 256, dtype=torch.float32, device=net.device)
    _lib.check(_lib.load().das_mse_residual(_p(net), net.shape[1], _p(base), _p(target), V, _p(grad),
                                            grad.shape[1] if grad is not None else 0, _p(pred), _p(loss_parts),
                                            _stream(stream)), learn=True)
    return loss_parts


def adam(w, m, v, g, w_bf16, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _lib.check(_lib.load().das_adam(_p(w), _p(m), _p(v), _p(g), _p(w_bf16), w.numel(), lr, beta1, beta2, eps,
                                    step, _stream(stream)), learn=True)


def f32_to_bf16(x, y, stream=None):
    _lib.check(_lib.load().das_f32_to_bf16(_p(x), _p(y), x.numel(), _stream(stream)), learn=True)


# ---------------------------------------------------------------- the U-Net
class UNet:
    """Buffers, forward, backward and Adam for one volume size (D, H, W divisible by 8)."""

    def __init__(self, dims, cin=8, chans=(16, 32, 48, 64), cout=16, device="cuda", wgrad_chunk=None):
        D, H, W = dims
        if D % 8 or H % 8 or W % 8:
            raise ValueError("volume dimensions must be divisible by 8, got %s" % (dims,))
        self.dims = [(D >> l, H >> l, W >> l) for l in range(4)]
        self.V = [d * h * w for d, h, w in self.dims]
        self.cin, self.chans, self.cout = cin, tuple(chans), cout
        self.shapes = layer_shapes(cin, chans, cout)
        self.device = torch.device(device)
        dev = self.device
        # flat parameter layout [w_0, b_0, w_1, b_1, ...] (every block a multiple of 8 elements)
        self.offsets = {}
        off = 0
        for name, ci, co in self.shapes:
            nw = co * 27 * ci
            self.offsets[name] = (off, nw, off + nw, co)
            off += nw + co
        self.n_params = off
        f32 = dict(dtype=torch.float32, device=dev)
        self.master = torch.zeros(off, **f32)
        self.grad = torch.zeros(off, **f32)
        self.m = torch.zeros(off, **f32)
        self.v = torch.zeros(off, **f32)
        self.wbf = torch.zeros(off, dtype=BF16, device=dev)
        self.wt = {name: torch.zeros(co * 27 * ci, dtype=BF16, device=dev) for name, ci, co in self.shapes}
        self.step_count = 0
        c = self.chans
        bf = dict(dtype=BF16, device=dev)
        V = self.V
        self.ea = [torch.zeros(V[l], c[l], **bf) for l in range(4)]
        self.cat = [torch.zeros(V[l], c[l] + c[l + 1], **bf) for l in range(3)]
        self.pool = [torch.zeros(V[l + 1], c[l], **bf) for l in range(3)]
        self.b3 = torch.zeros(V[3], c[3], **bf)
        self.da = [torch.zeros(V[l], c[l], **bf) for l in range(3)]
        self.db = [torch.zeros(V[l], c[l], **bf) for l in range(3)]
        self.net = torch.zeros(V[0], cout, **f32)
        # backward buffers
        self.gnet = torch.zeros(V[0], cout, **bf)
        self.g_db = [torch.zeros(V[l], c[l], **bf) for l in range(3)] + [torch.zeros(V[3], c[3], **bf)]
        self.g_da = [torch.zeros(V[l], c[l], **bf) for l in range(4)]
        self.gcat = [torch.zeros(V[l], c[l] + c[l + 1], **bf) for l in range(3)]
        self.g_pool = [torch.zeros(V[l + 1], c[l], **bf) for l in range(3)]
        self.g_tmp = [torch.zeros(V[l], c[l], **bf) for l in range(3)]
        self.g_s = [torch.zeros(V[l], c[l], **bf) for l in range(3)]
        self.loss_parts = torch.zeros((V[0] + 255) // 256, **f32)
        self.chunks = {}
        need = 0
        for name, ci, co in self.shapes:
            lv = self._level(name)
            chunk = wgrad_chunk or self._chunk(V[lv])
            self.chunks[name] = chunk
            need = max(need, wgrad_work_floats(self.dims[lv], ci, co, chunk))
        self.work = torch.zeros(need, **f32)

    @staticmethod
    def _level(name):
        return 0 if name == "out" else int(name[1])

    @staticmethod
    def _chunk(v):
        """Voxels per weight-gradient partial sum: at most 256 partial sums (the weight gradient runs one wave
        per chunk and tap, so fewer chunks leave CUs idle), at least 1024 voxels each."""
        return max(1024, ((v + 255) // 256 + 31) // 32 * 32)

    # -- parameters
    def w(self, name, dtype="bf16"):
        o, nw, ob, co = self.offsets[name]
        src = self.wbf if dtype == "bf16" else self.master
        return src[o:o + nw]

    def b(self, name):
        o, nw, ob, co = self.offsets[name]
        return self.master[ob:ob + co]

    def gw(self, name):
        o, nw, ob, co = self.offsets[name]
        return self.grad[o:o + nw], self.grad[ob:ob + co]

    def set_params(self, params):
        """params: {name: (w [Cout,27,Cin], b [Cout])} (numpy or torch); refreshes the bf16 copies."""
        for name, ci, co in self.shapes:
            w, b = params[name]
            o, nw, ob, _ = self.offsets[name]
            self.master[o:o + nw] = torch.as_tensor(np.asarray(w, dtype=np.float32).reshape(-1)).to(self.device)
            self.master[ob:ob + co] = torch.as_tensor(np.asarray(b, dtype=np.float32).reshape(-1)).to(self.device)
        self.refresh_copies()

    def get_params(self):
        out = {}
        host = self.master.cpu().numpy()
        for name, ci, co in self.shapes:
            o, nw, ob, _ = self.offsets[name]
            out[name] = (host[o:o + nw].reshape(co, 27, ci).copy(), host[ob:ob + co].copy())
        return out

    def get_grads(self):
        out = {}
        host = self.grad.cpu().numpy()
        for name, ci, co in self.shapes:
            o, nw, ob, _ = self.offsets[name]
            out[name] = (host[o:o + nw].reshape(co, 27, ci).copy(), host[ob:ob + co].copy())
        return out

    def init_params(self, seed, out_scale=0.1):
        """He-normal weights, zero biases, output layer scaled by out_scale (seeded, host generated)."""
        rng = np.random.default_rng(seed)
        p = {}
        for name, ci, co in self.shapes:
            std = np.sqrt(2.0 / (27 * ci)) * (out_scale if name == "out" else 1.0)
            p[name] = (rng.standard_normal((co, 27, ci)) * std, np.zeros(co))
        self.set_params(p)

    def refresh_copies(self, stream=None):
        f32_to_bf16(self.master, self.wbf, stream)
        self._transpose(stream)

    def _transpose(self, stream=None):
        for name, ci, co in self.shapes:
            transpose_weights(self.w(name), self.wt[name], ci, co, stream)

    # -- forward
    def forward(self, x, stream=None):
        """x: bfloat16 [V, cin] -> float32 net [V, cout] (self.net)."""
        if x.dtype != BF16 or tuple(x.shape) != (self.V[0], self.cin) or not x.is_contiguous():
            raise ValueError("x must be contiguous bfloat16 [%d, %d]" % (self.V[0], self.cin))
        c = self.chans
        h = x
        for l in range(3):
            d = self.dims[l]
            conv3d(h, self.w("e%da" % l), self.b("e%da" % l), self.ea[l], d, relu=True, stream=stream)
            s = Slice(self.cat[l], 0, c[l])
            conv3d(self.ea[l], self.w("e%db" % l), self.b("e%db" % l), s, d, relu=True, stream=stream)
            avgpool2(s, self.pool[l], self.dims[l + 1], stream)
            h = self.pool[l]
        d3 = self.dims[3]
        conv3d(h, self.w("e3a"), self.b("e3a"), self.ea[3], d3, relu=True, stream=stream)
        conv3d(self.ea[3], self.w("e3b"), self.b("e3b"), self.b3, d3, relu=True, stream=stream)
        prev = self.b3
        for l in (2, 1, 0):
            d = self.dims[l]
            upsample2(prev, Slice(self.cat[l], c[l], c[l + 1]), d, stream)
            conv3d(self.cat[l], self.w("d%da" % l), self.b("d%da" % l), self.da[l], d, relu=True, stream=stream)
            conv3d(self.da[l], self.w("d%db" % l), self.b("d%db" % l), self.db[l], d, relu=True, stream=stream)
            prev = self.db[l]
        conv3d(prev, self.w("out"), self.b("out"), self.net, self.dims[0], stream=stream)
        return self.net

    # -- loss and backward
    def loss(self, base, target, with_grad=True, pred=None, stream=None):
        """Mean squared error of base + net[:, :2] against target; fills self.gnet when with_grad.

        Returns the loss-part buffer (device); float(parts.sum()) / (2 V) is the loss."""
        return mse_residual(self.net, base, target, self.gnet if with_grad else None, pred, self.loss_parts, stream)

    def backward(self, x, stream=None):
        """Weight gradients into self.grad for d loss / d net = self.gnet (after forward and loss)."""
        c = self.chans
        ch = self.chunks

        def wgrad(name, inp, dy, lv):
            dw, dbias = self.gw(name)
            conv3d_wgrad(inp, dy, dw, dbias, self.work, self.dims[lv], ch[name], stream)

        def dgrad(name, dy, out, lv, mask=None):
            conv3d(dy, self.wt[name], None, out, self.dims[lv], flip=True, mask=mask, stream=stream)

        wgrad("out", self.db[0], self.gnet, 0)
        dgrad("out", self.gnet, self.g_db[0], 0, mask=self.db[0])
        for l in (0, 1, 2):
            wgrad("d%db" % l, self.da[l], self.g_db[l], l)
            dgrad("d%db" % l, self.g_db[l], self.g_da[l], l, mask=self.da[l])
            wgrad("d%da" % l, self.cat[l], self.g_da[l], l)
            dgrad("d%da" % l, self.g_da[l], self.gcat[l], l, mask=self.cat[l])
            # the upsampled channels' gradient (already masked by the ReLU of the coarser output)
            upsample2_bwd(Slice(self.gcat[l], c[l], c[l + 1]), self.g_db[l + 1], self.dims[l + 1], stream=stream)
        wgrad("e3b", self.ea[3], self.g_db[3], 3)
        dgrad("e3b", self.g_db[3], self.g_da[3], 3, mask=self.ea[3])
        wgrad("e3a", self.pool[2], self.g_da[3], 3)
        dgrad("e3a", self.g_da[3], self.g_pool[2], 3)
        for l in (2, 1, 0):
            avgpool2_bwd(self.g_pool[l], self.g_tmp[l], self.dims[l], stream=stream)
            add_mask(self.g_tmp[l], Slice(self.gcat[l], 0, c[l]), Slice(self.cat[l], 0, c[l]), self.g_s[l], stream)
            wgrad("e%db" % l, self.ea[l], self.g_s[l], l)
            dgrad("e%db" % l, self.g_s[l], self.g_da[l], l, mask=self.ea[l])
            wgrad("e%da" % l, self.pool[l - 1] if l > 0 else x, self.g_da[l], l)
            if l > 0:
                dgrad("e%da" % l, self.g_da[l], self.g_pool[l - 1], l)

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step_count += 1
        adam(self.master, self.m, self.v, self.grad, self.wbf, lr, self.step_count, beta1, beta2, eps, stream)
        self._transpose(stream)

    def train_step(self, x, base, target, lr, stream=None):
        """forward + loss + backward + Adam; returns the loss-part buffer of this step (before the update)."""
        self.forward(x, stream)
        parts = self.loss(base, target, True, stream=stream)
        self.backward(x, stream)
        self.adam_step(lr, stream=stream)
        return parts

    def flops_forward(self):
        """Multiply-add FLOPs of one forward pass (2 per MAC)."""
        total = 0
        for name, ci, co in self.shapes:
            total += 2 * 27 * ci * co * self.V[self._level(name)]
        return total
