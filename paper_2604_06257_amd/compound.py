"""Learned compounding: few-angle delay-and-sum + a 3D U-Net residual.

Compounding N plane waves multiplies the beamforming cost by N.  Here only a
few of the angles are beamformed (per-transmit output of one plan, so each
angle's volume is kept apart), the network reads their real and imaginary
parts (normalised by the RMS of their sum) and predicts the residual between
the N-angle compound and (N / n) times the few-angle sum.  The full N-angle
plan stays available as the reference and the fallback.

Argument marshalling only: beamforming, feature packing, the network and the
output run in the library's kernels (libdas.so).
"""

import ctypes

import torch

from . import _lib
from . import das as _das
from . import learn as _learn


def _p(t):
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    return ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def compound_features(ys, gain, x, base, work, scale, stream=None):
    """das_compound_features: ys complex64 [A, V] -> x bfloat16 [V, cin], base float32 [V, 2], scale {rms, 1/rms}."""
    A, V = ys.shape
    _lib.check(_lib.load().das_compound_features(_p(ys), A, V, float(gain), _p(x), x.shape[1], _p(base), _p(work),
                                                 _p(scale), _stream(stream)), learn=True)


def compound_rescale(y, scale, out, restore=False, stream=None):
    _lib.check(_lib.load().das_compound_rescale(_p(y), y.numel(), _p(scale), int(restore), _p(out), _stream(stream)),
               learn=True)


def compound_output(net, base, scale, out, stream=None):
    _lib.check(_lib.load().das_compound_output(_p(net), net.shape[1], _p(base), base.shape[0], _p(scale), _p(out),
                                               _stream(stream)), learn=True)


class LearnedCompounding:
    """Plans, buffers and network for one geometry.

    params: das.Params of the full acquisition (n_tx = all angles, n_frames = 1);
    elem_xyz [E, 3], vox_xyz [V, 3] float32 device tensors, voxels ordered as a
    dims = (D, H, W) lattice (last index fastest); tx_arrival [T, V] float32
    device (das.tx_plane_wave); input_idx: the transmits the network sees.
    """

    def __init__(self, params, elem_xyz, vox_xyz, tx_arrival, dims, input_idx, chans=(16, 32, 48, 64), cin=8):
        if params.n_frames != 1:
            raise ValueError("learned compounding works on single frames")
        D, H, W = dims
        if D * H * W != params.n_vox:
            raise ValueError("dims %s do not match %d voxels" % (dims, params.n_vox))
        self.params = params
        self.input_idx = list(input_idx)
        self.A = len(self.input_idx)
        if cin < 2 * self.A:
            raise ValueError("cin must hold 2 channels per input angle")
        self.gain = params.n_tx / self.A
        self.full = _das.Plan(params, elem_xyz, vox_xyz, tx_arrival)
        # the input angles: one plan whose per-transmit output keeps each angle's volume (the receive geometry
        # is then formed once for all of them), else one plan per angle
        tx_in = tx_arrival[self.input_idx].contiguous()
        self.inputs = _das.Plan(_das.Params(**{**params.__dict__, "n_tx": self.A}), elem_xyz, vox_xyz, tx_in)
        self.per_tx = self.A <= 4 and self.inputs.info()["kernel"][0] <= 2
        self.plans = [] if self.per_tx else [
            _das.Plan(_das.Params(**{**params.__dict__, "n_tx": 1}), elem_xyz, vox_xyz, tx_arrival[t:t + 1].contiguous())
            for t in self.input_idx]
        V = params.n_vox
        dev = vox_xyz.device
        self.V = V
        self.ys = torch.zeros((self.A, V), dtype=torch.complex64, device=dev)
        self.x = torch.zeros((V, cin), dtype=torch.bfloat16, device=dev)
        self.base = torch.zeros((V, 2), dtype=torch.float32, device=dev)
        self.scale = torch.zeros(2, dtype=torch.float32, device=dev)
        self.work = torch.zeros(max(1, int(_lib.load().das_compound_work(V))), dtype=torch.float32, device=dev)
        self.net = _learn.UNet(dims, cin=cin, chans=chans, cout=16, device=dev)

    def input_iq(self, iq):
        """The input angles' channel data [A, E, S, 1] out of a full acquisition [T, E, S, 1] (a copy)."""
        return iq[self.input_idx].contiguous()

    def beamform_inputs(self, iq_in, stream=None):
        """The input angles (channel data [A, E, S, 1]), one volume each: self.ys [A, V]."""
        if self.per_tx:
            self.inputs.execute_per_tx(iq_in, out=self.ys.view(self.A, self.V, 1), stream=stream)
        else:
            for a, plan in enumerate(self.plans):
                plan.execute(iq_in[a:a + 1], out=self.ys[a].view(self.V, 1), stream=stream)
        return self.ys

    def features(self, stream=None):
        compound_features(self.ys, self.gain, self.x, self.base, self.work, self.scale, stream)
        return self.x, self.base, self.scale

    def full_compound(self, iq, out=None, stream=None):
        """The reference: all plane waves beamformed and summed (complex64 [V, 1])."""
        return self.full.execute(iq, out=out, stream=stream)

    def normalised_target(self, y_full, out, stream=None):
        """y_full / rms (float32 [V, 2] view of a complex64 volume), with this input's scale."""
        compound_rescale(y_full, self.scale, out, restore=False, stream=stream)
        return out

    def predict(self, iq_in, out=None, stream=None):
        """Few-angle beamforming (channel data of the input angles, [A, E, S, 1]) + network: the estimated
        compound, complex64 [V, 1]."""
        self.beamform_inputs(iq_in, stream)
        self.features(stream)
        self.net.forward(self.x, stream)
        if out is None:
            out = torch.empty((self.V, 1), dtype=torch.complex64, device=self.x.device)
        compound_output(self.net.net, self.base, self.scale, out, stream)
        return out

    def close(self):
        self.full.close()
        self.inputs.close()
        for p in self.plans:
            p.close()
