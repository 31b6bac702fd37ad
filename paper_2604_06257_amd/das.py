"""Python binding of the gfx950 delay-and-sum library (argument marshalling only).

Device memory and streams come from PyTorch (ROCm build); every step of the
beamforming path runs in the library's HIP kernels.

    plan = Plan(params, elem_xyz, vox_xyz, tx_arrival)   # torch tensors on cuda
    y = plan.execute(iq)                                  # complex64 [V, F]

``iq`` is complex64 ``[T, E, S, F]`` or float16 / bfloat16 ``[T, E, S, F, 2]``
(interleaved real, imaginary).
"""

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import check


@dataclass
class Params:
    """Acquisition / reconstruction parameters (see ``das_params`` in das.h)."""

    n_tx: int
    n_elem: int
    n_samples: int
    n_frames: int
    n_vox: int
    sound_speed: float = 1540.0
    fs: float = 20e6
    f_demod: float = 5e6
    t0: float = 0.0
    f_number: float = 1.0
    tukey_alpha: float = 0.5

    def to_c(self):
        return _lib.DasParams(int(self.n_tx), int(self.n_elem), int(self.n_samples), int(self.n_frames),
                              int(self.n_vox), float(self.sound_speed), float(self.fs), float(self.f_demod),
                              float(self.t0), float(self.f_number), float(self.tukey_alpha))


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f32(t, name, shape):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) torch tensor" % name)
    if t.dtype != torch.float32:
        raise ValueError("%s must be float32, got %s" % (name, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def iq_dtype_code(iq):
    """das_iq_dtype for a tensor: complex64 [...], or fp16/bf16 [..., 2]."""
    if iq.dtype == torch.complex64:
        return _lib.DAS_IQ_C64
    if iq.dtype == torch.float16:
        return _lib.DAS_IQ_C16F
    if iq.dtype == torch.bfloat16:
        return _lib.DAS_IQ_C16BF
    raise ValueError("unsupported IQ dtype %s (complex64, float16 or bfloat16 [..., 2])" % iq.dtype)


class Plan:
    """An immutable beamforming plan (das_plan_create / das_execute)."""

    def __init__(self, params, elem_xyz, vox_xyz, tx_arrival, stream=None):
        lib = _lib.load()
        self.params = params
        E, V, T = params.n_elem, params.n_vox, params.n_tx
        pe = _dev_f32(elem_xyz, "elem_xyz", (E, 3))
        pv = _dev_f32(vox_xyz, "vox_xyz", (V, 3)) if V > 0 else ctypes.c_void_p(0)
        pt = _dev_f32(tx_arrival, "tx_arrival", (T, V)) if V > 0 else ctypes.c_void_p(0)
        handle = ctypes.c_void_p(0)
        cp = params.to_c()
        check(lib.das_plan_create(ctypes.byref(handle), ctypes.byref(cp), pe, pv, pt, _stream_ptr(stream)))
        self._h = handle

    def info(self):
        lib = _lib.load()
        inf = _lib.DasPlanInfo()
        check(lib.das_plan_query(self._h, ctypes.byref(inf)))
        return {"n_vox": inf.n_vox, "n_slots": inf.n_slots, "n_tiles": inf.n_tiles,
                "total_triples": inf.total_triples, "active_triples": inf.active_triples,
                "processed_triples": inf.processed_triples, "tile_dims": tuple(inf.tile_dims),
                "max_window": inf.max_window,
                "kernel": (inf.kernel_fc, inf.kernel_pitch, inf.kernel_groups)}

    def execute(self, iq, out=None, stream=None):
        """Beamform ``iq`` into ``out`` (complex64 [V, F], allocated if None)."""
        p = self.params
        code = iq_dtype_code(iq)
        want = (p.n_tx, p.n_elem, p.n_samples, p.n_frames) + (() if code == _lib.DAS_IQ_C64 else (2,))
        if not iq.is_cuda or tuple(iq.shape) != want or not iq.is_contiguous():
            raise ValueError("iq must be a contiguous CUDA tensor of shape %s, got %s" % (want, tuple(iq.shape)))
        if out is None:
            out = torch.empty((p.n_vox, p.n_frames), dtype=torch.complex64, device=iq.device)
        elif out.dtype != torch.complex64 or tuple(out.shape) != (p.n_vox, p.n_frames) or not out.is_contiguous():
            raise ValueError("out must be contiguous complex64 of shape %s" % ((p.n_vox, p.n_frames),))
        check(_lib.load().das_execute(self._h, ctypes.c_void_p(iq.data_ptr()), code,
                                      ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def execute_per_tx(self, iq, out=None, stream=None):
        """Each transmit's volume separately (das_execute_per_tx): complex64 [T, V, F]; T <= 4, F <= 2."""
        p = self.params
        code = iq_dtype_code(iq)
        want = (p.n_tx, p.n_elem, p.n_samples, p.n_frames) + (() if code == _lib.DAS_IQ_C64 else (2,))
        if not iq.is_cuda or tuple(iq.shape) != want or not iq.is_contiguous():
            raise ValueError("iq must be a contiguous CUDA tensor of shape %s, got %s" % (want, tuple(iq.shape)))
        shape = (p.n_tx, p.n_vox, p.n_frames)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex64, device=iq.device)
        elif out.dtype != torch.complex64 or tuple(out.shape) != shape or not out.is_contiguous():
            raise ValueError("out must be contiguous complex64 of shape %s" % (shape,))
        check(_lib.load().das_execute_per_tx(self._h, ctypes.c_void_p(iq.data_ptr()), code,
                                             ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(_lib.load().das_plan_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def tx_plane_wave(vox_xyz, angles, sound_speed, stream=None):
    """Plane-wave arrival table [T, V] float32 on the device (das_tx_plane_wave)."""
    ang = np.ascontiguousarray(np.asarray(angles, dtype=np.float64).reshape(-1, 2))
    V = vox_xyz.shape[0]
    pv = _dev_f32(vox_xyz, "vox_xyz", (V, 3))
    out = torch.empty((ang.shape[0], V), dtype=torch.float32, device=vox_xyz.device)
    check(_lib.load().das_tx_plane_wave(ctypes.c_void_p(out.data_ptr()), pv, V,
                                        ang.ctypes.data_as(ctypes.c_void_p), ang.shape[0], float(sound_speed),
                                        _stream_ptr(stream)))
    return out


def tile_order(vox_xyz):
    """Host-side voxel tiling (das_tile_order): (slot_to_vox int32 [slots], tile_dims)."""
    lib = _lib.load()
    v = np.ascontiguousarray(np.asarray(vox_xyz, dtype=np.float32).reshape(-1, 3))
    n_slots = ctypes.c_int64(0)
    dims = (ctypes.c_int32 * 3)()
    check(lib.das_tile_order(v.ctypes.data_as(ctypes.c_void_p), v.shape[0], None, 0, ctypes.byref(n_slots), dims))
    out = np.empty(n_slots.value, dtype=np.int32)
    check(lib.das_tile_order(v.ctypes.data_as(ctypes.c_void_p), v.shape[0], out.ctypes.data_as(ctypes.c_void_p),
                             out.size, ctypes.byref(n_slots), dims))
    return out, tuple(dims)


def kernel_variants():
    """The compiled kernel variants (das_kernel_variants): list of (fc, pitch, groups)."""
    lib = _lib.load()
    n = lib.das_kernel_variants(None, 0)
    if n < 0:
        check(n)
    buf = (ctypes.c_int32 * (3 * n))()
    n2 = lib.das_kernel_variants(buf, n)
    if n2 < 0:
        check(n2)
    return [(buf[3 * k], buf[3 * k + 1], buf[3 * k + 2]) for k in range(n)]


def choose_kernel_variant(n_frames, max_window, n_tiles, items_per_tile):
    """The variant a plan with these figures gets (das_choose_kernel_variant): (fc, pitch, groups)."""
    lib = _lib.load()
    buf = (ctypes.c_int32 * 3)()
    check(lib.das_choose_kernel_variant(int(n_frames), int(max_window), int(n_tiles), float(items_per_tile), buf))
    return (buf[0], buf[1], buf[2])


def beamform(iq, elem_xyz, vox_xyz, tx_arrival, params, out=None, stream=None):
    """One-shot convenience: plan, execute, destroy."""
    with Plan(params, elem_xyz, vox_xyz, tx_arrival, stream=stream) as plan:
        return plan.execute(iq, out=out, stream=stream)
