"""Post-processing of beamformed volumes (das_post.h): B-mode and Power Doppler.

Argument marshalling only; the kernels run in libdas.so.  ``y`` is the
beamformer's output, complex64 [V, F] on the device.
"""

import ctypes

import torch

from . import _lib


def _check_y(y):
    if not isinstance(y, torch.Tensor) or not y.is_cuda or y.dtype != torch.complex64 or y.dim() != 2 \
            or not y.is_contiguous():
        raise ValueError("y must be a contiguous complex64 [V, F] device tensor")


def _stream(stream=None):
    return ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def bmode(y, dynamic_range_db=60.0, out=None, stream=None):
    """Log-compressed envelope in dB (0 dB at each frame's peak, floored at -dynamic_range_db): float32 [V, F]."""
    _check_y(y)
    V, F = y.shape
    lib = _lib.load()
    if out is None:
        out = torch.empty((V, F), dtype=torch.float32, device=y.device)
    work = torch.empty(max(1, int(lib.das_bmode_work(V, F))), dtype=torch.float32, device=y.device)
    _lib.check(lib.das_bmode(ctypes.c_void_p(y.data_ptr()), V, F, float(dynamic_range_db),
                             ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(work.data_ptr()), work.numel(),
                             _stream(stream)), post=True)
    return out


def power_doppler(y, n_clutter, out=None, stream=None):
    """Energy per voxel after removing the n_clutter largest singular components over frames: float32 [V]."""
    _check_y(y)
    V, F = y.shape
    lib = _lib.load()
    if out is None:
        out = torch.empty(V, dtype=torch.float32, device=y.device)
    work = torch.empty(max(1, int(lib.das_power_doppler_work(V, F))), dtype=torch.float64, device=y.device)
    _lib.check(lib.das_power_doppler(ctypes.c_void_p(y.data_ptr()), V, F, int(n_clutter),
                                     ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(work.data_ptr()), work.numel(),
                                     _stream(stream)), post=True)
    return out


def power_doppler_noalloc(y, n_clutter, out, stream=None):
    """Power Doppler into the caller's float32 [V] ``out`` with the library's fixed scratch array (no work buffer;
    calls that overlap on one GPU race)."""
    _check_y(y)
    V, F = y.shape
    if not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.float32 or out.shape != (V,) \
            or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 [V] device tensor")
    lib = _lib.load()
    _lib.check(lib.das_power_doppler_noalloc(ctypes.c_void_p(y.data_ptr()), V, F, int(n_clutter),
                                             ctypes.c_void_p(out.data_ptr()), _stream(stream)), post=True)
    return out
