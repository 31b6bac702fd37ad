"""Analytic IQ echoes of point-scatterer phantoms (FP64 model, complex64 output).

Two implementations of the same forward model: ``echo_iq`` (compiled C with
OpenMP, for paper-sized phantoms) and ``echo_iq_numpy`` (direct evaluation,
for small cases and for checking the C code).
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "_echo.c")
_LIB = os.path.join(_HERE, "_echo.so")
_lib = None


def build_echo_lib(force=False):
    """Compile the C echo simulator in place (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build_echo_lib()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.synth_echo.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   dp, dp, dp, dp, ctypes.c_int] + [ctypes.c_double] * 7
        lib.synth_echo.restype = None
        _lib = lib
    return _lib


def plane_wave_normals(angles):
    """Unit propagation directions for plane waves.

    ``angles`` is ``[T, 2]`` radians: (theta, phi) = (lateral steering in x-z,
    elevation tilt towards y).  n = (sin th cos ph, sin ph, cos th cos ph).
    """
    a = np.asarray(angles, dtype=np.float64).reshape(-1, 2)
    th, ph = a[:, 0], a[:, 1]
    return np.stack([np.sin(th) * np.cos(ph), np.sin(ph), np.cos(th) * np.cos(ph)], axis=1)


def _per_frame(scat, amp, n_frames):
    scat = np.asarray(scat, dtype=np.float64)
    amp = np.asarray(amp, dtype=np.float64)
    if scat.ndim == 2:
        scat = np.broadcast_to(scat, (n_frames,) + scat.shape)
        amp = np.broadcast_to(amp, (n_frames,) + amp.shape)
    assert scat.shape[0] == n_frames and scat.shape[2] == 3 and amp.shape == scat.shape[:2]
    return np.ascontiguousarray(scat), np.ascontiguousarray(amp)


def echo_iq(elem_xyz, angles, scat, amp, *, n_samples, n_frames, c, fs, fc, fd, t0=0.0,
            sigma=None, trunc_sigmas=6.0):
    """Complex64 IQ ``[T, E, S, F]`` echoed by point scatterers.

    ``scat`` is ``[K, 3]`` (static) or ``[F, K, 3]`` (per frame) metres and
    ``amp`` the matching real amplitudes.  ``sigma`` defaults to 0.577 / fc.
    """
    lib = _load()
    if sigma is None:
        sigma = 0.577 / fc
    elem = np.ascontiguousarray(np.asarray(elem_xyz, dtype=np.float64))
    normals = np.ascontiguousarray(plane_wave_normals(angles))
    scat, amp = _per_frame(scat, amp, n_frames)
    T, E, S, F, K = normals.shape[0], elem.shape[0], int(n_samples), int(n_frames), scat.shape[1]
    out = np.empty((T, E, S, F), dtype=np.complex64)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.synth_echo(out.ctypes.data, T, E, S, F, elem.ctypes.data_as(dp), normals.ctypes.data_as(dp),
                   scat.ctypes.data_as(dp), amp.ctypes.data_as(dp), K,
                   float(c), float(fs), float(fc), float(fd), float(t0), float(sigma), float(trunc_sigmas))
    return out


def echo_iq_numpy(elem_xyz, angles, scat, amp, *, n_samples, n_frames, c, fs, fc, fd, t0=0.0,
                  sigma=None, trunc_sigmas=6.0):
    """Direct FP64 evaluation of the same model (small cases only)."""
    if sigma is None:
        sigma = 0.577 / fc
    elem = np.asarray(elem_xyz, dtype=np.float64)
    normals = plane_wave_normals(angles)
    scat, amp = _per_frame(scat, amp, n_frames)
    T, E, S, F = normals.shape[0], elem.shape[0], int(n_samples), int(n_frames)
    ts = t0 + np.arange(S) / fs
    out = np.zeros((T, E, S, F), dtype=np.complex128)
    for t in range(T):
        for f in range(F):
            x = scat[f]
            d_tx = x @ normals[t] / c
            for e in range(E):
                tau = d_tx + np.sqrt(((x - elem[e]) ** 2).sum(axis=1)) / c  # [K]
                dt = ts[:, None] - tau[None, :]                              # [S, K]
                g = np.exp(-dt ** 2 / (2 * sigma ** 2)) * (np.abs(dt) <= trunc_sigmas * sigma)
                ph = np.exp(-2j * np.pi * fd * tau)[None, :] * np.exp(2j * np.pi * (fc - fd) * dt)
                out[t, e, :, f] = (amp[f][None, :] * g * ph).sum(axis=1)
    return out.astype(np.complex64)
