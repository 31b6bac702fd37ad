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
_GPU_SRC = os.path.join(_HERE, "_echo_gpu.hip")
_GPU_LIB = os.path.join(_HERE, "_echo_gpu.so")
_gpu_lib = None


def build_echo_lib(force=False):
    """Compile the C echo simulator in place (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_echo_gpu_lib(force=False):
    """Compile the gfx950 echo simulator in place (hipcc)."""
    if force or not os.path.exists(_GPU_LIB) or os.path.getmtime(_GPU_LIB) < os.path.getmtime(_GPU_SRC):
        tmp = _GPU_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-x", "hip", _GPU_SRC,
                               "-o", tmp], stderr=subprocess.DEVNULL)
        os.replace(tmp, _GPU_LIB)
    return _GPU_LIB


def _load_gpu():
    global _gpu_lib
    if _gpu_lib is None:
        if not os.path.exists(_GPU_LIB):
            raise RuntimeError("synth/_echo_gpu.so is not built; run synth.echo.build_echo_gpu_lib()")
        lib = ctypes.CDLL(_GPU_LIB)
        vp = ctypes.c_void_p
        lib.synth_echo_gpu.argtypes = [vp] + [ctypes.c_int] * 4 + [vp] * 4 + [ctypes.c_int] + [ctypes.c_double] * 7 + [vp]
        lib.synth_echo_gpu.restype = ctypes.c_int
        _gpu_lib = lib
    return _gpu_lib


def echo_iq_gpu(elem_xyz, angles, scat, amp, *, n_samples, n_frames, c, fs, fc, fd, t0=0.0, sigma=None,
                trunc_sigmas=6.0, out=None, device="cuda"):
    """The same model as ``echo_iq`` evaluated on the GPU: complex64 torch tensor [T, E, S, F].

    Host arrays are copied to the device in float64; ``out`` may be a
    preallocated contiguous complex64 tensor of the right shape."""
    import torch
    lib = _load_gpu()
    if sigma is None:
        sigma = 0.577 / fc
    scat, amp = _per_frame(scat, amp, n_frames)
    dev = torch.device(device)
    d64 = dict(dtype=torch.float64, device=dev)
    elem_d = torch.as_tensor(np.ascontiguousarray(np.asarray(elem_xyz, dtype=np.float64)), **d64)
    nrm_d = torch.as_tensor(np.ascontiguousarray(plane_wave_normals(angles)), **d64)
    scat_d = torch.as_tensor(scat, **d64)
    amp_d = torch.as_tensor(amp, **d64)
    T, E, S, F, K = nrm_d.shape[0], elem_d.shape[0], int(n_samples), int(n_frames), scat.shape[1]
    if out is None:
        out = torch.empty((T, E, S, F), dtype=torch.complex64, device=dev)
    elif tuple(out.shape) != (T, E, S, F) or out.dtype != torch.complex64 or not out.is_contiguous():
        raise ValueError("out must be contiguous complex64 %s" % ((T, E, S, F),))
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    st = lib.synth_echo_gpu(ctypes.c_void_p(out.data_ptr()), T, E, S, F, ctypes.c_void_p(elem_d.data_ptr()),
                            ctypes.c_void_p(nrm_d.data_ptr()), ctypes.c_void_p(scat_d.data_ptr()),
                            ctypes.c_void_p(amp_d.data_ptr()), K, float(c), float(fs), float(fc), float(fd),
                            float(t0), float(sigma), float(trunc_sigmas), stream)
    if st != 0:
        raise RuntimeError("synth_echo_gpu failed with status %d" % st)
    # keep the inputs alive until the kernel has read them
    torch.cuda.current_stream(dev).synchronize()
    return out


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
