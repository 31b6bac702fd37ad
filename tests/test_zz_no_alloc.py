"""das_power_doppler_noalloc (the allocation-free Power Doppler) against das_power_doppler, through the C ABI.

Two calls in a row on the same GPU, the second with a smaller input, each compared with das_power_doppler on
the same frames: bitwise, since the scratch array holds the same voxel chunking as a caller's work buffer for
every frame count.  The scratch array keeps the first call's contents: the second call must not depend on them.
"""

import ctypes

import numpy as np
import pytest
import torch

from paper_2604_06257_amd import _lib

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _frames(seed, V, F):
    r = np.random.default_rng(seed)
    c = lambda *s: (r.standard_normal(s) + 1j * r.standard_normal(s)).astype(np.complex64)  # noqa: E731
    # a decaying spectrum of singular values, so the clutter subspace is well separated
    y = c(V, F) @ np.diag(np.geomspace(30.0, 1.0, F)).astype(np.complex64) @ np.linalg.qr(c(F, F))[0]
    return torch.as_tensor(y.astype(np.complex64), device=DEV)


def _with_work(lib, y, k):
    V, F = y.shape
    out = torch.empty(V, dtype=torch.float32, device=DEV)
    work = torch.empty(int(lib.das_power_doppler_work(V, F)), dtype=torch.float64, device=DEV)
    st = lib.das_power_doppler(ctypes.c_void_p(y.data_ptr()), V, F, k, ctypes.c_void_p(out.data_ptr()),
                               ctypes.c_void_p(work.data_ptr()), work.numel(), None)
    assert st == 0, lib.das_post_last_error()
    return out


def _no_alloc(lib, y, k):
    V, F = y.shape
    out = torch.full((V,), float("nan"), dtype=torch.float32, device=DEV)
    st = lib.das_power_doppler_noalloc(ctypes.c_void_p(y.data_ptr()), V, F, k, ctypes.c_void_p(out.data_ptr()),
                                       None)
    assert st == 0, lib.das_post_last_error()
    return out


@pytest.mark.parametrize("calls", [((65536, 32, 2), (3000, 12, 1)), ((20000, 16, 3), (700, 32, 5))])
def test_power_doppler_noalloc_matches_the_work_buffer_entry_point(calls):
    lib = _lib.load()
    for i, (V, F, k) in enumerate(calls):
        y = _frames(100 * i + V + F, V, F)
        got = _no_alloc(lib, y, k)
        torch.cuda.synchronize()
        ref = _with_work(lib, y, k)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy().astype(np.float64), ref.cpu().numpy().astype(np.float64)
        assert np.isfinite(g).all()
        np.testing.assert_array_equal(g, r)


def test_power_doppler_noalloc_rejects_bad_arguments():
    lib = _lib.load()
    y = _frames(1, 64, 4)
    out = torch.empty(64, dtype=torch.float32, device=DEV)
    yp, op = ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(out.data_ptr())
    assert lib.das_power_doppler_noalloc(None, 64, 4, 1, op, None) == _lib.DAS_EINVAL
    assert lib.das_power_doppler_noalloc(yp, 64, 33, 1, op, None) == _lib.DAS_ESHAPE
    assert lib.das_power_doppler_noalloc(yp, 0, 4, 1, op, None) == _lib.DAS_ESHAPE
    assert lib.das_power_doppler_noalloc(yp, 64, 4, 5, op, None) == _lib.DAS_EINVAL
