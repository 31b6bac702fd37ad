"""The GPU echo simulator (input generator) against the C simulator on small cases."""

import numpy as np
import pytest
import torch

from synth import echo_iq, echo_iq_gpu, matrix_array

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("T,E,S,F,K,t0", [(2, 16, 512, 2, 300, 0.0), (3, 9, 300, 1, 1000, 2e-6), (1, 4, 64, 3, 0, 0.0),
                                          (1, 5, 2048, 1, 20050, 0.0)])
def test_gpu_echo_matches_c(T, E, S, F, K, t0):
    r = np.random.default_rng(T * 100 + K)
    elem = matrix_array(int(np.ceil(np.sqrt(E))), int(np.ceil(np.sqrt(E))), 0.3e-3)[:E]
    ang = np.stack([r.uniform(-0.2, 0.2, T), r.uniform(-0.2, 0.2, T)], axis=1)
    # scatterers inside, before and beyond the record (partial and empty windows)
    scat = np.stack([r.uniform(-5e-3, 5e-3, (F, K)), r.uniform(-5e-3, 5e-3, (F, K)),
                     r.uniform(-1e-3, 13e-3, (F, K))], axis=2)
    amp = r.standard_normal((F, K)) * (1 + 9 * (r.uniform(size=(F, K)) < 0.01))
    kw = dict(n_samples=S, n_frames=F, c=1540.0, fs=60e6, fc=15e6, fd=15e6, t0=t0)
    ref = echo_iq(elem, ang, scat, amp, **kw)
    got = echo_iq_gpu(elem, ang, scat, amp, **kw).cpu().numpy()
    assert got.shape == ref.shape == (T, E, S, F)
    scale = max(np.abs(ref).max(), 1e-30)
    err = np.abs(got - ref).max()
    assert err <= 2e-6 * scale, (err, scale)
    if K == 0:
        assert not got.any()
    # deterministic: integer accumulation does not depend on thread arrival order
    again = echo_iq_gpu(elem, ang, scat, amp, **kw).cpu().numpy()
    assert np.array_equal(got, again)
