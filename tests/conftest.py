import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libdas.so")


@pytest.fixture(scope="session")
def rng():
    return np.random.default_rng(12345)


def small_case(seed, T=2, E=6, S=40, F=3, V=9, fs=20e6, fd=5e6, t0=-1e-7, f_number=0.8, alpha=0.5,
               depth=(0.3e-3, 1.2e-3)):
    """Random tiny problem whose delays fall inside (and at the edges of) the record."""
    r = np.random.default_rng(seed)
    iq = (r.standard_normal((T, E, S, F)) + 1j * r.standard_normal((T, E, S, F))).astype(np.complex64)
    elem = r.uniform(-0.6e-3, 0.6e-3, (E, 3)).astype(np.float32)
    elem[:, 2] = 0.0
    vox = np.stack([r.uniform(-1e-3, 1e-3, V), r.uniform(-0.5e-3, 0.5e-3, V),
                    r.uniform(depth[0], depth[1], V)], axis=1).astype(np.float32)
    tx = r.uniform(0.0, 4e-7, (T, V)).astype(np.float32)
    params = dict(c=1540.0, fs=fs, fd=fd, t0=t0, f_number=f_number, tukey_alpha=alpha)
    return iq, elem, vox, tx, params
