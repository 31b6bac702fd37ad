"""Pins of the post-processing oracle (B-mode, SVD clutter filter, Power Doppler) on the CPU."""

import numpy as np
import pytest

from oracle import post_oracle as P


def test_bmode_special_values():
    y = np.array([[2.0 + 0j, 1.0], [0.2j, 0.0], [-0.002, 1e-9]])
    db = P.bmode_db(y, dynamic_range_db=60.0)
    assert db[0, 0] == 0.0 and db[0, 1] == 0.0              # each frame's peak is 0 dB
    assert db[1, 0] == pytest.approx(-20.0, abs=1e-12)        # |0.2j| / 2
    assert db[2, 0] == pytest.approx(-60.0, abs=1e-12)        # |-0.002| / 2, right at the floor
    assert db[1, 1] == -60.0 and db[2, 1] == -60.0            # zero and below the floor
    # invariant to a complex scale of the frame
    np.testing.assert_allclose(P.bmode_db(y * (3 - 4j)), P.bmode_db(y), atol=1e-12)
    # an all-zero frame is the floor
    assert np.all(P.bmode_db(np.zeros((4, 1))) == -60.0)


def test_power_doppler_without_filter_is_the_frame_energy():
    r = np.random.default_rng(0)
    y = r.standard_normal((50, 8)) + 1j * r.standard_normal((50, 8))
    np.testing.assert_allclose(P.power_doppler(y, 0), (np.abs(y) ** 2).sum(1), rtol=1e-14)
    assert np.allclose(P.power_doppler(y, 8), 0.0, atol=1e-20 + 1e-12 * (np.abs(y) ** 2).sum())


def _tissue_plus_blood(seed, V=200, F=16, k=2, tissue_amp=100.0):
    """Tissue and blood with orthogonal frame patterns (row spaces) and orthogonal voxel maps (column
    spaces), so the SVD of their sum separates them exactly; tissue is the k strongest components."""
    r = np.random.default_rng(seed)
    cplx = lambda *s: r.standard_normal(s) + 1j * r.standard_normal(s)  # noqa: E731
    q, _ = np.linalg.qr(cplx(F, F))
    qv, _ = np.linalg.qr(cplx(V, F))
    tissue = qv[:, :k] @ (tissue_amp * cplx(k, k)) @ q[:, :k].conj().T
    blood = qv[:, k:] @ cplx(F - k, F - k) @ q[:, k:].conj().T
    return tissue, blood


def test_clutter_filter_removes_exactly_a_strong_orthogonal_tissue_subspace():
    tissue, blood = _tissue_plus_blood(1)
    pd = P.power_doppler(tissue + blood, 2)
    np.testing.assert_allclose(pd, (np.abs(blood) ** 2).sum(1), rtol=1e-9)
    # removing one component fewer leaves the weaker tissue component in
    assert P.power_doppler(tissue + blood, 1).sum() > 10 * pd.sum()


def test_clutter_filter_residual_is_orthogonal_and_energy_splits():
    r = np.random.default_rng(2)
    y = r.standard_normal((120, 10)) + 1j * r.standard_normal((120, 10))
    k = 3
    res = P.svd_clutter_filter(y, k)
    s = np.linalg.svd(y, compute_uv=False)
    # the residual is orthogonal to what was removed and carries exactly the trailing singular energy
    np.testing.assert_allclose((np.abs(res) ** 2).sum(), (s[k:] ** 2).sum(), rtol=1e-12)
    np.testing.assert_allclose(res.conj().T @ (y - res), 0.0, atol=1e-10)
    # invariant to a unitary mixing of the frames (the filter acts on the frame subspace)
    q, _ = np.linalg.qr(r.standard_normal((10, 10)) + 1j * r.standard_normal((10, 10)))
    np.testing.assert_allclose(P.power_doppler(y @ q, k), P.power_doppler(y, k), rtol=1e-10)


def test_pixel_error_db():
    ref = np.array([1.0, 0.5, 0.0])
    assert P.pixel_error_db(ref + np.array([0, 1e-6, 0]), ref, power=True) == pytest.approx(-60.0)
    assert P.pixel_error_db(ref + np.array([0, 1e-6, 0]), ref, power=False) == pytest.approx(-120.0)
    assert P.pixel_error_db(ref, ref, power=True) == -np.inf
