"""Pins of the FP64 oracle against facts fixed by the paper and the mathematics.

Each test holds the oracle to something other than itself: closed forms,
special cases, a brute-force scalar implementation, invariants and the
interpolation error bound of an analytic echo.  A dropped term, a wrong sign
of the phase, a swapped interpolation weight or an off-by-one sample index
fails at least one of them.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import das, tukey, apodization, tx_plane_wave, das_scalar
from synth import echo_iq, echo_iq_numpy, linear_array, matrix_array, grid_2d
from conftest import small_case

C = 1540.0


def _tau_scalar(tx_value, vox, elem, c=C):
    """Round-trip delay of one (voxel, element), written independently of the oracle."""
    d = math.sqrt(sum((float(a) - float(b)) ** 2 for a, b in zip(vox, elem)))
    return float(tx_value) + d / c


# ----------------------------------------------------------------- window
def test_tukey_special_values():
    a = 0.5
    assert tukey(np.array([0.0]), a)[0] == 1.0
    assert tukey(np.array([1.0 - a]), a)[0] == 1.0
    assert tukey(np.array([1.0 - a / 2]), a)[0] == pytest.approx(0.5, abs=1e-15)
    assert tukey(np.array([1.0]), a)[0] == 0.0
    assert tukey(np.array([1.5]), a)[0] == 0.0
    # alpha = 1 is the Hann window cos^2(pi rho / 2)
    rho = np.linspace(0, 0.999, 50)
    np.testing.assert_allclose(tukey(rho, 1.0), np.cos(np.pi * rho / 2) ** 2, atol=1e-15)
    # alpha = 0 is the boxcar
    np.testing.assert_array_equal(tukey(np.array([0.0, 0.5, 0.999, 1.0]), 0.0), [1, 1, 1, 0])
    # continuous at both ends of the taper
    for edge in (1.0 - a, 1.0):
        lo, hi = tukey(np.array([edge - 1e-9, edge + 1e-9]), a)
        assert abs(lo - hi) < 1e-8


def test_apodization_aperture():
    # element straight above the voxel: rho = 0 -> 1; at lateral distance depth/(2 f#): rho = 1 -> 0
    f_num, z = 1.5, 0.02
    vox = np.array([[0.0, 0.0, z], [z / (2 * f_num), 0.0, z], [0.0, z / (2 * f_num) * 0.5, z], [0.0, 0.0, -z]])
    w = apodization(vox, np.zeros(3), f_num, 0.5)
    assert w[0] == 1.0 and w[1] == 0.0 and w[2] == 1.0 and w[3] == 0.0
    assert (apodization(vox, np.zeros(3), 0.0, 0.5) == 1.0).all()


# --------------------------------------------------------------- tx table
def test_tx_plane_wave_closed_forms():
    vox = np.array([[1e-3, 2e-3, 3e-3], [-4e-3, 0.5e-3, 10e-3]])
    ang = np.array([[0.0, 0.0], [np.pi / 2, 0.0], [0.0, np.pi / 2], [0.3, 0.0], [0.0, -0.2]])
    tx = tx_plane_wave(vox, ang, C)
    np.testing.assert_allclose(tx[0], vox[:, 2] / C, rtol=1e-15)
    np.testing.assert_allclose(tx[1], vox[:, 0] / C, rtol=1e-12, atol=1e-20)
    np.testing.assert_allclose(tx[2], vox[:, 1] / C, rtol=1e-12, atol=1e-20)
    np.testing.assert_allclose(tx[3], (np.sin(0.3) * vox[:, 0] + np.cos(0.3) * vox[:, 2]) / C, rtol=1e-14)
    np.testing.assert_allclose(tx[4], (np.sin(-0.2) * vox[:, 1] + np.cos(-0.2) * vox[:, 2]) / C, rtol=1e-14)


# ------------------------------------------------------------- P1 zero
def test_p1_zero_in_zero_out():
    iq, elem, vox, tx, p = small_case(1)
    y = das(np.zeros_like(iq), elem, vox, tx, **p)
    assert (y == 0).all()


# ------------------------------------------------------------- P2 linearity
def test_p2_linearity():
    iq, elem, vox, tx, p = small_case(2)
    iq2, *_ = small_case(3)
    a, b = 0.7 - 0.2j, -1.3 + 0.4j
    lhs = das(a * iq.astype(np.complex128) + b * iq2.astype(np.complex128), elem, vox, tx, **p)
    rhs = a * das(iq, elem, vox, tx, **p) + b * das(iq2, elem, vox, tx, **p)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


# ---------------------------------------------------------- P3 CW point pin
@pytest.mark.parametrize("f_number", [0.0, 1.0])
def test_p3_cw_point_sum_of_weights(f_number):
    """iq = A exp(-j 2 pi fd tau_te(x_s)) for every sample -> y(x_s) = A sum_te w exactly."""
    T, E, S, F = 2, 16, 256, 2
    fs, fd = 20e6, 5e6
    elem = linear_array(E, 0.3e-3)
    vox = np.array([[0.4e-3, 0.0, 4e-3], [-0.6e-3, 0.0, 5e-3]], dtype=np.float32)
    tx = np.array([[4e-3 / C, 5e-3 / C], [4.2e-3 / C, 4.9e-3 / C]], dtype=np.float32)
    A = 0.8 - 0.3j
    for k in range(vox.shape[0]):
        iq = np.zeros((T, E, S, F), dtype=np.complex128)
        wsum = 0.0
        for t in range(T):
            for e in range(E):
                tau = _tau_scalar(tx[t, k], vox[k], elem[e])
                assert 0 <= (tau * fs) <= S - 1
                iq[t, e, :, :] = A * np.exp(-2j * np.pi * fd * tau)
                if f_number == 0.0:
                    wsum += 1.0
                else:
                    dx, dy = float(vox[k, 0]) - float(elem[e, 0]), float(vox[k, 1]) - float(elem[e, 1])
                    rho = 2 * f_number * math.hypot(dx, dy) / (float(vox[k, 2]) - float(elem[e, 2]))
                    wsum += 0.0 if rho >= 1 else (1.0 if rho <= 0.5 else 0.5 * (1 + math.cos(math.pi * (rho - 0.5) / 0.5)))
        y = das(iq, elem, vox[k:k + 1], tx[:, k:k + 1], c=C, fs=fs, fd=fd, f_number=f_number, tukey_alpha=0.5)
        if f_number == 0.0:
            assert wsum == T * E
        assert np.abs(y - A * wsum).max() < 1e-12 * abs(A) * wsum


# ------------------------------------------------- P4 Gaussian scatterer peak
@pytest.mark.parametrize("f_number", [0.0, 1.5])
def test_p4_gaussian_point_scatterer_peak(f_number):
    """Analytic echo of one scatterer on a voxel: the peak equals A * sum w up to the
    linear-interpolation error bound 1 / (8 (fs sigma)^2) of the Gaussian envelope."""
    fc = 7.6e6
    fs, fd = 4 * fc, fc
    sigma = 0.577 / fc
    E, S = 128, 1024
    elem = linear_array(E, 0.3e-3)
    xs = np.array([[1.2e-3, 0.0, 12e-3]], dtype=np.float32)
    A = 2.0
    angles = np.zeros((1, 2))
    iq = echo_iq(elem, angles, xs.astype(np.float64), np.array([A]), n_samples=S, n_frames=1, c=C, fs=fs,
                 fc=fc, fd=fd, sigma=sigma)
    tx = tx_plane_wave(xs, angles, C).astype(np.float32)
    y = das(iq, elem, xs, tx, c=C, fs=fs, fd=fd, f_number=f_number, tukey_alpha=0.5)[0, 0]
    wsum = 0.0
    for e in range(E):
        wsum += apodization(xs, elem[e], f_number, 0.5)[0]
    bound = A * wsum / (8 * (fs * sigma) ** 2)
    err = abs(y - A * wsum)
    assert err <= bound
    assert err > 0.05 * bound  # the interpolation loss is real, not hidden by a bug that returns A*sum w
    # the peak is the maximum of the image along depth
    zs = xs[0, 2] + np.arange(-6, 7) * 0.05e-3
    line = np.stack([np.full(zs.size, xs[0, 0]), np.zeros(zs.size), zs], axis=1).astype(np.float32)
    yl = das(iq, elem, line, tx_plane_wave(line, angles, C).astype(np.float32), c=C, fs=fs, fd=fd,
             f_number=f_number, tukey_alpha=0.5)[:, 0]
    assert np.argmax(np.abs(yl)) == 6


# ------------------------------------------------ P5 constant record, edges
def test_p5_constant_iq_ramps_at_record_edges():
    """fd = 0, f# = 0, iq = 1: y = sum L with L = 1 inside, u + 1 on [-1, 0), S - u on [S-1, S), else 0."""
    T, E, S, F = 1, 5, 12, 2
    elem = linear_array(E, 0.3e-3)
    fs = 20e6
    # voxels straight below the array at depths whose delays straddle both record edges
    depths = np.linspace(0.0, 0.8e-3, 41)
    vox = np.stack([np.zeros(depths.size), np.zeros(depths.size), depths], axis=1).astype(np.float32)
    tx = np.zeros((T, depths.size), dtype=np.float32)
    t0 = 0.6 / fs
    iq = np.ones((T, E, S, F), dtype=np.complex64)
    y = das(iq, elem, vox, tx, c=C, fs=fs, fd=0.0, t0=t0, f_number=0.0)
    seen = set()
    for v in range(depths.size):
        expect = 0.0
        for e in range(E):
            u = (_tau_scalar(0.0, vox[v], elem[e]) - t0) * fs
            if 0 <= u <= S - 1:
                expect += 1.0
            elif -1 < u < 0:
                expect += u + 1
            elif S - 1 < u < S:
                expect += S - u
            seen.add(int(np.floor(u)) if -1 <= u < S else (-9 if u < -1 else 99))
        np.testing.assert_allclose(y[v], expect, atol=1e-12)
    assert {-1, 0, S - 1, 99} <= seen  # both ramps, the interior and beyond the record are exercised


# --------------------------------------------- P6 linear record is exact
def test_p6_linear_in_sample_is_interpolated_exactly():
    T, E, S, F = 2, 7, 64, 2
    fs, fd, t0 = 20e6, 5e6, -2e-7
    elem = linear_array(E, 0.3e-3)
    r = np.random.default_rng(6)
    vox = np.stack([r.uniform(-1e-3, 1e-3, 11), np.zeros(11), r.uniform(0.5e-3, 1.5e-3, 11)], 1).astype(np.float32)
    tx = r.uniform(0, 3e-7, (T, 11)).astype(np.float32)
    a = np.array([0.3 + 0.1j, -0.2 + 0.5j])   # per frame
    b = np.array([0.01 - 0.02j, 0.03 + 0.0j])
    s = np.arange(S)
    iq = np.zeros((T, E, S, F), dtype=np.complex128)
    for f in range(F):
        iq[:, :, :, f] = a[f] + b[f] * s
    y = das(iq, elem, vox, tx, c=C, fs=fs, fd=fd, t0=t0, f_number=0.0)
    for v in range(vox.shape[0]):
        expect = np.zeros(F, dtype=np.complex128)
        for t in range(T):
            for e in range(E):
                tau = _tau_scalar(tx[t, v], vox[v], elem[e])
                u = (tau - t0) * fs
                assert 0 <= u <= S - 1
                expect += (a + b * u) * np.exp(2j * np.pi * fd * tau)
        np.testing.assert_allclose(y[v], expect, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------- P7 brute force
@pytest.mark.parametrize("seed", range(6))
def test_p7_oracle_matches_scalar_brute_force(seed):
    kw = [dict(), dict(f_number=0.0), dict(alpha=1.0), dict(alpha=0.0, f_number=0.3),
          dict(t0=3e-7), dict(T=3, E=4, S=24, F=4, V=8)][seed]
    iq, elem, vox, tx, p = small_case(100 + seed, **kw)
    y = das(iq, elem, vox, tx, **p)
    yb = np.array(das_scalar(iq, elem, vox, tx, p["c"], p["fs"], p["fd"], p["t0"], p["f_number"], p["tukey_alpha"]))
    scale = max(1.0, np.abs(yb).max())
    assert np.abs(y - yb).max() <= 1e-12 * scale
    assert np.abs(yb).max() > 0  # the case exercises non-zero output


# ------------------------------------------------------- P8 invariants
def test_p8_frame_permutation_equivariance():
    iq, elem, vox, tx, p = small_case(8, F=5)
    perm = np.array([3, 0, 4, 1, 2])
    y = das(iq, elem, vox, tx, **p)
    yp = das(iq[..., perm], elem, vox, tx, **p)
    np.testing.assert_array_equal(yp, y[:, perm])


def test_p8_transmit_additivity():
    iq, elem, vox, tx, p = small_case(9, T=3)
    y = das(iq, elem, vox, tx, **p)
    ys = sum(das(iq[t:t + 1], elem, vox, tx[t:t + 1], **p) for t in range(3))
    np.testing.assert_allclose(y, ys, rtol=0, atol=1e-13 * np.abs(y).max())


def test_p8_element_permutation_invariance():
    iq, elem, vox, tx, p = small_case(10, E=7)
    perm = np.array([6, 2, 0, 5, 1, 3, 4])
    y = das(iq, elem, vox, tx, **p)
    yp = das(iq[:, perm], elem[perm], vox, tx, **p)
    np.testing.assert_allclose(y, yp, rtol=0, atol=1e-13 * np.abs(y).max())


# ----------------------------------------------------------- P9 mirror
def test_p9_mirror_symmetry():
    E, S = 32, 512
    fc = 7.6e6
    fs = 4 * fc
    elem = linear_array(E, 0.3e-3)
    assert (elem[::-1, 0] == -elem[:, 0]).all()
    nx, nz = 9, 7
    xs = (np.arange(nx) - (nx - 1) / 2) * 0.2e-3
    zs = 4e-3 + np.arange(nz) * 0.3e-3
    vox = grid_2d(xs, zs)
    angles = np.zeros((1, 2))
    tx = tx_plane_wave(vox, angles, C).astype(np.float32)
    scat = np.array([[0.5e-3, 0, 4.6e-3], [-0.3e-3, 0, 5.3e-3]])
    amp = np.array([1.0, -0.7])
    kw = dict(n_samples=S, n_frames=1, c=C, fs=fs, fc=fc, fd=fc)
    iq_a = echo_iq(elem, angles, scat, amp, **kw)
    mirrored = scat * np.array([-1, 1, 1])
    iq_b = echo_iq(elem, angles, mirrored, amp, **kw)
    p = dict(c=C, fs=fs, fd=fc, f_number=1.5, tukey_alpha=0.5)
    ya = das(iq_a, elem, vox, tx, **p).reshape(nx, nz)
    yb = das(iq_b, elem, vox, tx, **p).reshape(nx, nz)
    np.testing.assert_allclose(yb, ya[::-1, :], rtol=0, atol=1e-9 * np.abs(ya).max())
    assert np.abs(ya).max() > 1.0


# ------------------------------------------------- P11 synth closed form
def test_p11_synth_single_scatterer():
    fc = 5e6
    fs, fd = 4 * fc, fc
    sigma = 0.577 / fc
    elem = linear_array(8, 0.3e-3)
    x = np.array([[0.7e-3, 0.0, 6e-3]])
    iq = echo_iq(elem, np.zeros((1, 2)), x, np.array([1.5]), n_samples=256, n_frames=1, c=C, fs=fs, fc=fc, fd=fd)
    for e in range(8):
        tau = _tau_scalar(x[0, 2] / C, x[0], elem[e].astype(np.float64))
        s_near = int(round(tau * fs))
        mag = np.abs(iq[0, e, :, 0])
        assert np.argmax(mag) == s_near
        for s in (s_near - 2, s_near, s_near + 3):
            expect = 1.5 * math.exp(-((s / fs - tau) ** 2) / (2 * sigma ** 2)) * np.exp(-2j * np.pi * fd * tau)
            assert abs(iq[0, e, s, 0] - expect) < 2e-6 * 1.5


def test_synth_c_matches_numpy_model():
    elem = matrix_array(3, 2, 0.3e-3)
    r = np.random.default_rng(4)
    scat = r.uniform([-1e-3, -1e-3, 3e-3], [1e-3, 1e-3, 5e-3], (2, 5, 3))
    amp = r.standard_normal((2, 5))
    kw = dict(n_samples=400, n_frames=2, c=C, fs=60e6, fc=15e6, fd=14e6)
    ang = np.array([[0.0, 0.05], [0.1, -0.05]])
    a = echo_iq(elem, ang, scat, amp, **kw)
    b = echo_iq_numpy(elem, ang, scat, amp, **kw)
    assert np.abs(a - b).max() <= 2e-6 * np.abs(b).max()


# ------------------------------------------------------------ metrics
def test_error_metrics():
    y = np.array([1.0, 2.0, 2.0], dtype=complex)
    assert oracle.nrmse_db(y * (1 + 1e-5), y) == pytest.approx(-100.0, abs=1e-6)
    assert oracle.peak_err_db(y + np.array([0, 2e-3, 0]), y) == pytest.approx(-60.0, abs=1e-6)
    assert oracle.nrmse_db(y, y) == -np.inf
