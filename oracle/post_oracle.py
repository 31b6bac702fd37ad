"""FP64 oracle of the post-processing steps.  TEST INFRASTRUCTURE ONLY.

The paper names two steps that follow beamforming (Sec. 3.3, after the
beamforming call): log compression for B-mode images and clutter filtering for
Doppler imaging, and states its validation errors in their terms (Sec. 5: Power
Doppler pixel errors in dB of power relative to the reference image's peak;
B-mode pixel errors in dB of amplitude).  The clutter filter is the SVD filter
of the cited Doppler work: the beamformed frames form a Casorati matrix
C [V, F] (voxels x frames), its k largest singular components (slow, coherent
tissue) are removed, and the Power Doppler image is the energy left per voxel.

    bmode_db(y)[v, f] = max(20 log10(|y[v, f]| / max_v |y[v, f]|), -dr)   (per frame)
    power_doppler(y, k)[v] = sum_f |(C - U_k S_k V_k^H)[v, f]|^2
    pixel_error_db(a, ref, power) = max_v 10 log10(|a - ref| / max ref)  (power images)
                                    max_v 20 log10(|a - ref| / max ref)  (amplitude images)
"""

import numpy as np


def envelope(y):
    return np.abs(np.asarray(y, dtype=np.complex128))


def bmode_db(y, dynamic_range_db=60.0):
    """Log-compressed envelope, 0 dB at each frame's peak, floored at -dynamic_range_db."""
    env = envelope(y)
    peak = env.max(axis=0, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        db = 20.0 * np.log10(env / peak)
    db = np.where(peak > 0, db, -dynamic_range_db)
    return np.maximum(db, -dynamic_range_db)


def svd_clutter_filter(y, n_clutter):
    """C minus its n_clutter largest singular components (C = y as [V, F])."""
    c = np.asarray(y, dtype=np.complex128)
    if n_clutter == 0:
        return c.copy()
    u, s, vh = np.linalg.svd(c, full_matrices=False)
    k = n_clutter
    return c - (u[:, :k] * s[:k]) @ vh[:k]


def power_doppler(y, n_clutter):
    """Energy per voxel of the clutter-filtered frames."""
    return (np.abs(svd_clutter_filter(y, n_clutter)) ** 2).sum(axis=1)


def pixel_error_db(a, ref, power):
    """Largest pixel error in dB relative to the reference's peak (power: 10 log10, amplitude: 20 log10)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(a - ref).max() / np.abs(ref).max()
    if err == 0:
        return -np.inf
    return (10.0 if power else 20.0) * np.log10(err)
