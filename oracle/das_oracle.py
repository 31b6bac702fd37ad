"""Delay-and-sum written out in FP64 (complex128).  TEST INFRASTRUCTURE ONLY.

For every frame f and voxel v (paper Sec. 2.1: delay, index/interpolate,
coherent sum over receive elements, repeated for every voxel and frame, and
compounded over transmits; Sec. 4.3: transmit arrival per voxel taken from a
precomputed table, receive delay |x_v - p_e| / c; Sec. 4.1: linear
interpolation, f-number apodization):

    y[v, f] = sum_t sum_e  w(v, e) * L_f(t, e, u) * exp(+j 2 pi fd tau)
    tau     = tau_tx[t, v] + |x_v - p_e| / c
    u       = (tau - t0) * fs
    L_f     = (1 - beta) q(i0) + beta q(i0 + 1),  i0 = floor(u), beta = u - i0,
              q(s) = iq[t, e, s, f] for 0 <= s < S and 0 outside the record
    w(v, e) = tukey_alpha(rho), rho = 2 f# |(x_v - p_e)_xy| / (z_v - z_e)

Readings where the paper is silent (each also listed in the design notes):
the window is Tukey(alpha) on the normalised lateral distance rho (rho >= 1
is outside the aperture); f# = 0 means no apodization; a voxel not below the
element (z_v - z_e <= 0) gets weight 0 when f# > 0; samples outside the
record are zero, so interpolation between sample S-1 and the zero past the
end (and between the zero before 0 and sample 0) is linear; the phase
rotation is exp(+j 2 pi fd tau) with the absolute delay, matching IQ data
demodulated as iq(t) = analytic(t) exp(-j 2 pi fd t); compounding is a plain
sum over transmits with no normalisation.

Inputs are promoted exactly from the float32/complex64 arrays handed to the
GPU, so their float32 quantisation is shared input, not oracle error.
"""

import numpy as np


def tukey(rho, alpha):
    """Tukey (tapered cosine) window on rho in [0, 1]; 0 for rho >= 1.

    1 for rho <= 1 - alpha; 0.5 (1 + cos(pi (rho - 1 + alpha) / alpha)) on
    the taper; alpha = 0 is the boxcar (1 for rho < 1), alpha = 1 is Hann.
    """
    rho = np.asarray(rho, dtype=np.float64)
    w = np.zeros_like(rho)
    if alpha <= 0.0:
        w[rho < 1.0] = 1.0
        return w
    flat = rho <= 1.0 - alpha
    taper = (~flat) & (rho < 1.0)
    w[flat] = 1.0
    w[taper] = 0.5 * (1.0 + np.cos(np.pi * (rho[taper] - 1.0 + alpha) / alpha))
    return w


def apodization(vox, elem_e, f_number, alpha):
    """f-number receive weight of one element for every voxel (paper Sec. 4.1).

    The aperture admits an element when its lateral distance from the voxel
    is below depth / (2 f#); rho is that ratio, the window tapers to 0 at
    rho = 1.  Lateral distance is radial in the array's x-y plane.
    """
    vox = np.asarray(vox, dtype=np.float64)
    if f_number == 0.0:
        return np.ones(vox.shape[0])
    d = vox - np.asarray(elem_e, dtype=np.float64)
    lat = np.hypot(d[:, 0], d[:, 1])
    depth = d[:, 2]
    w = np.zeros(vox.shape[0])
    below = depth > 0.0
    rho = 2.0 * f_number * lat[below] / depth[below]
    w[below] = tukey(rho, alpha)
    return w


def tx_plane_wave(vox, angles, c):
    """Plane-wave arrival time at each voxel, ``[T, V]`` seconds, FP64.

    The transmit table of the paper's hybrid delay strategy (Sec. 4.3): the
    wavefront with unit normal n crosses the array origin at t = 0 and
    reaches x at (n . x) / c.  ``angles`` [T, 2] = (theta, phi) radians:
    n = (sin th cos ph, sin ph, cos th cos ph).
    """
    vox = np.asarray(vox, dtype=np.float64)
    a = np.asarray(angles, dtype=np.float64).reshape(-1, 2)
    th, ph = a[:, 0], a[:, 1]
    n = np.stack([np.sin(th) * np.cos(ph), np.sin(ph), np.cos(th) * np.cos(ph)], axis=1)  # [T, 3]
    return (n @ vox.T) / c


def das(iq, elem_xyz, vox_xyz, tx_arrival, *, c, fs, fd, t0=0.0, f_number=1.0, tukey_alpha=0.5):
    """Beamform complex IQ ``[T, E, S, F]`` onto voxels; returns complex128 ``[V, F]``.

    ``elem_xyz`` [E, 3], ``vox_xyz`` [V, 3] metres; ``tx_arrival`` [T, V]
    seconds.  Loops over transmits and elements; vectorised over voxels and
    frames.
    """
    iq = np.asarray(iq)
    T, E, S, F = iq.shape
    vox = np.asarray(vox_xyz, dtype=np.float64).reshape(-1, 3)
    elem = np.asarray(elem_xyz, dtype=np.float64).reshape(-1, 3)
    tx = np.asarray(tx_arrival, dtype=np.float64).reshape(T, -1)
    V = vox.shape[0]
    assert elem.shape[0] == E and tx.shape[1] == V
    y = np.zeros((V, F), dtype=np.complex128)
    if V == 0 or F == 0:
        return y
    for e in range(E):
        w = apodization(vox, elem[e], f_number, tukey_alpha)
        r = np.sqrt(((vox - elem[e]) ** 2).sum(axis=1))
        for t in range(T):
            rec = iq[t, e].astype(np.complex128)  # [S, F]

            def q(idx):
                inside = (idx >= 0) & (idx < S)  # zero outside the record
                return np.where(inside[:, None], rec[np.clip(idx, 0, S - 1)], 0.0)

            tau = tx[t] + r / c
            u = (tau - t0) * fs
            i0f = np.floor(u)
            beta = u - i0f
            i0 = np.clip(i0f, -2, S + 1).astype(np.int64)
            lerp = (1.0 - beta)[:, None] * q(i0) + beta[:, None] * q(i0 + 1)
            rot = w * np.exp(2j * np.pi * fd * tau)
            y += rot[:, None] * lerp
    return y


def nrmse_db(y, y_ref):
    """20 log10(||y - y_ref||_2 / ||y_ref||_2) over all complex entries."""
    y = np.asarray(y, dtype=np.complex128)
    y_ref = np.asarray(y_ref, dtype=np.complex128)
    num = np.linalg.norm((y - y_ref).ravel())
    den = np.linalg.norm(y_ref.ravel())
    if num == 0.0:
        return -np.inf
    return 20.0 * np.log10(num / den)


def peak_err_db(y, y_ref):
    """20 log10(max |y - y_ref| / max |y_ref|): peak-normalised pixel error."""
    y = np.asarray(y, dtype=np.complex128)
    y_ref = np.asarray(y_ref, dtype=np.complex128)
    num = np.abs(y - y_ref).max()
    if num == 0.0:
        return -np.inf
    return 20.0 * np.log10(num / np.abs(y_ref).max())
