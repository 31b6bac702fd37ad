"""The five paper-shaped workloads, as seeded synthetic stand-ins.

c1  2D plane wave, 128-element linear array (pitch 0.3 mm, fc = fd = 7.6 MHz,
    fs = 4 fc), 1 transmit at 0 deg, 1 frame, 1024 samples, 20 seeded point
    scatterers plus circular Gaussian noise (std 0.01 per component), grid
    128 x 128 over x in [-19.05, 19.05] mm and z in [5, 35] mm, f-number 1.5.
c2  stand-in for the rotating-disk Doppler ensemble of the paper's benchmark
    (Sec. 4.1: 128-element linear array, 32 plane-wave frames, 0.1 mm grid,
    complex64, linear interpolation, f-number 1.0): fc = fd = 5 MHz,
    fs = 20 MHz, 2048 samples, 5000 scatterers in a disk of radius 5 mm
    centred at (0, 22.8) mm rotating 0.5 deg per frame inside 20000 static
    speckle scatterers, 256 x 256 grid at 0.1 mm (x = (i - 128) 0.1 mm,
    z = 10 + j 0.1 mm).  ``c2_251`` is the 251 x 251 grid the paper counts.
c3  3D: 32 x 32 matrix array (pitch 0.3 mm, fc = fd = 15 MHz, fs = 60 MHz),
    5 plane waves tilted in elevation (-6, -3, 0, 3, 6 deg), 2048 samples,
    8 frames of independent speckle (20000 scatterers) plus 50 fixed points
    (amplitude 10), 96^3 grid at 0.1 mm (x, y = (i - 48) 0.1 mm,
    z = 2 + k 0.1 mm), f-number 1.0.
c4  = c2 (the IQ is later stored as FP16 / BF16 by the caller).
c5  c3 geometry with 11 plane waves (-10 .. 10 deg in steps of 2 in
    elevation), 1 frame; the learned-compounding input uses -10, 0, +10 deg.

Every array is float32 / complex64 as the beamformer receives it.  All
randomness comes from ``numpy.random.default_rng(seed)``.
"""

import numpy as np

from .geometry import linear_array, matrix_array, grid_2d, grid_3d
from .echo import echo_iq

C_SOUND = 1540.0
MM = 1e-3
DEG = np.pi / 180.0

CONFIGS = ("c1", "c2", "c2_251", "c3", "c4", "c5")
DEFAULT_SEEDS = {"c1": 1, "c2": 2, "c2_251": 2, "c3": 3, "c4": 2, "c5": 10000}


def _params(fc, f_number, n_samples, n_frames, alpha=0.5):
    return dict(c=C_SOUND, fs=4.0 * fc, fc=fc, fd=fc, t0=0.0, f_number=f_number, tukey_alpha=alpha,
                n_samples=n_samples, n_frames=n_frames)


def _disk_phantom(rng, n_frames, grid_x, grid_z):
    """Rotating disk (radius 5 mm at (0, 22.8 mm)) inside static speckle."""
    cx, cz, rad = 0.0, 22.8 * MM, 5.0 * MM
    k_disk, k_bg = 5000, 20000
    r = rad * np.sqrt(rng.uniform(size=k_disk))
    th = rng.uniform(0.0, 2 * np.pi, size=k_disk)
    a_disk = rng.standard_normal(k_disk)
    bg = np.empty((0, 2))
    while bg.shape[0] < k_bg:
        cand = np.stack([rng.uniform(grid_x[0], grid_x[1], size=2 * k_bg),
                         rng.uniform(grid_z[0], grid_z[1], size=2 * k_bg)], axis=1)
        keep = (cand[:, 0] - cx) ** 2 + (cand[:, 1] - cz) ** 2 > rad ** 2
        bg = np.concatenate([bg, cand[keep]], axis=0)
    bg = bg[:k_bg]
    a_bg = rng.standard_normal(k_bg)
    scat = np.zeros((n_frames, k_disk + k_bg, 3))
    amp = np.zeros((n_frames, k_disk + k_bg))
    for f in range(n_frames):
        ang = th + 0.5 * DEG * f
        scat[f, :k_disk, 0] = cx + r * np.cos(ang)
        scat[f, :k_disk, 2] = cz + r * np.sin(ang)
        scat[f, k_disk:, 0] = bg[:, 0]
        scat[f, k_disk:, 2] = bg[:, 1]
        amp[f, :k_disk] = a_disk
        amp[f, k_disk:] = a_bg
    return scat, amp


def volume_phantom(rng, n_frames, lo, hi, n_speckle=20000, n_points=50, point_amp=10.0):
    """Per-frame independent speckle in a box plus fixed bright points."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    pts = lo + (hi - lo) * rng.uniform(size=(n_points, 3))
    scat = np.zeros((n_frames, n_speckle + n_points, 3))
    amp = np.zeros((n_frames, n_speckle + n_points))
    for f in range(n_frames):
        scat[f, :n_speckle] = lo + (hi - lo) * rng.uniform(size=(n_speckle, 3))
        amp[f, :n_speckle] = rng.standard_normal(n_speckle)
        scat[f, n_speckle:] = pts
        amp[f, n_speckle:] = point_amp
    return scat, amp


def make_config(name, seed=None, *, with_iq=True, n_frames=None, angles_deg=None):
    """Build one workload: geometry, grid, transmit angles, parameters, IQ.

    Returns a dict with ``elem`` [E,3] f32, ``vox`` [V,3] f32, ``angles``
    [T,2] radians (theta, phi), ``params`` (c, fs, fc, fd, t0, f_number,
    tukey_alpha, n_samples, n_frames), ``grid_shape`` and, if ``with_iq``,
    ``iq`` complex64 [T,E,S,F].  ``n_frames`` / ``angles_deg`` override the
    config's values (for smaller test cases of the same geometry).
    """
    if name not in CONFIGS:
        raise ValueError("unknown config %r" % (name,))
    seed = DEFAULT_SEEDS[name] if seed is None else seed
    rng = np.random.default_rng(seed)
    out = {"name": name, "seed": seed}
    if name == "c1":
        p = _params(7.6e6, 1.5, 1024, 1 if n_frames is None else n_frames)
        elem = linear_array(128, 0.3 * MM)
        xs = np.linspace(-19.05 * MM, 19.05 * MM, 128)
        zs = np.linspace(5 * MM, 35 * MM, 128)
        vox = grid_2d(xs, zs)
        grid_shape = (128, 128)
        ang = np.zeros((1, 2)) if angles_deg is None else np.asarray(angles_deg, float).reshape(-1, 2) * DEG
        k = 20
        sx = rng.uniform(-15 * MM, 15 * MM, size=k)
        sz = rng.uniform(5 * MM, 25 * MM, size=k)
        scat = np.stack([sx, np.zeros(k), sz], axis=1)
        amp = np.ones(k)
        noise_std = 0.01
    elif name in ("c2", "c2_251", "c4"):
        p = _params(5e6, 1.0, 2048, 32 if n_frames is None else n_frames)
        elem = linear_array(128, 0.3 * MM)
        n = 251 if name == "c2_251" else 256
        xs = (np.arange(n) - n // 2) * 0.1 * MM
        zs = 10 * MM + np.arange(n) * 0.1 * MM
        vox = grid_2d(xs, zs)
        grid_shape = (n, n)
        ang = np.zeros((1, 2)) if angles_deg is None else np.asarray(angles_deg, float).reshape(-1, 2) * DEG
        scat, amp = _disk_phantom(rng, p["n_frames"], (xs[0], xs[-1]), (zs[0], zs[-1]))
        noise_std = 0.0
    else:  # c3, c5
        nf = (8 if name == "c3" else 1) if n_frames is None else n_frames
        p = _params(15e6, 1.0, 2048, nf)
        elem = matrix_array(32, 32, 0.3 * MM)
        xs = (np.arange(96) - 48) * 0.1 * MM
        zs = 2 * MM + np.arange(96) * 0.1 * MM
        vox = grid_3d(xs, xs, zs)
        grid_shape = (96, 96, 96)
        if angles_deg is None:
            phis = [-6, -3, 0, 3, 6] if name == "c3" else list(range(-10, 11, 2))
            ang = np.array([[0.0, ph * DEG] for ph in phis])
        else:
            ang = np.asarray(angles_deg, float).reshape(-1, 2) * DEG
        lo = (xs[0], xs[0], zs[0])
        hi = (xs[-1], xs[-1], zs[-1])
        scat, amp = volume_phantom(rng, p["n_frames"], lo, hi)
        noise_std = 0.0
    out.update(elem=elem, vox=vox, angles=ang, params=p, grid_shape=grid_shape, scat=scat, amp=amp)
    if with_iq:
        iq = echo_iq(elem, ang, scat, amp, n_samples=p["n_samples"], n_frames=p["n_frames"],
                     c=p["c"], fs=p["fs"], fc=p["fc"], fd=p["fd"], t0=p["t0"])
        if noise_std > 0:
            nz = rng.standard_normal(iq.shape + (2,)) * noise_std
            iq = (iq + (nz[..., 0] + 1j * nz[..., 1])).astype(np.complex64)
        out["iq"] = iq
    return out


def random_iq(shape, seed, dtype=np.complex64):
    """Circular complex Gaussian IQ (std 1 per component), seeded."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(tuple(shape) + (2,), dtype=np.float32)
    return (x[..., 0] + 1j * x[..., 1]).astype(dtype)
