"""Parity of the gfx950 DAS path (through the C ABI) with the FP64 oracle.

Bar: normalised RMS error <= -100 dB and peak-normalised pixel error <= -100 dB
(the error style of the paper's Sec. 5: the largest pixel error relative to the
reference image's peak), FP32 path vs FP64 oracle on the same float32/complex64
inputs; exact zeros where the definition gives zero; bitwise determinism.
Full-size workloads run on the GPU in the same launch configuration the
benchmark times; the oracle checks every voxel (c1, c2, the paper's 251 x 251
grid), every 4th voxel per axis (c3: 13,824 voxels, all elements, transmits and
frames of each) or a seeded sample (the sweep extremes).
"""

import numpy as np
import pytest
import torch

import oracle
import paper_2604_06257_amd as das
from synth import make_config, grid_2d, linear_array, matrix_array
from synth.configs import random_iq
from conftest import small_case
from oracle_pool import oracle_job, quantize_iq, build_inputs

pytestmark = pytest.mark.gpu

DB_BAR = -100.0


def check_db(y, ref, what):
    """Both error measures against the bar; returns (nrmse dB, peak dB)."""
    db, pk = oracle.nrmse_db(y, ref), oracle.peak_err_db(y, ref)
    print(what, "nrmse %.1f dB, peak %.1f dB" % (db, pk))
    assert db <= DB_BAR and pk <= DB_BAR, (what, db, pk)
    return db, pk


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_das(iq, elem, vox, tx, p, iq_dtype="c64"):
    T, E, S, F = iq.shape
    params = das.Params(n_tx=T, n_elem=E, n_samples=S, n_frames=F, n_vox=vox.shape[0], sound_speed=p["c"],
                        fs=p["fs"], f_demod=p["fd"], t0=p.get("t0", 0.0), f_number=p["f_number"],
                        tukey_alpha=p["tukey_alpha"])
    if iq_dtype == "c64":
        iq_t = dev(iq.astype(np.complex64))
    else:
        ri = torch.view_as_real(dev(iq.astype(np.complex64)))
        iq_t = ri.to(torch.float16 if iq_dtype == "f16" else torch.bfloat16).contiguous()
    with das.Plan(params, dev(elem), dev(vox), dev(tx)) as plan:
        y = plan.execute(iq_t)
        torch.cuda.synchronize()
        info = plan.info()
    return y.cpu().numpy(), info, iq_t


def oracle_params(cfg):
    p = cfg["params"]
    return dict(c=p["c"], fs=p["fs"], fd=p["fd"], t0=p["t0"], f_number=p["f_number"], tukey_alpha=p["tukey_alpha"])


def tx_table(vox, angles, c):
    return oracle.tx_plane_wave(vox, angles, c).astype(np.float32)


# ------------------------------------------------------------ a0 tx table
def test_tx_plane_wave_kernel_matches_oracle():
    cfg = make_config("c3", with_iq=False, angles_deg=[[0, -6], [0, 3], [5, 2], [-10, 0]])
    vox = cfg["vox"]
    got = das.tx_plane_wave(dev(vox), cfg["angles"], 1540.0).cpu().numpy()
    ref = oracle.tx_plane_wave(vox, cfg["angles"], 1540.0)
    ulp = np.spacing(np.abs(ref).astype(np.float32))
    assert np.all(np.abs(got.astype(np.float64) - ref) <= ulp)   # correctly rounded up to one ulp
    assert (got == ref.astype(np.float32)).mean() > 0.99


# ------------------------------------------------------- small random shapes
CASES = [
    dict(), dict(F=1), dict(F=2), dict(F=5), dict(F=8, T=3), dict(F=17), dict(F=32), dict(F=33, V=40),
    dict(F=70, E=3), dict(f_number=0.0), dict(alpha=1.0), dict(t0=3e-7), dict(S=8, t0=5e-7),
    dict(V=300, E=5, F=4), dict(fd=0.0), dict(T=5, E=9, F=9, V=64),
]


@pytest.mark.parametrize("i", range(len(CASES)))
def test_parity_small_random(i):
    iq, elem, vox, tx, p = small_case(500 + i, **CASES[i])
    y, info, _ = gpu_das(iq, elem, vox, tx, p)
    ref = oracle.das(iq, elem, vox, tx, **p)
    assert np.abs(ref).max() > 0
    db = oracle.nrmse_db(y, ref)
    print("case", CASES[i], "nrmse dB", db, "info", info)
    assert db <= DB_BAR


# ------------------------------------------------------------ workloads
def _sampled_parity(cfg, n_sample, seed, iq=None):
    vox = cfg["vox"]
    iq = cfg["iq"] if iq is None else iq
    p = oracle_params(cfg)
    tx = tx_table(vox, cfg["angles"], p["c"])
    y, info, _ = gpu_das(iq, cfg["elem"], vox, tx, p)
    idx = np.sort(np.random.default_rng(seed).choice(vox.shape[0], n_sample, replace=False))
    ref = oracle.das(iq, cfg["elem"], vox[idx], tx[:, idx], **p)
    return y, y[idx], ref, info


def _job_parity(spec, idx, quant="c64"):
    """GPU run of job ``spec`` (inputs rebuilt from its seeds, IQ stored as ``quant``) against the oracle, run in
    a child process, on voxels ``idx``.  Returns (full GPU output, its rows idx, oracle rows, plan info)."""
    iq, elem, vox, tx, p = build_inputs(spec)
    iq_t, _ = quantize_iq(iq, quant)
    del iq
    F = iq_t.shape[3]
    params = das.Params(n_tx=iq_t.shape[0], n_elem=iq_t.shape[1], n_samples=iq_t.shape[2], n_frames=F,
                        n_vox=vox.shape[0], sound_speed=p["c"], fs=p["fs"], f_demod=p["fd"], t0=p["t0"],
                        f_number=p["f_number"], tukey_alpha=p["tukey_alpha"])
    with das.Plan(params, dev(elem), dev(vox), dev(tx)) as plan:
        y = plan.execute(iq_t.cuda()).cpu().numpy()
        info = plan.info()
    ref = oracle_job(dict(spec, quant=quant), idx)
    return y, y[idx], ref, info


def test_parity_c1_full():
    cfg = make_config("c1")
    p = oracle_params(cfg)
    tx = tx_table(cfg["vox"], cfg["angles"], p["c"])
    y, info, _ = gpu_das(cfg["iq"], cfg["elem"], cfg["vox"], tx, p)
    ref = oracle.das(cfg["iq"], cfg["elem"], cfg["vox"], tx, **p)
    check_db(y, ref, "c1 (all voxels) %s" % (info,))
    # voxels deeper than the record (25.9 mm at 0 deg) see zero channel data: exact zeros
    z = cfg["vox"][:, 2]
    deep = z > 1540.0 * (1024 + 1) / (2 * 30.4e6)  # round trip longer than the record plus one sample
    assert deep.any() and np.all(y[deep] == 0)
    assert info["kernel"] == (1, 0, 4)  # the launch configuration bench.py times for c1 (direct kernel)


_C2_REF = {}


def _c2_reference(quant):
    """GPU output and oracle reference of c2 on all 65,536 voxels for IQ stored as ``quant`` (cached)."""
    if quant not in _C2_REF:
        _C2_REF[quant] = _job_parity(dict(config="c2"), np.arange(65536), quant)
    return _C2_REF[quant]


def test_parity_c2_full():
    """c2, the benchmarked workload, in the benchmarked variant: every voxel against the oracle."""
    y, _, ref, info = _c2_reference("c64")
    check_db(y, ref, "c2 (all 65536 voxels) %s" % (info,))
    assert y.shape == (65536, 32) and np.isfinite(y).all()
    assert info["kernel"] == (16, 65, 2)  # the launch configuration of the bench line


def test_parity_c2_251_full():
    cfg = make_config("c2_251", n_frames=8)
    p = oracle_params(cfg)
    tx = tx_table(cfg["vox"], cfg["angles"], p["c"])
    y, info, _ = gpu_das(cfg["iq"], cfg["elem"], cfg["vox"], tx, p)
    ref = oracle_job(dict(config="c2_251", n_frames=8), np.arange(cfg["vox"].shape[0]))
    check_db(y, ref, "c2_251 (all 63001 voxels, 8 frames) %s" % (info,))


C3_STRIDE = np.array([(ix * 96 + iy) * 96 + iz for ix in range(0, 96, 4) for iy in range(0, 96, 4)
                      for iz in range(0, 96, 4)])  # every 4th voxel per axis of the depth-fastest 96^3 grid


@pytest.mark.parametrize("quant", ["c64", "f16", "bf16"])
def test_parity_c3_strided(quant):
    """c3 at full size in the benchmarked variant: every 4th voxel per axis (13,824 voxels, all 1024 elements,
    5 transmits and 8 frames each) against the oracle on the same (quantised) samples.  The channel data is
    circular Gaussian (speckle's value distribution), which parity needs, rather than the echo model."""
    assert C3_STRIDE.shape == (13824,)
    spec = dict(config="c3", random_iq=dict(shape=[5, 1024, 2048, 8], seed=33))
    y, ys, ref, info = _job_parity(spec, C3_STRIDE, quant)
    check_db(ys, ref, "c3 %s (13824 strided voxels) %s" % (quant, info))
    assert y.shape == (96 ** 3, 8) and np.isfinite(y).all()
    assert info["kernel"] == (8, 65, 1)  # one unpaired 8-frame chunk per tile, as bench.py times c3


def test_parity_c2_grid_many_frames_sampled():
    """The c2 grid with 200 frames: 13 chunks of 16 frames, the last one ragged (8 frames), at full grid size."""
    cfg = make_config("c2", with_iq=False, n_frames=200)
    p = cfg["params"]
    iq = random_iq((1, 128, p["n_samples"], 200), seed=36)
    y, ys, ref, info = _sampled_parity(cfg, 256, 37, iq=iq)
    check_db(ys, ref, "c2 grid, 200 frames %s" % (info["kernel"],))
    assert info["kernel"][0] == 16 and y.shape == (65536, 200) and np.isfinite(y).all()


def test_parity_32_frame_variant_chosen_by_the_plan():
    """A 512 x 512 grid at the c2 spacing with 32 frames has 1024 tiles whose windows fit 40 rows: the plan picks
    the 32-frame variant (32, 41, 3) by itself.  Sampled voxels against the oracle."""
    c, fc = 1540.0, 5e6
    p = dict(c=c, fs=4 * fc, fd=fc, t0=0.0, f_number=1.0, tukey_alpha=0.5)
    xs = (np.arange(512) - 256) * 0.1e-3
    zs = 10e-3 + np.arange(512) * 0.1e-3
    vox = grid_2d(xs, zs)
    elem = linear_array(128, 0.3e-3)
    tx = tx_table(vox, np.zeros((1, 2)), c)
    iq = random_iq((1, 128, 2048, 32), seed=43)
    y, info, _ = gpu_das(iq, elem, vox, tx, p)
    assert info["kernel"] == (32, 41, 3)
    idx = np.sort(np.random.default_rng(44).choice(vox.shape[0], 1024, replace=False))
    ref = oracle.das(iq, elem, vox[idx], tx[:, idx], **p)
    check_db(y[idx], ref, "512^2 grid, 32 frames %s" % (info["kernel"],))


def test_parity_40_row_items_in_the_32_frame_variant(monkeypatch):
    """Regression: (32, 41, 3) with complex64 IQ stages 40-row items, whose last fill thread's run of 3 rows
    passes row 39; the rows past the window must not be stored (they are the next frame slot's row 0).  A
    coarse grid makes every window longer than 40 rows, so most items are exactly 40 rows, and voxels read
    row 0 of every frame slot."""
    monkeypatch.setenv("DAS_VARIANT", "32,41,3")
    xs = (np.arange(64) - 32) * 0.3e-3
    zs = 8e-3 + np.arange(32) * 0.3e-3
    vox = grid_2d(xs, zs)
    elem = linear_array(64, 0.3e-3)
    c = 1540.0
    p = dict(c=c, fs=20e6, fd=5e6, t0=0.0, f_number=1.0, tukey_alpha=0.5)
    tx = tx_table(vox, np.zeros((1, 2)), c)
    iq = random_iq((1, 64, 1024, 48), seed=45)
    y, info, _ = gpu_das(iq, elem, vox, tx, p)
    assert info["kernel"] == (32, 41, 3) and info["max_window"] > 80
    check_db(y, oracle.das(iq, elem, vox, tx, **p), "coarse grid, 40-row items")


def test_parity_boxcar_window():
    """tukey_alpha = 0 (the boxcar aperture) on a geometry where no (voxel, element) pair has its normalised
    lateral distance within 1e-4 of the aperture edge, so FP32 and FP64 take the same in/out decision."""
    elem = linear_array(128, 0.3e-3)
    xs = (np.arange(96) - 48) * 0.13e-3
    zs = 6e-3 + np.arange(64) * 0.17e-3
    vox = grid_2d(xs, zs)
    d = vox.astype(np.float64)[:, None, :] - elem.astype(np.float64)[None, :, :]
    rho = 2.0 * 1.0 * np.abs(d[..., 0]) / d[..., 2]
    keep = np.all(np.abs(rho - 1.0) > 1e-4, axis=1)
    vox = vox[keep]
    assert vox.shape[0] > 3000
    c = 1540.0
    p = dict(c=c, fs=20e6, fd=5e6, t0=0.0, f_number=1.0, tukey_alpha=0.0)
    tx = tx_table(vox, np.zeros((1, 2)), c)
    iq = random_iq((1, 128, 1024, 4), seed=46)
    y, info, _ = gpu_das(iq, elem, vox, tx, p)
    check_db(y, oracle.das(iq, elem, vox, tx, **p), "boxcar aperture %s" % (info["kernel"],))


@pytest.mark.parametrize("n_side,E,F,kernel", [(256, 8192, 8, (8, 65, 4)), (2510, 128, 8, (8, 65, 1))])
def test_parity_sweep_extremes_sampled(n_side, E, F, kernel):
    """The largest points of the element and voxel sweeps (8192 elements over the 38.4 mm aperture; a 2510 x 2510
    grid, 6.3 M voxels) with 8 frames, against the oracle on sampled voxels."""
    c, fc = 1540.0, 5e6
    p = dict(c=c, fs=4 * fc, fd=fc, t0=0.0, f_number=1.0, tukey_alpha=0.5)
    vox = grid_2d(np.linspace(-12.8e-3, 12.8e-3, n_side), np.linspace(10e-3, 35.5e-3, n_side))
    elem = linear_array(E, 38.4e-3 / E)
    tx = tx_table(vox, np.zeros((1, 2)), c)
    iq = random_iq((1, E, 2048, F), seed=38)
    y, info, _ = gpu_das(iq, elem, vox, tx, p)
    idx = np.sort(np.random.default_rng(39).choice(vox.shape[0], 128, replace=False))
    ref = oracle.das(iq, elem, vox[idx], tx[:, idx], **p)
    check_db(y[idx], ref, "sweep extreme %d^2 voxels, %d elements, %d frames %s" % (n_side, E, F, info["kernel"]))
    assert info["kernel"] == kernel and np.isfinite(y).all()


# ---------------------------------------------------------- special cases
def test_zero_in_zero_out_bitwise():
    cfg = make_config("c2", with_iq=False, n_frames=4)
    p = oracle_params(cfg)
    iq = np.zeros((1, 128, 2048, 4), np.complex64)
    y, *_ = gpu_das(iq, cfg["elem"], cfg["vox"], tx_table(cfg["vox"], cfg["angles"], p["c"]), p)
    assert np.all(y == 0)


def test_outside_aperture_is_exactly_zero():
    # voxels above the array plane get weight 0 with f# > 0; far-lateral voxels see no element in their aperture
    elem = linear_array(16, 0.3e-3)
    vox = np.array([[0, 0, -2e-3], [0, 0, 0.0], [40e-3, 0, 2e-3], [1e-3, 0, 10e-3]], np.float32)
    iq = random_iq((1, 16, 512, 3), seed=4)
    p = dict(c=1540.0, fs=20e6, fd=5e6, t0=0.0, f_number=1.0, tukey_alpha=0.5)
    tx = tx_table(vox, np.zeros((1, 2)), 1540.0)
    y, *_ = gpu_das(iq, elem, vox, tx, p)
    assert np.all(y[:3] == 0) and np.abs(y[3]).max() > 0
    ref = oracle.das(iq, elem, vox, tx, **p)
    assert oracle.nrmse_db(y, ref) <= DB_BAR


def test_deterministic_bitwise_across_runs_and_streams():
    cfg = make_config("c1", n_frames=3)
    p = oracle_params(cfg)
    tx = tx_table(cfg["vox"], cfg["angles"], p["c"])
    params = das.Params(1, 128, 1024, 3, cfg["vox"].shape[0], p["c"], p["fs"], p["fd"], 0.0, p["f_number"], 0.5)
    iq = dev(cfg["iq"])
    with das.Plan(params, dev(cfg["elem"]), dev(cfg["vox"]), dev(tx)) as plan:
        a = plan.execute(iq).clone()
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            b = plan.execute(iq, stream=s)
        s.synchronize()
        c = plan.execute(iq)
        torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_point_cloud_voxels_parity():
    # voxels that are not a lattice are grouped along a Morton curve
    r = np.random.default_rng(7)
    vox = np.stack([r.uniform(-5e-3, 5e-3, 3000), np.zeros(3000), r.uniform(5e-3, 20e-3, 3000)], 1).astype(np.float32)
    elem = linear_array(64, 0.3e-3)
    iq = random_iq((1, 64, 1200, 6), seed=8)
    p = dict(c=1540.0, fs=20e6, fd=5e6, t0=0.0, f_number=1.0, tukey_alpha=0.5)
    tx = tx_table(vox, np.zeros((1, 2)), 1540.0)
    y, info, _ = gpu_das(iq, elem, vox, tx, p)
    assert info["tile_dims"] == (0, 0, 0)
    assert oracle.nrmse_db(y, oracle.das(iq, elem, vox, tx, **p)) <= DB_BAR


def test_wide_windows_take_several_passes():
    # a coarse grid (1 mm steps) makes tile windows far longer than one LDS pass
    xs = (np.arange(32) - 16) * 1e-3
    zs = 5e-3 + np.arange(8) * 1e-3
    vox = grid_2d(xs, zs)
    elem = linear_array(32, 0.3e-3)
    iq = random_iq((2, 32, 1500, 32), seed=9)
    p = dict(c=1540.0, fs=20e6, fd=5e6, t0=0.0, f_number=0.0, tukey_alpha=0.5)
    tx = tx_table(vox, np.array([[0.0, 0.0], [0.2, 0.0]]), 1540.0)
    y, info, _ = gpu_das(iq, elem, vox, tx, p)
    assert info["max_window"] > 64   # more than one pass of the 32-frame kernel
    assert oracle.nrmse_db(y, oracle.das(iq, elem, vox, tx, **p)) <= DB_BAR


def test_empty_voxel_list():
    params = das.Params(1, 4, 16, 2, 0)
    elem = dev(linear_array(4, 0.3e-3))
    with das.Plan(params, elem, torch.zeros((0, 3), device="cuda"), torch.zeros((1, 0), device="cuda")) as plan:
        out = plan.execute(torch.zeros((1, 4, 16, 2), dtype=torch.complex64, device="cuda"))
        assert out.shape == (0, 2)
        assert plan.info()["n_tiles"] == 0


def test_plan_outlives_its_inputs():
    cfg = make_config("c1")
    p = oracle_params(cfg)
    tx = tx_table(cfg["vox"], cfg["angles"], p["c"])
    params = das.Params(1, 128, 1024, 1, cfg["vox"].shape[0], p["c"], p["fs"], p["fd"], 0.0, p["f_number"], 0.5)
    e, v, t = dev(cfg["elem"]), dev(cfg["vox"]), dev(tx)
    plan = das.Plan(params, e, v, t)
    del e, v, t
    torch.cuda.empty_cache()
    y = plan.execute(dev(cfg["iq"])).cpu().numpy()
    plan.close()
    assert oracle.nrmse_db(y, oracle.das(cfg["iq"], cfg["elem"], cfg["vox"], tx, **p)) <= DB_BAR


def test_binding_rejects_wrong_shapes_and_dtypes():
    cfg = make_config("c1", with_iq=False)
    p = oracle_params(cfg)
    tx = tx_table(cfg["vox"], cfg["angles"], p["c"])
    params = das.Params(1, 128, 1024, 1, cfg["vox"].shape[0], p["c"], p["fs"], p["fd"], 0.0, p["f_number"], 0.5)
    with das.Plan(params, dev(cfg["elem"]), dev(cfg["vox"]), dev(tx)) as plan:
        with pytest.raises(ValueError):
            plan.execute(torch.zeros((1, 128, 1024, 2), dtype=torch.complex64, device="cuda"))
        with pytest.raises(ValueError):
            plan.execute(torch.zeros((1, 128, 1024, 1), dtype=torch.complex128, device="cuda"))
        with pytest.raises(ValueError):
            plan.execute(torch.zeros((1, 128, 1024, 1), dtype=torch.complex64))  # host tensor


# ------------------------------------------------------- 16-bit IQ storage
@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_16bit_iq_parity_and_storage_error(kind):
    """c2 as the benchmark times it (32 frames), with IQ stored as FP16 / BF16: every voxel against the oracle
    on the same quantised samples (the FP32 arithmetic bar), and the storage error against the oracle on the
    complex64 input, reported in dB."""
    y, _, ref_q, info = _c2_reference(kind)
    check_db(y, ref_q, "c2 %s on the quantised samples %s" % (kind, info["kernel"]))
    ref = _c2_reference("c64")[2]
    db = oracle.nrmse_db(y, ref)
    print(kind, info["kernel"], "storage error vs complex64 input: %.1f dB (peak %.1f dB)"
          % (db, oracle.peak_err_db(y, ref)))
    assert db <= (-65.0 if kind == "f16" else -45.0)


def test_one_plan_on_two_streams_concurrently():
    """The plan is immutable: executing it on two streams at once gives the same bits as one at a time."""
    cfg = make_config("c2", with_iq=False, n_frames=8)
    p = cfg["params"]
    E, S = 128, p["n_samples"]
    iqa = random_iq((1, E, S, 8), seed=41)
    iqb = random_iq((1, E, S, 8), seed=42)
    tx = tx_table(cfg["vox"], cfg["angles"], p["c"])
    params = das.Params(1, E, S, 8, cfg["vox"].shape[0], p["c"], p["fs"], p["fd"], p["t0"], p["f_number"],
                        p["tukey_alpha"])
    with das.Plan(params, dev(cfg["elem"]), dev(cfg["vox"]), dev(tx)) as plan:
        a, b = dev(iqa), dev(iqb)
        ya, yb = plan.execute(a), plan.execute(b)
        torch.cuda.synchronize()
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        outs = []
        for _ in range(3):
            oa = torch.empty_like(ya)
            ob = torch.empty_like(yb)
            s1.wait_stream(torch.cuda.current_stream())
            s2.wait_stream(torch.cuda.current_stream())
            plan.execute(a, out=oa, stream=s1)
            plan.execute(b, out=ob, stream=s2)
            outs.append((oa, ob))
        torch.cuda.synchronize()
        for oa, ob in outs:
            assert torch.equal(oa, ya) and torch.equal(ob, yb)


@pytest.mark.parametrize("T,F,dtype,force", [(3, 1, "c64", None), (4, 2, "c64", None), (2, 1, "f16", None),
                                             (1, 1, "c64", None), (3, 1, "c64", "1,129,1"), (4, 2, "c64", "2,129,1"),
                                             (3, 1, "bf16", "1,65,2"), (4, 2, "c64", "2,257,2")])
def test_per_transmit_output(T, F, dtype, force, monkeypatch):
    """das_execute_per_tx: each transmit's volume equals a one-transmit plan's output (bitwise for single-group
    plans) and the FP64 oracle's (T = 1) volume; the sum over transmits equals the compounded call.  `force`
    pins a variant (this small grid would otherwise take four element groups)."""
    if force:
        monkeypatch.setenv("DAS_VARIANT", force)
    iq, elem, vox, tx, p = small_case(500 + 10 * T + F, T=T, E=12, S=64, F=F, V=700)
    y_c, _, iq_t = gpu_das(iq, elem, vox, tx, p, iq_dtype=dtype)
    params = das.Params(n_tx=T, n_elem=12, n_samples=64, n_frames=F, n_vox=vox.shape[0], sound_speed=p["c"],
                        fs=p["fs"], f_demod=p["fd"], t0=p["t0"], f_number=p["f_number"], tukey_alpha=p["tukey_alpha"])
    with das.Plan(params, dev(elem), dev(vox), dev(tx)) as plan:
        fc, _, groups = plan.info()["kernel"]
        assert fc <= 2
        if force:
            assert (fc, groups) == (int(force.split(",")[0]), int(force.split(",")[2]))
        y_t = plan.execute_per_tx(iq_t).cpu().numpy()
    assert y_t.shape == (T, vox.shape[0], F)
    iq_q = iq if dtype == "c64" else iq_t.float().cpu().numpy().view(np.complex64)[..., 0]
    for t in range(T):
        y1, _, _ = gpu_das(iq_q[t:t + 1], elem, vox, tx[t:t + 1], p)
        if dtype == "c64" and groups == 1:  # the same items in the same order
            np.testing.assert_array_equal(y_t[t], y1)
        else:  # element groups fold their partial sums in another order; or the 16-bit staging path
            np.testing.assert_allclose(y_t[t], y1, rtol=1e-5, atol=1e-6 * np.abs(y1).max())
        ref = oracle.das(iq_q[t:t + 1], elem, vox, tx[t:t + 1], **p)
        assert oracle.nrmse_db(y_t[t], ref) <= DB_BAR
    s = y_t.astype(np.complex128).sum(0)
    assert np.linalg.norm(s - y_c) <= 1e-6 * np.linalg.norm(y_c)


def test_per_transmit_output_rejects_unsupported_plans():
    iq, elem, vox, tx, p = small_case(77, T=5, E=6, S=40, F=1, V=50)
    params = das.Params(n_tx=5, n_elem=6, n_samples=40, n_frames=1, n_vox=50, sound_speed=p["c"], fs=p["fs"],
                        f_demod=p["fd"], t0=p["t0"], f_number=p["f_number"], tukey_alpha=p["tukey_alpha"])
    with das.Plan(params, dev(elem), dev(vox), dev(tx)) as plan:
        with pytest.raises(ValueError):
            plan.execute_per_tx(dev(iq))


@pytest.mark.parametrize("kind,F", [("f16", 32), ("bf16", 16), ("c64", 24)])
def test_paired_stages_parity(kind, F, monkeypatch):
    """Variants with 16 frames per workgroup stage two element windows per step: parity against the oracle on
    the same (quantised) samples, for each IQ type (their fill threads cover different row counts).  The grid
    is small enough that the plan would pick smaller frame chunks, so the variant is pinned."""
    monkeypatch.setenv("DAS_VARIANT", "16,65,2")
    iq, elem, vox, tx, p = small_case(900 + F, T=2, E=24, S=96, F=F, V=600, depth=(0.3e-3, 2.0e-3))
    y, info, iq_t = gpu_das(iq, elem, vox, tx, p, iq_dtype=kind)
    assert info["kernel"][0] == 16
    iq_q = iq if kind == "c64" else iq_t.float().cpu().numpy().view(np.complex64)[..., 0]
    ref = oracle.das(iq_q, elem, vox, tx, **p)
    db = oracle.nrmse_db(y, ref)
    print(kind, F, "nrmse dB", db, info)
    assert db <= DB_BAR


_VARIANT_REFS = {}


@pytest.mark.parametrize("F", [24, 23])
@pytest.mark.parametrize("kind", ["c64", "f16"])
def test_paired_fill_at_record_edges(F, kind, monkeypatch):
    """The paired variants' fill reads a zero row for samples outside the record: a 12-sample record and t0 past
    some delays put windows over row -1 and past the last row (the record's zero padding), with aligned (F = 24)
    and per-sample (F = 23, odd) loads."""
    iq, elem, vox, tx, p = small_case(1700 + F, T=2, E=16, S=12, F=F, V=300, t0=4e-7, depth=(0.3e-3, 1.0e-3))
    if kind == "f16":
        iq_t = torch.view_as_real(torch.from_numpy(iq)).to(torch.float16).contiguous()
        iq_q = iq_t.float().numpy().view(np.complex64)[..., 0]
    else:
        iq_t, iq_q = torch.from_numpy(iq), iq
    ref = oracle.das(iq_q, elem, vox, tx, **p)
    # delays below t0 and past the record: both edges of the zero padding are in play
    u = (tx[:, :, None] + np.linalg.norm(vox[None, :, None, :] - elem[None, None, :, :], axis=-1) / p["c"]
         - p["t0"]) * p["fs"]
    assert (np.floor(u) == -1).any() and (np.floor(u) == 11).any() and np.abs(ref).max() > 0
    params = das.Params(n_tx=2, n_elem=16, n_samples=12, n_frames=F, n_vox=vox.shape[0], sound_speed=p["c"],
                        fs=p["fs"], f_demod=p["fd"], t0=p["t0"], f_number=p["f_number"],
                        tukey_alpha=p["tukey_alpha"])
    for forced in [(16, 65, 2), (16, 33, 2), (32, 65, 2), (32, 41, 3)]:
        monkeypatch.setenv("DAS_VARIANT", "%d,%d,%d" % forced)
        with das.Plan(params, dev(elem), dev(vox), dev(tx)) as plan:
            assert plan.info()["kernel"] == forced
            y = plan.execute(iq_t.cuda()).cpu().numpy()
        check_db(y, ref, "paired fill %s F=%d %s" % (forced, F, kind))


@pytest.mark.parametrize("kind", ["c64", "f16", "bf16"])
def test_every_kernel_variant(kind, monkeypatch):
    """Every compiled variant (forced through DAS_VARIANT), for each IQ type: parity with the FP64 oracle on the
    same (quantised) samples, with a ragged last frame chunk (F = FC + FC / 2) and two transmits."""
    failures = []
    for fc, pitch, groups in das.kernel_variants():
        F = fc + max(1, fc // 2)
        key = (F, kind)
        if key not in _VARIANT_REFS:
            iq, elem, vox, tx, p = small_case(1200 + F, T=2, E=24, S=96, F=F, V=600, depth=(0.3e-3, 2.0e-3))
            iq_t = None
            if kind != "c64":
                dt = torch.float16 if kind == "f16" else torch.bfloat16
                iq_t = torch.view_as_real(torch.from_numpy(iq.astype(np.complex64))).to(dt).contiguous()
                iq_q = iq_t.float().numpy().view(np.complex64)[..., 0]
            else:
                iq_q = iq
            _VARIANT_REFS[key] = (iq_q, iq_t, elem, vox, tx, p, oracle.das(iq_q, elem, vox, tx, **p))
        iq_q, iq_t, elem, vox, tx, p, ref = _VARIANT_REFS[key]
        monkeypatch.setenv("DAS_VARIANT", "%d,%d,%d" % (fc, pitch, groups))
        params = das.Params(n_tx=2, n_elem=24, n_samples=96, n_frames=F, n_vox=vox.shape[0], sound_speed=p["c"],
                            fs=p["fs"], f_demod=p["fd"], t0=p["t0"], f_number=p["f_number"],
                            tukey_alpha=p["tukey_alpha"])
        with das.Plan(params, dev(elem), dev(vox), dev(tx)) as plan:
            got = plan.info()["kernel"]
            x = dev(iq_q.astype(np.complex64)) if kind == "c64" else iq_t.cuda()
            y = plan.execute(x).cpu().numpy()
        db = oracle.nrmse_db(y, ref)
        if got != (fc, pitch, groups) or not db <= DB_BAR:
            failures.append(((fc, pitch, groups), got, db))
    assert not failures, failures


@pytest.mark.parametrize("kind", ["c64", "f16", "bf16"])
def test_every_per_transmit_variant(kind, monkeypatch):
    """Every variant that has a per-transmit form (1 or 2 frames per workgroup), forced, for each IQ type: each
    transmit's volume against the FP64 oracle of that transmit alone on the same (quantised) samples."""
    T, F = 3, 2
    iq, elem, vox, tx, p = small_case(1300, T=T, E=16, S=80, F=F, V=600, depth=(0.3e-3, 2.0e-3))
    if kind == "c64":
        iq_q, x_host = iq, None
    else:
        dt = torch.float16 if kind == "f16" else torch.bfloat16
        x_host = torch.view_as_real(torch.from_numpy(iq.astype(np.complex64))).to(dt).contiguous()
        iq_q = x_host.float().numpy().view(np.complex64)[..., 0]
    refs = [oracle.das(iq_q[t:t + 1], elem, vox, tx[t:t + 1], **p) for t in range(T)]
    params = das.Params(n_tx=T, n_elem=16, n_samples=80, n_frames=F, n_vox=vox.shape[0], sound_speed=p["c"],
                        fs=p["fs"], f_demod=p["fd"], t0=p["t0"], f_number=p["f_number"], tukey_alpha=p["tukey_alpha"])
    x = dev(iq_q.astype(np.complex64)) if kind == "c64" else x_host.cuda()
    failures = []
    for fc, pitch, groups in das.kernel_variants():
        if fc > 2:
            continue
        monkeypatch.setenv("DAS_VARIANT", "%d,%d,%d" % (fc, pitch, groups))
        with das.Plan(params, dev(elem), dev(vox), dev(tx)) as plan:
            got = plan.info()["kernel"]
            y = plan.execute_per_tx(x).cpu().numpy()
        dbs = [oracle.nrmse_db(y[t], refs[t]) for t in range(T)]
        if got != (fc, pitch, groups) or not max(dbs) <= DB_BAR:
            failures.append(((fc, pitch, groups), got, dbs))
    assert not failures, failures
