"""Throughput benchmark of the gfx950 delay-and-sum path.

One step = one das_execute of the whole workload: every voxel, element,
transmit and frame (paper Eq. 1 points), inputs resident in HBM.  Default
workload: the rotating-disk stand-in (128-element linear array, 1 plane
wave, 32 frames of 2048 complex64 samples, 256 x 256 grid at 0.1 mm,
f-number 1), i.e. 268,435,456 points per step.

Prints one JSON line with points/s, the roofline of the dominant kernel and
the FP64 oracle timed on the host cores (run before the GPU is touched).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from synth import make_config  # noqa: E402

WORKLOADS = {
    "c2": "rotating-disk stand-in: 128-el linear array (0.3 mm), 1 plane wave at 0 deg, 32 frames x 2048 samples "
          "complex64 IQ (fc = fd = 5 MHz, fs = 20 MHz), 256 x 256 grid at 0.1 mm, f# 1.0 Tukey(0.5)",
    "c2_251": "paper-exact grid of the rotating-disk benchmark: as c2 with 251 x 251 voxels",
    "c1": "2D plane wave, 128-el linear array, 1 transmit, 1 frame x 1024 samples, 128 x 128 grid, f# 1.5",
    "c3": "3D: 32 x 32 matrix array, 5 elevation plane waves, 8 frames x 2048 samples, 96^3 grid, f# 1.0",
    "c3_f1": "c3 with 1 frame: the per-GPU share when c3's frames are split over 8 GPUs",
    "c3_v8": "c3 on the central 12 of its 96 x columns (110592 voxels, all 8 frames): the heaviest per-GPU share "
             "when c3's voxels are split over 8 GPUs in lateral slabs",
    "c3_v4f4": "c3 on the central 24 x columns with 4 frames: the heaviest per-GPU share of 4 slabs x 2 frame groups",
    "c3_v2f2": "c3 on the central 48 x columns with 2 frames: the heaviest per-GPU share of 2 slabs x 4 frame groups",
}
# workloads that are a listed configuration with other settings: (config, make_config overrides, x-column slice)
WORKLOAD_CONFIG = {"c3_f1": ("c3", {"n_frames": 1}, None), "c3_v8": ("c3", {}, (42, 54)),
                   "c3_v4f4": ("c3", {"n_frames": 4}, (36, 60)), "c3_v2f2": ("c3", {"n_frames": 2}, (24, 72))}
FLOP_PER_POINT = 16          # two complex multiply-accumulates per (voxel, element, transmit, frame)
PEAK_FP32_TFLOPS = 157.3     # MI355X published FP32 vector peak (256 CU x 2.4 GHz x 256 FLOP/clk)
PEAK_HBM_GBPS = 8000.0       # MI355X published HBM3E bandwidth
PAPER_PTS_PER_S = 258052096 / 0.23e-3   # RTX 5090, 251 x 251 rotating disk (context only)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "das_kernel_traffic.txt")


def kernel_source_hash():
    """SHA-256 over the sources the delay-and-sum kernel is built from (csrc/das_*)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2604_06257_amd", "csrc", "das_*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per launch recorded by rocprofv3 for the current kernel sources, else None."""
    try:
        lines = [l.split() for l in open(TRAFFIC_FILE) if l.strip() and not l.startswith("#")]
    except OSError:
        return None
    rec = {l[0]: l[1:] for l in lines}
    if rec.get("source_sha256", [None])[0] != kernel_source_hash() or workload not in rec:
        return None
    f = dict(zip(rec[workload][::2], rec[workload][1::2]))
    return int(f["read_bytes"]) + int(f["write_bytes"])


def _host_cpus():
    """(os.cpu_count(), the CPUs in this process's affinity mask, as a compact range list)."""
    try:
        aff = sorted(os.sched_getaffinity(0))
    except AttributeError:
        aff = list(range(os.cpu_count() or 1))
    runs, start = [], None
    for i, c in enumerate(aff):
        if start is None:
            start = c
        if i + 1 == len(aff) or aff[i + 1] != c + 1:
            runs.append("%d" % start if start == c else "%d-%d" % (start, c))
            start = None
    return os.cpu_count(), aff, ",".join(runs)


def _cores():
    """Worker processes for the oracle: the CPUs this process may run on, at most 16 (the machine's CPU share
    of one GPU)."""
    return max(1, min(16, len(_host_cpus()[1])))


_SHARED = {}


def _oracle_chunk(bounds):
    import oracle
    a, b = bounds
    s = _SHARED
    return a, oracle.das(s["iq"], s["elem"], s["vox"][a:b], s["tx"][:, a:b], **s["p"])


def cpu_baseline(cfg, max_voxels, min_seconds=10.0):
    """FP64 oracle on the host cores (fork pool over voxel chunks), timed over at least min_seconds."""
    import multiprocessing as mp

    import oracle
    p = cfg["params"]
    vox = cfg["vox"][:max_voxels]
    tx = oracle.tx_plane_wave(vox, cfg["angles"], p["c"]).astype(np.float32)
    _SHARED.update(iq=cfg["iq"], elem=cfg["elem"], vox=vox, tx=tx,
                   p=dict(c=p["c"], fs=p["fs"], fd=p["fd"], t0=p["t0"], f_number=p["f_number"],
                          tukey_alpha=p["tukey_alpha"]))
    cores = _cores()
    V = vox.shape[0]
    chunk = max(1, -(-V // (4 * cores)))
    bounds = [(a, min(V, a + chunk)) for a in range(0, V, chunk)]
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    reps = 0
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        # repeat the sample until about min_seconds of host time have been measured (the first pass is kept)
        while True:
            out = pool.map(_oracle_chunk, bounds)
            if reps == 0:
                parts = out
            reps += 1
            if time.perf_counter() - t0 >= min_seconds:
                break
    dt = time.perf_counter() - t0
    y = np.zeros((V, p["n_frames"]), np.complex128)
    for a, part in parts:
        y[a:a + part.shape[0]] = part
    T, E = cfg["iq"].shape[:2]
    pts = V * E * T * p["n_frames"]
    # one core: the first voxels of the same sample in this process, repeated for about 3 s
    n1 = max(1, V // 64)
    reps1, t1 = 0, time.perf_counter()
    while True:
        _oracle_chunk((0, n1))
        reps1 += 1
        if time.perf_counter() - t1 >= 3.0:
            break
    dt1 = time.perf_counter() - t1
    pts1 = n1 * E * T * p["n_frames"]
    n_cpu, aff, aff_txt = _host_cpus()
    return y, {"value": reps * pts / dt, "unit": "points/s", "cores": cores, "kind": "oracle",
               "seconds": round(dt, 3), "repeats": reps,
               "host_cpu_count": n_cpu, "affinity_cpus": len(aff), "affinity_mask": aff_txt,
               "single_core": {"value": reps1 * pts1 / dt1, "unit": "points/s", "seconds": round(dt1, 3),
                               "sample": "%d voxels x all elements, transmits, frames = %d points, %d times"
                                         % (n1, pts1, reps1)},
               "sample": "%d voxels (all %d elements, %d transmit(s), %d frames) = %d points, computed %d times, "
                         "voxel chunks over %d processes" % (V, E, T, p["n_frames"], pts, reps, cores)}


def time_steps(plan, iq, out, steps, warmup, torch):
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.execute(iq, out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        plan.execute(iq, out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def time_launches(plan, iq, out, repeats, torch, flush=None):
    """Per-launch kernel times (HIP events around each launch on the launch stream): (median, min) in ms.

    With ``flush`` (a 1 GiB device buffer) the buffer is rewritten before every launch so that the
    launch starts with cold caches (L2 and the 256 MB Infinity Cache evicted)."""
    stream = torch.cuda.current_stream()
    times = []
    plan.execute(iq, out)
    for _ in range(repeats):
        if flush is not None:
            flush.fill_(1.0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.execute(iq, out)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2], times[0]


def iq16_range(iq):
    """Largest |component| of complex64 IQ and the fraction of nonzero components that are subnormal
    when stored as float16 / bfloat16 (round to nearest even; overflow needs max >= 65504 for float16)."""
    ri = np.abs(np.stack([iq.real, iq.imag]).ravel().astype(np.float32))
    nz = ri[ri > 0]
    with np.errstate(over="ignore"):  # components beyond float16's range become inf (reported by fits_fp16)
        f16 = np.abs(nz.astype(np.float16).astype(np.float32))
    sub16 = float(np.mean((f16 > 0) & (f16 < 2.0 ** -14))) if nz.size else 0.0
    # bfloat16 keeps float32's exponent range: subnormal below 2^-126
    subbf = float(np.mean(nz < 2.0 ** -126)) if nz.size else 0.0
    return {"max_abs_component": float(ri.max()) if ri.size else 0.0, "fits_fp16": bool(ri.max() < 65504.0),
            "fp16_subnormal_fraction": sub16, "bf16_subnormal_fraction": subbf,
            "fp16_flushed_to_zero_fraction": float(np.mean(f16 == 0)) if nz.size else 0.0}


def scaling_sweep(axis, steps, warmup):
    """Throughput while one size varies around the rotating-disk stand-in (paper Sec. 4.5, Fig. 5):
    voxels 63k-6.3M (finer grids over the same region), elements 128-8192 (same aperture), frames 1-512.
    IQ is seeded circular-Gaussian data generated on the device; one JSON line per point."""
    import torch

    import paper_2604_06257_amd as das
    from synth import grid_2d, linear_array

    c, fc = 1540.0, 5e6
    fs, S = 4 * fc, 2048
    base = dict(n_side=256, n_elem=128, frames=32)
    points = {"voxels": [("n_side", n) for n in (251, 502, 1004, 1587, 2510)],
              "elements": [("n_elem", e) for e in (128, 256, 512, 1024, 2048, 4096, 8192)],
              "frames": [("frames", f) for f in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512)]}[axis]
    gen = torch.Generator(device="cuda")
    for key, val in points:
        cfg = dict(base)
        cfg[key] = val
        n, E, F = cfg["n_side"], cfg["n_elem"], cfg["frames"]
        xs = np.linspace(-12.8e-3, 12.8e-3, n)
        zs = np.linspace(10e-3, 35.5e-3, n)
        vox = torch.from_numpy(grid_2d(xs, zs)).cuda()
        elem = torch.from_numpy(linear_array(E, 38.4e-3 / E)).cuda()
        tx = das.tx_plane_wave(vox, np.zeros((1, 2)), c)
        gen.manual_seed(1000 + val)
        iq = torch.randn((1, E, S, F), dtype=torch.complex64, device="cuda", generator=gen)
        params = das.Params(1, E, S, F, vox.shape[0], c, fs, fc, 0.0, 1.0, 0.5)
        with das.Plan(params, elem, vox, tx) as plan:
            info = plan.info()
            out = torch.empty((vox.shape[0], F), dtype=torch.complex64, device="cuda")
            ms, _ = time_steps(plan, iq, out, steps, warmup, torch)
        pts = vox.shape[0] * E * F
        print(json.dumps({"sweep": axis, "voxels": vox.shape[0], "elements": E, "frames": F, "ms_per_step": ms,
                          "points_per_s": pts / (ms * 1e-3), "active_fraction": info["active_triples"] /
                          max(1, info["total_triples"]), "kernel": "fc=%d pitch=%d groups=%d" % info["kernel"]}),
              flush=True)
        del iq, out


def c3_report(steps, warmup, torch, das, oracle):
    """c3 (the largest single-GPU workload: 96^3 voxels, 32 x 32 elements, 5 plane waves, 8 frames) timed in
    the same run: channel data from the GPU echo simulator (the input generator's model), the plan's variant, ms
    per launch, points/s (Eq. 1), the roofline fraction of its kernel and the error against the FP64 oracle on
    a sample of voxels."""
    from synth import echo_iq_gpu
    cfg = make_config("c3", with_iq=False)
    p = cfg["params"]
    T, E, S, F = cfg["angles"].shape[0], cfg["elem"].shape[0], p["n_samples"], p["n_frames"]
    V = cfg["vox"].shape[0]
    iq = echo_iq_gpu(cfg["elem"], cfg["angles"], cfg["scat"], cfg["amp"], n_samples=S, n_frames=F, c=p["c"],
                     fs=p["fs"], fc=p["fc"], fd=p["fd"], t0=p["t0"])
    vox = torch.from_numpy(cfg["vox"]).cuda()
    tx = das.tx_plane_wave(vox, cfg["angles"], p["c"])
    params = das.Params(T, E, S, F, V, p["c"], p["fs"], p["fd"], p["t0"], p["f_number"], p["tukey_alpha"])
    with das.Plan(params, torch.from_numpy(cfg["elem"]).cuda(), vox, tx) as plan:
        info = plan.info()
        out = torch.empty((V, F), dtype=torch.complex64, device="cuda")
        ms, _ = time_steps(plan, iq, out, steps, warmup, torch)
        y = out.cpu().numpy()
    idx = np.arange(0, V, V // 48)[:48]  # 48 voxels spread over the grid
    ref = oracle.das(iq.cpu().numpy(), cfg["elem"], cfg["vox"][idx], tx.cpu().numpy()[:, idx], c=p["c"], fs=p["fs"],
                     fd=p["fd"], t0=p["t0"], f_number=p["f_number"], tukey_alpha=p["tukey_alpha"])
    pts = V * E * T * F
    tflops = info["active_triples"] * F * FLOP_PER_POINT / (ms * 1e-3) / 1e12
    return {"workload": "c3: " + WORKLOADS["c3"], "ms_per_step": ms, "value": pts / (ms * 1e-3),
            "unit": "points/s", "points_per_step": pts,
            "active_points_per_s": info["active_triples"] * F / (ms * 1e-3),
            "kernel": "das_kernel<fc=%d, pitch=%d, groups=%d>" % info["kernel"],
            "roofline": {"bound": "alu", "achieved": tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / PEAK_FP32_TFLOPS, "traffic": measured_traffic("c3")},
            "nrmse_db_vs_fp64": oracle.nrmse_db(y[idx], ref), "peak_err_db_vs_fp64": oracle.peak_err_db(y[idx], ref),
            "parity_sample": "%d voxels (every %d-th), all elements, transmits and frames" % (len(idx), V // 48),
            "iq": "GPU echo simulator: 20000 speckle scatterers per frame + 50 points"}


def hbm_report(T, E, S, F, V, info, ms, traffic):
    """The HBM side of the roofline for one launch: compulsory bytes (IQ read once, output written once, the
    transmit table and the voxel and element coordinates), their rate against the 8 TB/s peak, the measured HBM
    bytes (PMC record) as a rate, and the kernel's on-chip gather rate (16 B of LDS operands per processed point
    and frame)."""
    compulsory = T * E * S * F * 8 + V * F * 8 + T * V * 4 + V * 12 + E * 12
    sec = ms * 1e-3
    rep = {"compulsory_bytes": compulsory, "compulsory_GBps": compulsory / sec / 1e9,
           "peak_GBps": PEAK_HBM_GBPS, "frac": compulsory / sec / 1e9 / PEAK_HBM_GBPS,
           "measured_bytes": traffic, "measured_GBps": None if traffic is None else traffic / sec / 1e9,
           "gather_GBps": info["processed_triples"] * F * 16 / sec / 1e9,
           "note": "the path is bound on chip (VALU, LDS), not by HBM: its intensity is far above the ridge"}
    return rep


C5_WEIGHTS = os.path.join(ROOT, "paper_2604_06257_amd", "weights", "unet_c5.npz")


def c5_report(n_test=20):
    """Learned compounding (c5: 96^3 voxels, 32 x 32 elements, 11 plane waves, 1 frame) with the stored weights of
    the network trained on 1800 phantoms, on n_test freshly generated held-out phantoms (the training run's test
    seeds): NRMSE against the 11-angle compound of (11/3) x the 3-angle sum and of the network, the 11-angle DAS
    time and the learned path's (3-angle per-transmit DAS + features + network)."""
    from paper_2604_06257_amd import train_compound
    r = train_compound.evaluate_checkpoint(C5_WEIGHTS, n_test=n_test)
    return {"workload": "c5: learned compounding of 3 of 11 plane waves (-10, 0, +10 deg), 96^3 grid, "
                        "32 x 32 array, 1 frame; stored weights, held-out phantoms generated here",
            "n_test": r["n_test"], "test_phantom_seeds": r["test_phantom_seeds"],
            "nrmse_db_vs_11_angle": r["nrmse_db_vs_full_compound"], "gain_db": r["gain_db"],
            "ms": r["ms"], "speedup_vs_11_angle_das": r["speedup"], "trained": r["trained"]}


def unet_forward_report(steps, warmup, dims=(96, 96, 96)):
    """Forward pass of the learned-compounding U-Net (random weights, random bfloat16 input) on a dims grid: the
    whole forward, then each convolution alone (HIP events around each call, median over the steps), with its
    FLOPs (2 x 27 x Cin x Cout per voxel) as a share of the 2.5 PFLOP/s dense BF16 MFMA peak."""
    import torch
    from paper_2604_06257_amd import learn
    U = learn.UNet(dims)
    V = dims[0] * dims[1] * dims[2]
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    x = torch.randn((V, U.cin), device="cuda", generator=g).to(torch.bfloat16)

    def timed_forward(n):
        for _ in range(warmup):
            U.forward(x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            U.forward(x)
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / n

    fw_ms = timed_forward(steps)
    orig, rec = learn.conv3d, []

    def conv_timed(xx, w, bias, out, d, **kw):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = orig(xx, w, bias, out, d, **kw)
        e1.record()
        rec.append((tuple(d), learn._whole(xx).c, learn._whole(out).c, e0, e1))
        return r

    learn.conv3d = conv_timed
    try:
        for _ in range(warmup):
            U.forward(x)
        torch.cuda.synchronize()
        rec.clear()
        for _ in range(steps):
            U.forward(x)
        torch.cuda.synchronize()
    finally:
        learn.conv3d = orig
    per = len(rec) // steps
    layers, flops = [], 0
    for i, (name, _, _) in enumerate(learn.layer_shapes(U.cin, U.chans, U.cout)[:per]):
        d, ci, co = rec[i][:3]
        ts = sorted(rec[i + j * per][3].elapsed_time(rec[i + j * per][4]) for j in range(steps))
        us = 1e3 * ts[steps // 2]
        fl = 2 * 27 * ci * co * d[0] * d[1] * d[2]
        flops += fl
        layers.append({"layer": name, "dims": list(d), "cin": ci, "cout": co, "us": us,
                       "tflops": fl / us / 1e6, "frac_bf16_peak": fl / us / 1e6 / 2500.0})
    return {"unet_forward": {"dims": list(dims), "gflop": flops / 1e9, "ms": fw_ms,
                             "tflops": flops / fw_ms / 1e9, "frac_bf16_peak": flops / fw_ms / 1e9 / 2500.0,
                             "steps": steps, "layers": layers,
                             "note": "random weights and input; forward only; the peak is the dense BF16 MFMA "
                                     "2.5 PFLOP/s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the FP16 / BF16 IQ timings")
    ap.add_argument("--no-c3", action="store_true", help="skip the c3 sub-object")
    ap.add_argument("--no-c5", action="store_true", help="skip the c5 (learned compounding) sub-object")
    ap.add_argument("--cpu-voxels", type=int, default=None, help="voxels in the oracle sample (default: all)")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="also run a torch copy of this many GiB (for HBM counter calibration)")
    ap.add_argument("--post", action="store_true",
                    help="also time B-mode and Power Doppler (SVD clutter filter, rank 1) on the beamformed frames")
    ap.add_argument("--sweep", choices=("voxels", "elements", "frames"), default=None,
                    help="print one JSON line per size along this axis instead of the benchmark line")
    ap.add_argument("--unet", action="store_true",
                    help="print the learned-compounding U-Net forward timing at 96^3 (one JSON line) instead")
    args = ap.parse_args()
    if args.unet:
        print(json.dumps(unet_forward_report(max(5, min(args.steps, 50)), max(2, min(args.warmup, 5)))))
        return
    if args.sweep:
        scaling_sweep(args.sweep, args.steps, args.warmup)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the beamforming path runs on a single MI355X "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    name, overrides, xcols = WORKLOAD_CONFIG.get(args.workload, (args.workload, {}, None))
    cfg = make_config(name, **overrides)
    if xcols is not None:
        xs = np.unique(cfg["vox"][:, 0])
        cfg["vox"] = np.ascontiguousarray(cfg["vox"][np.isin(cfg["vox"][:, 0], xs[xcols[0]:xcols[1]])])
    p = cfg["params"]
    iq_np = cfg["iq"]
    T, E, S, F = iq_np.shape
    V = cfg["vox"].shape[0]
    points = V * E * T * F

    ref = base = None
    if not args.no_cpu_baseline:
        nv = V if args.cpu_voxels is None else min(V, args.cpu_voxels)
        ref, base = cpu_baseline(cfg, nv)

    import torch

    import oracle
    import paper_2604_06257_amd as das

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    vox = dev(cfg["vox"])
    tx = das.tx_plane_wave(vox, cfg["angles"], p["c"])
    params = das.Params(T, E, S, F, V, p["c"], p["fs"], p["fd"], p["t0"], p["f_number"], p["tukey_alpha"])
    plan = das.Plan(params, dev(cfg["elem"]), vox, tx)
    info = plan.info()
    iq = dev(iq_np)
    out = torch.empty((V, F), dtype=torch.complex64, device="cuda")
    ms, wall = time_steps(plan, iq, out, args.steps, args.warmup, torch)
    value = points / (ms * 1e-3)
    warm_med, warm_min = time_launches(plan, iq, out, 51, torch)
    flush = torch.empty((1 << 30) // 4, dtype=torch.float32, device="cuda")
    cold_med, cold_min = time_launches(plan, iq, out, 21, torch, flush=flush)
    del flush

    active_pts = info["active_triples"] * F
    achieved_tflops = active_pts * FLOP_PER_POINT / (ms * 1e-3) / 1e12
    result = {
        "metric": "points/s (voxel x element x tx x frame) FP32 vs FP16-IQ, error in dB vs FP64",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload + ": " + WORKLOADS[args.workload], "voxels": V, "elements": E,
                   "transmits": T, "frames": F, "samples": S, "points_per_step": points, "iq": "complex64",
                   "parallelism": "single GPU"},
        "wall_ms_per_step": wall * 1e3 / args.steps,
        "per_launch_ms": {"warm_median": warm_med, "warm_min": warm_min, "cold_median": cold_med,
                          "cold_min": cold_min, "cold_points_per_s": points / (cold_med * 1e-3),
                          "cold": "1 GiB buffer rewritten before each launch (L2 and Infinity Cache evicted)"},
        "active_points_per_s": active_pts / (ms * 1e-3),
        "active_fraction": info["active_triples"] / max(1, info["total_triples"]),
        "processed_fraction": info["processed_triples"] / max(1, info["total_triples"]),
        "plan": {"tiles": info["n_tiles"], "tile_dims": info["tile_dims"], "max_window": info["max_window"],
                 "kernel": "das_kernel<fc=%d, pitch=%d, groups=%d>" % info["kernel"]},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / PEAK_FP32_TFLOPS, "traffic": measured_traffic(args.workload),
                     "kernel": "das_kernel<fc=%d, pitch=%d, complex64, groups=%d>" % info["kernel"],
                     "work": "%d FLOP x active points (w > 0, inside the record) per launch" % FLOP_PER_POINT},
        "hbm": hbm_report(T, E, S, F, V, info, ms, measured_traffic(args.workload)),
        "paper_context": {"points_per_s": PAPER_PTS_PER_S, "hardware": "NVIDIA GeForce RTX 5090",
                          "workload": "PyMUST rotating disk 251 x 251, 32 frames"},
    }
    y = out.cpu().numpy()
    if ref is not None:
        nv = ref.shape[0]
        result["nrmse_db_vs_fp64"] = oracle.nrmse_db(y[:nv], ref)
        result["peak_err_db_vs_fp64"] = oracle.peak_err_db(y[:nv], ref)
        result["cpu_baseline"] = base
    if not args.no_variants:
        var = {}
        ri = torch.view_as_real(iq)
        for name, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
            iq16 = ri.to(dt).contiguous()
            out16 = torch.empty_like(out)
            ms16, _ = time_steps(plan, iq16, out16, args.steps, args.warmup, torch)
            v = {"value": points / (ms16 * 1e-3), "ms_per_step": ms16, "dtype": "f32 (IQ stored %s)" % name}
            if ref is not None:
                y16 = out16.cpu().numpy()
                v["nrmse_db_vs_fp64"] = oracle.nrmse_db(y16[:ref.shape[0]], ref)
            var[name] = v
            del iq16
        var["iq_range"] = iq16_range(iq_np)
        result["iq16_variants"] = var
    if not args.no_c3 and args.workload != "c3":
        result["c3"] = c3_report(max(5, args.steps // 10), max(2, args.warmup // 4), torch, das, oracle)
        torch.cuda.empty_cache()
    if not args.no_c5 and args.workload == "c2":
        result["c5"] = c5_report()
        torch.cuda.empty_cache()
    if args.post:
        from paper_2604_06257_amd import post
        plan.execute(iq, out)
        pm = {}
        for name, fn in (("bmode_60db", lambda: post.bmode(out, 60.0)),
                         ("power_doppler_k1", lambda: post.power_doppler(out, 1))):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                fn()
            e1.record()
            e1.synchronize()
            pm[name] = e0.elapsed_time(e1) / 20
        pm["beamform"] = result["ms_per_step"]
        result["post_ms"] = pm
    if args.copy_calibration > 0:
        n = int(args.copy_calibration * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = 4 * n
    plan.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
