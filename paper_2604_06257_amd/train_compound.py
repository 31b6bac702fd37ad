"""Train and evaluate learned compounding on seeded synthetic phantoms.

    python -m paper_2604_06257_amd.train_compound --geometry c5 --n-train 1800 --n-val 100 --n-test 100 --steps 12000

Data: per phantom (seed base + i; training, validation and test phantoms in
that order) the GPU echo simulator writes the IQ of all
plane waves, the library beamforms the full compound (the target) and the
input angles one by one; features are normalised by the RMS of the
input-angle sum.  Everything stays in device memory.  Training is Adam on one
volume per step; the validation set picks the checkpoint; evaluation reports the normalised RMS error in dB against
the full compound for the scaled few-angle sum (no network) and for the
network, and the speedup t(full) / (t(input angles) + t(features) +
t(network) + t(output)); the input angles are beamformed from their own
channel data, [A, E, S, 1], as an acquisition of only those angles records it.

``--geometry small`` is a reduced case (8 x 8 array, 32^3 grid, 512 samples)
for quick runs.
"""

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import das as _das
from .compound import LearnedCompounding

MM = 1e-3
DEG = math.pi / 180.0


def geometry(name):
    """Array, grid, angles and acquisition parameters; phantom(seed) -> (scat, amp)."""
    from synth import make_config, matrix_array, grid_3d, volume_phantom
    if name == "c5":
        cfg = make_config("c5", with_iq=False)
        elem, vox, ang, p = cfg["elem"], cfg["vox"], cfg["angles"], cfg["params"]
        dims = cfg["grid_shape"]
        lo, hi = vox.min(0).astype(np.float64), vox.max(0).astype(np.float64)
        n_speckle, n_points, seed0 = 20000, 50, 10000
    elif name == "small":
        elem = matrix_array(8, 8, 0.3 * MM)
        xs = (np.arange(32) - 16) * 0.1 * MM
        zs = 2 * MM + np.arange(32) * 0.1 * MM
        vox = grid_3d(xs, xs, zs)
        dims = (32, 32, 32)
        ang = np.array([[0.0, ph * DEG] for ph in range(-10, 11, 2)])
        p = dict(c=1540.0, fs=60e6, fc=15e6, fd=15e6, t0=0.0, f_number=1.0, tukey_alpha=0.5, n_samples=512,
                 n_frames=1)
        lo, hi = vox.min(0).astype(np.float64), vox.max(0).astype(np.float64)
        n_speckle, n_points, seed0 = 1000, 10, 50000
    else:
        raise ValueError("unknown geometry %r" % name)

    def phantom(i):
        rng = np.random.default_rng(seed0 + i)
        return volume_phantom(rng, 1, lo, hi, n_speckle=n_speckle, n_points=n_points)
    # input angles: the two extremes and the centre
    T = ang.shape[0]
    return dict(elem=elem, vox=vox, angles=ang, params=p, dims=tuple(dims), phantom=phantom,
                input_idx=[0, T // 2, T - 1])


class Dataset:
    """Device-resident inputs, baselines and targets of n phantoms."""

    def __init__(self, lc, geo, n, first=0, log=None):
        from synth import echo_iq_gpu
        p = geo["params"]
        V = lc.V
        dev = lc.x.device
        self.n = n
        self.x = torch.zeros((n, V, lc.x.shape[1]), dtype=torch.bfloat16, device=dev)
        self.base = torch.zeros((n, V, 2), dtype=torch.float32, device=dev)
        self.target = torch.zeros((n, V, 2), dtype=torch.float32, device=dev)
        T, E = geo["angles"].shape[0], geo["elem"].shape[0]
        iq = torch.empty((T, E, p["n_samples"], 1), dtype=torch.complex64, device=dev)
        y_full = torch.empty((V, 1), dtype=torch.complex64, device=dev)
        t0 = time.time()
        for i in range(n):
            scat, amp = geo["phantom"](first + i)
            echo_iq_gpu(geo["elem"], geo["angles"], scat, amp, n_samples=p["n_samples"], n_frames=1, c=p["c"],
                        fs=p["fs"], fc=p["fc"], fd=p["fd"], t0=p["t0"], out=iq, device=dev)
            lc.full_compound(iq, out=y_full)
            lc.beamform_inputs(lc.input_iq(iq))
            lc.features()
            self.x[i].copy_(lc.x)
            self.base[i].copy_(lc.base)
            lc.normalised_target(y_full, self.target[i])
            if log and (i + 1) % max(1, n // 10) == 0:
                torch.cuda.synchronize()
                log("data %d/%d phantoms (%.1f s)" % (i + 1, n, time.time() - t0))
        torch.cuda.synchronize()


def nrmse_db(pred, target):
    """20 log10(||pred - target|| / ||target||) over a batch of volumes (float64 sums)."""
    num = (pred.double() - target.double()).pow(2).sum()
    den = target.double().pow(2).sum()
    return 10.0 * math.log10(float(num) / float(den))


def lr_at(step, steps, lr, warmup=100):
    if step < warmup:
        return lr * (step + 1) / warmup
    return lr * 0.5 * (1.0 + math.cos(math.pi * (step - warmup) / max(1, steps - warmup)))


def evaluate(lc, data):
    """(baseline dB, network dB) over the data set's volumes."""
    net = lc.net
    preds = torch.empty_like(data.base)
    for i in range(data.n):
        net.forward(data.x[i])
        torch.add(data.base[i], net.net[:, :2], out=preds[i])
    return nrmse_db(data.base, data.target), nrmse_db(preds, data.target)


def time_paths(lc, geo, reps=5):
    """Average ms of the full compound and of each stage of the learned path (HIP events)."""
    from synth import echo_iq_gpu
    p = geo["params"]
    dev = lc.x.device
    scat, amp = geo["phantom"](10 ** 6)
    iq = echo_iq_gpu(geo["elem"], geo["angles"], scat, amp, n_samples=p["n_samples"], n_frames=1, c=p["c"],
                     fs=p["fs"], fc=p["fc"], fd=p["fd"], t0=p["t0"], device=dev)
    iq_in = lc.input_iq(iq)  # what an acquisition of only the input angles records
    y = torch.empty((lc.V, 1), dtype=torch.complex64, device=dev)
    out = torch.empty((lc.V, 1), dtype=torch.complex64, device=dev)
    stages = {"full_das": lambda: lc.full_compound(iq, out=y),
              "input_das": lambda: lc.beamform_inputs(iq_in),
              "features": lambda: lc.features(),
              "network": lambda: lc.net.forward(lc.x),
              "learned_total": lambda: lc.predict(iq_in, out=out)}
    res = {}
    for name, fn in stages.items():
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        res[name] = a.elapsed_time(b) / reps
    return res


def run(args, log=print):
    geo = geometry(args.geometry)
    p = geo["params"]
    dev = torch.device("cuda")
    elem = torch.as_tensor(np.ascontiguousarray(geo["elem"], dtype=np.float32), device=dev)
    vox = torch.as_tensor(np.ascontiguousarray(geo["vox"], dtype=np.float32), device=dev)
    tx = _das.tx_plane_wave(vox, geo["angles"], p["c"])
    T, E, V = geo["angles"].shape[0], elem.shape[0], vox.shape[0]
    params = _das.Params(T, E, p["n_samples"], 1, V, p["c"], p["fs"], p["fd"], p["t0"], p["f_number"],
                         p["tukey_alpha"])
    lc = LearnedCompounding(params, elem, vox, tx, geo["dims"], geo["input_idx"])
    lc.net.init_params(seed=args.seed)
    n_val = getattr(args, "n_val", 0)
    eval_every = getattr(args, "eval_every", 0) or args.steps
    t0 = time.time()
    train = Dataset(lc, geo, args.n_train, first=0, log=log)
    val = Dataset(lc, geo, n_val, first=args.n_train, log=log) if n_val > 0 else None
    test = Dataset(lc, geo, args.n_test, first=args.n_train + n_val, log=log)
    t_data = time.time() - t0
    log("data: %d train + %d validation + %d test phantoms in %.1f s" % (args.n_train, n_val, args.n_test, t_data))
    base_db, net0_db = evaluate(lc, test)
    log("before training: baseline %.2f dB, network %.2f dB" % (base_db, net0_db))
    order = np.random.default_rng(args.seed).permutation(args.n_train)
    best = None  # (validation dB, step, master weights) of the best checkpoint
    val_curve = []
    t0 = time.time()
    run_loss = 0.0
    for step in range(args.steps):
        i = int(order[step % args.n_train])
        if step % args.n_train == args.n_train - 1:
            order = np.random.default_rng(args.seed + step).permutation(args.n_train)
        parts = lc.net.train_step(train.x[i], train.base[i], train.target[i], lr_at(step, args.steps, args.lr))
        if (step + 1) % args.log_every == 0:
            run_loss = float(parts.sum()) / (2 * V)
            log("step %d/%d loss %.4e lr %.2e (%.1f s)" % (step + 1, args.steps, run_loss,
                                                          lr_at(step, args.steps, args.lr), time.time() - t0))
        if val is not None and ((step + 1) % eval_every == 0 or step + 1 == args.steps):
            vdb = evaluate(lc, val)[1]
            val_curve.append((step + 1, round(vdb, 3)))
            log("step %d validation network %.3f dB" % (step + 1, vdb))
            if best is None or vdb < best[0]:
                best = (vdb, step + 1, lc.net.master.clone())
    torch.cuda.synchronize()
    t_train = time.time() - t0
    if best is not None:  # the checkpoint with the lowest validation error
        lc.net.master.copy_(best[2])
        lc.net.refresh_copies()
    base_db, net_db = evaluate(lc, test)
    train_base_db, train_net_db = evaluate(lc, train) if args.n_train <= 200 else (None, None)
    times = time_paths(lc, geo)
    speedup = times["full_das"] / times["learned_total"]
    res = {"geometry": args.geometry, "dims": list(geo["dims"]), "n_elem": E, "n_angles": T,
           "input_angles_deg": [round(float(geo["angles"][t, 1]) / DEG, 3) for t in geo["input_idx"]],
           "n_train": args.n_train, "n_val": n_val, "n_test": args.n_test, "steps": args.steps, "lr": args.lr,
           "validation_nrmse_db": val_curve, "checkpoint_step": best[1] if best is not None else args.steps,
           "test_nrmse_db": {"scaled_input_sum": round(base_db, 3), "network": round(net_db, 3),
                             "network_untrained": round(net0_db, 3)},
           "gain_db": round(base_db - net_db, 3),
           "train_nrmse_db": None if train_base_db is None else {"scaled_input_sum": round(train_base_db, 3),
                                                               "network": round(train_net_db, 3)},
           "ms": {k: round(v, 4) for k, v in times.items()}, "speedup": round(speedup, 3),
           "net_gflop_forward": round(lc.net.flops_forward() / 1e9, 2),
           "net_tflops_forward": round(lc.net.flops_forward() / (times["network"] * 1e-3) / 1e12, 2),
           "seconds": {"data": round(t_data, 1), "train": round(t_train, 1)},
           "ms_per_train_step": round(1e3 * t_train / max(1, args.steps), 3)}
    if getattr(args, "save_weights", None):
        save_weights(lc.net, args.save_weights, res)
    lc.close()
    return res


def save_weights(net, path, summary=None):
    """The network's FP32 master weights as a NumPy archive (no pickled objects): arrays '<layer>.w' [Cout, 27,
    Cin] and '<layer>.b' [Cout], plus 'summary' (the training record as JSON text)."""
    arrays = {}
    for name, (w, b) in net.get_params().items():
        arrays[name + ".w"] = w
        arrays[name + ".b"] = b
    arrays["summary"] = np.array(json.dumps(summary or {}))
    with open(path, "wb") as f:
        np.savez(f, **arrays)


def load_weights(net, path):
    """Weights written by save_weights into net (loaded without unpickling); returns the training record."""
    with np.load(path, allow_pickle=False) as z:
        net.set_params({name: (z[name + ".w"], z[name + ".b"]) for name, _, _ in net.shapes})
        return json.loads(str(z["summary"]))


def evaluate_checkpoint(path, n_test=20, geometry_name="c5", log=None):
    """The learned path with stored weights on freshly generated held-out phantoms (the test seeds of the training
    run that wrote them): NRMSE of (11/3) x the 3-angle sum and of the network against the 11-angle compound, and
    the timing of both paths."""
    geo = geometry(geometry_name)
    p = geo["params"]
    dev = torch.device("cuda")
    elem = torch.as_tensor(np.ascontiguousarray(geo["elem"], dtype=np.float32), device=dev)
    vox = torch.as_tensor(np.ascontiguousarray(geo["vox"], dtype=np.float32), device=dev)
    tx = _das.tx_plane_wave(vox, geo["angles"], p["c"])
    T, E, V = geo["angles"].shape[0], elem.shape[0], vox.shape[0]
    params = _das.Params(T, E, p["n_samples"], 1, V, p["c"], p["fs"], p["fd"], p["t0"], p["f_number"],
                         p["tukey_alpha"])
    lc = LearnedCompounding(params, elem, vox, tx, geo["dims"], geo["input_idx"])
    try:
        rec = load_weights(lc.net, path)
        first = int(rec.get("n_train", 0)) + int(rec.get("n_val", 0))
        test = Dataset(lc, geo, n_test, first=first, log=log)
        base_db, net_db = evaluate(lc, test)
        times = time_paths(lc, geo)
    finally:
        lc.close()
    return {"geometry": geometry_name, "dims": list(geo["dims"]), "n_angles": T, "n_test": n_test,
            "test_phantom_seeds": [first, first + n_test - 1],
            "nrmse_db_vs_full_compound": {"scaled_input_sum": base_db, "network": net_db},
            "gain_db": base_db - net_db, "ms": times, "speedup": times["full_das"] / times["learned_total"],
            "trained": {k: rec.get(k) for k in ("n_train", "n_val", "steps", "checkpoint_step", "test_nrmse_db")}}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--geometry", default="c5", choices=("c5", "small"))
    ap.add_argument("--n-train", type=int, default=1800)
    ap.add_argument("--n-val", type=int, default=100)
    ap.add_argument("--n-test", type=int, default=100)
    ap.add_argument("--eval-every", type=int, default=2000, help="validation interval in steps")
    ap.add_argument("--steps", type=int, default=12000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--log-every", type=int, default=500)
    ap.add_argument("--out", default=None, help="write the JSON summary here")
    ap.add_argument("--save-weights", default=None, help="write the trained weights (NumPy archive) here")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)
    res = run(args, log)
    line = json.dumps(res)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
