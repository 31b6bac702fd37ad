"""The FP64 oracle on many voxels, run in a child process that never touches the GPU.

The GPU tests hold a HIP context, so they do not fork worker pools themselves.  A job
names seeded inputs (a workload from ``synth`` with its echo IQ, or circular Gaussian
IQ of a given shape and seed, optionally stored as FP16 / BF16) and a list of voxel
indices; the child process rebuilds exactly those inputs from the seeds, splits the
voxels over a fork pool of host processes and returns the oracle's complex128
``[len(index), F]`` values.  ``quantize_iq`` is the one 16-bit storage routine used
both here and by the tests that upload the quantised samples, so the oracle sees the
very samples the GPU reads.

    python tests/oracle_pool.py JOBDIR      (the child's entry point)
"""

import json
import os
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def quantize_iq(iq, kind):
    """Store complex64 IQ as 2 x FP16 / 2 x BF16 (round to nearest even, on the CPU).

    Returns (torch CPU tensor [..., 2] of the storage type, complex128 array of the
    stored values).  For kind == "c64" the tensor is the complex64 array itself.
    """
    import torch
    iq = np.ascontiguousarray(iq, dtype=np.complex64)
    if kind == "c64":
        return torch.from_numpy(iq), iq.astype(np.complex128)
    dt = {"f16": torch.float16, "bf16": torch.bfloat16}[kind]
    q = torch.view_as_real(torch.from_numpy(iq)).to(dt).contiguous()
    back = q.float().numpy()
    return q, (back[..., 0].astype(np.float64) + 1j * back[..., 1].astype(np.float64))


def build_inputs(spec):
    """Seeded inputs of a job: (iq complex64 [T,E,S,F], elem, vox, tx float32 [T,V], oracle params)."""
    sys.path.insert(0, ROOT)
    import oracle
    from synth import make_config
    from synth.configs import random_iq
    kw = {}
    if spec.get("n_frames") is not None:
        kw["n_frames"] = spec["n_frames"]
    rnd = spec.get("random_iq")
    cfg = make_config(spec["config"], with_iq=rnd is None, **kw)
    p = cfg["params"]
    iq = cfg["iq"] if rnd is None else random_iq(tuple(rnd["shape"]), seed=rnd["seed"])
    tx = oracle.tx_plane_wave(cfg["vox"], cfg["angles"], p["c"]).astype(np.float32)
    op = dict(c=p["c"], fs=p["fs"], fd=p["fd"], t0=p["t0"], f_number=p["f_number"], tukey_alpha=p["tukey_alpha"])
    return iq, cfg["elem"], cfg["vox"], tx, op


_JOB = {}


def _chunk(bounds):
    import oracle
    a, b = bounds
    j = _JOB
    idx = j["idx"][a:b]
    return a, oracle.das(j["iq"], j["elem"], j["vox"][idx], j["tx"][:, idx], **j["p"])


def _child(jobdir):
    import multiprocessing as mp
    with open(os.path.join(jobdir, "job.json")) as fh:
        spec = json.load(fh)
    idx = np.load(os.path.join(jobdir, "idx.npy"))
    iq, elem, vox, tx, p = build_inputs(spec)
    iq_q = quantize_iq(iq, spec.get("quant", "c64"))[1]
    del iq
    _JOB.update(iq=iq_q, elem=elem, vox=vox, tx=tx, p=p, idx=idx)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(16, cores))
    n = idx.shape[0]
    chunk = max(1, -(-n // (4 * cores)))
    bounds = [(a, min(n, a + chunk)) for a in range(0, n, chunk)]
    with mp.get_context("fork").Pool(cores) as pool:
        parts = pool.map(_chunk, bounds)
    out = np.zeros((n, iq_q.shape[3]), np.complex128)
    for a, y in parts:
        out[a:a + y.shape[0]] = y
    np.save(os.path.join(jobdir, "ref.npy"), out)


def oracle_job(spec, idx, timeout=600):
    """Run the oracle for job ``spec`` on voxels ``idx`` in a child process; returns complex128 [len(idx), F]."""
    with tempfile.TemporaryDirectory(prefix="das_oracle_") as d:
        with open(os.path.join(d, "job.json"), "w") as fh:
            json.dump(spec, fh)
        np.save(os.path.join(d, "idx.npy"), np.asarray(idx, dtype=np.int64))
        proc = subprocess.run([sys.executable, os.path.abspath(__file__), d], timeout=timeout,
                              stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if proc.returncode != 0:
            raise RuntimeError("oracle child failed:\n" + proc.stdout[-4000:])
        return np.load(os.path.join(d, "ref.npy"))


if __name__ == "__main__":
    _child(sys.argv[1])
