"""Host-side checks of bench.py: argument contract, the traffic record's source-hash guard, workload table and
the 16-bit range report (no GPU needed)."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from synth.configs import CONFIGS  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus 2" in r.stderr and r.stdout == ""


def test_traffic_record_is_tied_to_the_kernel_sources(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) == 64
    rec = tmp_path / "traffic.txt"
    rec.write_text("# comment\nsource_sha256 %s\nc2 fetch_kib 1.0 write_kib 2.0 read_bytes 100 write_bytes 20\n" % h)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    assert bench.measured_traffic("c2") == 120
    assert bench.measured_traffic("c1") is None  # no record for this workload
    rec.write_text("source_sha256 %s\nc2 fetch_kib 1.0 write_kib 2.0 read_bytes 100 write_bytes 20\n" % ("0" * 64))
    assert bench.measured_traffic("c2") is None  # the kernel sources changed since the counters were taken
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("c2") is None


def test_workload_table():
    for name, (base, overrides, xcols) in bench.WORKLOAD_CONFIG.items():
        assert name in bench.WORKLOADS and base in CONFIGS
        assert set(overrides) <= {"n_frames"}
        assert xcols is None or 0 <= xcols[0] < xcols[1] <= 96
    for name in bench.WORKLOADS:
        assert name in CONFIGS or name in bench.WORKLOAD_CONFIG


def test_iq16_range_report():
    iq = np.array([1.0 + 2.0j, 70000.0 - 1e-6j, 0.0, 1e-40 + 0j], dtype=np.complex64)
    r = bench.iq16_range(iq)
    assert r["max_abs_component"] == 70000.0 and not r["fits_fp16"]
    assert 0.0 < r["fp16_flushed_to_zero_fraction"] < 1.0
    assert r["bf16_subnormal_fraction"] > 0.0  # 1e-40 is below float32's normal range


def test_hbm_report_compulsory_bytes():
    """c2's compulsory traffic: IQ once (1 x 128 x 2048 x 32 complex64), output once (65536 x 32 complex64), the
    transmit table (float32) and the voxel and element coordinates (3 float32 each)."""
    info = {"processed_triples": 1000}
    r = bench.hbm_report(1, 128, 2048, 32, 65536, info, 0.1, None)
    assert r["compulsory_bytes"] == 67108864 + 16777216 + 262144 + 786432 + 1536
    assert abs(r["compulsory_GBps"] - r["compulsory_bytes"] / 1e-4 / 1e9) < 1e-6
    assert abs(r["frac"] - r["compulsory_GBps"] / 8000.0) < 1e-12
    assert r["measured_GBps"] is None and r["gather_GBps"] == 1000 * 32 * 16 / 1e-4 / 1e9
    assert bench.hbm_report(1, 128, 2048, 32, 65536, info, 0.1, 2e8)["measured_GBps"] == 2e8 / 1e-4 / 1e9


def test_host_cpu_report():
    """cpu_baseline states the host's CPU count and the affinity mask the oracle pool runs on (as ranges)."""
    import bench
    n, aff, txt = bench._host_cpus()
    assert n >= 1 and len(aff) >= 1 and set(aff) <= set(range(max(n, max(aff) + 1)))
    expanded = []
    for part in txt.split(","):
        a, _, b = part.partition("-")
        expanded += list(range(int(a), int(b or a) + 1))
    assert expanded == aff
    assert 1 <= bench._cores() <= min(16, len(aff))
