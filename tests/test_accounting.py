"""The throughput (Eq. 1) and memory (Eq. 2 / Table 4) arithmetic against the
numbers the paper prints (tests/golden/paper_numbers.json, each cited)."""

import json
import math
import os

import pytest

from oracle import accounting

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_benchmark_points_eq1():
    g = GOLD["benchmark_points"]
    i = g["inputs"]
    assert 251 * 251 == i["voxels"]
    assert accounting.points(i["voxels"], i["channels"], i["compounding"], i["frames"]) == g["value"]


def test_benchmark_rate():
    g = GOLD["benchmark_rate"]
    r = g["inputs"]["points"] / g["inputs"]["seconds"]
    assert r == pytest.approx(g["value"], rel=g["rel_tol"])


@pytest.mark.parametrize("row", GOLD["table1"], ids=lambda r: r["mode"])
def test_table1_required_throughput(row):
    v = math.prod(row["voxels"])
    got = accounting.required_throughput(v, row["channels"], row["frame_rate"]) / 1e9
    assert got == pytest.approx(row["value_gpts"], rel=row["rel_tol"])


def test_table4_memory():
    g = GOLD["table4"]
    m = accounting.memory_bytes(g["voxels"], g["out_frames"], g["channels"], g["samples"], g["in_frames"])
    assert m["channel_data"] / 1e9 == pytest.approx(g["channel_data_gb"], abs=0.05)
    assert m["output"] / 1e9 == pytest.approx(g["output_gb"], abs=0.05)
    assert m["grid_coords"] / 1e9 == pytest.approx(g["grid_coords_gb"], abs=0.005)
    assert sum(m.values()) / 1e9 == pytest.approx(g["total_gb"], abs=0.1)


def test_fusi_and_ulm_points():
    g = GOLD["fusi_ensemble_points"]["inputs"]
    assert accounting.points(g["voxels"], g["channels"], g["compounding"], g["frames"]) == pytest.approx(
        GOLD["fusi_ensemble_points"]["value"], rel=GOLD["fusi_ensemble_points"]["rel_tol"])
    u = GOLD["ulm_rate"]
    assert math.prod(u["inputs"]["voxels"]) == u["inputs"]["voxels_total"]
    r = accounting.points(u["inputs"]["voxels_total"], u["inputs"]["channels"], u["inputs"]["compounding"],
                          u["inputs"]["frame_rate"])
    assert r == pytest.approx(u["value"], rel=u["rel_tol"])


def test_round_trip():
    g = GOLD["round_trip_ms"]
    i = g["inputs"]
    t = 2 * i["depth_m"] / i["c"] * i["frames"] * 1e3
    assert t == pytest.approx(g["value"], rel=g["rel_tol"])
    assert t / 0.23 > 6.0
