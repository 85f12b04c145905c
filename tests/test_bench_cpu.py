"""CPU checks of bench.py's host logic: the one-GPU contract, the rule that
counter-derived traffic is reported only while the counted sources are the
ones being run, and the per-unit counts behind every roofline, each against
its closed form."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_touching_a_device():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_committed_counters_are_reported_only_for_their_sources():
    with open(os.path.join(ROOT, "profiles", "traffic_counters.json")) as fh:
        kernels = json.load(fh)["kernels"]
    assert set(kernels) <= set(bench.KERNEL_SOURCES)
    for name, k in kernels.items():
        current = k["sources_sha256"] == bench.kernel_sources_sha256(name)
        assert bench.counter_traffic(name) == (float(k["bytes_per_launch"]) if current else None)
        assert os.path.exists(os.path.join(ROOT, k["summary"]))


def test_counter_traffic_is_dropped_when_a_counted_source_changes(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_1808_00128_amd").mkdir()
    os.symlink(os.path.join(ROOT, "paper_1808_00128_amd", "csrc"), tmp_path / "paper_1808_00128_amd" / "csrc")
    with open(os.path.join(ROOT, "profiles", "traffic_counters.json")) as fh:
        d = json.load(fh)
    name = next(iter(d["kernels"]))
    d["kernels"][name]["sources_sha256"] = "0" * 64
    (tmp_path / "profiles" / "traffic_counters.json").write_text(json.dumps(d))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic(name) is None
    assert bench.counter_traffic("no such kernel") is None


def test_evolution_counts():
    one = dict(H=0, CX=0, CZ=0, S=0, cond=0)
    for kind, own, table in (("H", 28 * 50 + 40, 35 * 50), ("CX", 12, 10), ("CZ", 4, 10), ("S", 3, 10),
                             ("cond", 12, 10)):
        st = dict(one, **{kind: 1})
        assert bench.algorithmic_ops_evolve(st, 50) == own
        assert bench.table_ops_evolve(st, 50) == table
    st = dict(H=3, CX=5, CZ=7, S=11, cond=13)
    assert bench.table_ops_evolve(st, 40) == 3 * 35 * 40 + (5 + 7 + 11 + 13) * 10


def test_amplitude_lds_bytes_per_pair():
    # n = 50: a term is packed when n - |v| <= 64 - n = 14; 13 chunks of x.
    packed = (1 << 49) - 1           # |v| = 49
    unpacked = (1 << 30) - 1         # |v| = 30
    assert bench.amp_lds_bytes_per_pair(50, [packed]) == (8.0 * 14, 1.0)
    assert bench.amp_lds_bytes_per_pair(50, [unpacked]) == (8.0 * 27, 0.0)
    b, f = bench.amp_lds_bytes_per_pair(50, [packed, unpacked])
    assert b == 8.0 * (14 + 27) / 2 and f == 0.5
    # the paper's per-pair count: 6 per set bit of x + 20
    assert bench.algorithmic_ops_amp([0b1011, 0]) == (6 * 3 + 20 + 20) / 2


def test_chain_step_bytes():
    chi, n, c = 1 << 20, 50, 64
    assert bench.table_chain_step_bytes(chi, c) == chi * (16 * c + 50)
    assert bench.chain_step_bytes(chi, n, c) == chi * (17 * n + 16 * c + 33)
    # window of 4: word read every step, written once per window, 2.5 pending rows
    assert bench.own_chain_step_bytes(chi, c, 4) == chi * (8 * c + 2 * c + 17 * 3.5 + 33)
    # a window of one step is the undeferred kernel: read and write every step
    assert bench.own_chain_step_bytes(chi, c, 1) == chi * (16 * c + 17 * 2 + 33)


def test_roofline_record():
    r = bench.roof("hbm", 4000.0, 8000.0, "GB/s", measured=5000.0, traffic=None)
    assert r["frac"] == 0.5 and r["frac_of_measured"] == 0.8 and r["traffic"] is None
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert bench.INT32_PEAK_OPS == pytest.approx(78.643e12, rel=1e-4)
    assert bench.LDS_PEAK_BPS == pytest.approx(78.643e12, rel=1e-4)
    assert bench.HBM_PEAK_BPS == 8.0e12
    assert np.isclose(bench.INT32_PEAK_OPS, 256 * 128 * 2.4e9)
