"""Host logic of bench.py (CPU only):

* a request for more than one GPU exits with status 2 and says why;
* an HBM-traffic record counts only while the kernel sources still hash to
  the version it was measured with: a record with the current hash is
  honoured, one with another hash or a missing file gives no figure, and the
  committed records' calibrated totals add up;
* every source a traffic record names exists, and the hash covers their
  bytes (a one-byte change of a copy changes it).
"""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("which", ["hh", "st57"])
def test_traffic_record_follows_the_source_hash(bench, tmp_path, which):
    path, sources = ((bench.TRAFFIC_FILE, bench.KERNEL_SOURCES) if which == "hh"
                     else (bench.SUR_TRAFFIC_FILE, bench.SUR_SOURCES))
    rec = json.load(open(path))
    # a record of the current sources counts (the committed one may lag a
    # kernel change until it is measured again: then bench.py reports none)
    cur = dict(rec, kernel_source_sha256=bench.kernel_source_hash(sources))
    q = tmp_path / "current.json"
    q.write_text(json.dumps(cur))
    assert bench.measured_traffic(str(q), sources) == rec["hbm_bytes_per_launch"]
    stale = dict(rec, kernel_source_sha256="0" * 64)
    p = tmp_path / "stale.json"
    p.write_text(json.dumps(stale))
    assert bench.measured_traffic(str(p), sources) is None
    assert bench.measured_traffic(str(tmp_path / "missing.json"), sources) is None
    # calibrated bytes: fetch scaled by the copy's ratio, writes as counted
    fetch = rec["fetch_kib_per_launch"] * rec["fetch_scale"] * 1024
    write = rec["write_kib_per_launch"] * rec["write_scale"] * 1024
    assert abs(rec["hbm_bytes_per_launch"] - (fetch + write)) <= 1e-6 * (fetch + write)


def test_source_hash_covers_the_bytes(bench, tmp_path, monkeypatch):
    for rel in bench.KERNEL_SOURCES + bench.SUR_SOURCES:
        assert os.path.isfile(os.path.join(ROOT, rel)), rel
    h0 = bench.kernel_source_hash(bench.KERNEL_SOURCES)
    assert h0 != bench.kernel_source_hash(bench.SUR_SOURCES)
    # the same hash from a copy of the sources, another after a one-byte change
    for rel in bench.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(ROOT, rel), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash(bench.KERNEL_SOURCES) == h0
    last = tmp_path / bench.KERNEL_SOURCES[-1]
    data = bytearray(last.read_bytes())
    data[-1] ^= 1
    last.write_bytes(bytes(data))
    assert bench.kernel_source_hash(bench.KERNEL_SOURCES) != h0


def test_trace_gap_analysis(bench, tmp_path):
    """Idle gaps between consecutive kernels of a kernel trace: gaps up to
    the threshold count as launch gaps, longer ones as host pauses."""
    rows = [("k_a(int)", 0, 1000), ("k_b(float)", 1200, 3200), ("k_a(int)", 3300, 4300),
            ("k_b(float)", 900000, 902000)]       # after a 895.7 us pause
    p = tmp_path / "kernel_trace.csv"
    with open(p, "w") as f:
        f.write("Kernel_Name,Start_Timestamp,End_Timestamp\n")
        for name, a, b in rows:
            f.write(f'"{name}",{a},{b}\n')
    r = bench.trace_gaps(str(p), max_gap_us=500.0)
    assert r["kernel_us"] == pytest.approx(1.0 + 2.0 + 1.0 + 2.0)
    assert r["idle_gap_us"] == pytest.approx(0.2 + 0.1)
    assert r["idle_share"] == pytest.approx(0.3 / 6.3)
    assert r["kernels"]["k_a"]["launches"] == 2
    assert r["kernels"]["k_b"]["mean_gap_before_us"] == pytest.approx(0.2)
    assert r["kernels"]["k_a"]["mean_gap_before_us"] == pytest.approx(0.1)
