"""Host logic of bench.py (no GPU): the algorithmic byte model of the stages and of Phi, the
lookup of a committed counter record (valid only while the kernel source and template
instance are unchanged), and the refusal of more than one GPU."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_byte_model_of_the_headline_workload(bench):
    n, M = 1024, 1 << 22
    N = n * n
    sb = bench.stage_bytes(n, M)
    # degridding: coordinates, y, v in and r out (32 B per visibility), the grid read once
    assert sb["degrid"] == 32 * M + 32 * N == 167772160
    # gridding of step 9: r and coordinates in, v out (24 B per visibility), the grid written once
    assert sb["grid"] == 24 * M + 32 * N == 134217728
    # the pruned forward FFT: x~ in, n x 2n complex rows out; the rows in, the 2n x 2n grid out
    assert sb["fft_rows"] == 20 * N and sb["fft_cols"] == 48 * N
    # Phi alone: x, the two FFT passes and the degridding with coordinates and y
    assert bench.phi_bytes(n, M) == 100 * N + 16 * M == 171966464
    # every stage scales with the active visibilities only through the gather / scatter terms
    sb4 = bench.stage_bytes(n, M // 4)
    for k in sb:
        assert (sb[k] - sb4[k]) == {"degrid": 24 * M, "grid": 18 * M}.get(k, 0)


def test_counter_record_follows_its_source(bench, tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("// a kernel\n")
    (tmp_path / "profiles").mkdir()
    rec = {"kernel": "k_x<32, 2>", "source": "kernel.hip",
           "source_sha256": hashlib.sha256(src.read_bytes()).hexdigest(), "bytes_per_launch": 123}
    (tmp_path / "profiles" / "grid_w_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    got = bench.profile_record("grid", "w", "k_x<32, 2>")
    assert got is not None and got["bytes_per_launch"] == 123
    assert bench.profile_record("grid", "w", "k_x<32, 0>") is None  # another template instance
    assert bench.profile_record("grid", "other", "k_x<32, 2>") is None  # no record
    src.write_text("// a kernel, edited\n")
    assert bench.profile_record("grid", "w", "k_x<32, 2>") is None  # the source changed


def test_committed_counter_record_is_consistent():
    rec = json.load(open(os.path.join(ROOT, "profiles", "grid_n1024_m4m_d64_traffic.json")))
    scaled = (rec["fetch_kib"] * rec["fetch_factor"] + rec["write_kib"] * rec["write_factor"]) * 1024
    assert abs(scaled - rec["bytes_per_launch"]) <= 1
    assert os.path.exists(os.path.join(ROOT, rec["source"]))
    for c in rec["commands"]:
        assert "rocprofv3 --pmc" in c and "bench.py" in c


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
