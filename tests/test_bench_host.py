"""Host logic of the benchmark: the counter-traffic records and the one-GPU guard.

CPU only: nothing here launches a kernel.
"""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _record(path):
    rec = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    return rec


def test_traffic_records_parse_and_are_keyed_by_their_own_sources():
    for precision, (path, sources) in bench.TRAFFIC.items():
        assert os.path.exists(path), path
        rec = _record(path)
        for key in ("workload", "source_hash", "fetch_factor", "write_factor",
                    "gemm1_bytes_per_launch", "gemm2_bytes_per_launch"):
            assert key in rec, (path, key)
        for f in sources:
            assert os.path.exists(os.path.join(ROOT, "paper_2509_08602_amd", "csrc", f)), f
        # a plain copy reads and writes close to its size once the factors are applied
        assert 0.5 <= float(rec["fetch_factor"]) <= 4.0
        assert 0.5 <= float(rec["write_factor"]) <= 4.0


def test_traffic_is_reported_only_for_the_measured_workload_and_sources(tmp_path, monkeypatch):
    path, sources = bench.TRAFFIC["f32"]
    rec = _record(path)
    wl = rec["workload"]
    # another workload or another precision never borrows this record
    assert bench.measured_traffic("gemm2", wl + "-other", "f32") is None
    assert bench.measured_traffic("gemm2", wl, "f64") is None
    # a record whose hash does not match the sources is ignored
    fake = tmp_path / "traffic.txt"
    fake.write_text(f"workload = {wl}\nsource_hash = 0000000000000000\ngemm2_bytes_per_launch = 123\n")
    monkeypatch.setitem(bench.TRAFFIC, "f32", (str(fake), sources))
    assert bench.measured_traffic("gemm2", wl, "f32") is None
    # and one whose hash matches is read
    fake.write_text(f"workload = {wl}\nsource_hash = {bench.kernel_source_hash('f32')}\n"
                    "gemm2_bytes_per_launch = 123\n")
    assert bench.measured_traffic("gemm2", wl, "f32") == 123.0
    assert bench.measured_traffic("gemm1", wl, "f32") is None


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 2
    assert "one GPU" in json.loads(out.stdout.strip().splitlines()[-1])["error"]


def test_algorithmic_bytes_of_the_hot_products():
    """The byte model of the roofline: the dose block once at its storage
    width, the plan-side operand and the result traffic."""
    N, n_t, k, kp = 1000, 192, 9, 32
    # BF16 refinement: 2-byte dose block; GEMM2 reads q, X_ref, W_ref and writes q and dW
    assert bench.product_bytes("gemm2", "bf16", N, n_t, k, kp) == 2 * N * n_t + 2 * n_t * kp + 18 * N * kp
    assert bench.product_bytes("gemm1", "bf16", N, n_t, k, kp) == 2 * N * n_t + 2 * N * kp + 4 * n_t * kp
    # FP32: 4-byte block, q read and written and W written
    assert bench.product_bytes("gemm2", "f32", N, n_t, k, kp) == 4 * N * n_t + 4 * n_t * kp + 12 * N * kp
    info = bench.host_cpu()
    assert info["nproc"] >= 1
