"""Host logic of bench.py, without a GPU: a run over several GPUs is refused, the
algorithmic flop counts follow their closed forms, and a counter-measured traffic figure
is reported only for the kernel source it was taken on."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_flop_counts():
    b = _bench()
    m, n, s = 1 << 20, 128, 256
    f = b.flops(m, n, s, "rqr", True)
    assert f["sketch"] == 2 * s * m * n              # B = S A, s x m times m x n
    assert f["trsm"] == m * n * n                    # X = Y T^{-1}, T n x n triangular
    assert f["gram"] == m * n * (n + 1)              # upper triangle of X^T X
    # Householder QR of the s x n sketch (Golub and Van Loan): 2 n^2 (s - n/3)
    assert f["sketch_factor"] == pytest.approx(2 * n * n * (s - n / 3))
    # + 1 pass: three solves, two Gram matrices, two Cholesky factors, two R products
    assert f["total"] == pytest.approx(f["sketch"] + f["sketch_factor"] + 3 * f["trsm"]
                                       + 2 * f["gram"] + 2 * f["potrf"] + 2 * f["trmm"])
    # the benchmark step's count, as its JSON line reports it
    assert f["total"] == pytest.approx(154897044821.33337, rel=1e-12)
    g = b.flops(m, n, s, "rlu", False)
    assert g["sketch_factor"] == pytest.approx(n * n * (s - n / 3))  # LU: half of QR
    assert g["total"] == pytest.approx(g["sketch"] + g["sketch_factor"] + 2 * g["trsm"]
                                       + g["gram"] + g["potrf"] + g["trmm"])


def test_traffic_only_for_the_measured_source(tmp_path, monkeypatch):
    b = _bench()
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    monkeypatch.setitem(b.KERNEL_SOURCES, "sketch", ["k.hip"])
    (tmp_path / "k.hip").write_text("kernel, first version\n")
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_sketch_w.json").write_text(
        json.dumps({"source_sha": b.source_hash(["k.hip"]), "bytes_per_launch": 123.0}))
    assert b.load_traffic("sketch", "w") == 123.0
    assert b.load_traffic("sketch", "other_workload") is None
    (tmp_path / "k.hip").write_text("kernel, changed\n")
    assert b.load_traffic("sketch", "w") is None


def test_kernel_roofs_and_step_bound():
    b = _bench()
    m, n, s = 1 << 20, 128, 256
    t = b.kernel_table(m, n, s, "rqr")
    # the TRSM moves 16mn bytes for mn^2 flops: 8 flop/B < 78.6/8 = 9.8, so HBM-bound
    r = b.roof_of(t["trsm"], 0.5)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(16 * m * n / 0.5e-3 / 1e9, rel=1e-4)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)
    # the sketch (64 flop/B) and the Gram (16 flop/B) are FP64 matrix-core bound
    assert b.roof_of(t["sketch"], 1.0)["bound"] == "mfma"
    g = b.roof_of(t["gram"], 0.4)
    assert g["bound"] == "mfma"
    assert g["achieved"] == pytest.approx(m * n * (n + 1) / 0.4e-3 / 1e12, rel=1e-4)
    assert b.roof_of(t["sketch_factor"], 0.2)["bound"] == "latency"
    # phase-sum roofline of the tall step (2.02 ms) and of the wide plain one (24.5 ms)
    assert b.step_t_roof(m, n, s, True) * 1e3 == pytest.approx(2.016, abs=0.01)
    assert b.step_t_roof(1 << 18, 1024, 2048, False) * 1e3 == pytest.approx(24.5, abs=0.1)
