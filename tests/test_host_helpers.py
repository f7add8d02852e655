"""Host-side helpers of the benchmark and the Section V runner (CPU only)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import lqrgen
import oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_gemv_counts_follow_section_4b():
    import bench
    from paper_2503_15269_amd import fig2
    for m in range(1, 5):
        assert fig2.gemv_per_iteration(0.0, m) == 2 * m + 2
        assert fig2.gemv_per_iteration(1.0, m) == 3 * m + 3
        assert fig2.gemv_per_iteration(0.5, m) == 5 * m + 1
        assert bench.gemv_count(1.0, m, "poly") == 3 * m + 3
        assert orc.gemv_per_iteration(orc.PC_OPT, 1.0, m) == 3 * m + 3
    assert bench.gemv_count(1.0, 2, "none") == 3
    # applications of the scaled operator C per iteration: A p, G, then H
    assert bench.apps_per_iteration(1.0, 2) == 4
    assert bench.apps_per_iteration(0.0, 2) == 2
    assert bench.apps_per_iteration(0.5, 3) == 6


def test_flop_and_byte_accounting():
    import bench
    h = np.array([10, 20])
    f = bench.solve_flops(h, 12, np.array([5, 7]), np.array([2, 3]))
    per_it = 4 * 2 * 2 * 144
    per_outer = 3 * 2 * 144 + 2 * 12 * 13
    assert f == 10 * (5 * per_it + 2 * per_outer) + 20 * (7 * per_it + 3 * per_outer)
    assert bench.solve_bytes(h, 12, np.zeros(2), np.zeros(2)) == 0.0


def test_dense_assembly_matches_oracle_spmv():
    from paper_2503_15269_amd import fig2
    d = lqrgen.lqr_instance(7, 4, 2, seed=3)
    A = fig2.dense_A(d["D"], d["O"])
    x = np.random.default_rng(0).standard_normal((7, 4))
    assert np.allclose(A @ x.reshape(-1), orc.spmv(d["D"], d["O"], x).reshape(-1))
    assert np.allclose(A, A.T)


def test_distinct_count_clusters():
    from paper_2503_15269_amd import fig2
    assert fig2.distinct_count([]) == 0
    assert fig2.distinct_count([1.0, 1.0 + 1e-9, 2.0, 2.0]) == 2
    assert fig2.distinct_count([0.1, 0.2, 0.3]) == 3


def test_measured_traffic_parsing(tmp_path, monkeypatch):
    import bench
    f = tmp_path / "traffic.md"
    f.write_text("x\n- kernel_source_sha256: `abc`\n"
                 "- hbm_bytes_per_launch[inner_tol=3e-06,kernel_config=13]: `123`\n"
                 "- hbm_bytes_per_launch[inner_tol=0.0001,kernel_config=14]: `456`\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.measured_traffic(3e-6, 13) == 123.0
    assert bench.measured_traffic(1e-4, 14) == 456.0
    assert bench.measured_traffic(1e-4, 13) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "other")
    assert bench.measured_traffic(3e-6, 13) is None


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_complexity_slope_and_crossover():
    from paper_2503_15269_amd import complexity as cx
    k, c = cx.fit_slope([1, 2, 3, 4], [3.0, 5.0, 7.0, 9.0])
    assert k == pytest.approx(2.0) and c == pytest.approx(1.0)
    rows = [dict(N=8, d=1.0, p=2.0), dict(N=32, d=3.0, p=2.0),
            dict(N=128, d=9.0, p=2.5), dict(N=512, d=30.0, p=3.0)]
    assert cx.crossover(rows, "d", "p") == 32
    # faster at one size but slower again above it: no lasting crossover
    rows[-1]["p"] = 40.0
    assert cx.crossover(rows, "d", "p") is None
    assert cx.crossover(rows[:1], "d", "p") is None
