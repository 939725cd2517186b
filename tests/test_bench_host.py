"""CPU-side checks of bench.py's bookkeeping (no GPU): the executed-MFMA
factor per precision mode and the one-GPU guard."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_exec_per_algo_single_precision_modes():
    st = {"matvecs_low": 1000, "fp64_tail": 0}
    assert bench.exec_per_algo("fp64", st, 20, 100) == 0.75
    assert bench.exec_per_algo("fp32", st, 20, 100) == 0.75
    assert bench.exec_per_algo("bf16x3", st, 20, 100) == 3.0


def test_exec_per_algo_two_term_mode_counts_three_term_start_pass():
    # start pass: (20 - 10) steps x 100 columns with three terms, then 500
    # defect-form products with two
    st = {"matvecs_low": 1500, "fp64_tail": 10}
    assert abs(bench.exec_per_algo("bf16x2", st, 20, 100) - (3.0 * 1000 + 2.0 * 500) / 1500) < 1e-15
    # only the start pass ran in low precision
    st = {"matvecs_low": 1000, "fp64_tail": 10}
    assert bench.exec_per_algo("bf16x2", st, 20, 100) == 3.0
    # odd degree: rounded up to even like the library
    st = {"matvecs_low": 2000, "fp64_tail": 0}
    assert bench.exec_per_algo("bf16x2", st, 19, 100) == 3.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "1 GPU" in r.stderr or "--gpus 1" in r.stderr


def test_mode_summary_fractions_and_speedup():
    m = {k: 0 for k in bench.MODE_KEYS}
    m.update(solve_s=2.0, filter_tflops=500.0, exec_per_algo=2.5, avg_launch_ms=20.0)
    out = bench.mode_summary(m, "bf16x2", 10.0)
    assert abs(out["filter_frac_peak"] - 0.2) < 1e-15
    assert abs(out["filter_executed_frac"] - 0.5) < 1e-15
    assert abs(out["speedup_vs_fp64"] - 5.0) < 1e-15
    assert "speedup_vs_fp64" not in bench.mode_summary(dict(m, exec_per_algo=0.75), "fp64", 10.0)


def test_cpu_baseline_pieces_on_a_small_matrix():
    # the CPU leg runs the oracle's pieces on the benchmark matrix; on a small
    # one it must finish and add them up as documented
    import numpy as np

    import gen
    p = gen.make_uniform(n=300, nev=20, nex=10)
    st = {"b_sup": 1.2, "mu_1": -1.0, "mu_ne": -0.5, "matvecs_fp64": 600, "matvecs_low": 0,
          "iterations": 2}
    cb = bench.cpu_baseline(p.H, p.V0, p.S, st, 300, 30, budget_s=0.05)
    pc = cb["pieces_s"]
    est = pc["lanczos"] + pc["filter"] + 2 * (pc["qr"] + pc["rr"] + pc["resid"])
    assert abs(cb["value"] - est) <= 1e-9 * est
    assert cb["kind"] == "oracle" and cb["cores"] >= 1
    assert cb["host"]["os_cpu_count"] == os.cpu_count()
    assert np.isfinite(cb["filter_gflops"])
