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
