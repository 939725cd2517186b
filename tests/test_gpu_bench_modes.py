"""The benchmark's single-step modes (`bench.py --eigensolver K` and
`--cholesky K`) at small sizes: they run through the library and report
consistent numbers (the same code paths the committed profiles come from)."""
import pytest

import bench
from gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2205_02491_amd as pk
    pk.lib()
    return pk


def test_eigensolver_mode(pk):
    announce("bench eigensolver mode k=96")
    out = bench.eigensolver_block(pk, 96, reps=1)
    assert out["k"] == 96 and set(out["cases"]) == {"dense", "near_diagonal_0.1",
                                                     "near_diagonal_0.01",
                                                     "near_diagonal_0.0001"}
    for name, row in out["cases"].items():
        assert row["jacobi_ms"] > 0 and row["library_ms"] > 0
        # Jacobi and the library agree on the eigenvalues to rounding
        assert row["eig_diff_rel"] < 1e-12, (name, row)
        assert row["jacobi_sweeps"] >= 1


def test_cholesky_mode(pk):
    announce("bench cholesky mode k=100")
    out = bench.cholesky_block(pk, 100, reps=2)
    assert out["k"] == 100 and set(out["cases"]) == {"c128", "f64"}
    for name, row in out["cases"].items():
        assert row["library_ms"] > 0 and row["torch_linalg_cholesky_ms"] > 0
        assert row["backward_err"] < 1e-13, (name, row)
