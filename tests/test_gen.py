"""CPU checks of the input generators used by the benchmark's Table 2 suite:
the closed-form and tridiagonal-solver spectra agree with a dense
eigendecomposition of the matrices they stand for."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import gen  # noqa: E402


@pytest.mark.parametrize("kind,builder", [("121", gen.tridiag_121),
                                          ("wilkinson", gen.tridiag_wilkinson)])
def test_tridiagonal_spectra_match_dense_eigensolver(kind, builder):
    n = 301
    lam = gen.spectrum_table1(kind, n)
    ref = np.linalg.eigvalsh(gen.dense_from_tridiag(*builder(n)))
    assert np.all(np.diff(lam) >= 0)
    assert np.max(np.abs(lam - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_table1_spectra_ranges():
    for kind in ("uniform", "geometric"):
        lam = gen.spectrum_table1(kind, 1000)
        assert lam[0] == pytest.approx(1e-4) and lam[-1] == pytest.approx(1.0)
        assert np.all(np.diff(lam) > 0)
    with pytest.raises(ValueError):
        gen.spectrum_table1("other", 10)
