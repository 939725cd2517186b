"""CPU pins of the blocked Cholesky factorisation the QR passes use
(chase_cholesky): a plain numpy model of its step order, checked against
LAPACK's potrf.  It shares no code with the library.  It pins the
choices the library documents:
- panels of 32 rows;
- the unscaled right-looking elimination inside a panel, with rows scaled
  by the square roots of their pivots at the end;
- the row panel by forward substitution with R11^H;
- the trailing update on the upper triangle only;
- the 1-based index of the first pivot that is not positive, or not a
  number, with nothing written after it.
"""
import numpy as np
import pytest
import scipy.linalg.lapack as lapack

CB = 32


def blocked_cholesky(a):
    """Upper R with R^H R = A, in the library's step order.  Reads the upper
    triangle of A only; returns (R over A's upper triangle with A's strict
    lower triangle kept, info)."""
    a = np.array(a, copy=True)
    k = a.shape[0]
    for j0 in range(0, k, CB):
        nb = min(CB, k - j0)
        d = np.triu(a[j0:j0 + nb, j0:j0 + nb]).copy()
        piv = np.zeros(nb)
        for j in range(nb):
            p = np.real(d[j, j])
            if not p > 0:
                return a, j0 + j + 1
            piv[j] = p
            for i in range(j + 1, nb):
                f = d[j, i] / p
                for c in range(i, nb):
                    d[i, c] -= np.conj(f) * d[j, c]
        r11 = np.zeros_like(d)
        for i in range(nb):
            r = np.sqrt(piv[i])
            r11[i, i] = r
            r11[i, i + 1:] = d[i, i + 1:] / r
        a[j0:j0 + nb, j0:j0 + nb] = np.where(np.triu(np.ones((nb, nb), bool)), r11,
                                             a[j0:j0 + nb, j0:j0 + nb])
        if j0 + nb == k:
            break
        # row panel: column c becomes R11^{-H} a_c, column-oriented substitution
        x = a[j0:j0 + nb, j0 + nb:].copy()
        for l in range(nb):
            x[l] = x[l] / np.real(r11[l, l])
            for i in range(l + 1, nb):
                x[i] -= np.conj(r11[l, i]) * x[l]
        a[j0:j0 + nb, j0 + nb:] = x
        # trailing update on the upper triangle only
        upd = x.conj().T @ x
        b = j0 + nb
        up = np.triu(np.ones((k - b, k - b), bool))
        a[b:, b:] = np.where(up, a[b:, b:] - upd, a[b:, b:])
    return a, 0


def _hpd(k, cplx, seed):
    g = np.random.default_rng(seed)
    b = g.standard_normal((2 * k + 8, k))
    if cplx:
        b = b + 1j * g.standard_normal((2 * k + 8, k))
    a = b.conj().T @ b
    return (a + a.conj().T) / 2


def _potrf(a):
    f = lapack.zpotrf if np.iscomplexobj(a) else lapack.dpotrf
    r, info = f(a, lower=0, clean=1)
    return np.triu(r), int(info)


@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("k", [1, 2, 31, 32, 33, 64, 65, 97])
def test_model_matches_lapack(cplx, k):
    a = _hpd(k, cplx, k)
    r, info = blocked_cholesky(a)
    assert info == 0
    r_ref, _ = _potrf(a)
    up = np.triu(np.ones((k, k), bool))
    assert np.max(np.abs(r[up] - r_ref[up])) <= 80 * k * 2.0 ** -53 * np.max(np.abs(r_ref))
    assert np.all(np.imag(np.diag(r)) == 0) and np.all(np.real(np.diag(r)) > 0)
    # the strict lower triangle is A's
    assert np.array_equal(r[~up], a[~up])


@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("p", [0, 7, 31, 32, 33, 70])
def test_model_info_is_lapacks(cplx, p):
    """First leading minor that is not positive definite: the same index as
    LAPACK's; the panels before the failing one are complete."""
    k = 80
    a = _hpd(k, cplx, 100 + p)
    a[p, p] -= 1e3 * np.max(np.abs(np.diag(a)))
    _, info_ref = _potrf(a)
    r, info = blocked_cholesky(a)
    assert info == info_ref == p + 1
    done = (p // CB) * CB
    if done:
        r_ref, _ = _potrf(a[:done, :done])
        assert np.allclose(np.triu(r[:done, :done]), r_ref, rtol=0, atol=1e-11 * np.abs(r_ref).max())


@pytest.mark.parametrize("where", [(3, 3), (2, 7), (40, 45), (0, 70)])
def test_model_nan_stops_at_first_reached_pivot(where):
    """A NaN at (i, j), i <= j, enters no pivot before j; pivot j becomes NaN
    and the factorisation reports j + 1."""
    k = 80
    a = _hpd(k, True, 5)
    i, j = where
    a[i, j] = np.nan
    a[j, i] = np.nan
    _, info = blocked_cholesky(a)
    assert info == j + 1


def test_model_reads_only_the_upper_triangle():
    k = 70
    a = _hpd(k, True, 9)
    b = a.copy()
    low = np.tril(np.ones((k, k), bool), -1)
    b[low] = 1e300  # garbage below the diagonal
    ra, ia = blocked_cholesky(a)
    rb, ib = blocked_cholesky(b)
    up = ~low
    assert ia == ib == 0 and np.array_equal(ra[up], rb[up])
