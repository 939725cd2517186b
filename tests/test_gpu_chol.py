"""The Cholesky factorisation of the QR step's Cholesky passes
(chase_cholesky) against LAPACK's potrf: the factor, the index of the first
leading minor that is not positive definite, non-finite pivots, and what the
call leaves untouched (the strict lower triangle, rows beyond k)."""
import ctypes

import numpy as np
import pytest
import scipy.linalg.lapack as lapack

from gpu_util import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2205_02491_amd as pk
    pk.lib()
    return pk


def _hpd(k, cplx, seed, cond_cols=1.0):
    """B^H B for a (2k + 8) x k Gaussian block B (condition of B about 6),
    its columns scaled from 1 down to 1 / cond_cols: Hermitian positive
    definite with condition about (6 cond_cols)^2."""
    g = np.random.Generator(np.random.PCG64(seed))
    b = g.standard_normal((2 * k + 8, k))
    if cplx:
        b = b + 1j * g.standard_normal((2 * k + 8, k))
    b = b * np.logspace(0, -np.log10(cond_cols), k)[None, :] if cond_cols > 1 else b
    a = b.conj().T @ b
    return (a + a.conj().T) / 2


def _potrf(a):
    """LAPACK's upper Cholesky factor and info (1-based, 0 on success)."""
    f = lapack.zpotrf if np.iscomplexobj(a) else lapack.dpotrf
    r, info = f(a, lower=0, clean=1)
    return np.triu(r), int(info)


@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("k", [1, 2, 31, 32, 33, 64, 65, 100, 257, 700])
def test_cholesky_matches_lapack(pk, cplx, k):
    announce(f"Cholesky k={k} cplx={cplx}")
    a = _hpd(k, cplx, 100 + k)
    r, info = pk.chase_cholesky(to_gpu(a))
    assert info == 0
    r = to_np(r)
    r_ref, info_ref = _potrf(a)
    assert info_ref == 0
    # well conditioned (condition of A about 40): forward error within a
    # small multiple of k u of the largest entry
    assert np.max(np.abs(r - r_ref)) <= 80 * k * U * np.max(np.abs(r_ref))
    assert np.all(np.real(np.diag(r)) > 0) and np.all(np.imag(np.diag(r)) == 0)
    # backward error of the factorisation
    assert np.max(np.abs(r.conj().T @ r - a)) <= 4 * k * U * np.max(np.abs(a))


@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("k", [1300, 2600])
def test_cholesky_at_subspace_sizes(pk, cplx, k):
    """The orders of the n = 20000 and n = 30000 solves' subspaces."""
    announce(f"Cholesky at subspace size k={k} cplx={cplx}")
    a = _hpd(k, cplx, 7 + k)
    r, info = pk.chase_cholesky(to_gpu(a))
    assert info == 0
    r = to_np(r)
    r_ref, _ = _potrf(a)
    assert np.max(np.abs(r - r_ref)) <= 80 * k * U * np.max(np.abs(r_ref))
    assert np.max(np.abs(r.conj().T @ r - a)) <= 4 * k * U * np.max(np.abs(a))


@pytest.mark.parametrize("cplx", [True, False])
def test_cholesky_ill_conditioned_gram(pk, cplx):
    """Gram matrix of a block whose columns span six decades (condition
    ~1e12, as in the first Cholesky QR pass on a filtered block): the
    backward error stays at rounding level."""
    k = 300
    announce(f"Cholesky ill conditioned k={k} cplx={cplx}")
    a = _hpd(k, cplx, 31, cond_cols=1e6)
    r, info = pk.chase_cholesky(to_gpu(a))
    assert info == 0
    r = to_np(r)
    assert np.max(np.abs(r.conj().T @ r - a)) <= 4 * k * U * np.max(np.abs(a))
    r_ref, _ = _potrf(a)
    # each row of R scaled by its diagonal: agrees with LAPACK to the
    # conditioning of the leading blocks
    d = np.abs(np.diag(r_ref))[:, None]
    assert np.max(np.abs(r - r_ref) / d) <= 1e-10


@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("p", [0, 5, 31, 32, 33, 63, 64, 150, 199])
def test_cholesky_info_matches_lapack(pk, cplx, p):
    """A matrix whose leading p x p block is positive definite and whose
    (p + 1) x (p + 1) block is not: info = p + 1, as LAPACK's."""
    k = 200
    announce(f"Cholesky info p={p} cplx={cplx}")
    a = _hpd(k, cplx, 55 + p)
    a[p, p] -= 1e3 * np.max(np.abs(np.diag(a)))
    _, info_ref = _potrf(a)
    assert info_ref == p + 1
    r, info = pk.chase_cholesky(to_gpu(a))
    assert info == p + 1
    # the columns before the failing panel are complete
    done = (p // 32) * 32
    if done:
        r_ref, _ = _potrf(a[:done, :done])
        assert np.max(np.abs(to_np(r)[:done, :done] - r_ref)) <= 1e-11 * np.max(np.abs(r_ref))


@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("where", [(3, 3), (2, 7), (40, 90), (0, 150)])
def test_cholesky_nonfinite_input(pk, cplx, where):
    """A NaN at (i, j), i <= j, first enters pivot j (through r_ij, or as
    a_jj itself): the factorisation stops there, info = j + 1, as LAPACK's
    reference potrf (which also treats a NaN pivot as not positive)."""
    k = 160
    announce(f"Cholesky NaN at {where} cplx={cplx}")
    a = _hpd(k, cplx, 9)
    i, j = where
    a[i, j] = np.nan
    a[j, i] = np.nan
    _, info = pk.chase_cholesky(to_gpu(a))
    assert info == j + 1


def test_cholesky_empty(pk):
    import torch
    r, info = pk.chase_cholesky(torch.zeros((0, 0), dtype=torch.complex128, device="cuda"))
    assert info == 0 and r.shape == (0, 0)


@pytest.mark.parametrize("cplx", [True, False])
def test_cholesky_leaves_lower_triangle_and_padding(pk, cplx):
    """Through the C-ABI on a column-major buffer with lda > k: the upper
    triangle becomes R, the strict lower triangle and the rows beyond k keep
    their bytes."""
    import torch
    k, lda = 77, 85
    announce(f"Cholesky lda={lda} k={k} cplx={cplx}")
    a = _hpd(k, cplx, 3)
    dt = np.complex128 if cplx else np.float64
    full = np.full((lda, k), 777.0 + (5.0j if cplx else 0.0), dtype=dt)  # column-major lda x k
    full[:k, :] = np.where(np.triu(np.ones((k, k), dtype=bool)), a, full[:k, :])
    buf = to_gpu(np.ascontiguousarray(full.T))  # row-major (k, lda) = column-major (lda, k)
    handle = pk.Handle(2, 1, 1, torch.complex128 if cplx else torch.float64)
    info = ctypes.c_int(-1)
    st = pk._stream()
    rc = pk.lib().chase_cholesky(handle.ptr, ctypes.c_void_p(buf.data_ptr()), lda, k,
                                 ctypes.byref(info), st)
    assert rc == 0 and info.value == 0
    out = to_np(buf).T  # column-major (lda, k)
    r_ref, _ = _potrf(a)
    upper = np.triu(np.ones((k, k), dtype=bool))
    assert np.max(np.abs(out[:k][upper] - r_ref[upper])) <= 1e-12 * np.max(np.abs(r_ref))
    assert np.all(out[:k][~upper] == full[:k][~upper])
    assert np.all(out[k:] == full[k:])


def test_cholesky_rejects_bad_arguments(pk):
    import torch
    handle = pk.Handle(2, 1, 1, torch.float64)
    buf = torch.eye(4, dtype=torch.float64, device="cuda")
    info = ctypes.c_int()
    st = pk._stream()
    L = pk.lib()
    assert L.chase_cholesky(handle.ptr, ctypes.c_void_p(buf.data_ptr()), 3, 4,
                            ctypes.byref(info), st) != 0
    assert L.chase_cholesky(handle.ptr, ctypes.c_void_p(buf.data_ptr()), 4, -1,
                            ctypes.byref(info), st) != 0
    assert L.chase_cholesky(handle.ptr, None, 4, 4, ctypes.byref(info), st) != 0
