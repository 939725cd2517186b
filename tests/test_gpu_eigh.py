"""The dense Hermitian eigensolver of the Rayleigh-Ritz step (chase_heev,
chase_opts.eig_solver): the library's block-cyclic Jacobi against the plain
definition (numpy's eigh), closed forms and invariants, and the solve with
the Jacobi eigensolver against the CPU oracle."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2205_02491_amd as pk
    pk.lib()
    return pk


def _random_herm(k, cplx, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    a = gen.gaussian(g, (k, k), cplx)
    return (a + a.conj().T) / 2


def _check_decomposition(G, ev, W, tol=1e-12):
    """Residual, orthonormality and eigenvalues against numpy's eigh."""
    k = G.shape[0]
    scale = max(np.max(np.abs(np.linalg.eigvalsh(G))), 1e-300)
    ref = np.linalg.eigvalsh(G)
    assert np.all(np.diff(ev) >= 0)
    assert np.max(np.abs(ev - ref)) <= tol * scale, np.max(np.abs(ev - ref)) / scale
    res = np.max(np.abs(G @ W - W * ev[None, :]))
    assert res <= tol * scale, res / scale
    orth = np.max(np.abs(W.conj().T @ W - np.eye(k)))
    assert orth <= tol, orth


@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("k", [1, 2, 3, 17, 31, 32, 33, 100, 257])
def test_jacobi_matches_dense_definition(pk, cplx, k):
    announce(f"heev Jacobi random Hermitian k={k} cplx={cplx}")
    G = _random_herm(k, cplx, 7000 + k)
    ev, W, sweeps = pk.chase_heev(to_gpu(G), method=pk.EIG_JACOBI)
    _check_decomposition(G, ev, to_np(W))
    if k > 1:
        assert 1 <= sweeps <= 20
    # the eigenvectors of simple eigenvalues agree with numpy's up to phase
    ref_ev, ref_w = np.linalg.eigh(G)
    gaps = np.diff(ref_ev)
    if k > 2 and np.min(gaps) > 1e-6 * np.max(np.abs(ref_ev)):
        ov = np.abs(np.sum(ref_w.conj() * to_np(W), axis=0))
        assert np.min(ov) > 1 - 1e-8


@pytest.mark.parametrize("cplx", [True, False])
def test_jacobi_and_library_agree(pk, cplx):
    k = 300
    announce(f"heev Jacobi vs library k={k} cplx={cplx}")
    G = _random_herm(k, cplx, 71)
    ev_j, W_j, sw = pk.chase_heev(to_gpu(G), method=pk.EIG_JACOBI)
    ev_l, W_l, sw_l = pk.chase_heev(to_gpu(G), method=pk.EIG_LIBRARY)
    assert sw >= 1 and sw_l == 0
    scale = np.max(np.abs(ev_l))
    assert np.max(np.abs(ev_j - ev_l)) <= 20 * k * 2.0 ** -53 * scale
    _check_decomposition(G, ev_l, to_np(W_l))


def test_jacobi_closed_form_121(pk):
    """The (1-2-1) tridiagonal matrix of order k: eigenvalues
    2 - 2 cos(j pi / (k + 1)), eigenvectors sin(i j pi / (k + 1))."""
    k = 75
    announce(f"heev Jacobi (1-2-1) closed form k={k}")
    G = 2.0 * np.eye(k) - np.eye(k, k=1) - np.eye(k, k=-1)
    ev, W, _ = pk.chase_heev(to_gpu(G), method=pk.EIG_JACOBI)
    j = np.arange(1, k + 1)
    lam = 2.0 - 2.0 * np.cos(j * np.pi / (k + 1))
    assert np.max(np.abs(ev - lam)) < 1e-13 * 4
    vec = np.sin(np.outer(j, j) * np.pi / (k + 1)) * np.sqrt(2.0 / (k + 1))
    ov = np.abs(np.sum(vec * to_np(W), axis=0))
    assert np.min(ov) > 1 - 1e-10


@pytest.mark.parametrize("cplx", [True, False])
def test_jacobi_diagonal_identity_and_multiple_eigenvalues(pk, cplx):
    announce(f"heev Jacobi degenerate cases cplx={cplx}")
    k = 40
    g = np.random.Generator(np.random.PCG64(9))
    # already diagonal (unsorted): no sweep, exact values, permuted unit vectors
    d = g.standard_normal(k)
    D = np.diag(d).astype(complex if cplx else float)
    ev, W, sweeps = pk.chase_heev(to_gpu(D), method=pk.EIG_JACOBI)
    assert sweeps == 0
    assert np.array_equal(ev, np.sort(d))
    assert np.array_equal(np.abs(to_np(W)), np.eye(k)[:, np.argsort(d, kind="stable")])
    # a multiple of the identity
    ev, W, sweeps = pk.chase_heev(to_gpu(3.0 * np.eye(k, dtype=D.dtype)), method=pk.EIG_JACOBI)
    assert sweeps == 0 and np.all(ev == 3.0)
    # eigenvalues of multiplicity 5 (planted): values exact to rounding, each
    # cluster's invariant subspace matches
    lam = np.repeat(np.arange(8, dtype=float), 5)
    q = gen.haar(k, g, cplx)
    G = gen.planted(lam, q)
    ev, W, _ = pk.chase_heev(to_gpu(G), method=pk.EIG_JACOBI)
    _check_decomposition(G, ev, to_np(W))
    W = to_np(W)
    for c in range(8):
        sl = slice(5 * c, 5 * c + 5)
        P = q[:, sl] @ q[:, sl].conj().T
        assert np.max(np.abs(P @ W[:, sl] - W[:, sl])) < 1e-12


@pytest.mark.parametrize("cplx", [True, False])
def test_auto_choice_follows_the_off_diagonal_norm(pk, cplx):
    announce(f"heev automatic choice cplx={cplx}")
    k = 200
    g = np.random.Generator(np.random.PCG64(11))
    near = np.diag(np.sort(g.uniform(-1, 1, k))) + 1e-4 * _random_herm(k, cplx, 12) / np.sqrt(k)
    ev, W, sweeps = pk.chase_heev(to_gpu(near), method=pk.EIG_AUTO)
    assert sweeps >= 1
    _check_decomposition(near, ev, to_np(W))
    dense = _random_herm(k, cplx, 13)
    ev, W, sweeps = pk.chase_heev(to_gpu(dense), method=pk.EIG_AUTO)
    assert sweeps == 0
    _check_decomposition(dense, ev, to_np(W))


def test_jacobi_rejects_nonfinite_input(pk):
    announce("heev Jacobi non-finite input")
    G = _random_herm(20, True, 3)
    G[4, 7] = np.nan
    G[7, 4] = np.nan
    with pytest.raises(pk.ChaseError, match="NUMERIC"):
        pk.chase_heev(to_gpu(G), method=pk.EIG_JACOBI)


@pytest.mark.parametrize("k", [1300, 2600])
def test_jacobi_at_full_block_size(pk, k):
    """Orders of the projected matrix at the n=20000 and n=100000 workloads
    (nev+nex = 1300 and 2600), complex: eigenvalues against the library's
    divide and conquer; residual and orthonormality on the GPU."""
    import torch
    announce(f"heev Jacobi full block size k={k}")
    g = np.random.Generator(np.random.PCG64(100 + k))
    # a Rayleigh quotient close to diagonal, as in the later iterations
    lam = np.sort(g.uniform(-1, 1, k))
    G = np.diag(lam) + 1e-3 * _random_herm(k, True, 101 + k) / np.sqrt(k)
    h = pk.Handle(k, k - 1, 1, torch.complex128)
    Gd = to_gpu(G)
    ev, W, sweeps = pk.chase_heev(Gd, method=pk.EIG_JACOBI, handle=h)
    ev_l, _, _ = pk.chase_heev(Gd, method=pk.EIG_LIBRARY, handle=h)
    assert 1 <= sweeps <= 8
    # both solvers are backward stable: each eigenvalue within a small
    # multiple of k u ||G||_2 of the host LAPACK's (a Jacobi whose rotation
    # products drift from unitary shifts the eigenvalues by ~1e-12 here)
    ref = np.linalg.eigvalsh(G)
    scale = np.max(np.abs(ref))
    bound = 2 * k * 2.0 ** -53 * scale
    err_j, err_l = np.max(np.abs(ev - ref)), np.max(np.abs(ev_l - ref))
    print(f"k={k}: Jacobi {err_j / scale:.2e}, library {err_l / scale:.2e} (relative)")
    assert err_j <= bound and err_l <= bound, (err_j / scale, err_l / scale)
    evd = torch.from_numpy(ev).to(W.device).to(W.dtype)
    res = torch.max(torch.abs(Gd @ W - W * evd[None, :])).item()
    orth = torch.max(torch.abs(W.mH @ W - torch.eye(k, dtype=W.dtype, device=W.device))).item()
    assert res <= 1e-12 * scale and orth <= 1e-12, (res, orth)


@pytest.mark.parametrize("cplx", [True, False])
def test_solve_with_jacobi_eigensolver_matches_oracle(pk, cplx):
    """The whole solve with every Rayleigh-Ritz eigensolve done by Jacobi:
    the same iterations and eigenvalues as the CPU oracle."""
    announce(f"solve with the Jacobi eigensolver cplx={cplx}")
    p = gen.make_uniform(n=1000, nev=100, nex=40, cplx=cplx)
    ev_o, _, _, st_o = oracle.solve(p.H, p.nev, p.nex, p.tol, p.deg, p.V0, p.S)
    ev, V, res, st = pk.chase_solve(to_gpu(p.H), p.nev, p.nex, tol=p.tol, degree=p.deg,
                                    V0=to_gpu(p.V0), S=to_gpu(p.S),
                                    opts=pk.default_opts(eig_solver=pk.EIG_JACOBI))
    assert st["converged"]
    assert st["eig_jacobi_calls"] == st["iterations"]
    assert st["eig_jacobi_sweeps"] >= st["iterations"]
    assert abs(st["iterations"] - st_o.iterations) <= 1
    scale = np.max(np.abs(p.lam))
    assert np.max(np.abs(ev - ev_o)) <= 1e-10 * scale
    assert np.max(res) <= p.tol
