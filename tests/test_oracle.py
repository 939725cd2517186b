"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these tests retypes an oracle formula: each compares the oracle with a
closed form, an invariant, a brute-force computation or a value printed in
the paper (tests/golden)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sl

import gen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_unitary(n, seed, cplx=True):
    g = np.random.Generator(np.random.PCG64(seed))
    return gen.haar(n, g, cplx)


# ------------------------------------------------------------ brute force
def test_jacobi_matches_121_closed_form():
    n = 9
    h = gen.dense_from_tridiag(*gen.tridiag_121(n))
    w, v = oracle.jacobi_eigh(h)
    k = np.arange(1, n + 1)
    lam = 2 - 2 * np.cos(np.pi * k / (n + 1))
    np.testing.assert_allclose(w, lam, atol=1e-14)
    vk = np.sin(np.outer(np.arange(1, n + 1), n + 1 - k) * np.pi / (n + 1)) * math.sqrt(2 / (n + 1))
    # eigenvectors agree up to a unit phase per column
    overlap = np.abs(np.sum(vk.conj() * v, axis=0))
    np.testing.assert_allclose(overlap, 1.0, atol=1e-12)


def test_jacobi_planted_complex():
    n = 10
    q = rand_unitary(n, 7)
    lam = np.linspace(-1.0, 2.0, n) ** 3
    w, v = oracle.jacobi_eigh(gen.planted(lam, q))
    np.testing.assert_allclose(w, np.sort(lam), atol=1e-13)


def test_dense_eigensolver_agrees_with_jacobi():
    """The Rayleigh-Ritz step's dense solver against brute force."""
    g = np.random.Generator(np.random.PCG64(3))
    a = gen.gaussian(g, (12, 12), True)
    a = (a + a.conj().T) / 2
    wj, vj = oracle.jacobi_eigh(a)
    theta, va = oracle.rayleigh_ritz(a, np.eye(12, dtype=complex))
    np.testing.assert_allclose(theta, wj, atol=1e-13)
    np.testing.assert_allclose(np.abs(np.sum(vj.conj() * va, axis=0)), 1.0, atol=1e-10)


# ------------------------------------------------------------ filter
def _degrees(k, seed=0):
    g = np.random.Generator(np.random.PCG64(seed))
    return 2 * g.integers(1, 11, size=k)


def test_filter_closed_form_diagonal():
    n, k = 60, 9
    lam = np.sort(np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, n))
    b_sup, mu_1, mu_ne = 1.05, -1.0, -0.6
    x = np.random.Generator(np.random.PCG64(2)).standard_normal((n, k))
    deg = _degrees(k)
    y, mv = oracle.chebyshev_filter(np.diag(lam), x, deg, b_sup, mu_1, mu_ne)
    assert mv == int(deg.sum())
    for a in range(k):
        p = oracle.cheb_poly_value(lam, int(deg[a]), b_sup, mu_1, mu_ne)
        ref = p * x[:, a]
        assert np.max(np.abs(y[:, a] - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_filter_closed_form_planted_complex():
    """On H = Q D Q^H the filter must equal Q p(D) Q^H X (a transposed or
    conjugated H, a wrong sign or a dropped three-term coefficient all fail)."""
    n, k = 50, 7
    q = rand_unitary(n, 11)
    lam = np.sort(np.random.Generator(np.random.PCG64(4)).uniform(-1, 1, n))
    h = gen.planted(lam, q)
    x = gen.gaussian(np.random.Generator(np.random.PCG64(5)), (n, k), True)
    b_sup, mu_1, mu_ne = 1.02, -0.99, -0.4
    deg = _degrees(k, 3)
    y, _ = oracle.chebyshev_filter(h, x, deg, b_sup, mu_1, mu_ne)
    for a in range(k):
        p = oracle.cheb_poly_value(lam, int(deg[a]), b_sup, mu_1, mu_ne)
        ref = q @ (p * (q.conj().T @ x[:, a]))
        assert np.max(np.abs(y[:, a] - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_filter_is_one_at_mu1():
    """The scaled polynomial is normalised at mu_1 (1x1 matrix [mu_1])."""
    b_sup, mu_1, mu_ne = 2.0, -1.3, 0.1
    for m in (2, 8, 20, 36):
        y, _ = oracle.chebyshev_filter(np.array([[mu_1]]), np.ones((1, 1)), [m], b_sup, mu_1, mu_ne)
        assert abs(y[0, 0] - 1.0) < 1e-12


def test_filter_bounded_on_damped_interval():
    """|C_m| <= 1 on [-1,1]: after scaling, values on [mu_ne, b_sup] are at most
    1/|C_m(t(mu_1))|, which is exactly 1/cosh(m acosh|t(mu_1)|)."""
    b_sup, mu_1, mu_ne, m = 1.0, -1.0, -0.5, 12
    lam = np.linspace(mu_ne, b_sup, 41)
    y, _ = oracle.chebyshev_filter(np.diag(lam), np.ones((41, 1)), [m], b_sup, mu_1, mu_ne)
    c, e = (b_sup + mu_ne) / 2, (b_sup - mu_ne) / 2
    bound = 1 / math.cosh(m * math.acosh(abs((mu_1 - c) / e)))
    assert np.max(np.abs(y)) <= bound * (1 + 1e-10)
    assert np.max(np.abs(y)) >= bound * (1 - 1e-10)  # attained at the ends


# ------------------------------------------------------------ Lanczos
def test_lanczos_full_length_exact_quadrature():
    """With an equal-weight start vector and a full-length run (re-orthogonal
    variant) the quadrature is exact: nodes = eigenvalues, weights = 1/n, so
    the DoS count reaches n_e exactly at lambda_{n_e}."""
    n = 24
    q = rand_unitary(n, 21)
    lam = np.sort(np.random.Generator(np.random.PCG64(22)).uniform(-1, 1, n))
    h = gen.planted(lam, q)
    s = (q @ np.ones(n)) / math.sqrt(n)
    runs = oracle.lanczos_runs(h, s[:, None], n, reorth=True)
    a, b = runs[0]
    th, y = oracle.tridiag_eig(a, b)
    np.testing.assert_allclose(th, lam, atol=1e-12)
    np.testing.assert_allclose(np.abs(y[0]) ** 2, 1 / n, atol=1e-12)
    assert abs(oracle.lanczos_norm(runs) - np.max(np.abs(lam))) < 1e-12
    for n_e in (1, 5, 11, 23):
        b_sup, mu_1, mu_ne, _ = oracle.spectral_bounds(h, s[:, None], n, n_e, reorth=True)
        assert abs(mu_ne - lam[n_e - 1]) < 1e-12
        assert abs(mu_1 - lam[0]) < 1e-12
        assert b_sup >= lam[-1] - 1e-12


@pytest.mark.parametrize("kind", ["uniform", "geometric", "cluster"])
def test_lanczos_bounds_enclose_spectrum(kind):
    n = 300
    for seed in range(3):
        g = np.random.Generator(np.random.PCG64(100 + seed))
        if kind == "uniform":
            lam = gen.spectrum_uniform_iid(n, g)
        elif kind == "geometric":
            lam = gen.spectrum_geometric_low(n, g, 30)
        else:
            lam = gen.spectrum_121_cluster(n, g, 40)
        h = gen.planted(lam, gen.haar(n, g, True))
        s = gen.gaussian(g, (n, 4), True)
        b_sup, mu_1, mu_ne, runs = oracle.spectral_bounds(h, s, 25, 40)
        assert b_sup >= lam[-1] - 1e-12          # Zhou-Li upper bound
        assert mu_1 >= lam[0] - 1e-12            # Ritz values interlace
        assert mu_1 <= mu_ne <= b_sup
        nrm = oracle.lanczos_norm(runs)   # residual normalisation: a lower bound
        assert 0.5 * np.max(np.abs(lam)) <= nrm <= np.max(np.abs(lam)) + 1e-12
        for a, b in runs:
            assert len(a) == 25


def test_lanczos_three_term_relation():
    """Re-run the recurrence implied by (a, b) on the same start vector: the
    vectors it produces must be orthonormal for a short plain run, and
    T = Q^H H Q must hold (checks the index pairing of alpha and beta)."""
    n, k = 80, 10
    g = np.random.Generator(np.random.PCG64(9))
    lam = gen.spectrum_uniform_iid(n, g)
    h = gen.planted(lam, gen.haar(n, g, True))
    s = gen.gaussian(g, (n, 1), True)
    (a, b), = oracle.lanczos_runs(h, s, k)
    # build Krylov basis independently by Gram-Schmidt on s, Hs, H^2 s, ...
    kry = np.empty((n, k), dtype=complex)
    v = s[:, 0] / np.linalg.norm(s[:, 0])
    for j in range(k):
        kry[:, j] = v
        v = h @ v
    qk, _ = np.linalg.qr(kry)
    t = qk.conj().T @ h @ qk
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(t)),
                               np.sort(oracle.tridiag_eig(a, b)[0]), atol=1e-10)
    np.testing.assert_allclose(np.abs(np.diag(t, 1)), b[: k - 1], atol=1e-10)


# ------------------------------------------------------------ QR
def test_qr_locked_invariants():
    n, L, k = 120, 6, 14
    g = np.random.Generator(np.random.PCG64(31))
    y = gen.haar(n, g, True)[:, :L]
    base = gen.gaussian(g, (n, k), True)
    # ill-conditioned active block: columns nearly parallel
    v = base[:, :1] + 1e-6 * base
    q = oracle.qr_locked(y, v)
    assert q.shape == (n, L + k)
    assert np.array_equal(q[:, :L], y)
    assert np.linalg.norm(q.conj().T @ q - np.eye(L + k)) < 1e-13 * math.sqrt(L + k)
    x = np.concatenate([y, v], axis=1)
    proj = x - q @ (q.conj().T @ x)
    assert np.linalg.norm(proj) < 1e-12 * np.linalg.norm(x)


# ------------------------------------------------------------ RR + residual
def test_rayleigh_ritz_exact_invariant_subspace():
    n, k = 40, 6
    q = rand_unitary(n, 41)
    lam = np.sort(np.random.Generator(np.random.PCG64(42)).uniform(-1, 1, n))
    h = gen.planted(lam, q)
    idx = np.array([3, 7, 8, 15, 22, 30])
    mix = rand_unitary(k, 43)
    qa = q[:, idx] @ mix
    theta, va = oracle.rayleigh_ritz(h, qa)
    np.testing.assert_allclose(theta, lam[idx], atol=1e-14)
    overlap = np.abs(np.sum(q[:, idx].conj() * va, axis=0))
    np.testing.assert_allclose(overlap, 1.0, atol=1e-12)
    r = oracle.residual_norms(h, va, theta, 1.0)
    assert r.max() < 1e-14


def test_residual_two_vector_closed_form():
    n = 30
    q = rand_unitary(n, 51)
    lam = np.linspace(-1, 1, n)
    h = gen.planted(lam, q)
    for phi in (0.1, 0.7, 1.3):
        v = math.cos(phi) * q[:, 2] + math.sin(phi) * q[:, 9]
        theta = lam[2] * math.cos(phi) ** 2 + lam[9] * math.sin(phi) ** 2
        r = oracle.residual_norms(h, v[:, None], np.array([theta]), 2.0)[0]
        exact = abs(lam[9] - lam[2]) * abs(math.sin(phi) * math.cos(phi)) / 2.0
        assert abs(r - exact) < 1e-14


# ------------------------------------------------------------ degrees
def test_degree_hand_values():
    opts = oracle.Options()
    # c=0, e=1; lambda=-2 -> rho = 2+sqrt(3); ln(1e8)/ln(3.7320508) = 13.99 -> 14 + 2 = 16
    # lambda=-1.5 -> rho = 1.5+sqrt(1.25) = 2.618; ln(1e7)/0.96242 = 16.75 -> 17 + 2 = 19 -> 20
    # lambda=-0.5 (inside the damped interval) -> max_deg
    # lambda=-1.01, res=1 -> huge -> capped at 36
    m = oracle.degrees([1e-2, 1e-3, 1e-3, 1.0], [-2.0, -1.5, -0.5, -1.01], 0.0, 1.0, 1e-10, opts, 20)
    assert list(m) == [16, 20, 36, 36]
    opts.optimize_degree = False
    assert list(oracle.degrees([1e-2], [-2.0], 0.0, 1.0, 1e-10, opts, 20)) == [20]


def test_degree_rate_matches_chebyshev_growth():
    """rho in the degree formula is the growth rate of C_m outside [-1,1]:
    C_m(t) = (rho^m + rho^-m)/2.  Recover rho from the closed form and check
    that the optimised degree is the smallest m (plus the extra) with
    rho^m >= res/tol."""
    opts = oracle.Options(deg_extra=0, max_deg=1000)
    for t in (-1.2, -2.5, -7.0):
        m = 9
        cm = math.cosh(m * math.acosh(abs(t)))
        rho = (cm + math.sqrt(cm * cm - 1)) ** (1 / m)
        ratio = 1e6
        d = int(oracle.degrees([ratio * 1e-10], [t], 0.0, 1.0, 1e-10, opts, 20)[0])
        mmin = math.ceil(math.log(ratio) / math.log(rho))
        assert d == mmin + (mmin % 2)


# ------------------------------------------------------------ whole solve
def _subspace_sin(a, b):
    qa, _ = np.linalg.qr(a)
    qb, _ = np.linalg.qr(b)
    # sine of the largest principal angle, from the projection residual
    return float(np.linalg.norm(qb - qa @ (qa.conj().T @ qb), 2))


@pytest.mark.parametrize("cplx", [True, False])
def test_solve_planted_spectrum(cplx):
    p = gen.make_uniform(n=400, nev=30, nex=12, cplx=cplx, cfg=7)
    ev, v, res, st = oracle.solve(p.H, p.nev, p.nex, p.tol, p.deg, p.V0, p.S)
    assert st.converged and st.locked >= p.nev
    norm = max(abs(p.lam[0]), abs(p.lam[-1]))
    assert np.all(res <= p.tol)
    # Weyl: each Ritz value is within its residual norm of an eigenvalue
    assert np.max(np.abs(ev - p.lam[: p.nev])) <= 2 * p.tol * norm
    assert np.linalg.norm(v.conj().T @ v - np.eye(p.nev)) <= 1e-12
    r = p.H @ v - v * ev[None, :]
    assert np.max(np.linalg.norm(r, axis=0)) <= p.tol * norm * 1.5
    gap = p.lam[p.nev] - p.lam[p.nev - 1]
    bound = np.linalg.norm(r) / gap
    assert _subspace_sin(v, p.Q[:, : p.nev]) <= max(bound, 1e-12) * 1.01


def test_solve_121_closed_form():
    n, nev, nex = 240, 8, 8
    p = gen.make_tridiag("121", n, nev, nex, cfg=8)
    ev, v, res, st = oracle.solve(p.H, nev, nex, 1e-10, 20, p.V0, p.S)
    assert st.converged
    np.testing.assert_allclose(ev, p.lam[:nev], atol=1e-10 * 4)
    overlap = np.abs(np.sum(p.Q[:, :nev] * v, axis=0))
    # gaps are ~ 1e-3 so eigenvector agreement is within res/gap
    np.testing.assert_allclose(overlap, 1.0, atol=1e-6)


def test_solve_tiny_matches_jacobi():
    n, nev, nex = 20, 3, 4
    g = np.random.Generator(np.random.PCG64(61))
    a = gen.gaussian(g, (n, n), True)
    h = (a + a.conj().T) / 2
    v0 = gen.gaussian(g, (n, nev + nex), True)
    s = gen.gaussian(g, (n, 4), True)
    ev, v, res, st = oracle.solve(h, nev, nex, 1e-12, 10, v0, s)
    wj, vj = oracle.jacobi_eigh(h)
    np.testing.assert_allclose(ev, wj[:nev], atol=1e-11)
    assert st.converged


def test_solve_reports_nonconvergence():
    p = gen.make_uniform(n=200, nev=10, nex=6, cfg=9)
    ev, v, res, st = oracle.solve(p.H, p.nev, p.nex, 1e-30, p.deg, p.V0, p.S,
                                  oracle.Options(max_iter=2))
    assert not st.converged and st.iterations == 2
    assert ev.shape == (10,) and np.all(np.diff(ev) >= 0)


# ------------------------------------------------------------ generators
def test_generator_condition_numbers_match_paper():
    """The paper prints the 2-norm condition numbers of its n=20k suite
    (Section 'Eigen-type tests'); they pin the readings of the Wilkinson
    diagonal and of eps in the Uniform/Geometric formulas."""
    with open(os.path.join(GOLDEN, "condition_numbers_20k.json")) as f:
        ref = json.load(f)
    n = ref["n"]
    k = np.arange(1, n + 1)
    lam121 = 2 - 2 * np.cos(np.pi * k / (n + 1))
    got = {"1-2-1": lam121[-1] / lam121[0]}
    uni = gen.table1_uniform(n)
    geo = gen.table1_geometric(n)
    got["Uniform"] = uni[-1] / uni[0]
    got["Geometric"] = geo[-1] / geo[0]
    d, e = gen.tridiag_wilkinson(n)
    lo = sl.eigvalsh_tridiagonal(d, e, select="i", select_range=(0, 1))
    hi = sl.eigvalsh_tridiagonal(d, e, select="i", select_range=(n - 1, n - 1))
    got["Wilkinson"] = abs(hi[0]) / np.min(np.abs(lo))
    for name, val in ref["cond"].items():
        # the paper prints two significant digits
        assert abs(got[name] - val) <= 0.051 * val, (name, got[name], val)
    assert lo[0] < 0 < lo[1]  # all eigenvalues positive but one


def test_haar_is_unitary_and_planted_is_hermitian():
    g = np.random.Generator(np.random.PCG64(71))
    q = gen.haar(64, g, True)
    assert np.linalg.norm(q.conj().T @ q - np.eye(64)) < 1e-13
    lam = np.linspace(-1, 1, 64)
    h = gen.planted(lam, q)
    assert np.array_equal(h, h.conj().T)
    np.testing.assert_allclose(np.linalg.eigvalsh(h), lam, atol=1e-14)


@pytest.mark.parametrize("cplx", [True, False])
def test_eigvec_adjoint_matches_finite_differences(cplx):
    """The eigenvector adjoint (first-order perturbation over the full
    eigendecomposition) against central differences of two phase-invariant
    losses, computed with numpy's eigendecomposition:
    L1 = ||V^H B||_F^2 (torch gradient 2 B B^H V) and
    L2 = sum_i w_i |v_i[0]|^2 (torch gradient 2 w_i v_i[0] at row 0)."""
    g = np.random.Generator(np.random.PCG64(901 + cplx))
    n, m = 40, 6
    A = gen.gaussian(g, (n, n), cplx)
    H = (A + A.conj().T) / 2
    B = gen.gaussian(g, (n, 3), cplx)
    w = g.standard_normal(m)

    def lowest(Hm):
        mu, U = np.linalg.eigh(Hm)
        return mu[:m], U[:, :m]

    def loss(Hm):
        _, V = lowest(Hm)
        return float(np.linalg.norm(V.conj().T @ B) ** 2 + np.sum(w * np.abs(V[0, :]) ** 2))

    lam, V = lowest(H)
    G = 2 * B @ (B.conj().T @ V)
    G[0, :] += 2 * w * V[0, :]
    dH = oracle.eigvec_adjoint(H, V, lam, G)
    assert np.allclose(dH, dH.conj().T)
    h = 1e-6
    for s in range(3):
        E = gen.gaussian(g, (n, n), cplx)
        E = (E + E.conj().T) / 2
        fd = (loss(H + h * E) - loss(H - h * E)) / (2 * h)
        an = float(np.real(np.sum(np.conj(dH) * E)))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1.0), (fd, an)
