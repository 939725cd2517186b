"""Plain CPU FP64 oracle of ChASE's subspace iteration (Algorithm 1).

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct
reference that the GPU library is checked against.  Only the test-suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the library
never does.  It shares no code with the GPU path: only the seeded input
generators (``gen``) feed both.

Every function follows a passage of the paper (Winkelmann-style ChASE as
summarised in Section 2.1 and Algorithm 1; the recurrence of Eq. (3)).  Where
the paper is silent the reading used is stated in the docstring; the same
readings are implemented independently on the GPU side.

Pin status
  lanczos_runs / spectral_bounds : pinned (interlacing, upper bound, exact
      quadrature on full-length runs with an equal-weight start).
  filter                         : pinned (Chebyshev closed form).
  qr_locked                      : pinned (invariants).
  rayleigh_ritz                  : pinned (exact invariant subspaces, Jacobi).
  residual_norms                 : pinned (two-vector closed form).
  degrees                        : pinned (hand values, cosh identity).
  solve                          : pinned (planted spectra, (1-2-1) closed
      form, brute-force Jacobi on tiny matrices).
  mu_ne from a short Lanczos run : parity unpinned (an estimate by design;
      only its exact limit on a full-length run is pinned).
  eigvec_adjoint                 : pinned (central finite differences through
      numpy's eigendecomposition; projector-loss invariance).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Options:
    """Settings Algorithm 1 takes as given without fixing their values."""
    max_deg: int = 36         # cap of the optimised degree (reading)
    deg_extra: int = 2        # safety margin added to the optimised degree
    optimize_degree: bool = True
    lanczos_steps: int = 25   # k_L, length of each Lanczos run
    lanczos_vecs: int = 4     # n_L, number of Lanczos runs
    max_iter: int = 50


@dataclasses.dataclass
class Stats:
    iterations: int = 0
    matvecs: int = 0
    locked: int = 0
    b_sup: float = 0.0
    mu_1: float = 0.0
    mu_ne: float = 0.0
    converged: bool = False


# ---------------------------------------------------------------- Lanczos
def lanczos_runs(H, S, steps, reorth=False):
    """Plain three-term Lanczos (Algorithm 1, spectral-bound step) started
    from each column of S.  Returns, per run, the diagonal ``a`` and the
    off-diagonal ``b`` of the tridiagonal T, where ``b[j]`` couples step j to
    j+1 (so ``b[-1]`` is the residual norm after the last step).  A run stops
    early when b_j <= 1e-14 * max|a_1..j| (invariant subspace found).
    ``reorth`` = full re-orthogonalisation, used only by the pins."""
    n = H.shape[0]
    steps = min(steps, n)
    runs = []
    for r in range(S.shape[1]):
        q = S[:, r] / np.linalg.norm(S[:, r])
        basis = [q]
        q_prev = np.zeros_like(q)
        beta_prev = 0.0
        a, b = [], []
        for _ in range(steps):
            w = H @ q - beta_prev * q_prev
            alpha = float(np.real(np.vdot(q, w)))
            w = w - alpha * q
            if reorth:
                for _pass in range(2):
                    for v in basis:
                        w = w - np.vdot(v, w) * v
            beta = float(np.linalg.norm(w))
            a.append(alpha)
            b.append(beta)
            if beta <= 1e-14 * max(abs(x) for x in a):
                break
            q_prev, q = q, w / beta
            basis.append(q)
            beta_prev = beta
        runs.append((np.array(a), np.array(b)))
    return runs


def tridiag_eig(a, b):
    """Eigen-decomposition of the symmetric tridiagonal matrix with diagonal a
    and off-diagonal b[:-1] (numpy's dense symmetric eigensolver)."""
    k = len(a)
    t = np.diag(a)
    if k > 1:
        t += np.diag(b[: k - 1], 1) + np.diag(b[: k - 1], -1)
    return np.linalg.eigh(t)


def dos_mu(nodes, weights, n, count):
    """Lanczos-quadrature density of states (the DoS estimate the paper cites
    from Lin et al.): the smallest node at which the estimated eigenvalue count
    n * cumulative_weight reaches ``count`` (step-function reading, no
    interpolation)."""
    order = np.argsort(nodes, kind="stable")
    cum = np.cumsum(weights[order]) * n
    idx = int(np.searchsorted(cum, count - 1e-9 * count))
    idx = min(idx, len(order) - 1)
    return float(nodes[order][idx])


def spectral_bounds(H, S, steps, n_e, reorth=False):
    """b_sup, mu_1, mu_{nev+nex} from the Lanczos runs (Algorithm 1, spectral
    bound step).  b_sup = max over runs of (largest Ritz value + |last beta|)
    (Zhou-Li upper bound), mu_1 = smallest Ritz value, mu_ne from the pooled
    quadrature nodes with weights |first eigenvector component|^2 / n_runs,
    clamped into [mu_1, b_sup]."""
    n = H.shape[0]
    runs = lanczos_runs(H, S, steps, reorth)
    b_sup, mu_1 = -np.inf, np.inf
    nodes, weights = [], []
    for a, b in runs:
        th, y = tridiag_eig(a, b)
        b_sup = max(b_sup, th[-1] + abs(b[len(a) - 1]))
        mu_1 = min(mu_1, th[0])
        nodes.append(th)
        weights.append(np.abs(y[0, :]) ** 2 / len(runs))
    nodes = np.concatenate(nodes)
    weights = np.concatenate(weights)
    mu_ne = dos_mu(nodes, weights, n, n_e)
    mu_ne = min(max(mu_ne, mu_1), b_sup)
    return float(b_sup), float(mu_1), float(mu_ne), runs


def lanczos_norm(runs):
    """Largest Ritz value in magnitude over the Lanczos runs: Ritz values lie
    in [lambda_min, lambda_max], so this is a lower bound of ||H||_2 (the
    residual normalisation of the solver)."""
    best = 0.0
    for a, b in runs:
        th, _ = tridiag_eig(a, b)
        best = max(best, abs(th[0]), abs(th[-1]))
    return float(best)


# ---------------------------------------------------------------- filter
def filter_coefficients(m, b_sup, mu_1, mu_ne):
    """Scalars (alpha_s, gamma_s, beta_s) of Eq. (3) for steps s = 1..m of the
    Chebyshev filter scaled so that the polynomial is 1 at mu_1 (Zhou & Saad
    scaled three-term recurrence).  Interval [mu_ne, b_sup] is damped:
    c = centre, e = half-width, sigma_1 = e / (mu_1 - c),
    sigma_{s+1} = 1 / (2/sigma_1 - sigma_s).
    Step 1:  X_1 = (sigma_1/e) (H - cI) X_0.
    Step s:  X_s = (2 sigma_s/e)(H - cI) X_{s-1} - sigma_{s-1} sigma_s X_{s-2}."""
    c = (b_sup + mu_ne) / 2.0
    e = (b_sup - mu_ne) / 2.0
    sigma1 = e / (mu_1 - c)
    coeffs = [(sigma1 / e, c, 0.0)]
    sigma = sigma1
    for _ in range(2, m + 1):
        sigma_new = 1.0 / (2.0 / sigma1 - sigma)
        coeffs.append((2.0 * sigma_new / e, c, -sigma * sigma_new))
        sigma = sigma_new
    return coeffs


def chebyshev_filter(H, X, degrees, b_sup, mu_1, mu_ne):
    """Filter step of Algorithm 1: column a of X is replaced by p_{m_a}(H) x_a,
    computed by the recurrence of Eq. (3).  Each column runs its own number of
    steps; the step count per column is its degree.  Returns (Y, matvecs)
    where matvecs counts matrix-vector products (one per column per step)."""
    degrees = np.asarray(degrees, dtype=np.int64)
    mmax = int(degrees.max()) if degrees.size else 0
    coeffs = filter_coefficients(max(mmax, 1), b_sup, mu_1, mu_ne)
    prev = np.array(X, dtype=np.result_type(X, np.float64), copy=True)  # X_{s-2}
    cur = prev.copy()                                                   # X_{s-1}
    matvecs = 0
    for s in range(1, mmax + 1):
        alpha, gamma, beta = coeffs[s - 1]
        act = np.nonzero(degrees >= s)[0]
        matvecs += act.size
        hx = H @ cur[:, act]
        nxt = alpha * (hx - gamma * cur[:, act]) + beta * prev[:, act]
        prev[:, act] = cur[:, act]
        cur[:, act] = nxt
    return cur, matvecs


def cheb_poly_value(lam, m, b_sup, mu_1, mu_ne):
    """Closed form of the scaled filter polynomial: C_m(t(lam)) / C_m(t(mu_1)),
    t(x) = (x - c)/e, C_m(t) = cos(m acos t) on |t|<=1 and
    sign^m cosh(m acosh|t|) outside.  Used by the pins only."""
    c = (b_sup + mu_ne) / 2.0
    e = (b_sup - mu_ne) / 2.0

    def cheb(t):
        t = np.asarray(t, dtype=np.float64)
        out = np.empty_like(t)
        inside = np.abs(t) <= 1
        out[inside] = np.cos(m * np.arccos(t[inside]))
        ti = t[~inside]
        out[~inside] = np.sign(ti) ** m * np.cosh(m * np.arccosh(np.abs(ti)))
        return out

    return cheb((np.asarray(lam) - c) / e) / cheb(np.array([(mu_1 - c) / e]))[0]


# ---------------------------------------------------------------- QR
def qr_locked(Y_locked, V):
    """QR step of Algorithm 1 on [Y V] (Householder, numpy), after which the
    locked columns are put back verbatim, so the returned block is
    [Y, Q_active] with Q_active orthonormal and orthogonal to Y."""
    L = Y_locked.shape[1]
    q, _ = np.linalg.qr(np.concatenate([Y_locked, V], axis=1))
    q[:, :L] = Y_locked
    return q


# ---------------------------------------------------------------- RR
def rayleigh_ritz(H, Qa):
    """Rayleigh-Ritz step (Algorithm 1; Section 2.3): G = Qa^H (H Qa), made
    exactly Hermitian, diagonalised with a dense solver (ascending), and the
    Ritz vectors Qa W returned with the Ritz values.  The projection is on the
    non-locked part only (the subspace yet to be diagonalised)."""
    g = Qa.conj().T @ (H @ Qa)
    g = (g + g.conj().T) / 2
    theta, w = np.linalg.eigh(g)
    return theta, Qa @ w


def residual_norms(H, V, theta, norm_est):
    """Residual step: ||H v_a - theta_a v_a||_2 / norm_est per column, with
    norm_est the largest Lanczos Ritz value in magnitude (a lower bound of
    ||H||_2, so res <= tol guarantees ||H v - theta v|| <= tol ||H||_2)."""
    r = H @ V - V * theta[None, :]
    return np.linalg.norm(r, axis=0) / norm_est


# ---------------------------------------------------------------- degrees
def degrees(res, ritz, c, e, tol, opts: Options, deg):
    """Degree step of Algorithm 1: per non-converged vector,
    m_a = ceil(|ln(res_a/tol)| / ln rho_a) + deg_extra, capped at max_deg and
    rounded up to even, with t_a = (ritz_a - c)/e and
    rho_a = max |t_a +- sqrt(t_a^2 - 1)| (the convergence factor of the
    Chebyshev polynomial at ritz_a).  rho_a <= 1 + 1e-12 gives max_deg."""
    res = np.asarray(res, dtype=np.float64)
    ritz = np.asarray(ritz, dtype=np.float64)
    out = np.empty(res.shape, dtype=np.int64)
    for a in range(res.size):
        if not opts.optimize_degree:
            m = deg
        else:
            t = (ritz[a] - c) / e
            root = np.sqrt(complex(t * t - 1.0))
            rho = max(abs(t + root), abs(t - root))
            if rho <= 1.0 + 1e-12:
                m = opts.max_deg
            else:
                m = int(math.ceil(abs(math.log(res[a] / tol)) / math.log(rho))) + opts.deg_extra
                m = min(m, opts.max_deg)
        m = max(m, 2)
        m += m % 2
        out[a] = m
    return out


# ---------------------------------------------------------------- solver
def solve(H, nev, nex, tol, deg, V0, S, opts: Options | None = None):
    """Algorithm 1 (ChASE): Lanczos bounds, then repeat Filter -> QR ->
    Rayleigh-Ritz -> Residual -> Deflation & Locking -> bound update ->
    Degrees -> Sort until nev pairs are locked or max_iter is reached.

    Readings: locking takes the longest converged prefix in ascending Ritz
    order; the bound update uses mu_1 = min and mu_ne = max of the locked and
    current Ritz values with b_sup fixed; residuals are relative to the
    largest Lanczos Ritz value in magnitude; degrees are even.
    Returns (evals[nev], evecs[n, nev], resid[nev], Stats)."""
    opts = opts or Options()
    n = H.shape[0]
    n_e = nev + nex
    deg = deg + deg % 2
    st = Stats()
    b_sup, mu_1, mu_ne, runs = spectral_bounds(H, S, opts.lanczos_steps, n_e)
    st.b_sup, st.mu_1, st.mu_ne = b_sup, mu_1, mu_ne
    norm_est = lanczos_norm(runs)
    c = (b_sup + mu_ne) / 2.0
    e = (b_sup - mu_ne) / 2.0

    V = np.array(V0, dtype=np.result_type(H, V0, np.float64), copy=True)
    m = np.full(n_e, deg, dtype=np.int64)
    lam = np.zeros(n_e)
    res = np.full(n_e, np.inf)
    L = 0
    for it in range(opts.max_iter):
        st.iterations = it + 1
        V[:, L:], mv = chebyshev_filter(H, V[:, L:], m[L:], b_sup, mu_1, mu_ne)
        st.matvecs += mv
        V = qr_locked(V[:, :L], V[:, L:])
        theta, Va = rayleigh_ritz(H, V[:, L:])
        V[:, L:] = Va
        lam[L:] = theta
        res[L:] = residual_norms(H, Va, theta, norm_est)
        nconv = 0
        while L + nconv < n_e and res[L + nconv] <= tol:
            nconv += 1
        L += nconv
        if L >= nev:
            st.converged = True
            break
        mu_1 = float(lam[:n_e].min())
        mu_ne = float(lam[:n_e].max())
        c = (b_sup + mu_ne) / 2.0
        e = (b_sup - mu_ne) / 2.0
        m[L:] = degrees(res[L:], lam[L:], c, e, tol, opts, deg)
        order = np.argsort(m[L:], kind="stable")
        V[:, L:] = V[:, L:][:, order]
        lam[L:] = lam[L:][order]
        res[L:] = res[L:][order]
        m[L:] = m[L:][order]
    st.locked = L
    st.mu_1, st.mu_ne = mu_1, mu_ne
    nout = L if L >= nev else n_e
    order = np.argsort(lam[:nout], kind="stable")[:nev]
    return lam[order], V[:, order], res[order], st


# ---------------------------------------------------------------- pins
def jacobi_eigh(A, sweeps=100, tol=1e-15):
    """Brute-force cyclic Jacobi diagonalisation of a small Hermitian matrix
    (Golub & Van Loan, symmetric Schur rotations; a complex pivot a_pq = g*ph
    is first made real by the phase D = diag(1, conj(ph)) on index q).
    Pure-Python loops over (p, q), for tiny matrices only.
    Returns (ascending eigenvalues, eigenvectors as columns)."""
    a = np.array(A, dtype=np.complex128, copy=True)
    n = a.shape[0]
    v = np.eye(n, dtype=np.complex128)
    for _ in range(sweeps):
        off = math.sqrt(sum(abs(a[i, j]) ** 2 for i in range(n) for j in range(n) if i != j))
        scale = math.sqrt(sum(abs(a[i, i]) ** 2 for i in range(n))) or 1.0
        if off <= tol * scale:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = a[p, q]
                g = abs(apq)
                if g == 0.0:
                    continue
                ph = apq / g
                tau = (a[q, q].real - a[p, p].real) / (2.0 * g)
                t = (1.0 if tau >= 0 else -1.0) / (abs(tau) + math.sqrt(1.0 + tau * tau))
                cs = 1.0 / math.sqrt(1.0 + t * t)
                sn = t * cs
                u = np.eye(n, dtype=np.complex128)
                u[p, p] = cs
                u[p, q] = sn
                u[q, p] = -sn * np.conj(ph)
                u[q, q] = cs * np.conj(ph)
                a = u.conj().T @ a @ u
                v = v @ u
    w = np.real(np.diagonal(a)).copy()
    order = np.argsort(w, kind="stable")
    return w[order], v[:, order]


def eigvec_adjoint(H, V, lam, G):
    """Gradient w.r.t. Hermitian H of a real loss L(V) on the lowest m
    eigenvectors V (n x m, eigenvalues lam ascending, simple) that does not
    depend on the vectors' phases, given G = dL/dV in torch's complex
    convention (dL = Re tr(G^H dV)).

    Definition used (first-order perturbation of a simple eigenpair, summed
    over the full eigendecomposition H = U diag(mu) U^H, which is the slow,
    plain part): dv_i = sum_{k != i} u_k (u_k^H dH v_i) / (lam_i - mu_k), so
        dL/dH = sym( sum_i sum_{k != i} u_k (u_k^H g_i) v_i^H / (lam_i - mu_k) ),
    sym(A) = (A + A^H)/2 (H ranges over Hermitian matrices).  The eigenpair
    u_i matching v_i is the i-th lowest.  Not in the paper: it extends the
    eigenvalue adjoint of the library's differentiation to losses on the
    eigenvectors.  Pinned by central finite differences through numpy's
    eigendecomposition on gauge-invariant losses."""
    n, m = V.shape
    mu, U = np.linalg.eigh(H)
    C = U.conj().T @ G                      # C[k, i] = u_k^H g_i
    D = np.zeros_like(C)
    for i in range(m):
        for k in range(n):
            if k != i:
                D[k, i] = C[k, i] / (lam[i] - mu[k])
    A = U @ D @ V.conj().T
    return (A + A.conj().T) / 2
