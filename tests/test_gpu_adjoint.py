"""Hand-written adjoints (through the C ABI) against central finite
differences and closed-form reference gradients.

Eigenvalue loss: dL/dH = sum_i w_i v_i v_i^H (first-order perturbation of
simple eigenvalues), referenced by the planted eigenvectors.
Filtered-block loss L = ||Y^H B||_F^2 with Y = p(H) X0 at frozen bounds and
degrees: referenced by the Daleckii-Krein formula
G = Q (F o (Q^H dL/dY X0^H Q)) Q^H, F_ij = (p_i - p_j)/(l_i - l_j), F_ii = p'(l_i).
Target: 1e-6 relative."""
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


def herm_dir(n, cplx, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    e = gen.gaussian(g, (n, n), cplx)
    e = (e + e.conj().T) / 2
    return e / np.linalg.norm(e)


def directional(G, E):
    return float(np.real(np.sum(np.conj(G) * E)))


@pytest.mark.parametrize("cplx", [True, False])
def test_eigval_adjoint_fd_and_reference(pk, cplx):
    import torch
    announce(f"eigval adjoint n=300 cplx={cplx}")
    p = gen.make_uniform(n=300, nev=12, nex=8, cplx=cplx, cfg=30)
    w = np.random.Generator(np.random.PCG64(31)).standard_normal(p.nev)
    V0, S = to_gpu(p.V0), to_gpu(p.S)

    def loss(Hn):
        lam, _ = pk.chase_eigh(to_gpu(Hn), p.nev, p.nex, 1e-12, 20, V0, S)
        return float(np.dot(w, to_np(lam)))

    H = to_gpu(p.H).requires_grad_(True)
    lam, vec = pk.chase_eigh(H, p.nev, p.nex, 1e-12, 20, V0, S)
    (torch.from_numpy(w).cuda() * lam).sum().backward()
    G = to_np(H.grad)
    q = p.Q[:, : p.nev]
    G_ref = (q * w[None, :]) @ q.conj().T
    assert np.linalg.norm(G - G_ref) <= 1e-8 * np.linalg.norm(G_ref)
    h = 1e-6
    for s in range(3):
        E = herm_dir(300, cplx, 40 + s)
        fd = (loss(p.H + h * E) - loss(p.H - h * E)) / (2 * h)
        an = directional(G, E)
        assert abs(fd - an) <= 1e-6 * max(abs(an), np.linalg.norm(G) * 1e-3), (fd, an)


def _cheb_deriv(lam, m, b_sup, mu_1, mu_ne):
    hstep = 1e-5 * (b_sup - mu_1)
    return (oracle.cheb_poly_value(lam + hstep, m, b_sup, mu_1, mu_ne)
            - oracle.cheb_poly_value(lam - hstep, m, b_sup, mu_1, mu_ne)) / (2 * hstep)


@pytest.mark.parametrize("cplx", [True, False])
def test_filter_adjoint_fd_and_daleckii_krein(pk, cplx):
    import torch
    announce(f"filter adjoint n=260 cplx={cplx}")
    n, k, m = 260, 24, 10
    g = np.random.Generator(np.random.PCG64(50 + cplx))
    lam = gen.spectrum_uniform_iid(n, g)
    q = gen.haar(n, g, cplx)
    Hn = gen.planted(lam, q)
    X0 = gen.gaussian(g, (n, k), cplx)
    B = gen.gaussian(g, (n, 5), cplx)
    b_sup, mu_1, mu_ne = 1.05, -1.0, -0.5
    deg = np.full(k, m, dtype=np.int32)
    Bt = to_gpu(B)

    def loss_np(Hm):
        y, _ = oracle.chebyshev_filter(Hm, X0, deg, b_sup, mu_1, mu_ne)
        return float(np.linalg.norm(y.conj().T @ B) ** 2)

    H = to_gpu(Hn).requires_grad_(True)
    Y = pk.filtered_block(H, to_gpu(X0), deg, b_sup, mu_1, mu_ne)
    L = (torch.linalg.matrix_norm(Y.mH @ Bt) ** 2)
    L.backward()
    G = to_np(H.grad)
    # Daleckii-Krein reference
    pv = oracle.cheb_poly_value(lam, m, b_sup, mu_1, mu_ne)
    dp = _cheb_deriv(lam, m, b_sup, mu_1, mu_ne)
    dl = lam[:, None] - lam[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        F = np.where(np.abs(dl) > 1e-9, (pv[:, None] - pv[None, :]) / dl, 0.0)
    F[np.diag_indices(n)] = dp
    Y_ref, _ = oracle.chebyshev_filter(Hn, X0, deg, b_sup, mu_1, mu_ne)
    gY = 2 * B @ (B.conj().T @ Y_ref)
    G_ref = q @ (F * (q.conj().T @ gY @ X0.conj().T @ q)) @ q.conj().T
    G_ref = (G_ref + G_ref.conj().T) / 2
    assert np.linalg.norm(G - G_ref) <= 1e-6 * np.linalg.norm(G_ref)
    h = 1e-6
    for s in range(3):
        E = herm_dir(n, cplx, 60 + s)
        fd = (loss_np(Hn + h * E) - loss_np(Hn - h * E)) / (2 * h)
        an = directional(G, E)
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9 * np.linalg.norm(G), (fd, an)


def test_filter_adjoint_mixed_degrees_input_gradient(pk):
    """Per-column degrees (sorted) and the gradient w.r.t. the filter input:
    Y = P X0 column-wise with P_a = p_{m_a}(H), so dL/dx_a = P_a^H g_a =
    p_{m_a}(H) g_a (p real, H Hermitian) -- the filter itself applied to gY."""
    import torch
    announce("filter adjoint per-column degrees + input gradient")
    n, k = 300, 16
    g = np.random.Generator(np.random.PCG64(70))
    lam = gen.spectrum_uniform_iid(n, g)
    q = gen.haar(n, g, True)
    Hn = gen.planted(lam, q)
    X0 = gen.gaussian(g, (n, k), True)
    deg = np.sort(2 * g.integers(1, 8, size=k)).astype(np.int32)
    b_sup, mu_1, mu_ne = 1.02, -1.0, -0.4
    gY = gen.gaussian(g, (n, k), True)
    H = to_gpu(Hn).requires_grad_(True)
    X = to_gpu(X0).requires_grad_(True)
    Y = pk.filtered_block(H, X, deg, b_sup, mu_1, mu_ne)
    torch.sum(torch.real(torch.conj(to_gpu(gY)) * Y)).backward()
    gx_ref, _ = oracle.chebyshev_filter(Hn, gY, deg, b_sup, mu_1, mu_ne)
    assert np.linalg.norm(to_np(X.grad) - gx_ref) <= 1e-10 * np.linalg.norm(gx_ref)
    # dH by FD on the linear functional
    Gd = to_np(H.grad)
    for s in range(2):
        E = herm_dir(n, True, 80 + s)
        yp, _ = oracle.chebyshev_filter(Hn + 1e-6 * E, X0, deg, b_sup, mu_1, mu_ne)
        ym, _ = oracle.chebyshev_filter(Hn - 1e-6 * E, X0, deg, b_sup, mu_1, mu_ne)
        fd = float(np.real(np.sum(np.conj(gY) * (yp - ym)))) / 2e-6
        an = directional(Gd, E)
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9 * np.linalg.norm(Gd), (fd, an)


@pytest.mark.parametrize("cplx", [True, False])
def test_filter_adjoint_full_size_daleckii_krein(pk, cplx):
    """Differentiation workload size (n=8000 complex128 and float64,
    nev+nex=260 columns, degree 20): the gradient of ||Y^H B||_F^2 against
    the Daleckii-Krein closed form built from the planted eigenvectors, on
    the GPU with torch."""
    import torch
    announce(f"filter adjoint n=8000 vs Daleckii-Krein cplx={cplx}")
    p = gen.make_uniform(n=8000, nev=200, nex=60, cplx=cplx, cfg=gen.CFG_DIFF8K)
    _, B = gen.loss_weights(gen.CFG_DIFF8K, 200, 16, 8000, cplx)
    b_sup, mu_1, mu_ne, m = 1.05, -1.0, -0.9, 20
    deg = np.full(260, m, dtype=np.int32)
    H = to_gpu(p.H).requires_grad_(True)
    X0, Bt = to_gpu(p.V0), to_gpu(B)
    Y = pk.filtered_block(H, X0, deg, b_sup, mu_1, mu_ne)
    (torch.linalg.matrix_norm(Y.mH @ Bt) ** 2).backward()
    G = H.grad
    lam = p.lam
    pv = oracle.cheb_poly_value(lam, m, b_sup, mu_1, mu_ne)
    dp = _cheb_deriv(lam, m, b_sup, mu_1, mu_ne)
    dl = lam[:, None] - lam[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        F = np.where(np.abs(dl) > 1e-7, (pv[:, None] - pv[None, :]) / dl,
                     0.5 * (dp[:, None] + dp[None, :]))
    q = to_gpu(p.Q)
    Ft = to_gpu(F).to(q.dtype)
    gY = 2.0 * Bt @ (Bt.mH @ Y.detach())
    M = (q.mH @ gY) @ (X0.mH @ q)
    G_ref = q @ (Ft * M) @ q.mH
    G_ref = (G_ref + G_ref.mH) / 2
    err = float(torch.linalg.matrix_norm(G - G_ref) / torch.linalg.matrix_norm(G_ref))
    # the reference's own divided differences are accurate to ~1e-8 here
    assert err < 1e-6, err


# ------------------------------------------------------------------ eigenvector adjoint
@pytest.mark.parametrize("cplx", [True, False])
def test_eigvec_adjoint_matches_oracle(pk, cplx):
    """chase_eigvec_adjoint (divided differences within the block,
    conjugate-gradient solves on the complement) against the oracle's
    definition (first-order perturbation over the full eigendecomposition),
    for the exact planted eigenpairs and an arbitrary G."""
    import torch
    announce(f"eigvec adjoint vs oracle n=320 cplx={cplx}")
    n, m = 320, 14
    g = np.random.Generator(np.random.PCG64(120 + cplx))
    lam = gen.spectrum_uniform_iid(n, g)
    q = gen.haar(n, g, cplx)
    Hn = gen.planted(lam, q)
    V = q[:, :m]
    G = gen.gaussian(g, (n, m), cplx)
    ref = oracle.eigvec_adjoint(Hn, V, lam[:m], G)
    dH = torch.zeros((n, n), dtype=to_gpu(Hn).dtype, device="cuda")
    its = pk.chase_eigvec_adjoint(to_gpu(Hn), to_gpu(V), lam[:m], to_gpu(G), dH, tol=1e-12)
    assert its > 0
    err = np.linalg.norm(to_np(dH) - ref) / np.linalg.norm(ref)
    assert err < 1e-8, err


@pytest.mark.parametrize("cplx", [True, False])
def test_eigvec_autograd_matches_finite_differences(pk, cplx):
    """Loss on eigenvalues and eigenvectors through chase_eigh's backward:
    L = sum_i w_i lam_i + ||V^H B||_F^2, against central differences of the
    same loss computed with numpy's eigendecomposition."""
    import torch
    announce(f"eigvec autograd FD n=300 cplx={cplx}")
    p = gen.make_uniform(n=300, nev=12, nex=8, cplx=cplx, cfg=32)
    g = np.random.Generator(np.random.PCG64(33))
    w = g.standard_normal(p.nev)
    B = gen.gaussian(g, (300, 3), cplx)
    Bt = to_gpu(B)
    H = to_gpu(p.H).requires_grad_(True)
    lam, vec = pk.chase_eigh(H, p.nev, p.nex, 1e-12, 20, to_gpu(p.V0), to_gpu(p.S), adj_tol=1e-12)
    L = (torch.from_numpy(w).cuda() * lam).sum() + torch.linalg.matrix_norm(vec.mH @ Bt) ** 2
    L.backward()
    G = to_np(H.grad)
    assert np.linalg.norm(G - G.conj().T) <= 1e-12 * np.linalg.norm(G)

    def loss_np(Hm):
        mu, U = np.linalg.eigh(Hm)
        V = U[:, : p.nev]
        return float(np.dot(w, mu[: p.nev]) + np.linalg.norm(V.conj().T @ B) ** 2)

    h = 1e-6
    for s in range(3):
        E = herm_dir(300, cplx, 140 + s)
        fd = (loss_np(p.H + h * E) - loss_np(p.H - h * E)) / (2 * h)
        an = directional(G, E)
        assert abs(fd - an) <= 1e-6 * max(abs(an), np.linalg.norm(G) * 1e-3), (fd, an)


@pytest.mark.parametrize("cplx", [True, False])
def test_eigvec_adjoint_full_size_planted(pk, cplx):
    """Differentiation workload size (n=8000 complex128 and float64, 200
    eigenvectors): the adjoint of ||V^H B||_F^2 against the first-order
    formula evaluated with torch from the planted eigendecomposition (all
    8000 pairs)."""
    import torch
    announce(f"eigvec adjoint n=8000 vs planted first-order formula cplx={cplx}")
    p = gen.make_uniform(n=8000, nev=200, nex=60, cplx=cplx, cfg=gen.CFG_DIFF8K)
    _, B = gen.loss_weights(gen.CFG_DIFF8K, 200, 16, 8000, cplx)
    Q = to_gpu(p.Q)
    lam = torch.from_numpy(p.lam).cuda()
    V = Q[:, :200].contiguous()
    Bt = to_gpu(B)
    G = 2.0 * Bt @ (Bt.mH @ V)
    H = to_gpu(p.H)
    dH = torch.zeros_like(H)
    its = pk.chase_eigvec_adjoint(H, V, p.lam[:200], G, dH, tol=1e-11)
    C = Q.mH @ G                                   # C[k, i] = q_k^H g_i
    den = lam[:200][None, :] - lam[:, None]        # lam_i - mu_k
    idx = torch.arange(200, device="cuda")
    den[idx, idx] = 1.0
    D = C / den
    D[idx, idx] = 0.0
    A = Q @ (D @ V.mH)
    ref = (A + A.mH) / 2
    err = float(torch.linalg.matrix_norm(dH - ref) / torch.linalg.matrix_norm(ref))
    print(f"[gpu-case] eigvec adjoint n=8000: {its} CG iterations, rel err {err:.2e}", flush=True)
    assert err < 1e-6, err


@pytest.mark.parametrize("cplx", [True, False])
def test_differentiation_workload_finite_differences(pk, cplx):
    """The differentiation workload end to end (n=8000, nev=200, nex=60):
    L = sum_i w_i lambda_i + ||Y^H B||_F^2 with lambda from the solve and Y
    the filtered start block at frozen bounds and degrees, gradient by the
    library's adjoints through autograd, against central differences
    (h = 1e-6) along two Hermitian directions: one built from B (so the
    directional derivative is a sizeable part of ||G||) and one Gaussian.
    The differences carry the forward evaluation's rounding over h, so the
    bar is 1e-6 of max(|derivative|, 1e-3 ||G||_F)."""
    import torch
    announce(f"differentiation workload FD n=8000 cplx={cplx}")
    n, nev, nex, tol, m = 8000, 200, 60, 1e-10, 20
    p = gen.make_uniform(n=n, nev=nev, nex=nex, cplx=cplx, cfg=gen.CFG_DIFF8K)
    w, B = gen.loss_weights(gen.CFG_DIFF8K, nev, 16, n, cplx)
    Hd, V0, S = to_gpu(p.H), to_gpu(p.V0), to_gpu(p.S)
    Bt, wt = to_gpu(B), to_gpu(w)
    _, _, _, st = pk.chase_solve(Hd, nev, nex, tol, m, V0, S)
    frozen = (st["b_sup"], st["mu_1"], st["mu_ne"])
    deg = np.full(nev + nex, m, dtype=np.int32)

    def loss(Hx):
        lam, _ = pk.chase_eigh(Hx, nev, nex, tol, m, V0, S)
        Y = pk.filtered_block(Hx, V0, deg, *frozen)
        return (wt * lam).sum() + torch.linalg.matrix_norm(Y.mH @ Bt) ** 2

    H = Hd.clone().requires_grad_(True)
    loss(H).backward()
    G = to_np(H.grad)
    gnorm = np.linalg.norm(G)
    g = np.random.Generator(np.random.PCG64(930 + cplx))
    c = gen.gaussian(g, (16, 16), cplx)
    E1 = B @ c @ B.conj().T
    E2 = gen.gaussian(g, (n, n), cplx)
    h = 1e-6
    for E in (E1, E2):
        E = (E + E.conj().T) / 2
        E /= np.linalg.norm(E)
        Et = to_gpu(E)
        with torch.no_grad():
            fd = (float(loss(Hd + h * Et)) - float(loss(Hd - h * Et))) / (2 * h)
        an = directional(G, E)
        announce(f"  FD {fd:.10e}  adjoint {an:.10e}  rel {abs(fd - an) / abs(an):.2e}")
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * gnorm), (fd, an, gnorm)


def test_adjoints_with_reserved_buffers_match(pk):
    """A handle created with adjoint_reserve holds the filter tape and the
    eigenvector adjoint's blocks from creation; the adjoints computed with it
    equal those of a handle that allocates them on first use."""
    import torch
    announce("adjoints with buffers reserved at creation")
    n, k, m, nev = 400, 30, 12, 10
    g = np.random.Generator(np.random.PCG64(77))
    lam = gen.spectrum_uniform_iid(n, g)
    q = gen.haar(n, g, True)
    H = to_gpu(gen.planted(lam, q))
    X0 = to_gpu(gen.gaussian(g, (n, k), True))
    gY = to_gpu(gen.gaussian(g, (n, k), True))
    Gv = to_gpu(gen.gaussian(g, (n, nev), True))
    V = to_gpu(q[:, :nev])
    deg = np.full(k, m, dtype=np.int32)
    out = []
    for reserve in (0, m):
        h = pk.Handle(n, k - 5, 5, H.dtype, pk.default_opts(adjoint_reserve=reserve))
        pk.chase_filter(H, X0, deg, 1.05, -1.0, -0.5, record_tape=True, handle=h)
        dF = torch.zeros_like(H)
        pk.chase_filter_adjoint(H, gY, dF, h)
        dV = torch.zeros_like(H)
        pk.chase_eigvec_adjoint(H, V, lam[:nev], Gv, dV, handle=h, tol=1e-12)
        out.append((to_np(dF), to_np(dV)))
        h.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
