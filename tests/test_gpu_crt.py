"""FP64 filter products on the INT8 matrix cores (chase_opts.fp64_emulation:
exact integer products modulo several moduli, recovered by Chinese
remaindering) against the CPU oracle's FP64 filter and solve."""
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


def _problem(n, cplx, seed, row_scale=False):
    g = np.random.Generator(np.random.PCG64(seed))
    lam = gen.spectrum_uniform_iid(n, g)
    q = gen.haar(n, g, cplx)
    h = gen.planted(lam, q)
    if row_scale:
        # a Hermitian D H D with D spanning six decades: rows of very
        # different magnitude (each row gets its own integer scale)
        d = np.exp(np.linspace(0.0, np.log(1e-6), n))
        h = (d[:, None] * h) * d[None, :]
    return h, g


@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("n,k,nm", [(300, 37, 14), (700, 150, 14), (1000, 140, 16),
                                    (1000, 140, 12), (333, 17, 14), (515, 64, 16),
                                    (40, 2, 14), (129, 5, 16)])
def test_int8_filter_matches_oracle(pk, cplx, n, k, nm):
    import torch
    announce(f"INT8 CRT filter n={n} k={k} moduli={nm} cplx={cplx}")
    # n = 333, 515 and 129 (not multiples of 4) take the one-entry-per-thread
    # conversion and reconstruction kernels, the others the four-wide ones;
    # (40, 2) and (129, 5) are the smallest blocks a handle takes
    h, g = _problem(n, cplx, 2000 + n + k + nm)
    x = gen.gaussian(g, (n, k), cplx)
    # columns of very different size (each column gets its own scale)
    x = x * np.exp(g.uniform(-8, 8, size=k))[None, :]
    deg = np.sort(2 * g.integers(1, 11, size=k)).astype(np.int32)
    b_sup, mu_1, mu_ne = 1.03, -1.0, -0.55
    y_ref, mv_ref = oracle.chebyshev_filter(h, x, deg, b_sup, mu_1, mu_ne)
    handle = pk.Handle(n, k - 1, 1, torch.complex128 if cplx else torch.float64,
                       pk.default_opts(fp64_emulation=nm))
    y, mv = pk.chase_filter(to_gpu(h), to_gpu(x), deg, b_sup, mu_1, mu_ne, handle=handle)
    assert mv == mv_ref
    y = to_np(y)
    # the integer forms keep about (log2 M - log2 n) / 2 bits: 14 and 16
    # moduli reach the FP64 filter's parity bar, 12 moduli about 2^-36
    tol = 1e-12 if nm >= 14 else 1e-9
    for a in range(k):
        err = np.max(np.abs(y[:, a] - y_ref[:, a])) / np.max(np.abs(y_ref[:, a]))
        assert err < tol, (a, deg[a], err)


@pytest.mark.parametrize("cplx", [True, False])
def test_int8_filter_rows_of_different_scale(pk, cplx):
    import torch
    n, k = 500, 33
    announce(f"INT8 CRT filter, rows over six decades, cplx={cplx}")
    h, g = _problem(n, cplx, 77, row_scale=True)
    x = gen.gaussian(g, (n, k), cplx)
    deg = np.full(k, 4, dtype=np.int32)
    nrm = np.max(np.abs(np.linalg.eigvalsh(h)))
    b_sup, mu_1, mu_ne = 1.01 * nrm, -nrm, -0.5 * nrm
    y_ref, _ = oracle.chebyshev_filter(h, x, deg, b_sup, mu_1, mu_ne)
    handle = pk.Handle(n, k - 1, 1, torch.complex128 if cplx else torch.float64,
                       pk.default_opts(fp64_emulation=14))
    y, _ = pk.chase_filter(to_gpu(h), to_gpu(x), deg, b_sup, mu_1, mu_ne, handle=handle)
    err = np.max(np.abs(to_np(y) - y_ref)) / np.max(np.abs(y_ref))
    assert err < 1e-12, err


@pytest.mark.parametrize("cplx", [True, False])
def test_int8_defect_form_matches_fp64(pk, cplx):
    """The defect-correction filter (chase_filter_ritz) with FP64 products
    on INT8 against the same call on the FP64 matrix cores."""
    import torch
    n, k = 600, 40
    announce(f"INT8 CRT defect-form filter cplx={cplx}")
    h, g = _problem(n, cplx, 91)
    w, q = np.linalg.eigh(h)
    v = q[:, :k] + 1e-6 * gen.gaussian(g, (n, k), cplx)
    v, _ = np.linalg.qr(v)
    theta = np.real(np.sum(v.conj() * (h @ v), axis=0))
    r = h @ v - v * theta[None, :]
    deg = np.full(k, 10, dtype=np.int32)
    b_sup, mu_1, mu_ne = 1.02, -1.0, float(w[k + 5])
    dt = torch.complex128 if cplx else torch.float64
    h64 = pk.Handle(n, k - 1, 1, dt)
    h8 = pk.Handle(n, k - 1, 1, dt, pk.default_opts(fp64_emulation=14))
    args = (to_gpu(h), to_gpu(v), to_gpu(r), theta, deg, b_sup, mu_1, mu_ne)
    y64, _ = pk.chase_filter_ritz(*args, handle=h64)
    y8, _ = pk.chase_filter_ritz(*args, handle=h8)
    y64, y8 = to_np(y64), to_np(y8)
    assert np.max(np.abs(y8 - y64)) / np.max(np.abs(y64)) < 1e-12


@pytest.mark.parametrize("cplx", [True, False])
def test_solve_with_int8_products_matches_oracle(pk, cplx):
    """The whole solve with every filter product on INT8 (14 moduli): the
    oracle's iterations, eigenvalues and residual bound."""
    announce(f"solve with FP64 products on INT8 cplx={cplx}")
    p = gen.make_uniform(n=1000, nev=100, nex=40, cplx=cplx)
    ev_o, _, _, st_o = oracle.solve(p.H, p.nev, p.nex, p.tol, p.deg, p.V0, p.S)
    ev, V, res, st = pk.chase_solve(to_gpu(p.H), p.nev, p.nex, tol=p.tol, degree=p.deg,
                                    V0=to_gpu(p.V0), S=to_gpu(p.S),
                                    opts=pk.default_opts(fp64_emulation=14))
    assert st["converged"]
    assert abs(st["iterations"] - st_o.iterations) <= 1
    scale = np.max(np.abs(p.lam))
    assert np.max(np.abs(ev - ev_o)) <= 1e-10 * scale
    assert np.max(res) <= p.tol


def test_mixed_solve_with_int8_fp64_tail(pk):
    """Split-BF16 filter whose FP64 steps (tail of the start pass, FP64
    ranks) run on INT8: converges to the planted eigenvalues."""
    announce("mixed split-BF16 solve with the FP64 tail on INT8")
    p = gen.make_geometric(n=3000, nev=150, nex=50)
    ev, V, res, st = pk.chase_solve(to_gpu(p.H), p.nev, p.nex, tol=p.tol, degree=p.deg,
                                    V0=to_gpu(p.V0), S=to_gpu(p.S),
                                    opts=pk.default_opts(filter_prec=pk.PREC_BF16X2,
                                                         fp64_emulation=14))
    assert st["converged"] and st["matvecs_low"] > 0
    scale = np.max(np.abs(p.lam))
    assert np.max(np.abs(ev - p.lam[:p.nev])) <= 2e-10 * scale
    assert np.max(res) <= p.tol


def test_int8_filter_step_at_full_size(pk):
    """n=20000 complex, 64 columns, one degree-2 filter call: INT8 products
    against the FP64 matrix cores on the same input."""
    import torch
    n, k = 20000, 64
    announce(f"INT8 CRT filter at n={n} against the FP64 kernels")
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    a = torch.randn((n, n), dtype=torch.complex128, device="cuda", generator=g)
    H = ((a + a.mH) / (2 * (2 * n) ** 0.5)).contiguous()
    del a
    X = torch.randn((n, k), dtype=torch.complex128, device="cuda", generator=g)
    deg = np.full(k, 2, dtype=np.int32)
    h64 = pk.Handle(n, k - 1, 1, torch.complex128)
    y64, _ = pk.chase_filter(H, X, deg, 1.1, -1.1, -0.7, handle=h64)
    y64 = y64.clone()
    h64.close()
    h8 = pk.Handle(n, k - 1, 1, torch.complex128, pk.default_opts(fp64_emulation=14))
    y8, _ = pk.chase_filter(H, X, deg, 1.1, -1.1, -0.7, handle=h8)
    err = (torch.max(torch.abs(y8 - y64)) / torch.max(torch.abs(y64))).item()
    h8.close()
    assert err < 1e-12, err
