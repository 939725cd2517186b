"""Per-step parity of the HIP path with the CPU oracle (through the C ABI)."""
import math

import numpy as np
import pytest

import gen
import oracle
from gpu_util import announce, rel_err, subspace_sin, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2205_02491_amd as pk
    pk.lib()
    return pk


def _problem(n, cplx, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    lam = gen.spectrum_uniform_iid(n, g)
    q = gen.haar(n, g, cplx)
    return gen.planted(lam, q), lam, q, g


# ------------------------------------------------------------------ filter
@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("n,k", [(300, 37), (700, 150), (1000, 140)])
def test_filter_matches_oracle(pk, cplx, n, k):
    announce(f"filter parity n={n} k={k} cplx={cplx}")
    h, lam, q, g = _problem(n, cplx, 1000 + n + k)
    x = gen.gaussian(g, (n, k), cplx)
    deg = np.sort(2 * g.integers(1, 11, size=k)).astype(np.int32)
    b_sup, mu_1, mu_ne = 1.03, -1.0, -0.55
    y_ref, mv_ref = oracle.chebyshev_filter(h, x, deg, b_sup, mu_1, mu_ne)
    y, mv = pk.chase_filter(to_gpu(h), to_gpu(x), deg, b_sup, mu_1, mu_ne)
    assert mv == mv_ref
    y = to_np(y)
    for a in range(k):
        err = np.max(np.abs(y[:, a] - y_ref[:, a])) / np.max(np.abs(y_ref[:, a]))
        assert err < 1e-12, (a, deg[a], err)


def test_filter_closed_form_diagonal(pk):
    announce("filter closed form on diag(lambda)")
    n, k = 513, 19
    lam = np.sort(np.random.Generator(np.random.PCG64(5)).uniform(-1, 1, n))
    x = np.random.Generator(np.random.PCG64(6)).standard_normal((n, k)) + 0j
    deg = np.full(k, 20, dtype=np.int32)
    b_sup, mu_1, mu_ne = 1.01, -1.0, -0.7
    y, _ = pk.chase_filter(to_gpu(np.diag(lam).astype(complex)), to_gpu(x), deg, b_sup, mu_1, mu_ne)
    p = oracle.cheb_poly_value(lam, 20, b_sup, mu_1, mu_ne)
    ref = p[:, None] * x
    assert rel_err(to_np(y), ref) < 1e-12


def test_filter_fp32_error_bound(pk):
    """Low-precision products: each step's error is bounded by ~ gamma_n of
    FP32 times ||H|| ||X||; over m steps of a bounded recurrence the relative
    error stays at a few 1e-6."""
    announce("filter fp32 error bound")
    n, k = 800, 64
    h, lam, q, g = _problem(n, True, 77)
    x = gen.gaussian(g, (n, k), True)
    deg = np.full(k, 8, dtype=np.int32)
    b_sup, mu_1, mu_ne = 1.02, -1.0, -0.6
    y_ref, _ = oracle.chebyshev_filter(h, x, deg, b_sup, mu_1, mu_ne)
    y, _ = pk.chase_filter(to_gpu(h), to_gpu(x), deg, b_sup, mu_1, mu_ne, prec=pk.PREC_FP32)
    err = rel_err(to_np(y), y_ref)
    assert 1e-9 < err < 5e-5, err


@pytest.mark.parametrize("cplx", [True, False])
def test_filter_ritz_defect_form_matches_oracle(pk, cplx):
    """The defect-correction form computes exactly p(H) v for any vector v and
    shift theta with r = H v - theta v (here: random v, random theta)."""
    announce(f"filter_ritz FP64 parity cplx={cplx}")
    n, k = 650, 70
    h, lam, q, g = _problem(n, cplx, 2200 + cplx)
    v = gen.gaussian(g, (n, k), cplx)
    theta = g.uniform(-1, 1, size=k)
    r = h @ v - v * theta[None, :]
    deg = np.sort(2 * g.integers(1, 12, size=k)).astype(np.int32)
    b_sup, mu_1, mu_ne = 1.04, -1.0, -0.5
    y_ref, mv_ref = oracle.chebyshev_filter(h, v, deg, b_sup, mu_1, mu_ne)
    y, mv = pk.chase_filter_ritz(to_gpu(h), to_gpu(v), to_gpu(r), theta, deg, b_sup, mu_1, mu_ne)
    assert mv == mv_ref - k          # the first step needs no product
    y = to_np(y)
    for a in range(k):
        err = np.max(np.abs(y[:, a] - y_ref[:, a])) / np.max(np.abs(y_ref[:, a]))
        assert err < 1e-11, (a, deg[a], err)


# Rounding model of a product computed from FP32 operands with FP32
# accumulation (three real products per complex product): the error of one
# column, H d, is at most C * u32 * sqrt(n) * ||H||_2 * ||d||_2 (the square-root
# growth of n accumulated roundings of random sign; the operands' own rounding
# adds u32 * ||H||_F / sqrt(n) * ||d||, below that), C = 1.  An error E_s made
# at step s of the recurrence of Eq. (3) enters as alpha_s E_s and is carried
# to the end by the same recurrence started from (x_{s-1}, x_s) = (0, 1), so
# ||P_{s,m}(H)||_2 = max over the spectrum of |x_m(lambda)|.  The plain filter
# multiplies X_{s-1} at steps 1..m; the defect form multiplies
# D_{s-1} = X_{s-1} - T_{s-1}(theta) v at steps 2..m, whose norm is of the order
# of the residual, so its bound (and error) scale with ||r|| instead of ||y||.
FP32_PRODUCT_C = 1.0


def _fp32_filter_bounds(h, lam, v, theta, m, b_sup, mu_1, mu_ne):
    """Per-column bounds of the relative error (2-norm) of the plain and the
    defect-form FP32 filter of degree m, from the model above; oracle FP64
    values for the multiplied blocks."""
    n = h.shape[0]
    k = v.shape[1]
    u32 = 2.0 ** -24
    coef = oracle.filter_coefficients(m, b_sup, mu_1, mu_ne)
    amp = np.zeros(m + 1)
    for s in range(1, m + 1):
        xp, xc = np.zeros_like(lam), np.ones_like(lam)
        for j in range(s + 1, m + 1):
            a, gmm, b = coef[j - 1]
            xp, xc = xc, a * (lam - gmm) * xc + b * xp
        amp[s] = np.max(np.abs(xc))
    y, _ = oracle.chebyshev_filter(h, v, np.full(k, m), b_sup, mu_1, mu_ne)
    ny = np.linalg.norm(y, axis=0)
    hn = float(np.max(np.abs(lam)))
    bp = np.zeros(k)
    bd = np.zeros(k)
    for s in range(1, m + 1):
        if s == 1:
            xs = v
            ts = np.ones(k)
        else:
            xs, _ = oracle.chebyshev_filter(h, v, np.full(k, s - 1), b_sup, mu_1, mu_ne)
            ts = oracle.cheb_poly_value(theta, s - 1, b_sup, mu_1, mu_ne)
        w = abs(coef[s - 1][0]) * amp[s] * FP32_PRODUCT_C * u32 * math.sqrt(n) * hn
        bp += w * np.linalg.norm(xs, axis=0)
        if s >= 2:
            bd += w * np.linalg.norm(xs - v * ts[None, :], axis=0)
    return y, bp / ny, bd / ny


def test_filter_ritz_fp32_error_bound(pk):
    """FP32 products, plain filter vs defect-correction form on Ritz-like
    vectors (residual ~1e-5): each column's error is below the bound of the
    rounding model above, and the defect form's bound and error are orders of
    magnitude below the plain filter's."""
    announce("filter_ritz FP32 error vs the rounding-model bound")
    n, k = 900, 40
    h, lam, q, g = _problem(n, True, 2300)
    v = q[:, :k] + 1e-6 * gen.gaussian(g, (n, k), True)
    v /= np.linalg.norm(v, axis=0)[None, :]
    theta = np.real(np.sum(v.conj() * (h @ v), axis=0))
    r = h @ v - v * theta[None, :]
    m = 20
    deg = np.full(k, m, dtype=np.int32)
    b_sup, mu_1, mu_ne = 1.02, -1.0, lam[60]
    y_ref, bnd_p, bnd_d = _fp32_filter_bounds(h, lam, v, theta, m, b_sup, mu_1, mu_ne)
    y_d, _ = pk.chase_filter_ritz(to_gpu(h), to_gpu(v), to_gpu(r), theta, deg, b_sup, mu_1,
                                  mu_ne, prec=pk.PREC_FP32)
    y_p, _ = pk.chase_filter(to_gpu(h), to_gpu(v), deg, b_sup, mu_1, mu_ne, prec=pk.PREC_FP32)
    ny = np.linalg.norm(y_ref, axis=0)
    e_d = np.linalg.norm(to_np(y_d) - y_ref, axis=0) / ny
    e_p = np.linalg.norm(to_np(y_p) - y_ref, axis=0) / ny
    print(f"[fp32-model] plain: err max {e_p.max():.3e} bound min {bnd_p.min():.3e} "
          f"ratio max {np.max(e_p / bnd_p):.3f} median {np.median(e_p / bnd_p):.3f}; "
          f"defect: err max {e_d.max():.3e} bound max {bnd_d.max():.3e} "
          f"ratio max {np.max(e_d / bnd_d):.3f} median {np.median(e_d / bnd_d):.3f}", flush=True)
    assert np.all(e_p <= bnd_p), np.max(e_p / bnd_p)
    assert np.all(e_d <= bnd_d), np.max(e_d / bnd_d)
    # the two bounds differ only in the multiplied blocks' norms: ||D|| is
    # of the order of the residual (here ~1e-5 of ||X||), times the growth
    assert np.max(bnd_d) < 1e-2 * np.min(bnd_p)
    assert np.max(e_d) < 1e-3 * np.max(e_p), (e_d.max(), e_p.max())


# ------------------------------------------------------------------ split BF16
# Split-BF16 products: hi = bf16(x), lo = bf16(x - hi) carry 16 significant
# bits; a product a*b is formed as hi*hi + hi*lo + lo*hi (dropped lo*lo and
# the split remainders: at most 3 * 2^-16 |ab|, typically ~2^-17) with FP32
# accumulation.  A dot product of random-sign terms then has relative error
# ~1e-5; over a bounded recurrence of m steps it stays below ~1e-4.
# The two-term form (CHASE_PREC_BF16X2) rounds the block to bf16 (2^-9
# relative per value, hi*hi + lo_H*hi): ~3e-3 per filter on these inputs in a
# CPU emulation of the rounding (max 4.4e-3).  Bounds: (max, minimum median).
ERR = {"bf16x3": (1e-4, 3e-7), "bf16x2": (2e-2, 5e-4)}


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x2"])
@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("n,k", [(810, 64), (1000, 300)])
def test_filter_bf16x3_error_bound(pk, cplx, n, k, prec):
    """n not a multiple of 16 (zero-padded K), several 256-row and 128-column
    tiles with ragged tails, per-column degrees (the active block shrinks)."""
    announce(f"filter {prec} n={n} k={k} cplx={cplx}")
    h, lam, q, g = _problem(n, cplx, 3000 + n + k + cplx)
    x = gen.gaussian(g, (n, k), cplx)
    deg = np.sort(2 * g.integers(1, 6, size=k)).astype(np.int32)
    b_sup, mu_1, mu_ne = 1.02, -1.0, -0.6
    y_ref, mv_ref = oracle.chebyshev_filter(h, x, deg, b_sup, mu_1, mu_ne)
    code = pk.PREC_BF16X3 if prec == "bf16x3" else pk.PREC_BF16X2
    y, mv = pk.chase_filter(to_gpu(h), to_gpu(x), deg, b_sup, mu_1, mu_ne, prec=code)
    assert mv == mv_ref
    y = to_np(y)
    err = np.linalg.norm(y - y_ref, axis=0) / np.linalg.norm(y_ref, axis=0)
    assert np.all(err < ERR[prec][0]), (err.max(), int(err.argmax()))
    # really this precision (not a more precise path): typical error ~1e-5
    # with three terms, ~3e-3 with two
    assert np.median(err) > ERR[prec][1], np.median(err)


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x2"])
@pytest.mark.parametrize("cplx", [True, False])
def test_filter_bf16x3_whole_tiles_and_split_tail(pk, cplx, prec):
    """n=4100, k=2100: 17 x 17 tiles of 256 x 128, more than one round of
    workgroups on the device, so a launch runs whole tiles and (when the
    last round is at most half full) a split-K tail whose FP32 partial tiles
    are summed afterwards; the active block shrinks with the degrees, so the
    tile count changes from step to step.  Sampled columns (first and last
    of column tiles, the ragged last tile) against the oracle's filter of
    those columns (the filter acts on each column separately)."""
    n, k = 4100, 2100
    announce(f"filter {prec} whole tiles + split tail n={n} k={k} cplx={cplx}")
    g = np.random.Generator(np.random.PCG64(4100 + cplx))
    a = gen.gaussian(g, (n, n), cplx)
    h = (a + a.conj().T) / (2.0 * np.sqrt(2.0 * n))  # semicircle on about [-1, 1]
    del a
    x = gen.gaussian(g, (n, k), cplx)
    deg = np.sort(2 * g.integers(1, 6, size=k)).astype(np.int32)
    b_sup, mu_1, mu_ne = 1.1, -1.1, -0.7
    code = pk.PREC_BF16X3 if prec == "bf16x3" else pk.PREC_BF16X2
    y, mv = pk.chase_filter(to_gpu(h), to_gpu(x), deg, b_sup, mu_1, mu_ne, prec=code)
    assert mv == int(deg.sum())
    cols = np.array([0, 1, 127, 128, 1000, 1791, 2047, 2048, 2099])
    y_ref, _ = oracle.chebyshev_filter(h, x[:, cols], deg[cols], b_sup, mu_1, mu_ne)
    y = to_np(y)[:, cols]
    err = np.linalg.norm(y - y_ref, axis=0) / np.linalg.norm(y_ref, axis=0)
    assert np.all(err < ERR[prec][0]), (err.max(), int(cols[err.argmax()]))
    assert np.median(err) > ERR[prec][1], np.median(err)


def _bf16(x):
    """Round to bf16 as the kernels do: to float32 first, then to nearest
    even on the upper 16 bits (finite values)."""
    u = np.asarray(x, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _split(x):
    """hi = bf16(x), lo = bf16(x - hi), componentwise for complex x."""
    if np.iscomplexobj(x):
        (hr, lr), (hi_, li) = _split(x.real), _split(x.imag)
        return hr + 1j * hi_, lr + 1j * li
    hi = _bf16(x)
    return hi, _bf16(x - hi)


def _dyadic(g, shape, cplx):
    """Entries i + f 2^-9 with i in {-2,-1,1,2} and f in {-1,0,1}: the split
    is exact (hi = i, lo = f 2^-9), and sums of products of such numbers stay
    multiples of 2^-9 (2^-18 for lo*lo, which no kernel forms)."""
    def part():
        return g.choice([-2.0, -1.0, 1.0, 2.0], size=shape) + g.integers(-1, 2, size=shape) * 2.0 ** -9
    return part() + 1j * part() if cplx else part()


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x2"])
@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("n,k", [(810, 64), (4100, 2100)])
def test_filter_split_bf16_matches_rounding_emulation(pk, cplx, n, k, prec):
    """The split-BF16 kernels against an FP64 emulation of their own operand
    rounding, on inputs that make the first step's sums exact in FP32
    arithmetic: H and X_0 with entries i + f 2^-9 (exact splits; every partial
    sum a multiple of 2^-9 far below 2^15), shift gamma = 0 and alpha_1 =
    -2^-9 (c = 0, e = 400, mu_1 = -512).  Step 2 multiplies the split of X_1
    (rounded to 16 bits, or to bf16 with two terms, the same way on both
    sides) and is the last one (degree 2), so what is left is the FP32
    accumulation of the products (measured 3.6e-7 at most, n=4100 complex),
    against 1e-6 (three terms, n=4100) to 7e-4 (two terms) for the operands'
    own rounding; a dropped or misplaced plane, 8-row group, K chunk or tile
    costs 1e-4 or more.  n=810 pads K; n=4100, k=2100 runs whole tiles and
    the split-K tail."""
    announce(f"filter {prec} vs rounding emulation n={n} k={k} cplx={cplx}")
    g = np.random.Generator(np.random.PCG64(7700 + n + cplx))
    a = np.triu(_dyadic(g, (n, n), cplx))
    h = a + np.triu(a, 1).conj().T
    if cplx:
        h[np.diag_indices(n)] = h.diagonal().real
    del a
    x = _dyadic(g, (n, k), cplx)
    deg = np.full(k, 2, dtype=np.int32)
    b_sup, mu_1, mu_ne = 400.0, -512.0, -400.0
    (a1, c1, b1), (a2, c2, b2) = oracle.filter_coefficients(2, b_sup, mu_1, mu_ne)
    assert a1 == -2.0 ** -9 and c1 == 0.0 and c2 == 0.0 and b1 == 0.0
    code = pk.PREC_BF16X3 if prec == "bf16x3" else pk.PREC_BF16X2
    y, mv = pk.chase_filter(to_gpu(h), to_gpu(x), deg, b_sup, mu_1, mu_ne, prec=code)
    assert mv == 2 * k
    cols = np.unique(np.concatenate([np.arange(0, k, max(1, k // 40)), [k - 1]]))
    h_hi, h_lo = _split(h)
    assert np.array_equal(h_hi + h_lo, h)

    def product(xs):
        x_hi, x_lo = _split(xs)
        p = h_hi @ x_hi + h_lo @ x_hi
        return p + h_hi @ x_lo if prec == "bf16x3" else p

    xc = x[:, cols]
    x1 = a1 * product(xc)
    y_emu = a2 * product(x1) + b2 * xc
    y_ref, _ = oracle.chebyshev_filter(h, xc, deg[cols], b_sup, mu_1, mu_ne)
    y = to_np(y)[:, cols]
    nrm = np.linalg.norm(y_ref, axis=0)
    e_emu = np.linalg.norm(y - y_emu, axis=0) / nrm
    e_ref = np.linalg.norm(y - y_ref, axis=0) / nrm
    announce(f"  max error vs emulation {e_emu.max():.2e}, vs FP64 {e_ref.max():.2e}")
    assert np.all(e_emu < 2e-6), (e_emu.max(), int(cols[e_emu.argmax()]))
    assert np.median(e_emu) < 0.5 * np.median(e_ref)

@pytest.mark.parametrize("n,k", [(17, 1), (256, 128), (257, 129), (300, 2)])
def test_filter_bf16x3_edge_shapes(pk, n, k):
    """Split-BF16 filter at edge shapes: a single column, exact tile
    multiples, one past them (ragged tails in rows, columns and K), and
    degrees that drop all but the last column after the first steps (the
    next-step split then covers one column)."""
    announce(f"filter bf16x3 edge n={n} k={k}")
    h, lam, q, g = _problem(n, True, 5100 + n + k)
    x = gen.gaussian(g, (n, k), True)
    deg = np.full(k, 2, dtype=np.int32)
    deg[-1] = 8
    b_sup, mu_1, mu_ne = 1.02, -1.0, -0.6
    y_ref, mv_ref = oracle.chebyshev_filter(h, x, deg, b_sup, mu_1, mu_ne)
    y, mv = pk.chase_filter(to_gpu(h), to_gpu(x), deg, b_sup, mu_1, mu_ne, prec=pk.PREC_BF16X3)
    assert mv == mv_ref
    err = np.linalg.norm(to_np(y) - y_ref, axis=0) / np.linalg.norm(y_ref, axis=0)
    assert np.all(err < 1e-4), (err.max(), int(err.argmax()))


def test_filter_bf16x3_closed_form_diagonal(pk):
    """H = diag(lambda): p(H) x = p(lambda) * x column by column."""
    announce("filter bf16x3 closed form on diag(lambda)")
    n, k = 530, 150
    lam = np.sort(np.random.Generator(np.random.PCG64(15)).uniform(-1, 1, n))
    x = np.random.Generator(np.random.PCG64(16)).standard_normal((n, k)) + 0j
    deg = np.full(k, 12, dtype=np.int32)
    b_sup, mu_1, mu_ne = 1.01, -1.0, -0.7
    y, _ = pk.chase_filter(to_gpu(np.diag(lam).astype(complex)), to_gpu(x), deg, b_sup, mu_1,
                           mu_ne, prec=pk.PREC_BF16X3)
    p = oracle.cheb_poly_value(lam, 12, b_sup, mu_1, mu_ne)
    ref = p[:, None] * x
    err = np.linalg.norm(to_np(y) - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert np.all(err < 1e-4), err.max()


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x2"])
def test_filter_ritz_bf16x3_error_scales_with_residual(pk, prec):
    """Defect-correction form with split-BF16 products: error relative to the
    residual (1e-6 here), so far below the plain split-BF16 filter's."""
    announce(f"filter_ritz {prec} vs plain {prec}")
    code = pk.PREC_BF16X3 if prec == "bf16x3" else pk.PREC_BF16X2
    n, k = 900, 40
    h, lam, q, g = _problem(n, True, 2300)
    v = q[:, :k] + 1e-6 * gen.gaussian(g, (n, k), True)
    v /= np.linalg.norm(v, axis=0)[None, :]
    theta = np.real(np.sum(v.conj() * (h @ v), axis=0))
    r = h @ v - v * theta[None, :]
    deg = np.full(k, 20, dtype=np.int32)
    b_sup, mu_1, mu_ne = 1.02, -1.0, lam[60]
    y_ref, _ = oracle.chebyshev_filter(h, v, deg, b_sup, mu_1, mu_ne)
    y_d, _ = pk.chase_filter_ritz(to_gpu(h), to_gpu(v), to_gpu(r), theta, deg, b_sup, mu_1,
                                  mu_ne, prec=code)
    y_p, _ = pk.chase_filter(to_gpu(h), to_gpu(v), deg, b_sup, mu_1, mu_ne, prec=code)
    e_d = rel_err(to_np(y_d), y_ref)
    e_p = rel_err(to_np(y_p), y_ref)
    assert e_p > (1e-7 if prec == "bf16x3" else 1e-5)
    assert e_d < (1e-8 if prec == "bf16x3" else 1e-6) and e_d < 1e-3 * e_p, (e_d, e_p)


def test_bf16x3_needs_split_handle(pk):
    """A handle created for FP64 filtering holds no split of H (either
    split-BF16 form is refused); a handle made for one split-BF16 form runs
    the other (same buffers)."""
    n = 300
    h, lam, q, g = _problem(n, True, 17)
    x = gen.gaussian(g, (n, 8), True)
    deg = np.full(8, 4, np.int32)
    handle = pk.Handle(n, 6, 2)
    for prec in (pk.PREC_BF16X3, pk.PREC_BF16X2):
        with pytest.raises(pk.ChaseError, match="split-BF16"):
            pk.chase_filter(to_gpu(h), to_gpu(x), deg, 1.02, -1.0, -0.6, prec=prec, handle=handle)
    h3 = pk.Handle(n, 6, 2, filter_prec=pk.PREC_BF16X3)
    y, mv = pk.chase_filter(to_gpu(h), to_gpu(x), deg, 1.02, -1.0, -0.6, prec=pk.PREC_BF16X2,
                            handle=h3)
    y_ref, _ = oracle.chebyshev_filter(h, x, deg, 1.02, -1.0, -0.6)
    err = np.linalg.norm(to_np(y) - y_ref, axis=0) / np.linalg.norm(y_ref, axis=0)
    assert mv == 32 and np.all(err < ERR["bf16x2"][0])


# ------------------------------------------------------------------ Lanczos
@pytest.mark.parametrize("cplx,nvec", [(True, 4), (False, 4), (True, 1)])
def test_lanczos_matches_oracle(pk, cplx, nvec):
    announce(f"lanczos parity cplx={cplx} nvec={nvec}")
    n = 900
    h, lam, q, g = _problem(n, cplx, 31 + cplx)
    s = gen.gaussian(g, (n, nvec), cplx)
    runs = oracle.lanczos_runs(h, s, 25)
    b_ref, m1_ref, mne_ref, _ = oracle.spectral_bounds(h, s, 25, 120)
    handle = pk.Handle(n, 80, 40, to_gpu(h).dtype)
    b_sup, mu_1, mu_ne, a, b, lens = pk.chase_lanczos(to_gpu(h), to_gpu(s), 25, handle=handle)
    for r, (ar, br) in enumerate(runs):
        assert lens[r] == len(ar)
        np.testing.assert_allclose(a[r, : len(ar)], ar, atol=1e-11)
        np.testing.assert_allclose(b[r, : len(br)], br, atol=1e-11)
    assert abs(b_sup - b_ref) < 1e-11 and abs(mu_1 - m1_ref) < 1e-11
    assert abs(mu_ne - mne_ref) < 1e-9
    assert b_sup >= lam[-1] - 1e-12 and mu_1 >= lam[0] - 1e-12


# ------------------------------------------------------------------ QR
@pytest.mark.parametrize("n,k,locked,cplx", [(1100, 150, 0, True), (1100, 150, 7, True),
                                             (1500, 400, 130, True), (1500, 400, 130, False)])
def test_qr_invariants_and_span(pk, n, k, locked, cplx):
    """k spans several 128-wide tiles: the Gram matrix is computed as the
    tiles on and above the diagonal and mirrored, and X R^-1 stops at the
    triangular factor's diagonal, offset by the locked columns (here also
    more than a tile)."""
    announce(f"qr n={n} k={k} locked={locked} cplx={cplx}")
    g = np.random.Generator(np.random.PCG64(41 + k + cplx))
    dt = complex if cplx else float
    y = gen.haar(n, g, cplx)[:, :locked] if locked else np.zeros((n, 0), dt)
    base = gen.gaussian(g, (n, k - locked), cplx)
    # columns with widely different scales and a near-dependency
    v = base * np.logspace(0, 6, k - locked)[None, :]
    v[:, 1] = v[:, 0] * 1e-3 + 1e-9 * base[:, 1]
    x = np.concatenate([y, v], axis=1)
    qd = to_np(pk.chase_qr(to_gpu(x), locked))
    assert np.array_equal(qd[:, :locked], y)
    assert np.linalg.norm(qd.conj().T @ qd - np.eye(k)) < 1e-12 * math.sqrt(k)
    q_ref = oracle.qr_locked(y, v)
    # same span: projector difference
    pdiff = qd @ qd.conj().T - q_ref @ q_ref.conj().T
    assert np.linalg.norm(pdiff, 2) < 1e-8


@pytest.mark.parametrize("cplx,locked", [(True, 0), (True, 9), (False, 9)])
def test_qr_householder_fallback_on_rank_deficient_block(pk, cplx, locked):
    """The last resort of the QR step: a non-locked column that is exactly
    zero (an exact linear combination of the others, with all coefficients
    0) gives the Gram matrix a zero diagonal entry, which no Cholesky pass,
    clean or shifted, can factor; the step then runs Householder QR (the
    paper's geqrf) and copies the locked columns back.  The result is
    orthonormal, keeps the locked columns bit for bit, contains span(X), and
    spans the same space as the oracle's Householder QR over the columns
    before the zero one (after it, a rank-deficient QR may complete the basis
    with any orthonormal direction)."""
    announce(f"qr Householder fallback cplx={cplx} locked={locked}")
    n, k = 700, 60
    g = np.random.Generator(np.random.PCG64(4242 + locked + cplx))
    dt = complex if cplx else float
    y = gen.haar(n, g, cplx)[:, :locked] if locked else np.zeros((n, 0), dt)
    v = gen.gaussian(g, (n, k - locked), cplx)
    jz = 23
    v[:, jz] = 0.0
    x = np.concatenate([y, v], axis=1)
    qt, qs = pk.chase_qr(to_gpu(x), locked, return_stats=True)
    qd = to_np(qt)
    assert qs["householder"] == 1, qs
    assert np.array_equal(qd[:, :locked], y)
    assert np.linalg.norm(qd.conj().T @ qd - np.eye(k)) < 1e-12 * math.sqrt(k)
    assert np.linalg.norm(x - qd @ (qd.conj().T @ x)) < 1e-12 * np.linalg.norm(x)
    q_ref = oracle.qr_locked(y, v)
    m = locked + jz
    pdiff = qd[:, :m] @ qd[:, :m].conj().T - q_ref[:, :m] @ q_ref[:, :m].conj().T
    assert np.linalg.norm(pdiff, 2) < 1e-12


def test_qr_exactly_duplicated_columns(pk):
    """Two exactly equal columns: rank deficient in exact arithmetic.  The QR
    step (shifted Cholesky passes, or Householder if those do not lead to
    clean ones) must still return an orthonormal basis that contains
    span(X) and agrees with the oracle up to the duplicated column."""
    announce("qr with exactly duplicated columns")
    n, k = 700, 60
    g = np.random.Generator(np.random.PCG64(4343))
    x = gen.gaussian(g, (n, k), True)
    x[:, 31] = x[:, 12]
    qt, qs = pk.chase_qr(to_gpu(x), 0, return_stats=True)
    qd = to_np(qt)
    announce(f"  shifted passes {qs['shifted_passes']}, householder {qs['householder']}")
    assert qs["shifted_passes"] > 0 or qs["householder"] == 1
    assert np.linalg.norm(qd.conj().T @ qd - np.eye(k)) < 1e-12 * math.sqrt(k)
    assert np.linalg.norm(x - qd @ (qd.conj().T @ x)) < 1e-10 * np.linalg.norm(x)
    q_ref = oracle.qr_locked(np.zeros((n, 0), complex), x)
    pdiff = qd[:, :31] @ qd[:, :31].conj().T - q_ref[:, :31] @ q_ref[:, :31].conj().T
    assert np.linalg.norm(pdiff, 2) < 1e-10


def test_single_vector_entry_points(pk):
    """One complex vector through QR, Rayleigh-Ritz and the eigenvalue
    adjoint: a single column is the case where a torch view of the caller's
    memory could reach the library unconjugated."""
    announce("single-vector QR / Rayleigh-Ritz / eigenvalue adjoint")
    import torch
    n = 200
    h, lam, q, g = _problem(n, True, 61)
    x = gen.gaussian(g, (n, 1), True)
    x_keep = x.copy()
    xt = to_gpu(x)
    qd = to_np(pk.chase_qr(xt))
    assert np.array_equal(to_np(xt), x_keep)          # the input is not modified
    ref = x / np.linalg.norm(x)
    ph = np.vdot(ref[:, 0], qd[:, 0])                 # same vector up to a phase
    assert abs(abs(ph) - 1.0) < 1e-12
    th, v, res = pk.chase_rayleigh_ritz(to_gpu(h), to_gpu(ref), 1.0)
    theta = float(np.real(np.vdot(ref[:, 0], h @ ref[:, 0])))
    assert abs(th[0] - theta) < 1e-13
    r = np.linalg.norm(h @ ref[:, 0] - theta * ref[:, 0])
    assert abs(res[0] - r) < 1e-12 * max(1.0, r)
    dH = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    pk.chase_eigval_adjoint(to_gpu(q[:, :1]), np.array([0.5]), dH)
    np.testing.assert_allclose(to_np(dH), 0.5 * np.outer(q[:, 0], q[:, 0].conj()), atol=1e-14)


# ------------------------------------------------------------------ RR + residual
@pytest.mark.parametrize("cplx,k", [(True, 140), (False, 140), (True, 300)])
def test_rayleigh_ritz_matches_oracle(pk, cplx, k):
    announce(f"rayleigh-ritz cplx={cplx} k={k}")
    n = 1000
    h, lam, q, g = _problem(n, cplx, 51 + cplx + k)
    qa, _ = np.linalg.qr(gen.gaussian(g, (n, k), cplx) + q[:, :k] * 5)
    th_ref, va_ref = oracle.rayleigh_ritz(h, qa)
    r_ref = oracle.residual_norms(h, va_ref, th_ref, 1.3)
    th, va, res = pk.chase_rayleigh_ritz(to_gpu(h), to_gpu(qa), 1.3)
    np.testing.assert_allclose(th, th_ref, atol=1e-13)
    np.testing.assert_allclose(res, r_ref, rtol=1e-8, atol=1e-14)
    va = to_np(va)
    # Ritz vectors agree up to a phase per (simple) column
    ov = np.abs(np.sum(va.conj() * va_ref, axis=0))
    gaps = np.minimum(np.diff(th_ref, prepend=-np.inf), np.diff(th_ref, append=np.inf))
    ok = gaps > 1e-6
    np.testing.assert_allclose(ov[ok], 1.0, atol=1e-8)
