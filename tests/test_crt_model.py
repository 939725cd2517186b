"""CPU pins of the arithmetic behind the FP64 products on INT8 (chase_opts.
fp64_emulation): a plain model written from the definitions (Chinese
remainder theorem, Garner's mixed-radix form, Gauss's three-product complex
form), checked against exact Python integers.  It shares no code with the
library; it pins the choices the library documents: the moduli are pairwise
coprime and fit int8 as balanced residues, the bit budget
pa + pb = floor(log2 M - 3 - log2 K) keeps every complex product part below
M / 2, and the reconstruction is exact there."""
import math
import random

import numpy as np
import pytest

MODULI = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191]


def budget(nm, K, cplx=True):
    log2m = sum(math.log2(m) for m in MODULI[:nm])
    total = math.floor(log2m - 2 - math.log2(K) - (1 if cplx else 0))
    pa = min(52, total // 2)
    return pa, min(52, total - pa)


def balanced(x, m):
    r = x % m
    return r - m if r > (m - 1) // 2 else r


def garner(residues, nm):
    """Balanced mixed-radix digits of the x with x = r_t (mod m_t), |x| < M/2."""
    digits = []
    for t in range(nm):
        m = MODULI[t]
        prod = 1
        for s in range(t):
            prod = prod * MODULI[s] % m
        partial = 0
        for s in range(t - 1, -1, -1):
            partial = partial * MODULI[s] + digits[s]
        d = (residues[t] - partial) * pow(prod, -1, m) % m
        digits.append(d - m if d > (m - 1) // 2 else d)
    return digits


def from_digits(digits, nm):
    x = 0
    for t in range(nm - 1, -1, -1):
        x = x * MODULI[t] + digits[t]
    return x


def test_moduli_pairwise_coprime_and_int8():
    for i, a in enumerate(MODULI):
        assert a <= 256
        for b in MODULI[i + 1:]:
            assert math.gcd(a, b) == 1
        # balanced residues lie in int8
        rs = [balanced(x, a) for x in range(-3 * a, 3 * a)]
        assert min(rs) >= -128 and max(rs) <= 127


@pytest.mark.parametrize("nm", [8, 12, 14, 16])
def test_garner_reconstructs_every_integer_below_half_the_product(nm):
    M = math.prod(MODULI[:nm])
    rng = random.Random(nm)
    for x in [0, 1, -1, M // 2 - 1, -(M // 2) + 1] + [rng.randrange(-(M // 2) + 1, M // 2)
                                                    for _ in range(200)]:
        digits = garner([x % m for m in MODULI[:nm]], nm)
        assert from_digits(digits, nm) == x
        # the digits are balanced (what the library evaluates in FP64)
        assert all(-(m // 2) <= d <= (m - 1) // 2 for d, m in zip(digits, MODULI[:nm]))


@pytest.mark.parametrize("nm,K", [(14, 20000), (14, 30000), (16, 65535), (12, 1000)])
def test_bit_budget_keeps_complex_products_exact(nm, K):
    """Worst case of the budget: every entry at its bound, all products of one
    sign.  Re = P1 - P2 and Im = P3 - P1 - P2 (combined in residue space)
    stay below M / 2, so Garner returns them exactly."""
    pa, pb = budget(nm, K)
    M = math.prod(MODULI[:nm])
    a, b = 2 ** pa, 2 ** pb
    re_max = K * (a * b + a * b)          # |sum a_re b_re - a_im b_im|
    im_max = K * (a * b + a * b)          # |sum a_re b_im + a_im b_re|
    assert max(re_max, im_max) < M // 2
    # the worst case through the residue form: Gauss P3 - P1 - P2 with P3 at
    # its own bound (2a)(2b) K, still reconstructed exactly
    p1, p2 = K * a * b, -K * a * b
    p3 = K * (2 * a) * (2 * b) - K * a * b
    im = p3 - p1 - p2
    res = [((p3 % m) - (p1 % m) - (p2 % m)) % m for m in MODULI[:nm]]
    assert from_digits(garner(res, nm), nm) == im


def test_complex_product_model_matches_exact_integers():
    """A small complex product through the whole scheme (scaling, integer
    forms, residues, three real products per modulus, Garner, Horner in
    FP64, unscaling) against the exact product of the integer forms and
    against numpy's FP64 product."""
    nm, n, k = 14, 64, 5
    rng = np.random.default_rng(3)
    H = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = (H + H.conj().T) / 2
    H[:4] *= 1e-5
    H[:, :4] *= 1e-5
    X = (rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))) * np.exp(
        rng.uniform(-6, 6, k))[None, :]
    pa, pb = budget(nm, n)
    rowmax = np.maximum(np.abs(H.real), np.abs(H.imag)).max(axis=1)
    colmax = np.maximum(np.abs(X.real), np.abs(X.imag)).max(axis=0)
    sig = pa - np.frexp(rowmax)[1]
    tau = pb - np.frexp(colmax)[1]
    ar = [[int(v) for v in row] for row in np.rint(np.ldexp(H.real, sig[:, None]))]
    ai = [[int(v) for v in row] for row in np.rint(np.ldexp(H.imag, sig[:, None]))]
    br = [[int(v) for v in row] for row in np.rint(np.ldexp(X.real, tau[None, :]))]
    bi = [[int(v) for v in row] for row in np.rint(np.ldexp(X.imag, tau[None, :]))]
    for i in (0, 3, 17, n - 1):
        for j in range(k):
            exact_re = sum(ar[i][l] * br[l][j] - ai[i][l] * bi[l][j] for l in range(n))
            exact_im = sum(ar[i][l] * bi[l][j] + ai[i][l] * br[l][j] for l in range(n))
            rr, ri = [], []
            for m in MODULI[:nm]:
                p1 = sum(balanced(ar[i][l], m) * balanced(br[l][j], m) for l in range(n)) % m
                p2 = sum(balanced(ai[i][l], m) * balanced(bi[l][j], m) for l in range(n)) % m
                p3 = sum(balanced(ar[i][l] + ai[i][l], m) * balanced(br[l][j] + bi[l][j], m)
                         for l in range(n)) % m
                rr.append((p1 - p2) % m)
                ri.append((p3 - p1 - p2) % m)
            dr, di = garner(rr, nm), garner(ri, nm)
            assert from_digits(dr, nm) == exact_re and from_digits(di, nm) == exact_im
            # Horner in FP64 from the top digit: within a few ulps of the integer
            vr = 0.0
            for t in range(nm - 1, -1, -1):
                vr = vr * MODULI[t] + dr[t]
            assert abs(vr - exact_re) <= 4 * nm * 2.0 ** -53 * abs(exact_re) + 1
            c = math.ldexp(vr, -int(sig[i] + tau[j]))
            ref = (H[i] @ X[:, j]).real
            scale = rowmax[i] * np.abs(X[:, j]).sum()
            # only the rounding of the integer forms remains (2^-pa, 2^-pb)
            assert abs(c - ref) <= 4 * (2.0 ** -pa + 2.0 ** -pb) * scale
