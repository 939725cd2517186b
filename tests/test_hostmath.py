"""The library's host-side logic of Algorithm 1 (Lanczos bounds and density
of states, Chebyshev coefficients, degree formula), compiled host-only with
g++, against the CPU oracle on the same inputs."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import gen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = tmp_path_factory.mktemp("shim") / "hostmath_shim.so"
    src = [os.path.join(ROOT, "tests", "hostmath_shim.cpp"),
           os.path.join(ROOT, "paper_2205_02491_amd", "csrc", "hostmath.cpp")]
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", str(out), *src],
                   check=True)
    lib = ctypes.CDLL(str(out))
    pd = ctypes.POINTER(ctypes.c_double)
    lib.shim_bounds.argtypes = [pd, pd, ctypes.c_int, ctypes.c_int, ctypes.c_long, ctypes.c_int,
                                pd, ctypes.POINTER(ctypes.c_int)]
    lib.shim_coefs.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, pd]
    lib.shim_degree.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int] * 4
    lib.shim_degree.restype = ctypes.c_int
    lib.shim_tail.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int]
    lib.shim_tail.restype = ctypes.c_int
    lib.shim_floor.argtypes = [ctypes.c_int, ctypes.c_long]
    lib.shim_floor.restype = ctypes.c_double
    return lib


def _pd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@pytest.mark.parametrize("kind", ["uniform", "geometric", "cluster", "breakdown"])
def test_lanczos_bounds_match_oracle(shim, kind):
    n, steps, nv, ne = 400, 25, 4, 60
    g = np.random.Generator(np.random.PCG64(hash(kind) % 1000))
    if kind == "geometric":
        lam = gen.spectrum_geometric_low(n, g, 50)
    elif kind == "cluster":
        lam = gen.spectrum_121_cluster(n, g, 60)
    elif kind == "breakdown":
        lam = np.repeat(np.linspace(-1, 1, 10), n // 10)   # 10 distinct values
    else:
        lam = gen.spectrum_uniform_iid(n, g)
    h = gen.planted(lam, gen.haar(n, g, True))
    s = gen.gaussian(g, (n, nv), True)
    runs = oracle.lanczos_runs(h, s, steps)
    b_ref, m1_ref, mne_ref, _ = oracle.spectral_bounds(h, s, steps, ne)
    a = np.zeros((steps, nv))
    b = np.zeros((steps, nv))
    for r, (ar, br) in enumerate(runs):
        a[: len(ar), r] = ar
        b[: len(br), r] = br       # entries past an early stop stay 0
    out = np.zeros(4)
    lens = (ctypes.c_int * nv)()
    shim.shim_bounds(_pd(np.ascontiguousarray(a)), _pd(np.ascontiguousarray(b)), nv, steps, n, ne,
                     _pd(out), lens)
    assert list(lens) == [len(ar) for ar, _ in runs]
    np.testing.assert_allclose(out, [b_ref, m1_ref, mne_ref, oracle.lanczos_norm(runs)], rtol=0,
                               atol=1e-13)


def test_chebyshev_coefficients_match_oracle(shim):
    for (b_sup, mu_1, mu_ne, m) in [(1.5, -1.0, -0.7, 36), (10.0, 1e-8, 0.044, 20), (2.0, -3.0, 1.9, 8)]:
        out = np.zeros(3 * m)
        shim.shim_coefs(m, b_sup, mu_1, mu_ne, _pd(out))
        ref = np.array(oracle.filter_coefficients(m, b_sup, mu_1, mu_ne)).ravel()
        np.testing.assert_allclose(out, ref, rtol=1e-15, atol=0)


def test_degree_formula_matches_oracle(shim):
    g = np.random.Generator(np.random.PCG64(5))
    opts = oracle.Options()
    for _ in range(2000):
        c, e = g.uniform(-1, 1), g.uniform(0.1, 2)
        ritz = g.uniform(c - 4 * e, c + 1.5 * e)
        res = 10 ** g.uniform(-11, 0)
        ref = int(oracle.degrees([res], [ritz], c, e, 1e-10, opts, 20)[0])
        got = shim.shim_degree(res, ritz, c, e, 1e-10, opts.max_deg, opts.deg_extra, 1, 20)
        assert got == ref, (res, ritz, c, e, got, ref)
    assert shim.shim_degree(1e-3, -5.0, 0.0, 1.0, 1e-10, 36, 2, 0, 17) == 18


def test_host_logic_under_sanitizers(tmp_path):
    """The same host code built as a standalone program with AddressSanitizer
    and UBSan (host only), driven through edge cases: one-step runs,
    immediate breakdown, degenerate intervals, huge and tiny residuals."""
    drv = tmp_path / "drv.cpp"
    drv.write_text(r"""
#include <cmath>
#include <cstdio>
#include <vector>
#include "hostmath.h"
int main() {
  chase_opts o{}; o.max_deg = 36; o.deg_extra = 2; o.optimize_degree = 1;
  for (int steps : {1, 2, 25}) {
    std::vector<double> a(steps * 3, 0.5), b(steps * 3, 1e-20);
    chase::Bounds bd = chase::lanczos_bounds(a, b, 3, steps, 100, 10, nullptr);
    if (!std::isfinite(bd.b_sup) || !std::isfinite(bd.mu_ne)) return 1;
  }
  for (double r : {1e-300, 1e-10, 1.0, 1e300})
    for (double t : {-1e6, -1.0000001, -1.0, 0.0, 0.999})
      if (chase::optimal_degree(r, t, 0.0, 1.0, 1e-10, o, 20) % 2) return 2;
  auto c = chase::cheb_coefficients(1, 1.0, -1.0, 0.0);
  if (c.size() != 1) return 3;
  std::puts("ok");
  return 0;
}
""")
    exe = tmp_path / "drv"
    csrc = os.path.join(ROOT, "paper_2205_02491_amd", "csrc")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", csrc, str(drv),
                    os.path.join(csrc, "hostmath.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr


def test_fp64_tail_rule(shim):
    """Automatic FP64 tail of a low-precision start pass: the fewest final
    steps j with floor / rho^j <= tol, rho the Chebyshev growth rate at the
    nev-th eigenvalue estimate (found here by counting steps, not by the
    library's logarithm formula); 0 when j would reach the degree, when the
    estimate is not below the damped interval [c - e, c + e], or when the
    floor is already below tol."""
    g = np.random.Generator(np.random.PCG64(8))
    for _ in range(3000):
        c, e = g.uniform(-1, 1), g.uniform(0.05, 2)
        lam = c - e * (1 + 10 ** g.uniform(-4, 1))
        floor, tol, deg = 2.0 ** -int(g.integers(6, 20)), 10.0 ** g.uniform(-12, -8), 20
        t = (lam - c) / e
        rho = abs(t) + np.sqrt(t * t - 1)
        j = 1
        while floor / rho ** j > tol * (1 + 1e-12) and j < 10 ** 6:
            j += 1
        want = j if j < deg else 0
        got = shim.shim_tail(floor, lam, c, e, tol, deg)
        assert got == want or abs(np.log(floor / tol) / np.log(rho) - round(np.log(floor / tol) / np.log(rho))) < 1e-9, \
            (floor, lam, c, e, tol, got, want)
    # off: estimate inside the damped interval, floor below tol, no interval
    assert shim.shim_tail(2.0 ** -14, 0.0, 0.0, 1.0, 1e-10, 20) == 0
    assert shim.shim_tail(1e-12, -5.0, 0.0, 1.0, 1e-10, 20) == 0
    assert shim.shim_tail(2.0 ** -14, -5.0, 0.0, 0.0, 1e-10, 20) == 0
    # the oracle's Lanczos estimates on gen.make_geometric(n=3000, nev=150,
    # nex=45, n_geo=180, cfg=41), the problem on which the floors were
    # calibrated (b_sup 1.51457, mu_ne 0.0074903, density-of-states estimate
    # of lambda_150 -0.857573; rho = 4.049): 10 steps for split BF16, 9 for
    # FP32, none once the degree is too small for that
    b_sup, mu_ne, lam_nev = 1.51457, 0.0074903, -0.857573
    c, e = (b_sup + mu_ne) / 2, (b_sup - mu_ne) / 2
    assert shim.shim_tail(2.0 ** -14, lam_nev, c, e, 1e-10, 20) == 10
    assert shim.shim_tail(2.0 ** -17, lam_nev, c, e, 1e-10, 20) == 9
    assert shim.shim_tail(2.0 ** -14, lam_nev, c, e, 1e-10, 10) == 0


def test_low_precision_floor(shim):
    """Rounding floor of a plain low-precision pass: split BF16 2^-14 at every
    n (the operands' 16-bit representation); FP32 2^-17 up to n=3000, the
    calibration size, then growing like sqrt(n) (n-term accumulation)."""
    for n in (1, 400, 3000, 20000, 100000):
        assert shim.shim_floor(1, n) == 2.0 ** -14
    for n in (1, 1000, 3000):
        assert shim.shim_floor(0, n) == 2.0 ** -17
    assert shim.shim_floor(0, 12000) == 2.0 ** -16
    np.testing.assert_allclose(shim.shim_floor(0, 20000), 2.0 ** -17 * np.sqrt(20000 / 3000),
                               rtol=1e-15)
    # with the calibration problem's estimates (see test_fp64_tail_rule):
    # the tail counted step by step, 9 at the calibration size and one or
    # two steps more at n=100000 (floor 5.8x higher, rho = 4.05)
    b_sup, mu_ne, lam_nev = 1.51457, 0.0074903, -0.857573
    c, e = (b_sup + mu_ne) / 2, (b_sup - mu_ne) / 2
    t = (lam_nev - c) / e
    rho = abs(t) + np.sqrt(t * t - 1)
    counted = {}
    for n in (3000, 20000, 100000):
        f = shim.shim_floor(0, n)
        j = 1
        while f / rho ** j > 1e-10:
            j += 1
        counted[n] = j
        assert shim.shim_tail(f, lam_nev, c, e, 1e-10, 20) == j
    assert counted[3000] == 9 and counted[100000] in (10, 11)
