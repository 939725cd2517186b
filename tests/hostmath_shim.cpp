// Test-only C wrappers around the library's host-side scalar logic
// (paper_2205_02491_amd/csrc/hostmath.cpp), built with g++ by the CPU tests.
#include <vector>

#include "../paper_2205_02491_amd/csrc/hostmath.h"

extern "C" {

void shim_bounds(const double* alpha, const double* beta, int nv, int steps, long n, int ne,
                 double* out3, int* lens) {
  std::vector<double> a(alpha, alpha + (size_t)nv * steps), b(beta, beta + (size_t)nv * steps);
  std::vector<int> l;
  chase::Bounds bd = chase::lanczos_bounds(a, b, nv, steps, n, ne, &l);
  out3[0] = bd.b_sup;
  out3[1] = bd.mu_1;
  out3[2] = bd.mu_ne;
  out3[3] = bd.norm_lower;
  for (int r = 0; r < nv; ++r) lens[r] = l[r];
}

void shim_coefs(int m, double b_sup, double mu_1, double mu_ne, double* out) {
  auto c = chase::cheb_coefficients(m, b_sup, mu_1, mu_ne);
  for (int i = 0; i < m; ++i) {
    out[3 * i] = c[i].alpha;
    out[3 * i + 1] = c[i].gamma;
    out[3 * i + 2] = c[i].beta;
  }
}

int shim_degree(double res, double ritz, double c, double e, double tol, int max_deg,
                int deg_extra, int optimize, int deg) {
  chase_opts o{};
  o.max_deg = max_deg;
  o.deg_extra = deg_extra;
  o.optimize_degree = optimize;
  return chase::optimal_degree(res, ritz, c, e, tol, o, deg);
}

double shim_floor(int split_bf16, long n) { return chase::low_precision_floor(split_bf16 != 0, n); }

int shim_tail(double floor, double lam_nev, double c, double e, double tol, int deg) {
  return chase::fp64_tail_steps(floor, lam_nev, c, e, tol, deg);
}
}
