// Host-side scalar logic of Algorithm 1 (see hostmath.cpp).
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/chase.h"

namespace chase {

struct Bounds {
  double b_sup, mu_1, mu_ne;
  double norm_lower;  // largest Ritz value in magnitude: a lower bound of ||H||_2
};

// One step of Eq. (3): X_s = alpha (H - gamma I) X_{s-1} + beta X_{s-2}.
struct Coef {
  double alpha, gamma, beta;
};

void sym_eig_small(std::vector<double> a, int k, std::vector<double>& val,
                   std::vector<double>& vec);

// alpha/beta are steps x nv, step-major (entry j*nv + r)
Bounds lanczos_bounds(const std::vector<double>& alpha, const std::vector<double>& beta, int nv,
                      int steps, int64_t n, int n_e, std::vector<int>* run_len);

std::vector<Coef> cheb_coefficients(int m, double b_sup, double mu_1, double mu_ne);

int optimal_degree(double res, double ritz, double c, double e, double tol, const chase_opts& o,
                   int deg);

// Number of final FP64 steps of a low-precision filter pass of degree deg
// (even) that damp a rounding floor `floor` down to tol at the growth rate
// rho = |t| + sqrt(t^2 - 1), t = (lam_nev - c)/e, of the nev-th wanted
// eigenvalue (estimate lam_nev); 0 when that takes deg steps or more, when
// lam_nev is not below the damped interval or floor <= tol.
int fp64_tail_steps(double floor, double lam_nev, double c, double e, double tol, int deg);

// Relative rounding floor of a plain low-precision filter pass over an
// n x n matrix, the `floor` of fp64_tail_steps: 2^-14 for split-BF16
// products (set by the operands' 16-bit representation, independent of n);
// 2^-17 sqrt(max(1, n/3000)) for FP32 products (set by the accumulation of
// n-term sums, whose rounding grows like sqrt(n); calibrated at n = 3000).
double low_precision_floor(bool split_bf16, int64_t n);

}  // namespace chase
