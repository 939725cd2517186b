// Host-side scalar logic of Algorithm 1: the Lanczos bound estimates (small
// tridiagonal eigenproblems and the density-of-states quadrature), the
// Chebyshev coefficients, the degree formula and the locking / sorting
// bookkeeping.  Plain C++ on arrays of at most nev+nex entries.
#include "hostmath.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace chase {

// Cyclic Jacobi for a small real symmetric matrix (row-major, k x k).
// Returns ascending eigenvalues and the eigenvectors as columns of `vec`.
void sym_eig_small(std::vector<double> a, int k, std::vector<double>& val,
                   std::vector<double>& vec) {
  vec.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) vec[(size_t)i * k + i] = 1.0;
  auto A = [&](int i, int j) -> double& { return a[(size_t)i * k + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) (i == j ? diag : off) += A(i, j) * A(i, j);
    if (off <= 1e-32 * (diag > 0 ? diag : 1.0)) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = A(p, q);
        if (apq == 0.0) continue;
        const double tau = (A(q, q) - A(p, p)) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int r = 0; r < k; ++r) {  // columns p, q
          const double arp = A(r, p), arq = A(r, q);
          A(r, p) = c * arp - s * arq;
          A(r, q) = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {  // rows p, q
          const double apr = A(p, r), aqr = A(q, r);
          A(p, r) = c * apr - s * aqr;
          A(q, r) = s * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double vrp = vec[(size_t)r * k + p], vrq = vec[(size_t)r * k + q];
          vec[(size_t)r * k + p] = c * vrp - s * vrq;
          vec[(size_t)r * k + q] = s * vrp + c * vrq;
        }
      }
  }
  std::vector<int> idx(k);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return A(x, x) < A(y, y); });
  val.resize(k);
  std::vector<double> v2((size_t)k * k);
  for (int c = 0; c < k; ++c) {
    val[c] = A(idx[c], idx[c]);
    for (int r = 0; r < k; ++r) v2[(size_t)r * k + c] = vec[(size_t)r * k + idx[c]];
  }
  vec.swap(v2);
}

Bounds lanczos_bounds(const std::vector<double>& alpha, const std::vector<double>& beta, int nv,
                      int steps, int64_t n, int n_e, std::vector<int>* run_len) {
  Bounds b;
  b.b_sup = -INFINITY;
  b.mu_1 = INFINITY;
  b.norm_lower = 0.0;
  std::vector<std::pair<double, double>> nodes;  // (theta, weight)
  if (run_len) run_len->assign(nv, 0);
  for (int r = 0; r < nv; ++r) {
    // length of the run: stop at the first beta_j <= 1e-14 max|alpha_0..j|
    int len = steps;
    double amax = 0.0;
    for (int j = 0; j < steps; ++j) {
      amax = std::max(amax, std::fabs(alpha[(size_t)j * nv + r]));
      if (beta[(size_t)j * nv + r] <= 1e-14 * amax) {
        len = j + 1;
        break;
      }
    }
    if (run_len) (*run_len)[r] = len;
    std::vector<double> t((size_t)len * len, 0.0);
    for (int j = 0; j < len; ++j) {
      t[(size_t)j * len + j] = alpha[(size_t)j * nv + r];
      if (j + 1 < len) {
        t[(size_t)j * len + j + 1] = beta[(size_t)j * nv + r];
        t[(size_t)(j + 1) * len + j] = beta[(size_t)j * nv + r];
      }
    }
    std::vector<double> th, y;
    sym_eig_small(t, len, th, y);
    b.b_sup = std::max(b.b_sup, th[len - 1] + std::fabs(beta[(size_t)(len - 1) * nv + r]));
    b.mu_1 = std::min(b.mu_1, th[0]);
    b.norm_lower = std::max(b.norm_lower, std::max(std::fabs(th[0]), std::fabs(th[len - 1])));
    for (int j = 0; j < len; ++j) nodes.emplace_back(th[j], y[j] * y[j] / nv);
  }
  // density of states: smallest node where n * cumulative weight reaches n_e
  std::stable_sort(nodes.begin(), nodes.end(),
                   [](const std::pair<double, double>& x, const std::pair<double, double>& y) {
                     return x.first < y.first;
                   });
  const double target = (double)n_e - 1e-9 * (double)n_e;
  double cum = 0.0;
  b.mu_ne = nodes.back().first;
  for (auto& nw : nodes) {
    cum += nw.second;
    if (cum * (double)n >= target) {
      b.mu_ne = nw.first;
      break;
    }
  }
  b.mu_ne = std::min(std::max(b.mu_ne, b.mu_1), b.b_sup);
  return b;
}

std::vector<Coef> cheb_coefficients(int m, double b_sup, double mu_1, double mu_ne) {
  const double c = 0.5 * (b_sup + mu_ne), e = 0.5 * (b_sup - mu_ne);
  const double s1 = e / (mu_1 - c);
  std::vector<Coef> out;
  out.push_back({s1 / e, c, 0.0});
  double s = s1;
  for (int i = 2; i <= m; ++i) {
    const double sn = 1.0 / (2.0 / s1 - s);
    out.push_back({2.0 * sn / e, c, -s * sn});
    s = sn;
  }
  return out;
}

int optimal_degree(double res, double ritz, double c, double e, double tol, const chase_opts& o,
                   int deg) {
  int m;
  if (!o.optimize_degree) {
    m = deg;
  } else {
    const double t = (ritz - c) / e;
    double rho;
    if (std::fabs(t) <= 1.0) {
      rho = 1.0;  // |t +- i sqrt(1 - t^2)| = 1
    } else {
      const double r = std::sqrt(t * t - 1.0);
      rho = std::max(std::fabs(t + r), std::fabs(t - r));
    }
    if (rho <= 1.0 + 1e-12) {
      m = o.max_deg;
    } else {
      const double x = std::ceil(std::fabs(std::log(res / tol)) / std::log(rho));
      m = x > 1e6 ? o.max_deg : (int)x + o.deg_extra;
      m = std::min(m, o.max_deg);
    }
  }
  m = std::max(m, 2);
  m += m % 2;
  return m;
}

int fp64_tail_steps(double floor, double lam_nev, double c, double e, double tol, int deg) {
  if (!(e > 0.0) || !(floor > tol) || !(tol > 0.0)) return 0;
  const double t = (lam_nev - c) / e;
  if (!(t < -1.0)) return 0;
  const double rho = -t + std::sqrt(t * t - 1.0);
  const double j = std::ceil(std::log(floor / tol) / std::log(rho));
  return (std::isfinite(j) && j < deg) ? (int)j : 0;
}

double low_precision_floor(bool split_bf16, int64_t n) {
  if (split_bf16) return 0x1p-14;
  return 0x1p-17 * std::sqrt(std::max(1.0, (double)n / 3000.0));
}

}  // namespace chase
