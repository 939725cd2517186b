// Cholesky factorisation A = R^H R of the Gram matrix in the QR step's
// Cholesky passes (Algorithm 1's QR step, done as Cholesky QR with a shifted
// pass and a Householder fallback; the paper's own QR is geqrf, Section
// 2.3).  R is upper triangular with a positive real diagonal.
//
// Right-looking blocked algorithm with panels of CB rows.  Per panel two
// launches:
//  - chol_panel_k: every workgroup factors the CB x CB diagonal block in
//    LDS (the same arithmetic in each, so they agree bit for bit), then
//    solves R11^H X = A12 for its own PC columns of the row panel, staged
//    through LDS, one column per thread held in registers (forward
//    substitution).  Workgroup 0 also stores R11.
//  - chol_update_k: A22 -= R12^H R12 on the upper triangle, in UT x UT
//    tiles staged through LDS.
// The order of a k x k factorisation is about k / CB panel steps; at the
// sizes of the subspace (k ~ 10^3) each launch is short and the chain is
// latency bound, which the one-launch panel keeps to two launches a panel.
//
// A pivot that is not positive (or not a number) stops the factorisation:
// info receives its 1-based order (as LAPACK's potrf) and every later
// launch returns at once; R then holds partial results.
#include "common.h"

#include <algorithm>

namespace chase {
namespace {

constexpr int CB = 32;        // panel rows
constexpr int CLD = CB + 1;   // LDS leading dimension of the diagonal block
constexpr int CT = 256;       // threads per workgroup
constexpr int CG = CT / CB;   // column groups of the (row, column-group) thread map
constexpr int PC = 128;       // row-panel columns per workgroup
constexpr int PLD = PC + 1;
constexpr int UT = 32;        // trailing-update tile
constexpr int ULD = UT + 1;

struct cd {
  double x, y;
};
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd operator*(cd a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ double real_(double a) { return a; }
__device__ __forceinline__ double real_(cd a) { return a.x; }
__device__ __forceinline__ double scaled(double a, double s) { return a * s; }
__device__ __forceinline__ cd scaled(cd a, double s) { return a * s; }
template <class T>
__device__ __forceinline__ T from_real(double a);
template <>
__device__ __forceinline__ double from_real<double>(double a) { return a; }
template <>
__device__ __forceinline__ cd from_real<cd>(double a) { return {a, 0.0}; }
// acc -= conj(a) * b
__device__ __forceinline__ void msub_conj(double& acc, double a, double b) {
  acc = fma(-a, b, acc);
}
__device__ __forceinline__ void msub_conj(cd& acc, cd a, cd b) {
  acc.x = fma(-a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(-a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
__device__ __forceinline__ void mac_conj(double& acc, double a, double b) { acc = fma(a, b, acc); }
__device__ __forceinline__ void mac_conj(cd& acc, cd a, cd b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

// Panel j0: factor the diagonal block and solve the row panel.  Grid:
// ceil((k - j0 - CB) / PC) workgroups (at least one).  Thread (ti, tg) =
// (tid % CB, tid / CB) owns row ti of the diagonal block at the columns
// tg + CG q (q < CB / CG), in registers.
template <class T>
__global__ __launch_bounds__(CT) void chol_panel_k(T* __restrict__ A, int64_t lda, int k, int j0,
                                                   int* __restrict__ info) {
  constexpr int NQ = CB / CG;
  __shared__ T D[CB * CLD];    // R11, column-major: D[i + c * CLD]
  __shared__ T P[CB * PLD];    // this workgroup's row-panel columns: P[i * PLD + c]
  __shared__ T row[2][CB];     // the pivot row of the current and the next step
  __shared__ double piv[CB];   // pivots a_jj = r_jj^2
  __shared__ double rdg[CB];   // 1 / r_jj
  const int bad = *info;       // loaded with the tiles below, tested after them
  const int tid = threadIdx.x;
  const int ti = tid % CB, tg = tid / CB;
  const int nb = min(CB, k - j0);
  // only full panels have columns to the right (nb < CB means j0 + nb == k)
  const int64_t c0 = (int64_t)j0 + nb + (int64_t)blockIdx.x * PC;
  const int pc = nb == CB ? (int)max<int64_t>(0, min<int64_t>(PC, k - c0)) : 0;
  T v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = tg + CG * q;
    v[q] = (ti <= c && c < nb) ? A[(int64_t)(j0 + ti) + (int64_t)(j0 + c) * lda]
                               : from_real<T>(0.0);
  }
  for (int c = tg; c < pc; c += CG) P[ti * PLD + c] = A[(int64_t)(j0 + ti) + (c0 + c) * lda];
  if (bad != 0) return;
  if (ti == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) row[0][tg + CG * q] = v[q];
  __syncthreads();
  // Unscaled right-looking elimination: step j takes conj(a_ji) a_jc / a_jj
  // off every a_ic, j < i <= c, and the owners of row j + 1 (final after
  // this step) publish it for the next step.  Row j ends as r_jj * (row j
  // of R) with a_jj = r_jj^2.
  for (int j = 0; j < nb; ++j) {
    const T* rj = row[j & 1];
    const double d = real_(rj[j]);
    if (!(d > 0.0)) {  // the same value in every thread: a uniform exit
      if (tid == 0 && blockIdx.x == 0) *info = j0 + j + 1;
      return;
    }
    if (tid == 0) piv[j] = d;
    if (ti > j && ti < nb) {
      const T f = scaled(rj[ti], 1.0 / d);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int c = tg + CG * q;
        if (c >= ti && c < nb) msub_conj(v[q], f, rj[c]);
      }
      if (ti == j + 1)
#pragma unroll
        for (int q = 0; q < NQ; ++q) row[(j + 1) & 1][tg + CG * q] = v[q];
    }
    __syncthreads();
  }
  if (ti < nb) {
    const double r = sqrt(piv[ti]);
    const double rs = 1.0 / r;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int c = tg + CG * q;
      if (c > ti && c < nb) D[ti + c * CLD] = scaled(v[q], rs);
      if (c == ti) D[ti + c * CLD] = from_real<T>(r);
    }
    if (tg == 0) rdg[ti] = rs;
  }
  __syncthreads();
  if (blockIdx.x == 0 && ti < nb)
    for (int c = tg; c < nb; c += CG)
      if (ti <= c) A[(int64_t)(j0 + ti) + (int64_t)(j0 + c) * lda] = D[ti + c * CLD];
  // Row panel: column c of A12 becomes R11^{-H} a_c (forward substitution,
  // column-oriented, in registers).
  if (tid < pc) {
    T x[CB];
#pragma unroll
    for (int i = 0; i < CB; ++i) x[i] = P[i * PLD + tid];
#pragma unroll
    for (int l = 0; l < CB; ++l) {
      x[l] = scaled(x[l], rdg[l]);
#pragma unroll
      for (int i = l + 1; i < CB; ++i) msub_conj(x[i], D[l + i * CLD], x[l]);
    }
#pragma unroll
    for (int i = 0; i < CB; ++i) P[i * PLD + tid] = x[i];
  }
  __syncthreads();
  for (int c = tg; c < pc; c += CG) A[(int64_t)(j0 + ti) + (c0 + c) * lda] = P[ti * PLD + c];
}

// A22 -= R12^H R12 on the upper triangle of the trailing block (rows and
// columns from j0 + CB), R12 in rows j0 .. j0 + CB - 1.  Grid t x t with
// t = ceil(m / UT); workgroups below the diagonal return.
template <class T>
__global__ __launch_bounds__(CT) void chol_update_k(T* __restrict__ A, int64_t lda, int k, int j0,
                                                    const int* __restrict__ info) {
  __shared__ T Ri[CB * ULD];  // Ri[l * ULD + q] = R12(l, i0 + q)
  __shared__ T Rc[CB * ULD];
  const int ti = blockIdx.x, tc = blockIdx.y;
  if (ti > tc || *info != 0) return;
  const int tid = threadIdx.x;
  const int b = j0 + CB;  // first row and column of the trailing block
  const int m = k - b;
  const int i0 = ti * UT, c0 = tc * UT;
  const int ni = min(UT, m - i0), nc = min(UT, m - c0);
  for (int e = tid; e < CB * UT; e += CT) {
    const int l = e % CB, q = e / CB;
    const T* row = A + (int64_t)(j0 + l);
    T vi = from_real<T>(0.0), vc = from_real<T>(0.0);
    if (q < ni) vi = row[(int64_t)(b + i0 + q) * lda];
    if (q < nc) vc = row[(int64_t)(b + c0 + q) * lda];
    Ri[l * ULD + q] = vi;
    Rc[l * ULD + q] = vc;
  }
  __syncthreads();
  const int ii = tid % UT;
  const int cg = tid / UT;  // column group
  constexpr int NG = CT / UT;
  constexpr int PER = UT / NG;
  T acc[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) acc[p] = from_real<T>(0.0);
#pragma unroll 4
  for (int l = 0; l < CB; ++l) {
    const T a = Ri[l * ULD + ii];
#pragma unroll
    for (int p = 0; p < PER; ++p) mac_conj(acc[p], a, Rc[l * ULD + cg + p * NG]);
  }
  if (ii >= ni) return;
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int cc = cg + p * NG;
    if (cc >= nc || (ti == tc && ii > cc)) continue;
    T* dst = A + (int64_t)(b + i0 + ii) + (int64_t)(b + c0 + cc) * lda;
    *dst = *dst - acc[p];
  }
}

template <class T>
void cholesky_launch(T* A, int64_t lda, int k, int* info, hipStream_t st) {
  for (int j0 = 0; j0 < k; j0 += CB) {
    const int nb = std::min(CB, k - j0);
    const int m = k - j0 - nb;
    const unsigned gp = (unsigned)std::max(1, (m + PC - 1) / PC);
    hipLaunchKernelGGL(chol_panel_k<T>, dim3(gp), dim3(CT), 0, st, A, lda, k, j0, info);
    CHASE_HIP(hipGetLastError());
    if (m > 0) {
      const unsigned t = (unsigned)((m + UT - 1) / UT);
      hipLaunchKernelGGL(chol_update_k<T>, dim3(t, t), dim3(CT), 0, st, A, lda, k, j0, info);
      CHASE_HIP(hipGetLastError());
    }
  }
}

}  // namespace

void cholesky_upper(bool cplx, void* A, int64_t lda, int k, int* d_info, hipStream_t st) {
  CHASE_REQUIRE(k >= 0 && lda >= std::max(1, k), "Cholesky: bad order or leading dimension");
  fill_zero(d_info, sizeof(int), st);
  if (k == 0) return;
  if (cplx)
    cholesky_launch(static_cast<cd*>(A), lda, k, d_info, st);
  else
    cholesky_launch(static_cast<double*>(A), lda, k, d_info, st);
}

}  // namespace chase
