// Dense Hermitian eigensolver of the Rayleigh-Ritz step (Algorithm 1;
// Section 2.3: the projected matrix G = Q^H H Q is diagonalised), on the GPU.
//
// Block-cyclic two-sided Jacobi (Golub & Van Loan, symmetric Schur rotations
// with a parallel round-robin ordering, block form).  The k x k matrix is cut
// into blocks of JB indices.  A sweep is the round-robin tournament over the
// blocks: in each round every pair of blocks (p, q) gets one cyclic Jacobi
// sweep over its 2 JB indices, run by one workgroup in LDS and accumulated
// into a 2JB x 2JB unitary U_pq; one launch then applies all pairs' U to the
// whole matrix (G <- J^H G J, J the block-diagonal product of the U_pq) and
// to the eigenvector block (V <- V J).  The convergence is quadratic; in the
// subspace iteration the projected matrix is close to diagonal once the
// Ritz vectors settle, and then a few sweeps suffice.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace chase {
namespace {

constexpr int JB = 16;       // indices per block
constexpr int JM = 2 * JB;   // order of a pair's subproblem
constexpr int JLD = JM + 1;  // LDS leading dimension (padded against bank conflicts)
constexpr int JT = 256;      // threads per workgroup
constexpr int JCG = JT / JM; // column groups of the tile stores (8)
constexpr int NPART = 256;   // workgroups of the norm reduction

struct cd {
  double x, y;
};
__device__ __forceinline__ cd operator+(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd operator*(cd a, cd b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cd operator*(cd a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ double conj_(double a) { return a; }
__device__ __forceinline__ cd conj_(cd a) { return {a.x, -a.y}; }
__device__ __forceinline__ double abs2(double a) { return a * a; }
__device__ __forceinline__ double abs2(cd a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double real_(double a) { return a; }
__device__ __forceinline__ double real_(cd a) { return a.x; }
template <class T>
__device__ __forceinline__ T from_real(double a);
template <>
__device__ __forceinline__ double from_real<double>(double a) { return a; }
template <>
__device__ __forceinline__ cd from_real<cd>(double a) { return {a, 0.0}; }
// acc += a * b
__device__ __forceinline__ void mac(double& acc, double a, double b) { acc = fma(a, b, acc); }
__device__ __forceinline__ void mac(cd& acc, cd a, cd b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

// Round-robin tournament over m players (m even), rounds r = 0 .. m-2:
// player 0 stays, the others rotate; pair t of round r is
// (rr_player(m, r, t), rr_player(m, r, m - 1 - t)).  Over the m - 1 rounds
// every two players meet exactly once.
__host__ __device__ inline int rr_player(int m, int r, int j) {
  return j == 0 ? 0 : (j - 1 + r) % (m - 1) + 1;
}

// Rotation that zeroes the (a, b) entry of the 2 x 2 Hermitian
// [[app, apq], [conj(apq), aqq]]: with apq = g ph (g = |apq|, |ph| = 1),
// u = [[cs, sn], [-sn conj(ph), cs conj(ph)]] = diag(1, conj(ph)) R, R the
// real rotation [[cs, sn], [-sn, cs]], and u^H A u is diagonal.  t = sn / cs
// is the root of smaller magnitude of t^2 + 2 tau t - 1 = 0, tau = (aqq -
// app) / (2 g), written as t = sign(d) 2 g / (|d| + sqrt(d^2 + 4 g^2)),
// d = aqq - app (one square root and one division on the dependent path).
// Entries with g <= thr are left alone (identity).
template <class T>
__device__ __forceinline__ int jac_rotation(double app, double aqq, T apq, double thr, double& cs,
                                            double& sn, T& ph) {
  const double g2 = abs2(apq);
  if (!(g2 > thr * thr)) {
    cs = 1.0;
    sn = 0.0;
    ph = from_real<T>(1.0);
    return 0;
  }
  const double d = aqq - app;
  const double rg = rsqrt(g2);
  const double r = sqrt(fma(d, d, 4.0 * g2));
  const double t = copysign(2.0 * g2 * rg, d) / (fabs(d) + r);
  cs = rsqrt(fma(t, t, 1.0));
  sn = t * cs;
  ph = apq * rg;
  return 1;
}

// Pair of blocks `pair` of round `round`: load its 2JB x 2JB subproblem,
// run one cyclic Jacobi sweep over its indices (round-robin over 2JB
// players: JB disjoint rotations per inner round, applied together), and
// write the accumulated unitary U (column-major, JM x JM) and whether any
// rotation was made.  Indices >= k are padding: zero rows and columns that
// never rotate.  S and U: JM x JLD arrays in LDS.
template <class T>
__device__ void pair_body(const T* __restrict__ G, int64_t ldg, int k, int nb, int round,
                          int pair, double thr, T* __restrict__ ubuf, int* __restrict__ flags,
                          T* S, T* U) {
  __shared__ double rcs[JB], rsn[JB];
  __shared__ T rph[JB];
  __shared__ int ra[JB], rb[JB], rrot[JB];
  __shared__ int any;
  const int tid = threadIdx.x;
  const int bp = rr_player(nb, round, pair), bq = rr_player(nb, round, nb - 1 - pair);
  auto gidx = [&](int l) { return l < JB ? bp * JB + l : bq * JB + (l - JB); };
  if (tid == 0) any = 0;
  for (int e = tid; e < JM * JM; e += JT) {
    const int r = e % JM, c = e / JM;
    const int gr = gidx(r), gc = gidx(c);
    T v = from_real<T>(0.0);
    if (gr < k && gc < k) v = G[gr + (int64_t)gc * ldg];
    S[c * JLD + r] = v;
    U[c * JLD + r] = from_real<T>(r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int rr = 0; rr < JM - 1; ++rr) {
    if (tid < JB) {
      const int a = rr_player(JM, rr, tid), b = rr_player(JM, rr, JM - 1 - tid);
      double cs, sn;
      T ph;
      const int rot = jac_rotation(real_(S[a * JLD + a]), real_(S[b * JLD + b]), S[b * JLD + a],
                                   thr, cs, sn, ph);
      rcs[tid] = cs;
      rsn[tid] = sn;
      rph[tid] = ph;
      ra[tid] = a;
      rb[tid] = b;
      rrot[tid] = rot;
      if (rot) any = 1;
    }
    __syncthreads();
    // S <- u^H S u on the 2 x 2 blocks (rows of pair i, columns of pair j)
    for (int e = tid; e < JB * JB; e += JT) {
      const int j = e / JB, i = e % JB;
      const int ai = ra[i], bi = rb[i], aj = ra[j], bj = rb[j];
      const double ci = rcs[i], si = rsn[i], cj = rcs[j], sj = rsn[j];
      const T pi_ = rph[i], pjc = conj_(rph[j]);
      // u_i^H M u_j = R_i^T (D_i^H M D_j) R_j: phases first, then the real
      // rotations
      const T m00 = S[aj * JLD + ai];
      const T m01 = S[bj * JLD + ai] * pjc;
      const T m10 = pi_ * S[aj * JLD + bi];
      const T m11 = S[bj * JLD + bi] * (pi_ * pjc);
      const T r00 = m00 * cj - m01 * sj, r01 = m00 * sj + m01 * cj;
      const T r10 = m10 * cj - m11 * sj, r11 = m10 * sj + m11 * cj;
      T n00 = r00 * ci - r10 * si, n01 = r01 * ci - r11 * si;
      T n10 = r00 * si + r10 * ci, n11 = r01 * si + r11 * ci;
      if (i == j) {
        // the pivot block: exactly diagonal and real after its rotation
        n00 = from_real<T>(real_(n00));
        n11 = from_real<T>(real_(n11));
        if (rrot[i]) {
          n01 = from_real<T>(0.0);
          n10 = from_real<T>(0.0);
        }
      }
      S[aj * JLD + ai] = n00;
      S[bj * JLD + ai] = n01;
      S[aj * JLD + bi] = n10;
      S[bj * JLD + bi] = n11;
    }
    // U <- U u on the columns of each pair
    for (int e = tid; e < JM * JB; e += JT) {
      const int rho = e % JM, j = e / JM;
      const int aj = ra[j], bj = rb[j];
      const double cj = rcs[j], sj = rsn[j];
      const T u0 = U[aj * JLD + rho], u1 = U[bj * JLD + rho] * conj_(rph[j]);
      U[aj * JLD + rho] = u0 * cj - u1 * sj;
      U[bj * JLD + rho] = u0 * sj + u1 * cj;
    }
    __syncthreads();
  }
  // One Newton-Schulz step towards the nearest unitary, U <- U (3 I - U^H U) / 2:
  // the rounding of the rotations leaves U unitary only to a few ulps per
  // inner round, and applying a non-unitary J^H G J shifts the eigenvalues by
  // that much in every round; the step brings it back to rounding level.
  // M = U^H U goes into S (no longer needed).
  const int i = tid % JM, cg = tid / JM;
  if (any) {
#pragma unroll
    for (int m = 0; m < JM / JCG; ++m) {
      const int c = cg + JCG * m;
      T acc = from_real<T>(0.0);
#pragma unroll 4
      for (int l = 0; l < JM; ++l) mac(acc, conj_(U[i * JLD + l]), U[c * JLD + l]);
      S[c * JLD + i] = acc;
    }
    __syncthreads();
    T nu[JM / JCG];
#pragma unroll
    for (int m = 0; m < JM / JCG; ++m) {
      const int c = cg + JCG * m;
      T acc = from_real<T>(0.0);
#pragma unroll 4
      for (int l = 0; l < JM; ++l) mac(acc, U[l * JLD + i], S[c * JLD + l]);
      nu[m] = U[c * JLD + i] * 1.5 - acc * 0.5;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < JM / JCG; ++m) U[(cg + JCG * m) * JLD + i] = nu[m];
    __syncthreads();
  }
  T* Uo = ubuf + (int64_t)pair * JM * JM;
  for (int e = tid; e < JM * JM; e += JT) Uo[e] = U[(e / JM) * JLD + (e % JM)];
  if (tid == 0) flags[pair] = any;
}

typedef double d4v __attribute__((ext_vector_type(4)));

// Y = A B for JM x JM tiles in LDS on the FP64 matrix cores (16x16x4 MFMA),
// A(i, l) at As[l * JLD + i] and B(l, c) at Bs[l * JLD + c].  Wave w of the
// four computes the quadrant of rows 16 (w & 1) and columns 16 (w >> 1).
// The operands go in swapped (B first), so the instruction produces the
// quadrant transposed: lane L holds Y(16 (w & 1) + L % 16, 16 (w >> 1) +
// L / 16 + 4 r) in out[r] (rows run along the lanes, as stores want them).
__device__ __forceinline__ void tile_mma(const double* As, const double* Bs, double (&out)[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = 16 * (w & 1), c0 = 16 * (w >> 1), l16 = lane & 15, lk = lane >> 4;
  d4v acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < JM; k0 += 4) {
    const double a = As[(k0 + lk) * JLD + i0 + l16];
    const double b = Bs[(k0 + lk) * JLD + c0 + l16];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) out[r] = acc[r];
}
__device__ __forceinline__ void tile_mma(const cd* As, const cd* Bs, cd (&out)[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = 16 * (w & 1), c0 = 16 * (w >> 1), l16 = lane & 15, lk = lane >> 4;
  d4v re = {0.0, 0.0, 0.0, 0.0}, im = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < JM; k0 += 4) {
    const cd a = As[(k0 + lk) * JLD + i0 + l16];
    const cd b = Bs[(k0 + lk) * JLD + c0 + l16];
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(b.x, a.x, re, 0, 0, 0);
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(-b.y, a.y, re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(b.y, a.x, im, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(b.x, a.y, im, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) out[r] = cd{re[r], im[r]};
}

// Position of out[r] of tile_mma in this thread: row, column.
__device__ __forceinline__ int mma_row() { return 16 * ((threadIdx.x >> 6) & 1) + (threadIdx.x & 15); }
__device__ __forceinline__ int mma_col(int r) {
  return 16 * (threadIdx.x >> 7) + ((threadIdx.x & 63) >> 4) + 4 * r;
}

// JM rows of V (row chunk `chunk`) times the columns of pair b of round
// `round`: V <- V U_b (nothing if the pair did not rotate).  Xs, Bs: LDS.
template <class T>
__device__ void vtile_body(T* __restrict__ V, int64_t ldv, int k, int nb, int round, int b,
                           int chunk, const T* __restrict__ ubuf, const int* __restrict__ flags,
                           T* Xs, T* Bs) {
  if (!flags[b]) return;
  const int tid = threadIdx.x;
  const int b0 = rr_player(nb, round, b), b1 = rr_player(nb, round, nb - 1 - b);
  auto gb = [&](int l) { return l < JB ? b0 * JB + l : b1 * JB + (l - JB); };
  const T* Ub = ubuf + (int64_t)b * JM * JM;
  const int64_t r0 = (int64_t)chunk * JM;
  for (int e = tid; e < JM * JM; e += JT) {
    const int r = e % JM, c = e / JM;
    const int gc = gb(c);
    T v = from_real<T>(0.0);
    if (r0 + r < k && gc < k) v = V[r0 + r + (int64_t)gc * ldv];
    Xs[c * JLD + r] = v;
    Bs[r * JLD + c] = Ub[e];
  }
  __syncthreads();
  T out[4];
  tile_mma(Xs, Bs, out);
  const int64_t row = r0 + mma_row();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int gc = gb(mma_col(r));
    if (row < k && gc < k) V[row + (int64_t)gc * ldv] = out[r];
  }
}

// First launch of a round: workgroups [0, npairs) solve the pairs of round
// `round` into the buffers (ubuf, flags); the next ones apply the previous
// round's unitaries (ubuf_v, flags_v, round_v) to the eigenvector block.
// The two halves touch disjoint memory (G is only read, V only by the
// second), so they run side by side.
template <class T>
__global__ __launch_bounds__(JT) void jac_stage1_k(const T* __restrict__ G, int64_t ldg,
                                                   T* __restrict__ V, int64_t ldv, int k, int nb,
                                                   int round, int npairs, double thr,
                                                   T* __restrict__ ubuf, int* __restrict__ flags,
                                                   int round_v, const T* __restrict__ ubuf_v,
                                                   const int* __restrict__ flags_v) {
  __shared__ T sm0[JM * JLD];
  __shared__ T sm1[JM * JLD];
  const int w = blockIdx.x;
  if (w < npairs) {
    pair_body<T>(G, ldg, k, nb, round, w, thr, ubuf, flags, sm0, sm1);
  } else {
    const int P = nb / 2, t = w - npairs;
    vtile_body<T>(V, ldv, k, nb, round_v, t % P, t / P, ubuf_v, flags_v, sm0, sm1);
  }
}

// Second launch of a round: the tile of G at (pair a rows, pair b columns),
// a <= b, becomes U_a^H X U_b and its mirror (b, a) the conjugate transpose
// (a == b: the Hermitian part); tiles whose two pairs did not rotate are
// left as they are.
template <class T>
__global__ __launch_bounds__(JT) void jac_stage2_k(T* __restrict__ G, int64_t ldg, int k, int nb,
                                                   int round, const T* __restrict__ ubuf,
                                                   const int* __restrict__ flags) {
  __shared__ T Xs[JM * JLD];  // X(i, l) at Xs[l * JLD + i]; later the result Y
  __shared__ T Bs[JM * JLD];  // U_b (B(l, c) at Bs[l * JLD + c]), then A = U_a^H
  __shared__ T Ts[JM * JLD];  // X U_b, T(l, c) at Ts[l * JLD + c]
  const int tid = threadIdx.x;
  const int i = tid % JM, cg = tid / JM;
  const int t = blockIdx.x;
  int b = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  if ((b + 1) * (b + 2) / 2 <= t) ++b;
  if (b * (b + 1) / 2 > t) --b;
  const int a = t - b * (b + 1) / 2;
  const int fa = flags[a], fb = flags[b];
  if (!fa && !fb) return;
  const int a0 = rr_player(nb, round, a), a1 = rr_player(nb, round, nb - 1 - a);
  const int b0 = rr_player(nb, round, b), b1 = rr_player(nb, round, nb - 1 - b);
  auto ga = [&](int l) { return l < JB ? a0 * JB + l : a1 * JB + (l - JB); };
  auto gb = [&](int l) { return l < JB ? b0 * JB + l : b1 * JB + (l - JB); };
  const T* Ua = ubuf + (int64_t)a * JM * JM;
  const T* Ub = ubuf + (int64_t)b * JM * JM;
  for (int e = tid; e < JM * JM; e += JT) {
    const int r = e % JM, c = e / JM;
    const int gr = ga(r), gc = gb(c);
    T v = from_real<T>(0.0);
    if (gr < k && gc < k) v = G[gr + (int64_t)gc * ldg];
    Xs[c * JLD + r] = v;
    Bs[r * JLD + c] = fb ? Ub[e] : from_real<T>(r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  T out[4];
  tile_mma(Xs, Bs, out);  // T = X U_b, stored as T(l, c) at Ts[l * JLD + c]
#pragma unroll
  for (int r = 0; r < 4; ++r) Ts[mma_row() * JLD + mma_col(r)] = out[r];
  __syncthreads();
  // A(c, r) = conj(U_a(r, c)) at Bs[r * JLD + c]
  for (int e = tid; e < JM * JM; e += JT) {
    const int r = e % JM, c = e / JM;
    Bs[r * JLD + c] = fa ? conj_(Ua[e]) : from_real<T>(r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  tile_mma(Bs, Ts, out);  // Y = U_a^H T, stored as Y(i, c) at Xs[c * JLD + i]
#pragma unroll
  for (int r = 0; r < 4; ++r) Xs[mma_col(r) * JLD + mma_row()] = out[r];
  __syncthreads();
  if (a == b) {
    const int gi = ga(i);
#pragma unroll
    for (int m = 0; m < JM / JCG; ++m) {
      const int c = cg + JCG * m;
      const int gc = ga(c);
      T v = (Xs[c * JLD + i] + conj_(Xs[i * JLD + c])) * 0.5;
      if (i == c) v = from_real<T>(real_(v));
      if (gi < k && gc < k) G[gi + (int64_t)gc * ldg] = v;
    }
  } else {
    const int gi = ga(i);
#pragma unroll
    for (int m = 0; m < JM / JCG; ++m) {
      const int c = cg + JCG * m;
      const int gc = gb(c);
      if (gi < k && gc < k) G[gi + (int64_t)gc * ldg] = Xs[c * JLD + i];
    }
    // mirror: lanes run over the rows of the (b, a) tile
    const int cr = tid % JM, ig = tid / JM;
    const int gcr = gb(cr);
#pragma unroll
    for (int m = 0; m < JM / JCG; ++m) {
      const int ii = ig + JCG * m;
      const int gii = ga(ii);
      if (gcr < k && gii < k) G[gcr + (int64_t)gii * ldg] = conj_(Xs[cr * JLD + ii]);
    }
  }
}

// part[2 w] = sum of |G_ij|^2 off the diagonal, part[2 w + 1] on it, over
// the entries workgroup w visits.
template <class T>
__global__ __launch_bounds__(JT) void jac_norms_k(const T* __restrict__ G, int64_t ldg, int k,
                                                  double* __restrict__ part) {
  __shared__ double so[JT], sd[JT];
  double off = 0.0, dia = 0.0;
  const int64_t total = (int64_t)k * k;
  for (int64_t e = (int64_t)blockIdx.x * JT + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * JT) {
    const int64_t r = e % k, c = e / k;
    const double v = abs2(G[r + c * ldg]);
    if (r == c)
      dia += v;
    else
      off += v;
  }
  so[threadIdx.x] = off;
  sd[threadIdx.x] = dia;
  __syncthreads();
  for (int s = JT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      so[threadIdx.x] += so[threadIdx.x + s];
      sd[threadIdx.x] += sd[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = so[0];
    part[2 * blockIdx.x + 1] = sd[0];
  }
}

template <class T>
__global__ void jac_eye_k(T* __restrict__ V, int64_t ldv, int k) {
  const int64_t total = (int64_t)k * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % k, c = e / k;
    V[r + c * ldv] = from_real<T>(r == c ? 1.0 : 0.0);
  }
}

inline int jac_blocks(int k) {
  int nb = (k + JB - 1) / JB;
  if (nb < 2) nb = 2;
  return nb + (nb & 1);
}

// Workspace layout for orders up to kmax (byte offsets): the pairs'
// unitaries, their rotation flags, the norm partials, the diagonal.
struct JacLayout {
  size_t ubuf[2], flags[2], part, diag, total;
  JacLayout(bool cplx, int kmax) {
    const int P = jac_blocks(std::max(kmax, 1)) / 2;
    const size_t esz = cplx ? 16 : 8;
    const size_t ub = ((size_t)P * JM * JM * esz + 255) / 256 * 256;
    const size_t fl = ((size_t)P * 4 + 255) / 256 * 256;
    ubuf[0] = 0;
    ubuf[1] = ub;
    flags[0] = 2 * ub;
    flags[1] = 2 * ub + fl;
    part = 2 * ub + 2 * fl;
    diag = part + 2 * NPART * 8;
    total = diag + (size_t)std::max(kmax, 1) * 8;
  }
};

template <class T>
struct JacobiRunner {
  static void norms(const void* G, int64_t ldg, int k, double* d_part, double* off2,
                    double* dia2, hipStream_t st) {
    std::vector<double> h(2 * NPART, 0.0);
    hipLaunchKernelGGL(jac_norms_k<T>, dim3(NPART), dim3(JT), 0, st, static_cast<const T*>(G),
                       ldg, k, d_part);
    CHASE_HIP(hipGetLastError());
    CHASE_HIP(hipMemcpyAsync(h.data(), d_part, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                             st));
    CHASE_HIP(hipStreamSynchronize(st));
    double o = 0.0, d = 0.0;
    for (int w = 0; w < NPART; ++w) {
      o += h[2 * w];
      d += h[2 * w + 1];
    }
    *off2 = o;
    *dia2 = d;
  }

  static int run(void* G, int64_t ldg, int k, void* V, int64_t ldv, void* ws,
                 const JacLayout& lay, double tol, int max_sweeps, double off2, double dia2,
                 hipStream_t st) {
    const int nb = jac_blocks(k), P = nb / 2;
    char* base = static_cast<char*>(ws);
    T* ubuf[2] = {reinterpret_cast<T*>(base + lay.ubuf[0]), reinterpret_cast<T*>(base + lay.ubuf[1])};
    int* flags[2] = {reinterpret_cast<int*>(base + lay.flags[0]),
                     reinterpret_cast<int*>(base + lay.flags[1])};
    double* d_part = reinterpret_cast<double*>(base + lay.part);
    const int tiles_g = P * (P + 1) / 2;
    const int tiles_v = ((k + JM - 1) / JM) * P;
    T* Gt = static_cast<T*>(G);
    T* Vt = static_cast<T*>(V);
    hipLaunchKernelGGL(jac_eye_k<T>, dim3(std::min<int64_t>(1024, ((int64_t)k * k + 255) / 256)),
                       dim3(256), 0, st, Vt, ldv, k);
    CHASE_HIP(hipGetLastError());
    const double fro2 = off2 + dia2;
    const double thr = tol * std::sqrt(fro2) / (double)k;
    int sweeps = 0;
    while (!(off2 <= tol * tol * fro2)) {
      if (sweeps >= max_sweeps)
        throw Error(CHASE_ERR_NUMERIC, "Jacobi eigensolver did not converge in " +
                                           std::to_string(max_sweeps) + " sweeps");
      // round r: pairs of r with the eigenvector update of r - 1, then G;
      // the last round's eigenvector update closes the sweep
      for (int r = 0; r <= nb - 1; ++r) {
        const bool pairs = r < nb - 1, vupd = r > 0;
        const int cur = r & 1, prev = (r + 1) & 1;
        hipLaunchKernelGGL(jac_stage1_k<T>, dim3((pairs ? P : 0) + (vupd ? tiles_v : 0)),
                           dim3(JT), 0, st, static_cast<const T*>(Gt), ldg, Vt, ldv, k, nb, r,
                           pairs ? P : 0, thr, ubuf[cur], flags[cur], r - 1,
                           static_cast<const T*>(ubuf[prev]),
                           static_cast<const int*>(flags[prev]));
        if (pairs)
          hipLaunchKernelGGL(jac_stage2_k<T>, dim3(tiles_g), dim3(JT), 0, st, Gt, ldg, k, nb, r,
                             static_cast<const T*>(ubuf[cur]),
                             static_cast<const int*>(flags[cur]));
      }
      CHASE_HIP(hipGetLastError());
      ++sweeps;
      double d2;
      norms(G, ldg, k, d_part, &off2, &d2, st);
      if (!std::isfinite(off2)) throw Error(CHASE_ERR_NUMERIC, "non-finite entries in Jacobi");
    }
    return sweeps;
  }
};

}  // namespace

size_t jacobi_ws_bytes(bool cplx, int kmax) { return JacLayout(cplx, kmax).total; }

void jacobi_norms(bool cplx, const void* G, int64_t ldg, int k, void* ws, int kmax,
                  double* off2, double* dia2, hipStream_t st) {
  CHASE_REQUIRE(k >= 1 && k <= kmax, "Jacobi eigensolver: order out of range");
  double* d_part = reinterpret_cast<double*>(static_cast<char*>(ws) + JacLayout(cplx, kmax).part);
  if (cplx)
    JacobiRunner<cd>::norms(G, ldg, k, d_part, off2, dia2, st);
  else
    JacobiRunner<double>::norms(G, ldg, k, d_part, off2, dia2, st);
}

int jacobi_heev(bool cplx, void* G, int64_t ldg, int k, void* V, int64_t ldv, void* W,
                int64_t ldw, double* d_evals, int* d_perm, void* ws, int kmax, double* evals_host,
                hipStream_t st, double off2, double dia2, double tol, int max_sweeps) {
  CHASE_REQUIRE(k >= 1 && k <= kmax, "Jacobi eigensolver: order out of range");
  CHASE_REQUIRE(ldg >= k && ldv >= k && ldw >= k, "Jacobi eigensolver: leading dimension < k");
  CHASE_REQUIRE(V != G && V != W, "Jacobi eigensolver: V must be a separate buffer");
  if (!std::isfinite(off2) || !std::isfinite(dia2))
    throw Error(CHASE_ERR_NUMERIC, "non-finite entries in the projected matrix");
  const JacLayout lay(cplx, kmax);
  int sweeps;
  if (cplx)
    sweeps = JacobiRunner<cd>::run(G, ldg, k, V, ldv, ws, lay, tol, max_sweeps, off2, dia2, st);
  else
    sweeps = JacobiRunner<double>::run(G, ldg, k, V, ldv, ws, lay, tol, max_sweeps, off2, dia2, st);
  // eigenvalues: the diagonal, ascending (stable), eigenvectors gathered to match
  double* d_diag = reinterpret_cast<double*>(static_cast<char*>(ws) + lay.diag);
  diag_real(cplx, G, ldg, k, d_diag, st);
  std::vector<double> w(k);
  CHASE_HIP(hipMemcpyAsync(w.data(), d_diag, (size_t)k * 8, hipMemcpyDeviceToHost, st));
  CHASE_HIP(hipStreamSynchronize(st));
  std::vector<int> perm(k);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return w[x] < w[y]; });
  for (int j = 0; j < k; ++j) evals_host[j] = w[perm[j]];
  CHASE_HIP(hipMemcpyAsync(d_perm, perm.data(), (size_t)k * sizeof(int), hipMemcpyHostToDevice,
                           st));
  CHASE_HIP(hipMemcpyAsync(d_evals, evals_host, (size_t)k * 8, hipMemcpyHostToDevice, st));
  gather_cols(cplx, V, ldv, W, ldw, k, k, d_perm, st);
  // the host arrays above must outlive the copies
  CHASE_HIP(hipStreamSynchronize(st));
  return sweeps;
}

}  // namespace chase
