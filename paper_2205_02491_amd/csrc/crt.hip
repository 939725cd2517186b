// FP64-accurate filter products on the INT8 matrix cores (an integer
// modular emulation of a floating-point matrix product: Ozaki, Uchino and
// Imamura's "Ozaki scheme II").
//
// C = H X with H (n x n) and X (n x k) in FP64.  Each row i of H is scaled by
// 2^sigma_i and each column j of X by 2^tau_j and rounded to integers of at
// most pa and pb bits; the integer product is then exact modulo each of N
// pairwise coprime moduli m_t <= 256, whose residues fit int8: one INT8
// GEMM with exact INT32 accumulation per modulus.  Chinese remaindering
// (Garner's mixed-radix form with balanced digits) recovers the integer
// product, exact because its magnitude stays below M / 2, M = prod m_t;
// scaling back gives C with the rounding error of the integer forms only
// (2^-pa of a row's largest entry, 2^-pb of a column's), which with N = 14
// moduli is about 2^-46: the accuracy class of an FP64 product.
//
// Complex products use Gauss's three real products (Re H + Im H)(Re X +
// Im X), Re H Re X, Im H Im X, combined in residue space, so the real and
// imaginary parts are each reconstructed once.  H is Hermitian: row i of H is
// the conjugate of column i, which makes the conversion of H read contiguous
// memory.  The residue planes of H are built once per solve; those of the
// block at every step.  The N (complex: 3N) INT8 products of a step are one
// strided-batched rocBLAS call; the reconstruction kernel applies the
// Chebyshev step of Eq. (3) (and the defect-correction term) on the way out.
#include "common.h"

#include <rocblas/rocblas.h>

#include <cmath>
#include <vector>

namespace chase {
namespace {

constexpr int TPB = 256;
// pairwise coprime moduli <= 256 (256 = 2^8; 255 = 3 5 17; 253 = 11 23;
// 247 = 13 19; the rest prime), largest first
constexpr int kModuli[kCrtMaxModuli] = {256, 255, 253, 251, 247, 241, 239, 233,
                                        229, 227, 223, 211, 199, 197, 193, 191};

// balanced residue of an integer-valued double |x| < 2^53 modulo m
__device__ __forceinline__ int bres(double x, int m, double minv) {
  const double q = rint(x * minv);
  int r = (int)fma(-q, (double)m, x);  // exact: the result is small
  if (r > (m - 1) / 2) r -= m;
  if (r < -(m / 2)) r += m;
  return r;
}

// x mod m in [0, m) for |x| < 2^31 (int32 GEMM output)
__device__ __forceinline__ int ures32(int x, int m, double minv) {
  const double q = floor((double)x * minv);
  int r = (int)((double)x - q * (double)m);
  if (r < 0) r += m;
  if (r >= m) r -= m;
  return r;
}

// exponent e with |v| < 2^e (frexp), 0 for v == 0
__device__ __forceinline__ int exp2_above(double v) {
  int e = 0;
  if (v > 0.0) (void)frexp(v, &e);
  return e;
}

// sigma[i] = pa - e_i, 2^(e_i - 1) <= max_j |H_ij| (real and imaginary parts)
// < 2^e_i, from column i (row i of a Hermitian H is its conjugate).
template <bool CPLX>
__global__ __launch_bounds__(TPB) void crt_rowexp_k(const double* __restrict__ H, int64_t ldh,
                                                    int64_t n, int pa, int* __restrict__ sigma) {
  __shared__ double red[TPB];
  const int64_t i = blockIdx.x;
  const int W = CPLX ? 2 : 1;
  double m = 0.0;
  for (int64_t e = threadIdx.x; e < n * W; e += TPB) m = fmax(m, fabs(H[i * ldh * W + e]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) sigma[i] = red[0] > 0.0 ? pa - exp2_above(red[0]) : 0;
}

// tau[j] = pb - e_j for column j of X (n rows).
template <bool CPLX>
__global__ __launch_bounds__(TPB) void crt_colexp_k(const double* __restrict__ X, int64_t ldx,
                                                    int64_t n, int pb, int* __restrict__ tau) {
  __shared__ double red[TPB];
  const int64_t j = blockIdx.x;
  const int W = CPLX ? 2 : 1;
  double m = 0.0;
  for (int64_t e = threadIdx.x; e < n * W; e += TPB) m = fmax(m, fabs(X[j * ldx * W + e]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) tau[j] = red[0] > 0.0 ? pb - exp2_above(red[0]) : 0;
}

// Residue planes of H, row-major (element (i, j) at i n + j: the column-major
// transpose, the A operand of a transposed GEMM).  Complex: planes 3t+0 (Re),
// 3t+1 (Im), 3t+2 (Re + Im) of modulus t; real: plane t.  Row i of H is
// conj(column i): Re H_ij = Re H[j + i ldh], Im H_ij = -Im H[j + i ldh].
template <bool CPLX>
__global__ __launch_bounds__(TPB) void crt_hplanes_k(const double* __restrict__ H, int64_t ldh,
                                                     int64_t n, const int* __restrict__ sigma,
                                                     CrtBasis B, int8_t* __restrict__ planes) {
  const int64_t i = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (j >= n) return;
  const int s = sigma[i];
  const int64_t o = i * n + j;
  const int64_t plane = n * n;
  if constexpr (CPLX) {
    const double re = rint(ldexp(H[2 * (j + i * ldh)], s));
    const double im = rint(ldexp(-H[2 * (j + i * ldh) + 1], s));
    const double sm = re + im;
    for (int t = 0; t < B.n_mod; ++t) {
      const int m = B.m[t];
      const double minv = 1.0 / (double)m;
      planes[(3 * t + 0) * plane + o] = (int8_t)bres(re, m, minv);
      planes[(3 * t + 1) * plane + o] = (int8_t)bres(im, m, minv);
      planes[(3 * t + 2) * plane + o] = (int8_t)bres(sm, m, minv);
    }
  } else {
    const double v = rint(ldexp(H[j + i * ldh], s));
    for (int t = 0; t < B.n_mod; ++t)
      planes[t * plane + o] = (int8_t)bres(v, B.m[t], 1.0 / (double)B.m[t]);
  }
}

// Residue planes of the block X (n x cols, column-major, ld n per plane).
template <bool CPLX>
__global__ __launch_bounds__(TPB) void crt_xplanes_k(const double* __restrict__ X, int64_t ldx,
                                                     int64_t n, int cols,
                                                     const int* __restrict__ tau, CrtBasis B,
                                                     int8_t* __restrict__ planes) {
  const int64_t j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const int s = tau[j];
  const int64_t o = j * n + i;
  const int64_t plane = n * (int64_t)cols;
  if constexpr (CPLX) {
    const double re = rint(ldexp(X[2 * (i + j * ldx)], s));
    const double im = rint(ldexp(X[2 * (i + j * ldx) + 1], s));
    const double sm = re + im;
    for (int t = 0; t < B.n_mod; ++t) {
      const int m = B.m[t];
      const double minv = 1.0 / (double)m;
      planes[(3 * t + 0) * plane + o] = (int8_t)bres(re, m, minv);
      planes[(3 * t + 1) * plane + o] = (int8_t)bres(im, m, minv);
      planes[(3 * t + 2) * plane + o] = (int8_t)bres(sm, m, minv);
    }
  } else {
    const double v = rint(ldexp(X[i + j * ldx], s));
    for (int t = 0; t < B.n_mod; ++t)
      planes[t * plane + o] = (int8_t)bres(v, B.m[t], 1.0 / (double)B.m[t]);
  }
}

// Four consecutive entries per thread (n a multiple of 4): the residues of
// each plane go out as one packed 32-bit store (byte e = entry e).
template <bool CPLX>
__global__ __launch_bounds__(TPB) void crt_hplanes4_k(const double* __restrict__ H, int64_t ldh,
                                                      int64_t n, const int* __restrict__ sigma,
                                                      CrtBasis B, int8_t* __restrict__ planes) {
  const int64_t i = blockIdx.y;
  const int64_t j0 = 4 * ((int64_t)blockIdx.x * TPB + threadIdx.x);
  if (j0 >= n) return;
  const int s = sigma[i];
  const int64_t o = i * n + j0;
  const int64_t plane = n * n;
  if constexpr (CPLX) {
    double re[4], im[4], sm[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      re[e] = rint(ldexp(H[2 * (j0 + e + i * ldh)], s));
      im[e] = rint(ldexp(-H[2 * (j0 + e + i * ldh) + 1], s));
      sm[e] = re[e] + im[e];
    }
    for (int t = 0; t < B.n_mod; ++t) {
      const int m = B.m[t];
      const double minv = 1.0 / (double)m;
      uint32_t wr = 0, wi = 0, ws = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        wr |= (uint32_t)(uint8_t)bres(re[e], m, minv) << (8 * e);
        wi |= (uint32_t)(uint8_t)bres(im[e], m, minv) << (8 * e);
        ws |= (uint32_t)(uint8_t)bres(sm[e], m, minv) << (8 * e);
      }
      *reinterpret_cast<uint32_t*>(planes + (3 * t + 0) * plane + o) = wr;
      *reinterpret_cast<uint32_t*>(planes + (3 * t + 1) * plane + o) = wi;
      *reinterpret_cast<uint32_t*>(planes + (3 * t + 2) * plane + o) = ws;
    }
  } else {
    double v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = rint(ldexp(H[j0 + e + i * ldh], s));
    for (int t = 0; t < B.n_mod; ++t) {
      uint32_t w = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        w |= (uint32_t)(uint8_t)bres(v[e], B.m[t], 1.0 / (double)B.m[t]) << (8 * e);
      *reinterpret_cast<uint32_t*>(planes + t * plane + o) = w;
    }
  }
}

template <bool CPLX>
__global__ __launch_bounds__(TPB) void crt_xplanes4_k(const double* __restrict__ X, int64_t ldx,
                                                      int64_t n, int cols,
                                                      const int* __restrict__ tau, CrtBasis B,
                                                      int8_t* __restrict__ planes) {
  const int64_t j = blockIdx.y;
  const int64_t i0 = 4 * ((int64_t)blockIdx.x * TPB + threadIdx.x);
  if (i0 >= n) return;
  const int s = tau[j];
  const int64_t o = j * n + i0;
  const int64_t plane = n * (int64_t)cols;
  if constexpr (CPLX) {
    double re[4], im[4], sm[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      re[e] = rint(ldexp(X[2 * (i0 + e + j * ldx)], s));
      im[e] = rint(ldexp(X[2 * (i0 + e + j * ldx) + 1], s));
      sm[e] = re[e] + im[e];
    }
    for (int t = 0; t < B.n_mod; ++t) {
      const int m = B.m[t];
      const double minv = 1.0 / (double)m;
      uint32_t wr = 0, wi = 0, ws = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        wr |= (uint32_t)(uint8_t)bres(re[e], m, minv) << (8 * e);
        wi |= (uint32_t)(uint8_t)bres(im[e], m, minv) << (8 * e);
        ws |= (uint32_t)(uint8_t)bres(sm[e], m, minv) << (8 * e);
      }
      *reinterpret_cast<uint32_t*>(planes + (3 * t + 0) * plane + o) = wr;
      *reinterpret_cast<uint32_t*>(planes + (3 * t + 1) * plane + o) = wi;
      *reinterpret_cast<uint32_t*>(planes + (3 * t + 2) * plane + o) = ws;
    }
  } else {
    double v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = rint(ldexp(X[i0 + e + j * ldx], s));
    for (int t = 0; t < B.n_mod; ++t) {
      uint32_t w = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        w |= (uint32_t)(uint8_t)bres(v[e], B.m[t], 1.0 / (double)B.m[t]) << (8 * e);
      *reinterpret_cast<uint32_t*>(planes + t * plane + o) = w;
    }
  }
}

// Garner: the integer x with x = r_t (mod m_t), |x| < M / 2, from residues
// r_t in [0, m_t): balanced mixed-radix digits v_t, x = v_0 + m_0 (v_1 + m_1
// (v_2 + ...)), evaluated in FP64 from the top digit (error <= ~NM u |x|).
// The moduli are compile-time constants.
// x mod m in [0, m) for an integer-valued float |x| < 2^24 (exact: the
// quotient estimate is off by at most one, which the two corrections undo)
__device__ __forceinline__ float fmod_m(float x, float m, float minv) {
  const float q = floorf(x * minv);
  float r = fmaf(-q, m, x);
  if (r < 0.f) r += m;
  if (r >= m) r -= m;
  return r;
}

template <int NM>
__device__ __forceinline__ double garner(const int (&r)[NM], const CrtBasis& B) {
  // every intermediate is an integer below 2^17 in magnitude, exact in FP32,
  // whose multiply-adds run at full rate (32-bit integer multiplies do not)
  float v[NM];
#pragma unroll
  for (int t = 0; t < NM; ++t) {
    const float m = (float)kModuli[t], minv = 1.0f / (float)kModuli[t];
    // (v_0 + m_0 (v_1 + ... + m_{t-2} v_{t-1})) mod m_t
    float acc = 0.f;
#pragma unroll
    for (int s = t - 1; s >= 0; --s) acc = fmod_m(fmaf(acc, (float)kModuli[s], v[s]), m, minv);
    float d = fmod_m((float)r[t] - acc, m, minv);
    d = fmod_m(d * (float)B.inv[t], m, minv);
    if (d > (m - 1.f) * 0.5f) d -= m;
    v[t] = d;
  }
  double x = 0.0;
#pragma unroll
  for (int t = NM - 1; t >= 0; --t) x = fma(x, (double)kModuli[t], (double)v[t]);
  return x;
}

// out(i, j) = alpha (C(i, j) - gamma Xs(i, j)) + beta out(i, j)
//             [+ colcoef[j] F(i, j)],  C = H Xs from the INT32 residue products.
template <bool CPLX, int NM>
__global__ __launch_bounds__(TPB) void crt_cheb_k(const int32_t* __restrict__ P, int64_t n,
                                                  int cols, CrtBasis B,
                                                  const int* __restrict__ sigma,
                                                  const int* __restrict__ tau, GemmArgs g) {
  const int64_t j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const int64_t plane = n * (int64_t)cols;
  const int64_t o = j * n + i;
  const int e = -(sigma[i] + tau[j]);
  const double* Xs = static_cast<const double*>(g.B);
  double* Cd = static_cast<double*>(g.C);
  const int64_t oc = i + j * g.ldc;
  if constexpr (CPLX) {
    int rr[NM], ri[NM];
#pragma unroll
    for (int t = 0; t < NM; ++t) {
      const int m = kModuli[t];
      const double minv = 1.0 / (double)m;
      const int p1 = ures32(P[(3 * t + 0) * plane + o], m, minv);
      const int p2 = ures32(P[(3 * t + 1) * plane + o], m, minv);
      const int p3 = ures32(P[(3 * t + 2) * plane + o], m, minv);
      rr[t] = (p1 - p2 + m) % m;
      ri[t] = (p3 - p1 - p2 + 2 * m) % m;
    }
    double vr = ldexp(garner<NM>(rr, B), e), vi = ldexp(garner<NM>(ri, B), e);
    vr = g.alpha * (vr - g.gamma * Xs[2 * (i + j * g.ldb)]);
    vi = g.alpha * (vi - g.gamma * Xs[2 * (i + j * g.ldb) + 1]);
    if (g.beta != 0.0) {
      vr += g.beta * Cd[2 * oc];
      vi += g.beta * Cd[2 * oc + 1];
    }
    if (g.colcoef) {
      const double cj = g.colcoef[j];
      const double* Fd = static_cast<const double*>(g.F);
      vr += cj * Fd[2 * (i + j * g.ldf)];
      vi += cj * Fd[2 * (i + j * g.ldf) + 1];
    }
    Cd[2 * oc] = vr;
    Cd[2 * oc + 1] = vi;
  } else {
    int r[NM];
#pragma unroll
    for (int t = 0; t < NM; ++t)
      r[t] = ures32(P[t * plane + o], kModuli[t], 1.0 / (double)kModuli[t]);
    double v = ldexp(garner<NM>(r, B), e);
    v = g.alpha * (v - g.gamma * Xs[i + j * g.ldb]);
    if (g.beta != 0.0) v += g.beta * Cd[oc];
    if (g.colcoef) v += g.colcoef[j] * static_cast<const double*>(g.F)[i + j * g.ldf];
    Cd[oc] = v;
  }
}

// The epilogue of one entry: out = alpha (c - gamma Xs) + beta out [+ cj F].
template <bool CPLX>
__device__ __forceinline__ void cheb_store(const GemmArgs& g, int64_t i, int64_t j, double vr,
                                           double vi) {
  const double* Xs = static_cast<const double*>(g.B);
  double* Cd = static_cast<double*>(g.C);
  const int64_t oc = i + j * g.ldc;
  if constexpr (CPLX) {
    vr = g.alpha * (vr - g.gamma * Xs[2 * (i + j * g.ldb)]);
    vi = g.alpha * (vi - g.gamma * Xs[2 * (i + j * g.ldb) + 1]);
    if (g.beta != 0.0) {
      vr += g.beta * Cd[2 * oc];
      vi += g.beta * Cd[2 * oc + 1];
    }
    if (g.colcoef) {
      const double cj = g.colcoef[j];
      const double* Fd = static_cast<const double*>(g.F);
      vr += cj * Fd[2 * (i + j * g.ldf)];
      vi += cj * Fd[2 * (i + j * g.ldf) + 1];
    }
    Cd[2 * oc] = vr;
    Cd[2 * oc + 1] = vi;
  } else {
    double v = g.alpha * (vr - g.gamma * Xs[i + j * g.ldb]);
    if (g.beta != 0.0) v += g.beta * Cd[oc];
    if (g.colcoef) v += g.colcoef[j] * static_cast<const double*>(g.F)[i + j * g.ldf];
    Cd[oc] = v;
  }
}

// Four consecutive rows per thread (n a multiple of 4): 16-byte loads of the
// INT32 products; the residues of the four entries are kept packed (one
// byte each) until each entry's reconstruction.
template <bool CPLX, int NM>
__global__ __launch_bounds__(TPB) void crt_cheb4_k(const int32_t* __restrict__ P, int64_t n,
                                                   int cols, CrtBasis B,
                                                   const int* __restrict__ sigma,
                                                   const int* __restrict__ tau, GemmArgs g) {
  typedef int i4v __attribute__((ext_vector_type(4)));
  const int64_t j = blockIdx.y;
  const int64_t i0 = 4 * ((int64_t)blockIdx.x * TPB + threadIdx.x);
  if (i0 >= n) return;
  const int64_t plane = n * (int64_t)cols;
  const int64_t o = j * n + i0;
  uint32_t pr[NM], pi[NM];
#pragma unroll
  for (int t = 0; t < NM; ++t) {
    const int m = kModuli[t];
    const double minv = 1.0 / (double)m;
    uint32_t wr = 0, wi = 0;
    if constexpr (CPLX) {
      const i4v a = *reinterpret_cast<const i4v*>(P + (3 * t + 0) * plane + o);
      const i4v b = *reinterpret_cast<const i4v*>(P + (3 * t + 1) * plane + o);
      const i4v c = *reinterpret_cast<const i4v*>(P + (3 * t + 2) * plane + o);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int p1 = ures32(a[e], m, minv), p2 = ures32(b[e], m, minv);
        const int p3 = ures32(c[e], m, minv);
        wr |= (uint32_t)((p1 - p2 + m) % m) << (8 * e);
        wi |= (uint32_t)((p3 - p1 - p2 + 2 * m) % m) << (8 * e);
      }
    } else {
      const i4v a = *reinterpret_cast<const i4v*>(P + t * plane + o);
#pragma unroll
      for (int e = 0; e < 4; ++e) wr |= (uint32_t)ures32(a[e], m, minv) << (8 * e);
    }
    pr[t] = wr;
    pi[t] = wi;
  }
  const int ej = tau[j];
  // one entry at a time (the reconstructions of four entries side by side
  // would hold four sets of digits)
#pragma unroll 1
  for (int e = 0; e < 4; ++e) {
    const int64_t i = i0 + e;
    const int sc = -(sigma[i] + ej);
    int r[NM];
#pragma unroll
    for (int t = 0; t < NM; ++t) r[t] = (int)((pr[t] >> (8 * e)) & 0xffu);
    const double vr = ldexp(garner<NM>(r, B), sc);
    double vi = 0.0;
    if constexpr (CPLX) {
#pragma unroll
      for (int t = 0; t < NM; ++t) r[t] = (int)((pi[t] >> (8 * e)) & 0xffu);
      vi = ldexp(garner<NM>(r, B), sc);
    }
    cheb_store<CPLX>(g, i, j, vr, vi);
  }
}

template <bool CPLX, int NM>
void launch_cheb(const int32_t* prod, int64_t n, int cols, const CrtBasis& B, const int* sigma,
                 const int* tau, const GemmArgs& g, hipStream_t st) {
  if (n % 4 == 0) {
    const dim3 grid((unsigned)((n / 4 + TPB - 1) / TPB), (unsigned)cols);
    hipLaunchKernelGGL((crt_cheb4_k<CPLX, NM>), grid, dim3(TPB), 0, st, prod, n, cols, B, sigma,
                       tau, g);
  } else {
    const dim3 grid((unsigned)((n + TPB - 1) / TPB), (unsigned)cols);
    hipLaunchKernelGGL((crt_cheb_k<CPLX, NM>), grid, dim3(TPB), 0, st, prod, n, cols, B, sigma,
                       tau, g);
  }
}

template <bool CPLX>
void launch_cheb_nm(const int32_t* prod, int64_t n, int cols, const CrtBasis& B,
                    const int* sigma, const int* tau, const GemmArgs& g, hipStream_t st) {
  switch (B.n_mod) {
    case 8: return launch_cheb<CPLX, 8>(prod, n, cols, B, sigma, tau, g, st);
    case 10: return launch_cheb<CPLX, 10>(prod, n, cols, B, sigma, tau, g, st);
    case 12: return launch_cheb<CPLX, 12>(prod, n, cols, B, sigma, tau, g, st);
    case 14: return launch_cheb<CPLX, 14>(prod, n, cols, B, sigma, tau, g, st);
    case 16: return launch_cheb<CPLX, 16>(prod, n, cols, B, sigma, tau, g, st);
  }
  throw Error(CHASE_ERR_ARG, "fp64_emulation: moduli must be 8, 10, 12, 14 or 16");
}

int inv_mod(int a, int m) {
  // extended Euclid; a and m coprime
  int t = 0, nt = 1, r = m, nr = ((a % m) + m) % m;
  while (nr != 0) {
    const int q = r / nr;
    int tmp = t - q * nt;
    t = nt;
    nt = tmp;
    tmp = r - q * nr;
    r = nr;
    nr = tmp;
  }
  return ((t % m) + m) % m;
}

}  // namespace

CrtBasis crt_basis(int n_mod, int64_t K, bool cplx) {
  CHASE_REQUIRE(n_mod == 8 || n_mod == 10 || n_mod == 12 || n_mod == 14 || n_mod == 16,
                "fp64_emulation: moduli must be 8, 10, 12, 14 or 16");
  CrtBasis b{};
  b.n_mod = n_mod;
  double log2M = 0.0;
  for (int t = 0; t < n_mod; ++t) {
    b.m[t] = kModuli[t];
    log2M += std::log2((double)kModuli[t]);
    // inverse of m_0 ... m_{t-1} modulo m_t
    int prod = 1;
    for (int s = 0; s < t; ++s) prod = (int)(((int64_t)prod * (kModuli[s] % kModuli[t])) % kModuli[t]);
    b.inv[t] = t == 0 ? 1 : inv_mod(prod, kModuli[t]);
  }
  // |C| <= 2 K 2^(pa + pb) (complex parts; real: K 2^(pa + pb)) must stay
  // below M / 2, one bit of margin
  const int total = (int)std::floor(log2M - 1.0 - 1.0 - std::log2((double)std::max<int64_t>(K, 1)) -
                                    (cplx ? 1.0 : 0.0));
  b.pa = std::min(52, total / 2);
  b.pb = std::min(52, total - b.pa);
  CHASE_REQUIRE(b.pa >= 16 && b.pb >= 16, "fp64_emulation: too few moduli for this size");
  return b;
}

namespace {
inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }
// byte offsets within the buffers: H planes | row exponents;
// block planes | INT32 products | column exponents
inline size_t h_planes_bytes(bool cplx, int64_t n, int n_mod) {
  return align256((size_t)(cplx ? 3 : 1) * n_mod * n * n);
}
inline size_t x_planes_bytes(bool cplx, int64_t n, int kmax, int n_mod) {
  return align256((size_t)(cplx ? 3 : 1) * n_mod * n * kmax);
}
inline size_t x_prod_bytes(bool cplx, int64_t n, int kmax, int n_mod) {
  return align256((size_t)(cplx ? 3 : 1) * n_mod * n * kmax * 4);
}
}  // namespace

size_t crt_h_bytes(bool cplx, int64_t n, int n_mod) {
  return h_planes_bytes(cplx, n, n_mod) + (size_t)n * 4;
}
size_t crt_x_bytes(bool cplx, int64_t n, int kmax, int n_mod) {
  return x_planes_bytes(cplx, n, kmax, n_mod) + x_prod_bytes(cplx, n, kmax, n_mod) +
         (size_t)kmax * 4 + 256;
}

void crt_prepare_h(bool cplx, const void* H, int64_t ldh, int64_t n, const CrtBasis& B,
                   void* hbuf, hipStream_t st) {
  CHASE_REQUIRE(n <= 65535, "fp64_emulation: n above 65535");
  int8_t* planes = static_cast<int8_t*>(hbuf);
  int* sigma = reinterpret_cast<int*>(planes + h_planes_bytes(cplx, n, B.n_mod));
  const double* Hd = static_cast<const double*>(H);
  const bool v4 = n % 4 == 0;
  const dim3 grid((unsigned)(((v4 ? n / 4 : n) + TPB - 1) / TPB), (unsigned)n);
  if (cplx) {
    hipLaunchKernelGGL(crt_rowexp_k<true>, dim3((unsigned)n), dim3(TPB), 0, st, Hd, ldh, n, B.pa,
                       sigma);
    if (v4)
      hipLaunchKernelGGL(crt_hplanes4_k<true>, grid, dim3(TPB), 0, st, Hd, ldh, n,
                         static_cast<const int*>(sigma), B, planes);
    else
      hipLaunchKernelGGL(crt_hplanes_k<true>, grid, dim3(TPB), 0, st, Hd, ldh, n,
                         static_cast<const int*>(sigma), B, planes);
  } else {
    hipLaunchKernelGGL(crt_rowexp_k<false>, dim3((unsigned)n), dim3(TPB), 0, st, Hd, ldh, n, B.pa,
                       sigma);
    if (v4)
      hipLaunchKernelGGL(crt_hplanes4_k<false>, grid, dim3(TPB), 0, st, Hd, ldh, n,
                         static_cast<const int*>(sigma), B, planes);
    else
      hipLaunchKernelGGL(crt_hplanes_k<false>, grid, dim3(TPB), 0, st, Hd, ldh, n,
                         static_cast<const int*>(sigma), B, planes);
  }
  CHASE_HIP(hipGetLastError());
}

void crt_cheb(bool cplx, const GemmArgs& g, const CrtBasis& B, const void* hbuf, void* xbuf,
              int kmax, rocblas_handle rb, hipStream_t st) {
  const int64_t n = g.M;
  const int cols = (int)g.N;
  CHASE_REQUIRE(g.K == n && cols >= 1 && cols <= kmax, "INT8 filter step: shape");
  const int P = (cplx ? 3 : 1) * B.n_mod;
  const int8_t* hplanes = static_cast<const int8_t*>(hbuf);
  const int* sigma = reinterpret_cast<const int*>(hplanes + h_planes_bytes(cplx, n, B.n_mod));
  int8_t* xplanes = static_cast<int8_t*>(xbuf);
  int32_t* prod =
      reinterpret_cast<int32_t*>(xplanes + x_planes_bytes(cplx, n, kmax, B.n_mod));
  int* tau = reinterpret_cast<int*>(reinterpret_cast<char*>(prod) +
                                    x_prod_bytes(cplx, n, kmax, B.n_mod));
  const double* Xs = static_cast<const double*>(g.B);
  const bool v4 = n % 4 == 0;
  const dim3 grid((unsigned)(((v4 ? n / 4 : n) + TPB - 1) / TPB), (unsigned)cols);
  if (cplx) {
    hipLaunchKernelGGL(crt_colexp_k<true>, dim3(cols), dim3(TPB), 0, st, Xs, g.ldb, n, B.pb, tau);
    if (v4)
      hipLaunchKernelGGL(crt_xplanes4_k<true>, grid, dim3(TPB), 0, st, Xs, g.ldb, n, cols,
                         static_cast<const int*>(tau), B, xplanes);
    else
      hipLaunchKernelGGL(crt_xplanes_k<true>, grid, dim3(TPB), 0, st, Xs, g.ldb, n, cols,
                         static_cast<const int*>(tau), B, xplanes);
  } else {
    hipLaunchKernelGGL(crt_colexp_k<false>, dim3(cols), dim3(TPB), 0, st, Xs, g.ldb, n, B.pb, tau);
    if (v4)
      hipLaunchKernelGGL(crt_xplanes4_k<false>, grid, dim3(TPB), 0, st, Xs, g.ldb, n, cols,
                         static_cast<const int*>(tau), B, xplanes);
    else
      hipLaunchKernelGGL(crt_xplanes_k<false>, grid, dim3(TPB), 0, st, Xs, g.ldb, n, cols,
                         static_cast<const int*>(tau), B, xplanes);
  }
  CHASE_HIP(hipGetLastError());
  // P exact integer products, one per (modulus, Gauss term): H planes are
  // row-major, i.e. the transposed operand of a column-major GEMM
  const int32_t one = 1, zero = 0;
  const rocblas_status rs = rocblas_gemm_strided_batched_ex(
      rb, rocblas_operation_transpose, rocblas_operation_none, n, cols, n, &one, hplanes,
      rocblas_datatype_i8_r, n, n * n, xplanes, rocblas_datatype_i8_r, n, n * (int64_t)cols,
      &zero, prod, rocblas_datatype_i32_r, n, n * (int64_t)cols, prod, rocblas_datatype_i32_r, n,
      n * (int64_t)cols, P, rocblas_datatype_i32_r, rocblas_gemm_algo_standard, 0, 0);
  if (rs != rocblas_status_success)
    throw Error(CHASE_ERR_HIP, std::string("rocblas INT8 GEMM: ") + rocblas_status_to_string(rs));
  if (cplx)
    launch_cheb_nm<true>(prod, n, cols, B, sigma, tau, g, st);
  else
    launch_cheb_nm<false>(prod, n, cols, B, sigma, tau, g, st);
  CHASE_HIP(hipGetLastError());
}

}  // namespace chase
