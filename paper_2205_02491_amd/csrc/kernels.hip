// Bandwidth-bound helper kernels of the ChASE hot path: block copies and
// column gathers (the degree sort of Algorithm 1), split-K reductions,
// Cholesky-QR scaling, residual-norm finishing, and the Lanczos block
// matrix-vector product with its wavefront reductions.
#include "common.h"

#include <algorithm>
#include <utility>

namespace chase {
namespace {

typedef double d2v __attribute__((ext_vector_type(2)));

constexpr int TPB = 256;

inline int blocks_for(int64_t work, int per_block, int cap = 65535 * 8) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

__global__ void fill_zero_k(uint32_t* p, int64_t words) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}
__global__ void fill_zero_bytes_k(unsigned char* p, int64_t bytes) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < bytes;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// one scalar = double; complex elements are 2 scalars (w = 2)
template <int W>
__global__ void copy_cols_k(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                            int64_t ldd, int64_t n, int64_t k, const int* __restrict__ perm) {
  const int64_t rows = n * W;
  for (int64_t j = blockIdx.y; j < k; j += gridDim.y) {
    const int64_t sj = perm ? perm[j] : j;
    const double* s = src + sj * lds * W;
    double* d = dst + j * ldd * W;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x)
      d[i] = s[i];
  }
}

template <bool CPLX>
__global__ void splitk_reduce_k(const double* __restrict__ ws, int splits, int64_t M, int64_t N,
                                double* __restrict__ C, int64_t ldc, bool herm, int tri_tile) {
  const int64_t total = M * N;
  const int W = CPLX ? 2 : 1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % M, j = e / M;
    // triangular products (Hermitian, square): tiles below the diagonal were
    // not computed; their entries are the conjugates of the mirrored ones
    const bool mirror = tri_tile > 0 && i / tri_tile > j / tri_tile;
    const bool diag = tri_tile > 0 && i / tri_tile == j / tri_tile;
    const int64_t src = mirror ? j + i * M : e;
    double sr = 0, si = 0;
    for (int z = 0; z < splits; ++z) {
      sr += ws[(z * total + src) * W];
      if (CPLX) si += ws[(z * total + src) * W + 1];
    }
    if (mirror) {
      si = -si;
    } else if (herm && (tri_tile == 0 || diag)) {
      // (S + S^H)/2 at (i, j): needs S(j, i) as well
      const int64_t et = j + i * M;
      double tr = 0, ti = 0;
      for (int z = 0; z < splits; ++z) {
        tr += ws[(z * total + et) * W];
        if (CPLX) ti += ws[(z * total + et) * W + 1];
      }
      sr = 0.5 * (sr + tr);
      si = 0.5 * (si - ti);
    }
    C[(i + j * ldc) * W] = sr;
    if (CPLX) C[(i + j * ldc) * W + 1] = si;
  }
}

template <bool CPLX>
__global__ void gram_diag_k(const double* __restrict__ S, int64_t lds, int64_t k, double* d,
                            int* flags) {
  const int W = CPLX ? 2 : 1;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < k;
       j += (int64_t)gridDim.x * blockDim.x) {
    const double s = S[(j + j * lds) * W];
    if (!(s > 0.0) || !isfinite(s)) {
      flags[0] = 1;
      d[j] = 1.0;
    } else {
      d[j] = 1.0 / sqrt(s);
    }
  }
}

template <bool CPLX>
__global__ void gram_apply_k(double* __restrict__ S, int64_t lds, int64_t k,
                             const double* __restrict__ d, double shift) {
  const int W = CPLX ? 2 : 1;
  const int64_t total = k * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % k, j = e / k;
    const double f = d[i] * d[j];
    double* p = S + (i + j * lds) * W;
    p[0] *= f;
    if (CPLX) p[1] *= f;
    if (i == j) {
      p[0] += shift;
      if (CPLX) p[1] = 0.0;
    }
  }
}

template <int W>
__global__ void add_diag_k(double* __restrict__ A, int64_t lda, int64_t k, double shift) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < k;
       j += (int64_t)gridDim.x * blockDim.x)
    A[(j + j * lda) * W] += shift;
}

template <bool CPLX>
__global__ void triu_rowscale_k(double* __restrict__ R, int64_t ldr, int64_t k,
                                const double* __restrict__ d) {
  const int W = CPLX ? 2 : 1;
  const int64_t total = k * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % k, j = e / k;
    double* p = R + (i + j * ldr) * W;
    if (i > j) {
      p[0] = 0.0;
      if (CPLX) p[1] = 0.0;
    } else {
      p[0] *= d[i];
      if (CPLX) p[1] *= d[i];
    }
  }
}

template <bool CPLX>
__global__ void diag_real_k(const double* __restrict__ A, int64_t lda, int64_t k, double* out) {
  const int W = CPLX ? 2 : 1;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < k;
       j += (int64_t)gridDim.x * blockDim.x)
    out[j] = A[(j + j * lda) * W];
}

__global__ void resid_finish_k(const double* __restrict__ partial, int tiles, int64_t N,
                               double inv_scale, double* __restrict__ res) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N;
       j += (int64_t)gridDim.x * blockDim.x) {
    double s = 0;
    for (int t = 0; t < tiles; ++t) s += partial[(int64_t)t * N + j];
    res[j] = sqrt(s) * inv_scale;
  }
}

template <bool CPLX>
__global__ void scale_cols_k(double* __restrict__ V, int64_t ldv, int64_t n, int64_t k,
                             const double* __restrict__ g) {
  const int W = CPLX ? 2 : 1;
  for (int64_t j = blockIdx.y; j < k; j += gridDim.y) {
    const double f = g[j];
    double* c = V + j * ldv * W;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * W;
         i += (int64_t)gridDim.x * blockDim.x)
      c[i] *= f;
  }
}

template <int W>
__global__ void axpby_cols_k(const double* __restrict__ a, const double* __restrict__ X, int64_t ldx,
                             const double* __restrict__ b, double* __restrict__ Y, int64_t ldy,
                             int64_t n, int64_t k) {
  for (int64_t j = blockIdx.y; j < k; j += gridDim.y) {
    const double aj = a ? a[j] : 1.0;
    const double* x = X + j * ldx * W;
    double* y = Y + j * ldy * W;
    if (b) {
      const double bj = b[j];
      for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * W;
           i += (int64_t)gridDim.x * blockDim.x)
        y[i] = aj * x[i] + bj * y[i];
    } else {
      for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * W;
           i += (int64_t)gridDim.x * blockDim.x)
        y[i] = aj * x[i];
    }
  }
}

template <int W>
__global__ void axpy_cols_k(double a, const double* __restrict__ X, int64_t ldx,
                            double* __restrict__ Y, int64_t ldy, int64_t n, int64_t k) {
  for (int64_t j = blockIdx.y; j < k; j += gridDim.y) {
    const double* x = X + j * ldx * W;
    double* y = Y + j * ldy * W;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * W;
         i += (int64_t)gridDim.x * blockDim.x)
      y[i] += a * x[i];
  }
}

// A = (A + A^H)/2, each unordered pair handled once (i <= j)
template <bool CPLX>
__global__ void herm_part_k(double* __restrict__ A, int64_t lda, int64_t n) {
  const int W = CPLX ? 2 : 1;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= j;
         i += (int64_t)gridDim.x * blockDim.x) {
      double* a = A + (i + j * lda) * W;
      double* b = A + (j + i * lda) * W;
      if (CPLX) {
        const double re = 0.5 * (a[0] + b[0]);
        const double im = 0.5 * (a[1] - b[1]);
        a[0] = re;
        a[1] = im;
        b[0] = re;
        b[1] = -im;
      } else {
        const double v = 0.5 * (a[0] + b[0]);
        a[0] = v;
        b[0] = v;
      }
    }
  }
}

__global__ void to_f32_k(const double* __restrict__ src, int64_t lds, float* __restrict__ dst,
                         int64_t rows_scalars, int64_t n, int W) {
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
    const double* s = src + j * lds * W;
    float* d = dst + j * rows_scalars;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows_scalars;
         i += (int64_t)gridDim.x * blockDim.x)
      d[i] = (float)s[i];
  }
}

__global__ void check_finite_k(const double* __restrict__ X, int64_t ldx, int64_t rows_scalars,
                               int64_t k, int W, int* flags) {
  for (int64_t j = blockIdx.y; j < k; j += gridDim.y) {
    const double* c = X + j * ldx * W;
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows_scalars;
         i += (int64_t)gridDim.x * blockDim.x)
      bad |= !isfinite(c[i]);
    if (bad) flags[0] = 1;
  }
}

// ------------------------------------------------------------------ start blocks
// Counter-based normal draws for start blocks the caller does not supply:
// scalar c of the stream (column-major, re/im interleaved) takes two
// uniforms from SplitMix64 (Steele, Lea and Flood, 2014: a Weyl sequence
// through a 64-bit finaliser) at counters 2c and 2c+1 of its key, and the
// Box-Muller transform turns them into one N(0, 1) value.
__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void fill_gaussian_k(double* __restrict__ X, int64_t ld_scalars, int64_t rows_scalars,
                                int64_t k, uint64_t key) {
  const int64_t total = rows_scalars * k;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < total;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = c / rows_scalars, i = c - j * rows_scalars;
    const uint64_t a = splitmix64(key + 2 * (uint64_t)c), b = splitmix64(key + 2 * (uint64_t)c + 1);
    const double u1 = (double)((a >> 11) + 1) * 0x1.0p-53;  // (0, 1]
    const double u2 = (double)(b >> 11) * 0x1.0p-53;        // [0, 1)
    X[i + j * ld_scalars] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
  }
}

// ------------------------------------------------------------------ debug checks
// Largest |A_ij - conj(A_ji)| (mode 0, square A) or |A_ij - delta_ij| (mode
// 1) into out[0] and largest |A_ij| into out[1], over 32 x 32 tiles staged
// through LDS so that both reads are coalesced.  out[] must start at zero;
// maxima of non-negative doubles are taken on their bit patterns.
template <bool CPLX>
__global__ __launch_bounds__(TPB) void max_defect_k(const double* __restrict__ A, int64_t lda,
                                                     int64_t n, int mode,
                                                     unsigned long long* out) {
  constexpr int W = CPLX ? 2 : 1;
  __shared__ double tile[32][33][W];
  __shared__ double red[2][TPB];
  const int64_t ti = (int64_t)blockIdx.x * 32, tj = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  double dmax = 0.0, amax = 0.0;
  if (mode == 0) {
    // tile (tj, ti) into LDS, read back transposed
    for (int r = ty; r < 32; r += 8) {
      const int64_t i = tj + tx, j = ti + r;
      for (int w = 0; w < W; ++w)
        tile[r][tx][w] = (i < n && j < n) ? A[(i + j * lda) * W + w] : 0.0;
    }
    __syncthreads();
  }
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = ti + tx, j = tj + r;
    if (i >= n || j >= n) continue;
    double re = A[(i + j * lda) * W], im = CPLX ? A[(i + j * lda) * W + 1] : 0.0;
    amax = fmax(amax, CPLX ? hypot(re, im) : fabs(re));
    if (mode == 0) {
      // A(j, i) = tile[tx][r]
      re -= tile[tx][r][0];
      if (CPLX) im += tile[tx][r][W - 1];
    } else if (i == j) {
      re -= 1.0;
    }
    dmax = fmax(dmax, CPLX ? hypot(re, im) : fabs(re));
  }
  red[0][threadIdx.x] = dmax;
  red[1][threadIdx.x] = amax;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(red[0][0]));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(red[1][0]));
  }
}

// ------------------------------------------------------------------ Lanczos
// Block matrix-vector product W = H Q for nv <= 8 vectors, H read once from
// HBM (column-major, coalesced along rows).  The columns of H are split over
// gridDim.y slices; each slice writes its partial sums, which the reduction
// kernel adds in a fixed order (deterministic).
constexpr int LZ_ROWS_PER_THREAD = 2;
constexpr int LZ_ROWS = TPB * LZ_ROWS_PER_THREAD;
constexpr int LZ_COLS_STAGE = 64;

template <bool CPLX, int NV>
__global__ __launch_bounds__(TPB) void lz_gemv_k(const double* __restrict__ H, int64_t ldh,
                                                 int64_t n, const double* __restrict__ Q,
                                                 double* __restrict__ part, int64_t cols_per) {
  // NV vectors (compile time: the accumulators stay in registers and the
  // occupancy high enough to keep HBM busy)
  const int W = CPLX ? 2 : 1;
  __shared__ double qs[LZ_COLS_STAGE][NV][2];
  const int64_t r0 = (int64_t)blockIdx.x * LZ_ROWS;
  const int64_t c0 = (int64_t)blockIdx.y * cols_per;
  const int64_t c1 = c0 + cols_per < n ? c0 + cols_per : n;
  double accr[LZ_ROWS_PER_THREAD][NV], acci[LZ_ROWS_PER_THREAD][NV];
#pragma unroll
  for (int r = 0; r < LZ_ROWS_PER_THREAD; ++r)
#pragma unroll
    for (int v = 0; v < NV; ++v) accr[r][v] = acci[r][v] = 0.0;

  for (int64_t cs = c0; cs < c1; cs += LZ_COLS_STAGE) {
    const int ncs = (int)(c1 - cs < LZ_COLS_STAGE ? c1 - cs : LZ_COLS_STAGE);
    __syncthreads();
    for (int e = threadIdx.x; e < ncs * NV; e += TPB) {
      const int c = e % ncs, v = e / ncs;
      const double* q = Q + ((cs + c) + (int64_t)v * n) * W;
      qs[c][v][0] = q[0];
      qs[c][v][1] = CPLX ? q[1] : 0.0;
    }
    __syncthreads();
    // 8 columns of H per round: 16 independent 16-byte loads in flight per
    // thread before the arithmetic that consumes them (16 columns or more
    // workgroups measured no faster).  H is streamed once per step, far
    // larger than the caches: nontemporal loads (the same column-block read
    // pattern alone: 6.9 TB/s with them, 6.1 TB/s without, at n=20000).
    constexpr int CU = 8;
    int c = 0;
    for (; c + CU <= ncs; c += CU) {
      double hr[CU][LZ_ROWS_PER_THREAD], hi[CU][LZ_ROWS_PER_THREAD];
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        const double* hc = H + (cs + c + u) * ldh * W;
#pragma unroll
        for (int r = 0; r < LZ_ROWS_PER_THREAD; ++r) {
          const int64_t i = r0 + threadIdx.x + r * TPB;
          hr[u][r] = 0.0;
          hi[u][r] = 0.0;
          if (i < n) {
            if (CPLX) {
              const d2v h = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(hc + 2 * i));
              hr[u][r] = h.x;
              hi[u][r] = h.y;
            } else {
              hr[u][r] = __builtin_nontemporal_load(hc + i);
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < CU; ++u)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double qr = qs[c + u][v][0], qi = qs[c + u][v][1];
#pragma unroll
          for (int r = 0; r < LZ_ROWS_PER_THREAD; ++r) {
            accr[r][v] += hr[u][r] * qr - hi[u][r] * qi;
            if (CPLX) acci[r][v] += hr[u][r] * qi + hi[u][r] * qr;
          }
        }
    }
    for (; c < ncs; ++c) {
      const double* hc = H + (cs + c) * ldh * W;
#pragma unroll
      for (int r = 0; r < LZ_ROWS_PER_THREAD; ++r) {
        const int64_t i = r0 + threadIdx.x + r * TPB;
        if (i < n) {
          double hr, hi = 0.0;
          if (CPLX) {
            const d2v h = *reinterpret_cast<const d2v*>(hc + 2 * i);
            hr = h.x;
            hi = h.y;
          } else {
            hr = hc[i];
          }
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const double qr = qs[c][v][0], qi = qs[c][v][1];
            accr[r][v] += hr * qr - hi * qi;
            if (CPLX) acci[r][v] += hr * qi + hi * qr;
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < LZ_ROWS_PER_THREAD; ++r) {
    const int64_t i = r0 + threadIdx.x + r * TPB;
    if (i < n) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double* p = part + (((int64_t)blockIdx.y * NV + v) * n + i) * W;
        p[0] = accr[r][v];
        if (CPLX) p[1] = acci[r][v];
      }
    }
  }
}

// block-wide sum of nv values per thread into out[blockIdx.x*nv + v]
__device__ inline void block_sum_store(double* vals, int nv, double* out) {
  __shared__ double red[TPB / 64][8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int v = 0; v < nv; ++v) {
    double x = vals[v];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[wave][v] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    double s = 0;
    for (int w = 0; w < TPB / 64; ++w) s += red[w][threadIdx.x];
    out[(int64_t)blockIdx.x * nv + threadIdx.x] = s;
  }
}

// W = sum of gemv partials - beta_prev * Q_prev ; dotp = Re(Q_cur^H W) partials
template <bool CPLX>
__global__ __launch_bounds__(TPB) void lz_reduce_k(const double* __restrict__ part, int splits,
                                                   int64_t n, int nv,
                                                   const double* __restrict__ qprev,
                                                   const double* __restrict__ qcur,
                                                   const double* __restrict__ beta_prev,
                                                   double* __restrict__ w, double* dotp) {
  const int W = CPLX ? 2 : 1;
  double dots[8];
  for (int v = 0; v < 8; ++v) dots[v] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    for (int v = 0; v < nv; ++v) {
      double sr = 0, si = 0;
      for (int z = 0; z < splits; ++z) {
        const double* p = part + (((int64_t)z * nv + v) * n + i) * W;
        sr += p[0];
        if (CPLX) si += p[1];
      }
      const int64_t o = (i + (int64_t)v * n) * W;
      const double bp = beta_prev ? beta_prev[v] : 0.0;
      sr -= bp * qprev[o];
      if (CPLX) si -= bp * qprev[o + 1];
      w[o] = sr;
      if (CPLX) w[o + 1] = si;
      dots[v] += qcur[o] * sr + (CPLX ? qcur[o + 1] * si : 0.0);
    }
  }
  block_sum_store(dots, nv, dotp);
}

// alpha = sum(dotp); W -= alpha * Q_cur (skipped when with_alpha == 0);
// nrmp = partial ||W||^2
template <bool CPLX>
__global__ __launch_bounds__(TPB) void lz_orth_k(const double* __restrict__ dotp, int nblk,
                                                 int64_t n, int nv, int with_alpha,
                                                 const double* __restrict__ qcur,
                                                 double* __restrict__ w, double* alpha_out,
                                                 double* nrmp) {
  const int W = CPLX ? 2 : 1;
  double alpha[8], nrm[8];
  for (int v = 0; v < 8; ++v) {
    alpha[v] = 0.0;
    nrm[v] = 0.0;
  }
  if (with_alpha) {
    for (int v = 0; v < nv; ++v) {
      double s = 0;
      for (int b = 0; b < nblk; ++b) s += dotp[(int64_t)b * nv + v];
      alpha[v] = s;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < nv) alpha_out[threadIdx.x] = alpha[threadIdx.x];
  }
  for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    for (int v = 0; v < nv; ++v) {
      const int64_t o = (i + (int64_t)v * n) * W;
      double xr = w[o], xi = CPLX ? w[o + 1] : 0.0;
      if (with_alpha) {
        xr -= alpha[v] * qcur[o];
        if (CPLX) xi -= alpha[v] * qcur[o + 1];
        w[o] = xr;
        if (CPLX) w[o + 1] = xi;
      }
      nrm[v] += xr * xr + xi * xi;
    }
  }
  block_sum_store(nrm, nv, nrmp);
}

// beta = sqrt(sum(nrmp)); Q_next = W / beta (0 if beta == 0)
template <bool CPLX>
__global__ __launch_bounds__(TPB) void lz_normalize_k(const double* __restrict__ nrmp, int nblk,
                                                      int64_t n, int nv,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ qnext,
                                                      double* beta_out) {
  const int W = CPLX ? 2 : 1;
  double inv[8];
  for (int v = 0; v < nv; ++v) {
    double s = 0;
    for (int b = 0; b < nblk; ++b) s += nrmp[(int64_t)b * nv + v];
    const double beta = sqrt(s);
    inv[v] = beta > 0.0 ? 1.0 / beta : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && beta_out) beta_out[v] = beta;
  }
  for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    for (int v = 0; v < nv; ++v) {
      const int64_t o = (i + (int64_t)v * n) * W;
      qnext[o] = w[o] * inv[v];
      if (CPLX) qnext[o + 1] = w[o + 1] * inv[v];
    }
  }
}

// ------------------------------------------------------------------ CG helpers
// (eigenvector adjoint: batched conjugate gradients, one system per column)
// Block-wide sum of one value per thread (fixed order: deterministic).
__device__ inline double block_sum1(double x) {
  __shared__ double red1[TPB / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  __syncthreads();
  if (lane == 0) red1[wave] = x;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < TPB / 64; ++w) s += red1[w];
  return s;
}

// out[j] = Re(x_j^H y_j); one block per column
template <int W>
__global__ __launch_bounds__(TPB) void col_dots_k(const double* __restrict__ X, int64_t ldx,
                                                  const double* __restrict__ Y, int64_t ldy,
                                                  int64_t n, double* out) {
  const int64_t j = blockIdx.x;
  const double* x = X + j * ldx * W;
  const double* y = Y + j * ldy * W;
  double s = 0;
  for (int64_t i = threadIdx.x; i < n * W; i += TPB) s += x[i] * y[i];
  s = block_sum1(s);
  if (threadIdx.x == 0) out[j] = s;
}

// A column is live while rr > tol2 rr0 and pq > 0.  Iterating a converged
// column on rounding-level residuals makes p^H A p noise and alpha blow up,
// so converged (or broken-down) columns are frozen.
__device__ inline bool cg_live(const double* rr, const double* rr0, const double* pq, double tol2,
                               int64_t j) {
  return rr[j] > tol2 * rr0[j] && pq[j] > 0.0;
}

// live columns: alpha = rr / pq; x += alpha p; r -= alpha q; rr_new = |r|^2
// (frozen columns: rr_new = rr, nothing else changes)
template <int W>
__global__ __launch_bounds__(TPB) void cg_step_k(double* __restrict__ X, double* __restrict__ R,
                                                 const double* __restrict__ P,
                                                 const double* __restrict__ Q, int64_t ld,
                                                 int64_t n, const double* rr, const double* rr0,
                                                 const double* pq, double tol2, double* rr_new) {
  const int64_t j = blockIdx.x;
  if (!cg_live(rr, rr0, pq, tol2, j)) {
    if (threadIdx.x == 0) rr_new[j] = rr[j];
    return;
  }
  const double a = rr[j] / pq[j];
  double* x = X + j * ld * W;
  double* r = R + j * ld * W;
  const double* p = P + j * ld * W;
  const double* q = Q + j * ld * W;
  double s = 0;
  for (int64_t i = threadIdx.x; i < n * W; i += TPB) {
    x[i] += a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  s = block_sum1(s);
  if (threadIdx.x == 0) rr_new[j] = s;
}

// live columns (same test as cg_step_k, on the values before the step):
// beta = rr_new / rr; p = r + beta p; rr = rr_new
template <int W>
__global__ __launch_bounds__(TPB) void cg_dir_k(double* __restrict__ P,
                                                const double* __restrict__ R, int64_t ld,
                                                int64_t n, double* rr, const double* rr0,
                                                const double* pq, double tol2,
                                                const double* rr_new) {
  const int64_t j = blockIdx.x;
  if (!cg_live(rr, rr0, pq, tol2, j)) return;
  const double b = rr_new[j] / rr[j];
  double* p = P + j * ld * W;
  const double* r = R + j * ld * W;
  for (int64_t i = threadIdx.x; i < n * W; i += TPB) p[i] = r[i] + b * p[i];
  __syncthreads();
  if (threadIdx.x == 0) rr[j] = rr_new[j];
}

// E(i, j) = (M(i, j) - conj(M(j, i))) / (2 (lam_j - lam_i)) for i != j with
// distinct eigenvalues, else 0 (k x k)
template <int W>
__global__ void sym_divdiff_k(const double* __restrict__ M, int64_t ldm,
                              const double* __restrict__ lam, int64_t k, double* __restrict__ E,
                              int64_t lde) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < k * k;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % k, j = idx / k;
    const double d = lam[j] - lam[i];
    const double scale = fmax(fabs(lam[i]), fabs(lam[j])) + 1e-300;
    double er = 0.0, ei = 0.0;
    if (i != j && fabs(d) > 1e-14 * scale) {
      const double* mij = M + (i + j * ldm) * W;
      const double* mji = M + (j + i * ldm) * W;
      er = (mij[0] - mji[0]) / (2.0 * d);
      if (W == 2) ei = (mij[1] + mji[1]) / (2.0 * d);
    }
    double* e = E + (i + j * lde) * W;
    e[0] = er;
    if (W == 2) e[1] = ei;
  }
}

constexpr int LZ_VEC_BLOCKS = 128;

// Column splits of the block GEMV: about 512 workgroups, two per CU of the
// 256-CU MI355X, all resident at once (each streams a long range of
// columns).  Measured at n=20000 with nontemporal loads: 6.7-6.9 TB/s with
// 480 workgroups, 5.9 TB/s with ~2048 (two rounds of resident workgroups).
int lz_splits(int64_t n) {
  const int64_t row_blocks = (n + LZ_ROWS - 1) / LZ_ROWS;
  int64_t s = 512 / row_blocks;
  const int64_t smax = (n + 63) / 64;
  if (s > smax) s = smax;
  if (s > 64) s = 64;
  if (s < 1) s = 1;
  return (int)s;
}

}  // namespace

// ------------------------------------------------------------------ host launchers
void fill_zero(void* p, int64_t bytes, hipStream_t st) {
  if (bytes <= 0) return;
  if (bytes % 4 == 0 && (reinterpret_cast<uintptr_t>(p) & 3) == 0)
    hipLaunchKernelGGL(fill_zero_k, dim3(blocks_for(bytes / 4, TPB * 4, 4096)), dim3(TPB), 0, st,
                       static_cast<uint32_t*>(p), bytes / 4);
  else
    hipLaunchKernelGGL(fill_zero_bytes_k, dim3(blocks_for(bytes, TPB * 4, 4096)), dim3(TPB), 0,
                       st, static_cast<unsigned char*>(p), bytes);
  CHASE_HIP(hipGetLastError());
}

static void copy_impl(bool cplx, const void* src, int64_t lds, void* dst, int64_t ldd, int64_t n,
                      int64_t k, const int* perm, hipStream_t st) {
  if (n <= 0 || k <= 0) return;
  const int64_t rows = n * (cplx ? 2 : 1);
  dim3 grid(blocks_for(rows, TPB * 4, 64), (unsigned)(k < 65535 ? k : 65535));
  if (cplx)
    hipLaunchKernelGGL(copy_cols_k<2>, grid, dim3(TPB), 0, st, static_cast<const double*>(src),
                       lds, static_cast<double*>(dst), ldd, n, k, perm);
  else
    hipLaunchKernelGGL(copy_cols_k<1>, grid, dim3(TPB), 0, st, static_cast<const double*>(src),
                       lds, static_cast<double*>(dst), ldd, n, k, perm);
  CHASE_HIP(hipGetLastError());
}

void copy_cols(bool cplx, const void* src, int64_t lds, void* dst, int64_t ldd, int64_t n,
               int64_t k, hipStream_t st) {
  copy_impl(cplx, src, lds, dst, ldd, n, k, nullptr, st);
}

void gather_cols(bool cplx, const void* src, int64_t lds, void* dst, int64_t ldd, int64_t n,
                 int64_t k, const int* perm_dev, hipStream_t st) {
  copy_impl(cplx, src, lds, dst, ldd, n, k, perm_dev, st);
}

void splitk_reduce(bool cplx, const void* ws, int splits, int64_t M, int64_t N, void* C,
                   int64_t ldc, bool herm, hipStream_t st, int tri_tile) {
  CHASE_REQUIRE(tri_tile == 0 || (herm && M == N), "triangular reduction of a non-Hermitian product");
  const int nb = blocks_for(M * N, TPB, 8192);
  if (cplx)
    hipLaunchKernelGGL(splitk_reduce_k<true>, dim3(nb), dim3(TPB), 0, st,
                       static_cast<const double*>(ws), splits, M, N, static_cast<double*>(C),
                       ldc, herm, tri_tile);
  else
    hipLaunchKernelGGL(splitk_reduce_k<false>, dim3(nb), dim3(TPB), 0, st,
                       static_cast<const double*>(ws), splits, M, N, static_cast<double*>(C),
                       ldc, herm, tri_tile);
  CHASE_HIP(hipGetLastError());
}

void gram_scale(bool cplx, void* S, int64_t lds, int64_t k, double shift, double* d, int* flags,
                hipStream_t st) {
  const int nb1 = blocks_for(k, TPB, 1024);
  const int nb2 = blocks_for(k * k, TPB, 8192);
  if (cplx) {
    hipLaunchKernelGGL(gram_diag_k<true>, dim3(nb1), dim3(TPB), 0, st,
                       static_cast<const double*>(S), lds, k, d, flags);
    hipLaunchKernelGGL(gram_apply_k<true>, dim3(nb2), dim3(TPB), 0, st, static_cast<double*>(S),
                       lds, k, d, shift);
  } else {
    hipLaunchKernelGGL(gram_diag_k<false>, dim3(nb1), dim3(TPB), 0, st,
                       static_cast<const double*>(S), lds, k, d, flags);
    hipLaunchKernelGGL(gram_apply_k<false>, dim3(nb2), dim3(TPB), 0, st, static_cast<double*>(S),
                       lds, k, d, shift);
  }
  CHASE_HIP(hipGetLastError());
}

void add_diag(bool cplx, void* A, int64_t lda, int64_t k, double shift, hipStream_t st) {
  const int nb = blocks_for(k, TPB, 1024);
  if (cplx)
    hipLaunchKernelGGL(add_diag_k<2>, dim3(nb), dim3(TPB), 0, st, static_cast<double*>(A), lda, k,
                       shift);
  else
    hipLaunchKernelGGL(add_diag_k<1>, dim3(nb), dim3(TPB), 0, st, static_cast<double*>(A), lda, k,
                       shift);
  CHASE_HIP(hipGetLastError());
}

void triu_rowscale(bool cplx, void* R, int64_t ldr, int64_t k, const double* d, hipStream_t st) {
  const int nb = blocks_for(k * k, TPB, 8192);
  if (cplx)
    hipLaunchKernelGGL(triu_rowscale_k<true>, dim3(nb), dim3(TPB), 0, st,
                       static_cast<double*>(R), ldr, k, d);
  else
    hipLaunchKernelGGL(triu_rowscale_k<false>, dim3(nb), dim3(TPB), 0, st,
                       static_cast<double*>(R), ldr, k, d);
  CHASE_HIP(hipGetLastError());
}

void diag_real(bool cplx, const void* A, int64_t lda, int64_t k, double* out, hipStream_t st) {
  const int nb = blocks_for(k, TPB, 1024);
  if (cplx)
    hipLaunchKernelGGL(diag_real_k<true>, dim3(nb), dim3(TPB), 0, st,
                       static_cast<const double*>(A), lda, k, out);
  else
    hipLaunchKernelGGL(diag_real_k<false>, dim3(nb), dim3(TPB), 0, st,
                       static_cast<const double*>(A), lda, k, out);
  CHASE_HIP(hipGetLastError());
}

void resid_finish(const double* partial, int tiles, int64_t N, double inv_scale, double* res,
                  hipStream_t st) {
  hipLaunchKernelGGL(resid_finish_k, dim3(blocks_for(N, TPB, 1024)), dim3(TPB), 0, st, partial,
                     tiles, N, inv_scale, res);
  CHASE_HIP(hipGetLastError());
}

void scale_cols(bool cplx, void* V, int64_t ldv, int64_t n, int64_t k, const double* g,
                hipStream_t st) {
  if (n <= 0 || k <= 0) return;
  dim3 grid(blocks_for(n * (cplx ? 2 : 1), TPB * 4, 64), (unsigned)(k < 65535 ? k : 65535));
  if (cplx)
    hipLaunchKernelGGL(scale_cols_k<true>, grid, dim3(TPB), 0, st, static_cast<double*>(V), ldv,
                       n, k, g);
  else
    hipLaunchKernelGGL(scale_cols_k<false>, grid, dim3(TPB), 0, st, static_cast<double*>(V), ldv,
                       n, k, g);
  CHASE_HIP(hipGetLastError());
}

void axpby_cols(bool cplx, const double* a, const void* X, int64_t ldx, const double* b, void* Y,
                int64_t ldy, int64_t n, int64_t k, hipStream_t st) {
  if (n <= 0 || k <= 0) return;
  dim3 grid(blocks_for(n * (cplx ? 2 : 1), TPB * 4, 64), (unsigned)(k < 65535 ? k : 65535));
  if (cplx)
    hipLaunchKernelGGL(axpby_cols_k<2>, grid, dim3(TPB), 0, st, a, static_cast<const double*>(X),
                       ldx, b, static_cast<double*>(Y), ldy, n, k);
  else
    hipLaunchKernelGGL(axpby_cols_k<1>, grid, dim3(TPB), 0, st, a, static_cast<const double*>(X),
                       ldx, b, static_cast<double*>(Y), ldy, n, k);
  CHASE_HIP(hipGetLastError());
}

void axpy_cols(bool cplx, double a, const void* X, int64_t ldx, void* Y, int64_t ldy, int64_t n,
               int64_t k, hipStream_t st) {
  if (n <= 0 || k <= 0) return;
  dim3 grid(blocks_for(n * (cplx ? 2 : 1), TPB * 4, 64), (unsigned)(k < 65535 ? k : 65535));
  if (cplx)
    hipLaunchKernelGGL(axpy_cols_k<2>, grid, dim3(TPB), 0, st, a, static_cast<const double*>(X),
                       ldx, static_cast<double*>(Y), ldy, n, k);
  else
    hipLaunchKernelGGL(axpy_cols_k<1>, grid, dim3(TPB), 0, st, a, static_cast<const double*>(X),
                       ldx, static_cast<double*>(Y), ldy, n, k);
  CHASE_HIP(hipGetLastError());
}

void herm_part(bool cplx, void* A, int64_t lda, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  dim3 grid(blocks_for(n, TPB, 64), (unsigned)(n < 65535 ? n : 65535));
  if (cplx)
    hipLaunchKernelGGL(herm_part_k<true>, grid, dim3(TPB), 0, st, static_cast<double*>(A), lda, n);
  else
    hipLaunchKernelGGL(herm_part_k<false>, grid, dim3(TPB), 0, st, static_cast<double*>(A), lda,
                       n);
  CHASE_HIP(hipGetLastError());
}

void to_f32(bool cplx, const void* src, int64_t lds, void* dst, int64_t n, hipStream_t st) {
  const int W = cplx ? 2 : 1;
  dim3 grid(blocks_for(n * W, TPB * 4, 64), (unsigned)(n < 65535 ? n : 65535));
  hipLaunchKernelGGL(to_f32_k, grid, dim3(TPB), 0, st, static_cast<const double*>(src), lds,
                     static_cast<float*>(dst), n * W, n, W);
  CHASE_HIP(hipGetLastError());
}

void fill_gaussian(bool cplx, void* X, int64_t ldx, int64_t n, int64_t k, uint64_t seed,
                   uint64_t stream_id, hipStream_t st) {
  if (n <= 0 || k <= 0) return;
  const int W = cplx ? 2 : 1;
  // one key per (seed, stream), scrambled by the same (bijective) finaliser:
  // distinct pairs give distinct keys, and two streams' counter ranges
  // (below 2^41 for any block the library draws) overlap with probability
  // about 2^-22
  uint64_t z = seed ^ (stream_id << 32) ^ 0xD1B54A32D192ED03ull;
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  const uint64_t key = z ^ (z >> 31);
  hipLaunchKernelGGL(fill_gaussian_k, dim3(blocks_for(n * W * k, TPB * 4, 65536)), dim3(TPB), 0,
                     st, static_cast<double*>(X), ldx * W, n * W, k, key);
  CHASE_HIP(hipGetLastError());
}

void max_defect(bool cplx, const void* A, int64_t lda, int64_t n, int mode, double* out2,
                hipStream_t st) {
  fill_zero(out2, 2 * sizeof(double), st);
  if (n <= 0) return;
  const unsigned t = (unsigned)((n + 31) / 32);
  CHASE_REQUIRE(t <= 65535, "matrix too large for the debug check");
  if (cplx)
    hipLaunchKernelGGL(max_defect_k<true>, dim3(t, t), dim3(TPB), 0, st,
                       static_cast<const double*>(A), lda, n, mode,
                       reinterpret_cast<unsigned long long*>(out2));
  else
    hipLaunchKernelGGL(max_defect_k<false>, dim3(t, t), dim3(TPB), 0, st,
                       static_cast<const double*>(A), lda, n, mode,
                       reinterpret_cast<unsigned long long*>(out2));
  CHASE_HIP(hipGetLastError());
}

void check_finite(bool cplx, const void* X, int64_t ldx, int64_t n, int64_t k, int* flags,
                  hipStream_t st) {
  if (n <= 0 || k <= 0) return;
  const int W = cplx ? 2 : 1;
  dim3 grid(blocks_for(n * W, TPB * 4, 64), (unsigned)(k < 65535 ? k : 65535));
  hipLaunchKernelGGL(check_finite_k, grid, dim3(TPB), 0, st, static_cast<const double*>(X), ldx,
                     n * W, k, W, flags);
  CHASE_HIP(hipGetLastError());
}

void col_dots(bool cplx, const void* X, int64_t ldx, const void* Y, int64_t ldy, int64_t n,
              int64_t k, double* out, hipStream_t st) {
  if (k <= 0) return;
  if (cplx)
    hipLaunchKernelGGL(col_dots_k<2>, dim3((unsigned)k), dim3(TPB), 0, st,
                       static_cast<const double*>(X), ldx, static_cast<const double*>(Y), ldy, n,
                       out);
  else
    hipLaunchKernelGGL(col_dots_k<1>, dim3((unsigned)k), dim3(TPB), 0, st,
                       static_cast<const double*>(X), ldx, static_cast<const double*>(Y), ldy, n,
                       out);
  CHASE_HIP(hipGetLastError());
}

void cg_step(bool cplx, void* X, void* R, const void* P, const void* Q, int64_t ld, int64_t n,
             int64_t k, const double* rr, const double* rr0, const double* pq, double tol2,
             double* rr_new, hipStream_t st) {
  if (k <= 0) return;
  if (cplx)
    hipLaunchKernelGGL(cg_step_k<2>, dim3((unsigned)k), dim3(TPB), 0, st, static_cast<double*>(X),
                       static_cast<double*>(R), static_cast<const double*>(P),
                       static_cast<const double*>(Q), ld, n, rr, rr0, pq, tol2, rr_new);
  else
    hipLaunchKernelGGL(cg_step_k<1>, dim3((unsigned)k), dim3(TPB), 0, st, static_cast<double*>(X),
                       static_cast<double*>(R), static_cast<const double*>(P),
                       static_cast<const double*>(Q), ld, n, rr, rr0, pq, tol2, rr_new);
  CHASE_HIP(hipGetLastError());
}

void cg_dir(bool cplx, void* P, const void* R, int64_t ld, int64_t n, int64_t k, double* rr,
            const double* rr0, const double* pq, double tol2, const double* rr_new,
            hipStream_t st) {
  if (k <= 0) return;
  if (cplx)
    hipLaunchKernelGGL(cg_dir_k<2>, dim3((unsigned)k), dim3(TPB), 0, st, static_cast<double*>(P),
                       static_cast<const double*>(R), ld, n, rr, rr0, pq, tol2, rr_new);
  else
    hipLaunchKernelGGL(cg_dir_k<1>, dim3((unsigned)k), dim3(TPB), 0, st, static_cast<double*>(P),
                       static_cast<const double*>(R), ld, n, rr, rr0, pq, tol2, rr_new);
  CHASE_HIP(hipGetLastError());
}

void sym_divdiff(bool cplx, const void* M, int64_t ldm, const double* lam, int64_t k, void* E,
                 int64_t lde, hipStream_t st) {
  if (k <= 0) return;
  const unsigned blocks = (unsigned)blocks_for(k * k, TPB, 4096);
  if (cplx)
    hipLaunchKernelGGL(sym_divdiff_k<2>, dim3(blocks), dim3(TPB), 0, st,
                       static_cast<const double*>(M), ldm, lam, k, static_cast<double*>(E), lde);
  else
    hipLaunchKernelGGL(sym_divdiff_k<1>, dim3(blocks), dim3(TPB), 0, st,
                       static_cast<const double*>(M), ldm, lam, k, static_cast<double*>(E), lde);
  CHASE_HIP(hipGetLastError());
}

size_t lanczos_bytes(bool cplx, int64_t n, int nv, int steps, int* max_splits) {
  const int W = cplx ? 2 : 1;
  const int s = lz_splits(n);
  if (max_splits) *max_splits = s;
  size_t b = 0;
  b += 3 * (size_t)n * nv * W * 8;            // q_prev, q_cur, w
  b += (size_t)s * nv * n * W * 8;            // gemv partials
  b += 2 * (size_t)LZ_VEC_BLOCKS * nv * 8;    // dot / norm partials
  b += 2 * (size_t)steps * nv * 8;            // alpha, beta
  return b;
}

void lanczos_run(bool cplx, const void* Hv, int64_t ldh, int64_t n, const void* Sv, int nv,
                 int steps, LanczosBufs& b, hipStream_t st) {
  const int W = cplx ? 2 : 1;
  const double* H = static_cast<const double*>(Hv);
  double* qprev = static_cast<double*>(b.q_prev);
  double* qcur = static_cast<double*>(b.q_cur);
  double* w = static_cast<double*>(b.w);
  double* part = static_cast<double*>(b.wpart);
  const int splits = b.max_splits;
  const int64_t cols_per = (n + splits - 1) / splits;
  const int row_blocks = (int)((n + LZ_ROWS - 1) / LZ_ROWS);
  const int vb = (int)std::min<int64_t>(LZ_VEC_BLOCKS, (n + TPB - 1) / TPB);

  // q_1 = s / ||s|| ; q_0 = 0
  if (Sv != w)
    CHASE_HIP(hipMemcpyAsync(w, Sv, (size_t)n * nv * W * 8, hipMemcpyDeviceToDevice, st));
  fill_zero(qprev, (int64_t)n * nv * W * 8, st);
  auto orth = [&](int with_alpha, double* alpha_out) {
    if (cplx)
      hipLaunchKernelGGL(lz_orth_k<true>, dim3(vb), dim3(TPB), 0, st, b.dotp, vb, n, nv,
                         with_alpha, qcur, w, alpha_out, b.nrmp);
    else
      hipLaunchKernelGGL(lz_orth_k<false>, dim3(vb), dim3(TPB), 0, st, b.dotp, vb, n, nv,
                         with_alpha, qcur, w, alpha_out, b.nrmp);
  };
  auto normalize = [&](double* dst, double* beta_out) {
    if (cplx)
      hipLaunchKernelGGL(lz_normalize_k<true>, dim3(vb), dim3(TPB), 0, st, b.nrmp, vb, n, nv, w,
                         dst, beta_out);
    else
      hipLaunchKernelGGL(lz_normalize_k<false>, dim3(vb), dim3(TPB), 0, st, b.nrmp, vb, n, nv, w,
                         dst, beta_out);
  };
  auto gemv = [&](const double* q) {
#define CHASE_LZ_GEMV(NVC)                                                                   \
  if (cplx)                                                                                \
    hipLaunchKernelGGL((lz_gemv_k<true, NVC>), dim3(row_blocks, splits), dim3(TPB), 0, st, H, \
                       ldh, n, q, part, cols_per);                                          \
  else                                                                                     \
    hipLaunchKernelGGL((lz_gemv_k<false, NVC>), dim3(row_blocks, splits), dim3(TPB), 0, st,   \
                       H, ldh, n, q, part, cols_per);
    switch (nv) {
      case 1: CHASE_LZ_GEMV(1) break;
      case 2: CHASE_LZ_GEMV(2) break;
      case 3: CHASE_LZ_GEMV(3) break;
      case 4: CHASE_LZ_GEMV(4) break;
      case 5: CHASE_LZ_GEMV(5) break;
      case 6: CHASE_LZ_GEMV(6) break;
      case 7: CHASE_LZ_GEMV(7) break;
      default: CHASE_LZ_GEMV(8) break;
    }
#undef CHASE_LZ_GEMV
  };
  orth(0, nullptr);
  normalize(qcur, nullptr);
  for (int j = 0; j < steps; ++j) {
    if (b.gemv_ev) CHASE_HIP(hipEventRecord(b.gemv_ev[2 * j], st));
    gemv(qcur);
    if (b.gemv_ev) CHASE_HIP(hipEventRecord(b.gemv_ev[2 * j + 1], st));
    const double* bprev = j > 0 ? b.beta + (int64_t)(j - 1) * nv : nullptr;
    if (cplx)
      hipLaunchKernelGGL(lz_reduce_k<true>, dim3(vb), dim3(TPB), 0, st, part, splits, n, nv,
                         qprev, qcur, bprev, w, b.dotp);
    else
      hipLaunchKernelGGL(lz_reduce_k<false>, dim3(vb), dim3(TPB), 0, st, part, splits, n, nv,
                         qprev, qcur, bprev, w, b.dotp);
    orth(1, b.alpha + (int64_t)j * nv);
    // q_{j+1} overwrites q_{j-1}
    normalize(qprev, b.beta + (int64_t)j * nv);
    std::swap(qprev, qcur);
    CHASE_HIP(hipGetLastError());
  }
}

}  // namespace chase
