// Split-BF16 ("bf16x3") products for the Chebyshev filter step on the CDNA4
// BF16 matrix cores.  Every operand value x is carried as two bf16 numbers,
// hi = bf16(x) and lo = bf16(x - hi) (16 significant bits together), and a
// real product is formed from three BF16 MFMAs with FP32 accumulation:
//   a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi
// (the dropped a_lo b_lo term is below 2^-16 |a b|).  A complex product is
// four real ones, i.e. twelve MFMAs.
//
// Operand storage (the "s8" layout, made by split_s8): a K x C matrix is
// stored column by column; the K rows are zero-padded to a multiple of 16 and
// grouped by 8, and group g of column c occupies (planes x 16) bytes at
// byte offset (c * groups + g) * planes * 16 as
//   complex: re_hi[8] re_lo[8] im_hi[8] im_lo[8]     real: hi[8] lo[8].
// One 16-byte plane of a group is exactly what a lane feeds to a
// 32x32x16 MFMA (eight consecutive k), so LDS fragments are single 16-byte
// reads and the K loop needs no bounds checks.
//
// The filter product C = H X (H Hermitian) uses the split of
// T = conj(H) = H^T: column i of T is row i of H, contiguous along k.
// The MFMA is fed the X fragment in its first slot and the T fragment in its
// second, so the 32 x 32 result is C^T and each lane's sixteen accumulators
// lie along one row of C: 32 lanes then write 32 consecutive rows of a
// column-major output.
//
// Workgroup tile 256 rows (of C) x 128 columns, K chunk 16, 512 threads =
// 8 wave64 in a 4 x 2 grid, each owning 64 x 64 as 2 x 2 fragments of
// 32 x 32; the chunk is staged through double-buffered LDS with a 16-byte pad
// per column (144-byte stride: eight lanes reading 16 bytes each hit 32
// distinct banks).  Workgroup ids are remapped so that each of the 8 XCDs
// works on a contiguous range of tiles (the same few row panels of H).
#include "common.h"

namespace chase {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

constexpr int TBM = S8_COLS_A;  // rows of C per workgroup (columns of the T split)
constexpr int TBN = S8_COLS_B;  // columns of C per workgroup (columns of the X split)
constexpr int NTHR = 512;
constexpr int KC = S8_KPAD;     // K per chunk = one MFMA k-step

__device__ inline bf8 as_bf8(u4v v) { return __builtin_bit_cast(bf8, v); }
__device__ inline u4v neg_u4(u4v v) {
  return v ^ u4v{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
}
__device__ inline f16v mfma(u4v a, u4v b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf8(a), as_bf8(b), c, 0, 0, 0);
}

template <bool CPLX>
__global__ __launch_bounds__(NTHR) void gemm_bf16x3_kernel(GemmArgs g, int tiles_n, int ntiles) {
  constexpr int P = CPLX ? 4 : 2;               // 16-byte planes per 8-row group
  constexpr int CB = (KC / 8) * P * 16;         // bytes of one column in one chunk
  constexpr int CS = CB + 16;                   // LDS column stride
  constexpr int NCOL = TBM + TBN;
  constexpr int PIECES = CB / 16;
  constexpr int LOADS = NCOL * PIECES / NTHR;
  static_assert(LOADS * NTHR == NCOL * PIECES, "chunk / threads");
  __shared__ __attribute__((aligned(16))) char lds[2][NCOL * CS];

  const int per_xcd = gridDim.x >> 3;
  const int t = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (t >= ntiles) return;
  const int tm = t / tiles_n, tn = t - tm * tiles_n;
  const int64_t i0 = (int64_t)tm * TBM, j0 = (int64_t)tn * TBN;
  const int64_t colbytes = g.s8_groups * P * 16;
  const char* __restrict__ Ta = static_cast<const char*>(g.a_s8) + i0 * colbytes;
  const char* __restrict__ Xb = static_cast<const char*>(g.b_s8) + j0 * colbytes;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int l32 = lane & 31, h = lane >> 5;

  u4v rg[LOADS];
  auto load_chunk = [&](int64_t c) {
#pragma unroll
    for (int e = 0; e < LOADS; ++e) {
      const int idx = tid + e * NTHR;
      const int col = idx / PIECES, pc = idx - col * PIECES;
      const char* src = col < TBM ? Ta + col * colbytes : Xb + (col - TBM) * colbytes;
      rg[e] = *reinterpret_cast<const u4v*>(src + c * CB + pc * 16);
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int e = 0; e < LOADS; ++e) {
      const int idx = tid + e * NTHR;
      const int col = idx / PIECES, pc = idx - col * PIECES;
      *reinterpret_cast<u4v*>(&lds[buf][col * CS + pc * 16]) = rg[e];
    }
  };

  f16v acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc_re[a][b] = f16v{};
      acc_im[a][b] = f16v{};
    }

  const int64_t nchunks = g.s8_groups / (KC / 8);
  load_chunk(0);
  store_chunk(0);
  __syncthreads();
  for (int64_t c = 0; c < nchunks; ++c) {
    const int buf = (int)(c & 1);
    const bool more = c + 1 < nchunks;
    if (more) load_chunk(c + 1);
    // fragments: lane reads the 16-byte planes of 8-row group h of its column
    u4v tf[2][P], xf[2][P];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const char* pt = &lds[buf][(wi * 64 + f * 32 + l32) * CS + h * P * 16];
      const char* px = &lds[buf][(TBM + wj * 64 + f * 32 + l32) * CS + h * P * 16];
#pragma unroll
      for (int p = 0; p < P; ++p) {
        tf[f][p] = *reinterpret_cast<const u4v*>(pt + p * 16);
        xf[f][p] = *reinterpret_cast<const u4v*>(px + p * 16);
      }
    }
    if constexpr (CPLX) {
      // C = T X: re = Tr Xr - Ti Xi, im = Tr Xi + Ti Xr; planes 0,1 = re hi/lo,
      // 2,3 = im hi/lo.  Each product as hi*hi + hi*lo + lo*hi.
#pragma unroll
      for (int fj = 0; fj < 2; ++fj) {
        const u4v nxi_h = neg_u4(xf[fj][2]), nxi_l = neg_u4(xf[fj][3]);
#pragma unroll
        for (int fi = 0; fi < 2; ++fi) {
          f16v re = acc_re[fi][fj], im = acc_im[fi][fj];
          re = mfma(xf[fj][1], tf[fi][0], re);
          im = mfma(xf[fj][3], tf[fi][0], im);
          re = mfma(xf[fj][0], tf[fi][1], re);
          im = mfma(xf[fj][2], tf[fi][1], im);
          re = mfma(nxi_l, tf[fi][2], re);
          im = mfma(xf[fj][1], tf[fi][2], im);
          re = mfma(nxi_h, tf[fi][3], re);
          im = mfma(xf[fj][0], tf[fi][3], im);
          re = mfma(xf[fj][0], tf[fi][0], re);
          im = mfma(xf[fj][2], tf[fi][0], im);
          re = mfma(nxi_h, tf[fi][2], re);
          im = mfma(xf[fj][0], tf[fi][2], im);
          acc_re[fi][fj] = re;
          acc_im[fi][fj] = im;
        }
      }
    } else {
#pragma unroll
      for (int fj = 0; fj < 2; ++fj)
#pragma unroll
        for (int fi = 0; fi < 2; ++fi) {
          f16v re = acc_re[fi][fj];
          re = mfma(xf[fj][1], tf[fi][0], re);
          re = mfma(xf[fj][0], tf[fi][1], re);
          re = mfma(xf[fj][0], tf[fi][0], re);
          acc_re[fi][fj] = re;
        }
    }
    if (more) store_chunk(buf ^ 1);
    __syncthreads();
  }

  // ---------------------------------------------------------------- epilogue
  // accumulator r of fragment (fi, fj) in lane (l32, h):
  //   row i = i0 + wi*64 + fi*32 + l32, column j = j0 + wj*64 + fj*32 + 8*(r/4) + 4*h + r%4
  double* __restrict__ Cd = static_cast<double*>(g.C);
  const double* __restrict__ B = static_cast<const double*>(g.B);
  const double* __restrict__ Fd = static_cast<const double*>(g.F);
#pragma unroll
  for (int fi = 0; fi < 2; ++fi) {
    const int64_t i = i0 + wi * 64 + fi * 32 + l32;
    if (i >= g.M) continue;
#pragma unroll
    for (int fj = 0; fj < 2; ++fj)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t j = j0 + wj * 64 + fj * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (j >= g.N) continue;
        const int64_t o = i + j * g.ldc;
        double vr = (double)acc_re[fi][fj][r];
        if constexpr (CPLX) {
          double vi = (double)acc_im[fi][fj][r];
          const d2v x = *reinterpret_cast<const d2v*>(B + 2 * (i + j * g.ldb));
          vr = g.alpha * (vr - g.gamma * x.x);
          vi = g.alpha * (vi - g.gamma * x.y);
          if (g.beta != 0.0) {
            const d2v y = *reinterpret_cast<const d2v*>(Cd + 2 * o);
            vr += g.beta * y.x;
            vi += g.beta * y.y;
          }
          if (g.colcoef) {
            const double cj = g.colcoef[j];
            const d2v f = *reinterpret_cast<const d2v*>(Fd + 2 * (i + j * g.ldf));
            vr += cj * f.x;
            vi += cj * f.y;
          }
          *reinterpret_cast<d2v*>(Cd + 2 * o) = d2v{vr, vi};
        } else {
          vr = g.alpha * (vr - g.gamma * B[i + j * g.ldb]);
          if (g.beta != 0.0) vr += g.beta * Cd[o];
          if (g.colcoef) vr += g.colcoef[j] * Fd[i + j * g.ldf];
          Cd[o] = vr;
        }
      }
  }
}

// ------------------------------------------------------------------ split
// Round-to-nearest-even float -> bf16 (finite inputs; NaN stays NaN).
__device__ inline unsigned bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ inline double bf16_value(unsigned b) { return (double)__uint_as_float(b << 16); }

template <bool CPLX>
__global__ void split_s8_k(const double* __restrict__ src, int64_t lds, int64_t rows,
                           int64_t cols, int64_t cols_pad, int64_t groups, int conj,
                           char* __restrict__ dst) {
  constexpr int P = CPLX ? 4 : 2;
  const int64_t total = cols_pad * groups;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = idx / groups, gr = idx - c * groups;
    unsigned hi[P / 2][8], lo[P / 2][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t r = gr * 8 + e;
      double x[2] = {0.0, 0.0};
      if (c < cols && r < rows) {
        if constexpr (CPLX) {
          const d2v v = *reinterpret_cast<const d2v*>(src + 2 * (r + c * lds));
          x[0] = v.x;
          x[1] = conj ? -v.y : v.y;
        } else {
          x[0] = src[r + c * lds];
        }
      }
#pragma unroll
      for (int q = 0; q < P / 2; ++q) {
        const unsigned bh = bf16_bits((float)x[q]);
        hi[q][e] = bh;
        lo[q][e] = bf16_bits((float)(x[q] - bf16_value(bh)));
      }
    }
    u4v* out = reinterpret_cast<u4v*>(dst + idx * P * 16);
#pragma unroll
    for (int q = 0; q < P / 2; ++q) {
      u4v vh, vl;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        vh[w] = hi[q][2 * w] | (hi[q][2 * w + 1] << 16);
        vl[w] = lo[q][2 * w] | (lo[q][2 * w + 1] << 16);
      }
      out[2 * q] = vh;
      out[2 * q + 1] = vl;
    }
  }
}

}  // namespace

void split_s8(bool cplx, bool conj, const void* src, int64_t lds, int64_t rows, int64_t cols,
              int64_t cols_pad, void* dst, int64_t groups, hipStream_t st) {
  CHASE_REQUIRE(groups * 8 >= rows && groups % (S8_KPAD / 8) == 0 && cols_pad >= cols,
                "split layout too small");
  const int64_t total = cols_pad * groups;
  if (total <= 0) return;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  if (cplx)
    hipLaunchKernelGGL(split_s8_k<true>, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<const double*>(src), lds, rows, cols, cols_pad, groups,
                       conj ? 1 : 0, static_cast<char*>(dst));
  else
    hipLaunchKernelGGL(split_s8_k<false>, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<const double*>(src), lds, rows, cols, cols_pad, groups, 0,
                       static_cast<char*>(dst));
  CHASE_HIP(hipGetLastError());
}

void gemm_bf16x3(bool cplx, const GemmArgs& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return;
  CHASE_REQUIRE(g.a_s8 && g.b_s8 && g.s8_groups > 0 && g.s8_groups % (S8_KPAD / 8) == 0,
                "split-BF16 operands missing");
  CHASE_REQUIRE(g.s8_groups * 8 >= g.K, "split-BF16 operands shorter than K");
  const int tiles_m = (int)((g.M + TBM - 1) / TBM);
  const int tiles_n = (int)((g.N + TBN - 1) / TBN);
  const int ntiles = tiles_m * tiles_n;
  const int grid_x = (ntiles + 7) / 8 * 8;
  if (cplx)
    hipLaunchKernelGGL(gemm_bf16x3_kernel<true>, dim3(grid_x), dim3(NTHR), 0, st, g, tiles_n,
                       ntiles);
  else
    hipLaunchKernelGGL(gemm_bf16x3_kernel<false>, dim3(grid_x), dim3(NTHR), 0, st, g, tiles_n,
                       ntiles);
  CHASE_HIP(hipGetLastError());
}

}  // namespace chase
