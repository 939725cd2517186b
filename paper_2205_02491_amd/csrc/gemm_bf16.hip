// Split-BF16 ("bf16x3") products for the Chebyshev filter step on the CDNA4
// BF16 matrix cores.  Every operand value x is carried as two bf16 numbers,
// hi = bf16(x) and lo = bf16(x - hi) (16 significant bits together), and a
// real product is formed from three BF16 MFMAs with FP32 accumulation:
//   a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi
// (the dropped a_lo b_lo term is below 2^-16 |a b|).  A complex product is
// four real ones, i.e. twelve MFMAs.  The two-term form (TERMS = 2) uses the
// block operand's hi part only, a b ~ a_hi b_hi + a_lo b_hi (the block
// rounded to bf16, 2^-9 relative): eight MFMAs per complex product; the
// block's lo planes are neither copied to LDS nor read (the operand layout
// is shared with TERMS = 3).
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
// Workgroup tile 256 rows (of C) x 128 columns, K chunk 16 (one MFMA
// k-step), 512 threads = 8 wave64 in a 4 x 2 grid, each owning 64 x 64 as
// 2 x 2 fragments of 32 x 32 (230 VGPRs: two waves per SIMD).  Chunks are
// copied global -> LDS by the gfx950 direct LDS loads (global_load_lds_dwordx4:
// lane t of a wave writes 16 bytes at the wave's LDS base + 16 t), one chunk
// ahead, into two 48 KB stages; the waits are explicit counters before a
// bare barrier (an LDS release fence would treat the in-flight direct loads
// as pending LDS stores and wait for all of them).  Each column's chunk is
// stored unpadded; its 16-byte piece p sits in slot p ^ ((c >> 1) & 7) so
// the 16 lanes of an LDS read cycle (consecutive columns, one piece) cover
// all 64 banks.  Workgroup ids are remapped so that each of the 8 XCDs works
// on a contiguous range of tiles (the same few row panels of H).
//
// The Chebyshev-step epilogue (FP64) can also write the split of its
// output, the next filter step's operand, into a second s8 buffer with
// 2-byte stores, so a filter call splits its block once instead of once per
// step.
//
// One workgroup fits a CU (98 KB of LDS), so a launch runs in rounds of one
// tile per CU and a last round that is at most half full would leave most
// of the chip idle.  Those tiles are run as a split-K tail instead: each in
// up to (CUs / tiles) K slices, every slice writing its FP32 accumulators to
// a workspace, and a second kernel sums the slices in FP64 and applies the
// Chebyshev-step update.
//
// Measured on one MI355X (n=30000, 2000 columns, 1888 tiles): 32.9 ms per
// step with the tail (34.3 ms without), 438 TFLOP/s algorithmic (1.3
// PFLOP/s of BF16 MFMA work); two-term form 23.5 ms.  n=20000 with 1300 columns: 10.4 ms (11.2 ms
// without the tail).  The matrix cores are busy 54% of the time at the
// clock this kernel runs at (about 1.95 GHz with random operands:
// power-limited; 2.3 GHz in a pure-MFMA loop); the same MFMA block alone
// reaches 94% of peak, and the kernel without its global loads 82%.
#include <algorithm>
#include <atomic>
#include <cstdlib>

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
constexpr int KC = 16;          // K per chunk = one MFMA k-step
constexpr int NSTAGE = 2;       // LDS stages (stage of chunk c: c & 1)

__device__ inline bf8 as_bf8(u4v v) { return __builtin_bit_cast(bf8, v); }
__device__ inline u4v neg_u4(u4v v) {
  return v ^ u4v{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
}
__device__ inline f16v mfma(u4v a, u4v b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf8(a), as_bf8(b), c, 0, 0, 0);
}

// Round-to-nearest-even float -> bf16 (finite inputs; NaN stays NaN).
__device__ inline unsigned bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ inline double bf16_value(unsigned b) { return (double)__uint_as_float(b << 16); }

// hi and lo halves of x (value), as 2-byte stores into plane q of the 8-row
// group holding row r: out points at the row's slot in the group's first
// plane (planes 16 bytes apart: hi of component q at plane 2q, lo at 2q+1).
__device__ inline void put_split(unsigned short* out, int q, double x) {
  const unsigned bh = bf16_bits((float)x);
  out[(2 * q) * 8] = (unsigned short)bh;
  out[(2 * q + 1) * 8] = (unsigned short)bf16_bits((float)(x - bf16_value(bh)));
}

// The split of output element (i, j) into the next step's operand.
template <bool CPLX>
__device__ inline void emit_next_split(const GemmArgs& g, int64_t i, int64_t j, double vr,
                                       double vi) {
  constexpr int P = CPLX ? 4 : 2;
  if (!g.s8_next || j < g.s8_next_col0) return;
  unsigned short* out = reinterpret_cast<unsigned short*>(
                            static_cast<char*>(g.s8_next) +
                            ((j - g.s8_next_col0) * g.s8_groups + (i >> 3)) * P * 16) +
                        (i & 7);
  put_split(out, 0, vr);
  if constexpr (CPLX) put_split(out, 1, vi);
}

// Chebyshev-step update of one element (FP64): out = alpha (acc - gamma X)
// + beta out [+ colcoef_j F]; with s8_next set, also its split.
template <bool CPLX>
__device__ inline void cheb_elem(const GemmArgs& g, int64_t i, int64_t j, double vr, double vi) {
  double* __restrict__ Cd = static_cast<double*>(g.C);
  const double* __restrict__ B = static_cast<const double*>(g.B);
  const double* __restrict__ Fd = static_cast<const double*>(g.F);
  const int64_t o = i + j * g.ldc;
  if constexpr (CPLX) {
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
  emit_next_split<CPLX>(g, i, j, vr, vi);
}

// Epilogue of a whole tile.  Accumulator r of fragment (fi, fj) in lane
// (l32, h) is C(i0 + wi*32*FI + fi*32 + l32, j0 + wj*32*FJ + fj*32 +
// 8*(r/4) + 4*h + r%4) (the 32x32x16 MFMA result layout, measured on the
// hardware).
template <bool CPLX, int FI = 2, int FJ = 2>
__device__ inline void epilogue(const GemmArgs& g, const f16v (&acc_re)[FI][FJ],
                                const f16v (&acc_im)[FI][FJ], int64_t i0, int64_t j0, int wi,
                                int wj, int l32, int h) {
#pragma unroll
  for (int fi = 0; fi < FI; ++fi) {
    const int64_t i = i0 + wi * (32 * FI) + fi * 32 + l32;
    if (i >= g.M) continue;
#pragma unroll
    for (int fj = 0; fj < FJ; ++fj)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t j = j0 + wj * (32 * FJ) + fj * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (j >= g.N) continue;
        cheb_elem<CPLX>(g, i, j, (double)acc_re[fi][fj][r],
                        CPLX ? (double)acc_im[fi][fj][r] : 0.0);
      }
  }
}

// Split-K tail: the FP32 partial tile of one K slice, column-major within
// the tile (TBM rows), re then im.
template <bool CPLX, int FI = 2, int FJ = 2>
__device__ inline void store_partial(float* __restrict__ ws, const f16v (&acc_re)[FI][FJ],
                                     const f16v (&acc_im)[FI][FJ], int wi, int wj, int l32,
                                     int h) {
#pragma unroll
  for (int fi = 0; fi < FI; ++fi) {
    const int il = wi * (32 * FI) + fi * 32 + l32;
#pragma unroll
    for (int fj = 0; fj < FJ; ++fj)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int jl = wj * (32 * FJ) + fj * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        ws[jl * TBM + il] = acc_re[fi][fj][r];
        if constexpr (CPLX) ws[TBM * TBN + jl * TBM + il] = acc_im[fi][fj][r];
      }
  }
}

// Launch plan: tiles [0, ntiles) whole, then (split-K tail) tiles
// [tile0, tile0 + rem) in K slices of cps chunks, partial tiles to ws.
struct TailPlan {
  int tile0, rem, slices;
  int64_t cps;
  float* ws;
};

template <bool CPLX, bool SPLIT, int TERMS>
__global__ __launch_bounds__(NTHR) void gemm_bf16x3_kernel(GemmArgs g, int tiles_n, int ntiles,
                                                           TailPlan tp) {
  static_assert(TERMS == 2 || TERMS == 3, "two or three split terms");
  constexpr int P = CPLX ? 4 : 2;
  constexpr int CB = (KC / 8) * P * 16;  // bytes of one column in one chunk
  constexpr int PIECES = CB / 16;
  constexpr int NW = NTHR / 64;
  constexpr int NCOL = TBM + TBN;
  constexpr int STAGE = NCOL * CB;
  constexpr int BLK_COLS = 1024 / CB;    // columns per 1 KB wave load
  constexpr int NBLK = NCOL / BLK_COLS;
  constexpr int LOADS = NBLK / NW;       // wave loads per chunk
  constexpr int WGI = TBM / 64;          // waves along the rows of C
  static_assert(WGI * (TBN / 64) == NW, "64 x 64 per wave");
  static_assert(LOADS * NW == NBLK && LOADS <= 15, "chunk / waves, vmcnt immediate");
  __shared__ __attribute__((aligned(1024))) char lds[NSTAGE * STAGE];

  // Workgroup ids are remapped so that each XCD takes a contiguous range of
  // work items.  Whole tiles: item = tile.  Tail: item = slice * rem + tile
  // offset, so one XCD works on one K slice of neighbouring tiles.
  const int per_xcd = gridDim.x >> 3;
  const int u = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (u >= (SPLIT ? tp.rem * tp.slices : ntiles)) return;
  const int slice = SPLIT ? u / tp.rem : 0;
  const int tr = SPLIT ? u - slice * tp.rem : 0;
  const int t = SPLIT ? tp.tile0 + tr : u;
  const int tm = t / tiles_n, tn = t - tm * tiles_n;
  const int64_t i0 = (int64_t)tm * TBM, j0 = (int64_t)tn * TBN;
  const int64_t colbytes = g.s8_groups * P * 16;
  const char* __restrict__ Ta = static_cast<const char*>(g.a_s8) + i0 * colbytes;
  const char* __restrict__ Xb = static_cast<const char*>(g.b_s8) + j0 * colbytes;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wi = wave % WGI, wj = wave / WGI;
  const int l32 = lane & 31, h = lane >> 5;
  auto slot = [](int c, int p) { return p ^ ((c >> 1) & (PIECES - 1)); };

  // lane's column within a 1 KB block; the piece it fetches is the one whose
  // slot (in its absolute column col0 + bc) is the lane's position lane % PIECES
  const int bc = lane / PIECES;
  const char* srcT = Ta + bc * colbytes;
  const char* srcX = Xb + bc * colbytes;
  auto issue = [&](int64_t c) {
    char* base = lds + (int)(c & 1) * STAGE;
#pragma unroll
    for (int e = 0; e < LOADS; ++e) {
      const int blk = wave * LOADS + e;
      const int col0 = blk * BLK_COLS;
      const int pc = slot(col0 + bc, lane % PIECES);  // slot() is an involution in p
      // two terms: the block's lo planes (odd pieces) are never read, so they
      // are not copied (the wait before the barrier drains all loads, so the
      // count of issued loads does not matter)
      if (TERMS == 2 && col0 >= TBM && (pc & 1)) continue;
      const char* src = (col0 < TBM ? srcT + (int64_t)col0 * colbytes
                                    : srcX + (int64_t)(col0 - TBM) * colbytes) + c * CB + pc * 16;
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                       (__attribute__((address_space(3))) void*)(base + blk * 1024),
                                       16, 0, 0);
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
  const int64_t cb = SPLIT ? slice * tp.cps : 0;
  const int64_t ce = SPLIT ? (cb + tp.cps < nchunks ? cb + tp.cps : nchunks) : nchunks;
  issue(cb);
  for (int64_t c = cb; c < ce; ++c) {
    // chunk c has landed (no other loads are in flight); the barrier also
    // retires every wave's LDS reads of chunk c-1, whose stage chunk c+1
    // reuses.  Compiler-only memory barriers keep the LDS accesses on their
    // side of it.
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0x70);  // vmcnt(0) lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (c + 1 < ce) issue(c + 1);
    const char* st = lds + (int)(c & 1) * STAGE;
    u4v tf[2][P], xf[2][P];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const int ct = wi * 64 + f * 32 + l32;
      const int cx = TBM + wj * 64 + f * 32 + l32;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const int pc = h * P + p;
        tf[f][p] = *reinterpret_cast<const u4v*>(st + ct * CB + slot(ct, pc) * 16);
        xf[f][p] = *reinterpret_cast<const u4v*>(st + cx * CB + slot(cx, pc) * 16);
      }
    }
    if constexpr (CPLX) {
#pragma unroll
      for (int fj = 0; fj < 2; ++fj) {
        const u4v nxi_h = neg_u4(xf[fj][2]), nxi_l = neg_u4(xf[fj][3]);
#pragma unroll
        for (int fi = 0; fi < 2; ++fi) {
          f16v re = acc_re[fi][fj], im = acc_im[fi][fj];
          if constexpr (TERMS == 3) {  // block lo planes
            re = mfma(xf[fj][1], tf[fi][0], re);
            im = mfma(xf[fj][3], tf[fi][0], im);
          }
          re = mfma(xf[fj][0], tf[fi][1], re);
          im = mfma(xf[fj][2], tf[fi][1], im);
          if constexpr (TERMS == 3) {
            re = mfma(nxi_l, tf[fi][2], re);
            im = mfma(xf[fj][1], tf[fi][2], im);
          }
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
          if constexpr (TERMS == 3) re = mfma(xf[fj][1], tf[fi][0], re);
          re = mfma(xf[fj][0], tf[fi][1], re);
          re = mfma(xf[fj][0], tf[fi][0], re);
          acc_re[fi][fj] = re;
        }
    }
  }
  if constexpr (SPLIT)
    store_partial<CPLX>(tp.ws + (int64_t)u * (CPLX ? 2 : 1) * (TBM * TBN), acc_re, acc_im, wi, wj,
                        l32, h);
  else
    epilogue<CPLX>(g, acc_re, acc_im, i0, j0, wi, wj, l32, h);
}

// Two-term products with a 32-deep K chunk per barrier.  The block operand
// enters the two-term products through its hi planes only, so only those are
// copied to LDS: a chunk takes 256 x 256 B of T and 128 x 128 B of the block
// (complex), 80 KB, and two stages fill the CU's 160 KB.  Per barrier a wave
// issues 64 MFMAs (twice the 16-deep kernel's), and a chunk's copies are
// issued a whole chunk (two MFMA k-steps) before they are needed.  T columns
// are 256 B (one row of the 64 banks): piece p of column c sits in slot
// p ^ (c & 15); the block's 128-B columns use p ^ ((c >> 1) & 7).  Requires
// s8_groups to be a multiple of 4 (K padded to 32).
constexpr int KC2 = 32;

template <int CB, int PIECES>
__device__ inline int lds_slot(int c, int p) {
  constexpr int R = 256 / CB;  // columns per 256-byte row of the banks
  return p ^ ((c / R) & (PIECES - 1));
}

template <bool CPLX, bool SPLIT>
__global__ __launch_bounds__(NTHR) void gemm_bf16x2_k32_kernel(GemmArgs g, int tiles_n,
                                                               int ntiles, TailPlan tp) {
  constexpr int P = CPLX ? 4 : 2;   // planes of a group in the s8 layout
  constexpr int PX = P / 2;         // the block's hi planes (re_hi, im_hi)
  constexpr int GPC = KC2 / 8;      // 8-row groups per chunk
  constexpr int CBT = GPC * P * 16;   // bytes of a T column per chunk
  constexpr int CBX = GPC * PX * 16;  // bytes of a block column per chunk (hi planes)
  constexpr int PT = CBT / 16, PXN = CBX / 16;
  constexpr int NW = NTHR / 64;
  constexpr int TBYTES = TBM * CBT;
  constexpr int STAGE = TBYTES + TBN * CBX;
  constexpr int TBLK = TBYTES / 1024, XBLK = TBN * CBX / 1024;
  constexpr int LOADS = (TBLK + XBLK) / NW;
  constexpr int WGI = TBM / 64;
  static_assert(WGI * (TBN / 64) == NW, "64 x 64 per wave");
  static_assert(LOADS * NW == TBLK + XBLK && LOADS <= 15, "chunk / waves, vmcnt immediate");
  static_assert(2 * STAGE <= 160 * 1024, "two stages in the CU's LDS");
  __shared__ __attribute__((aligned(1024))) char lds[2 * STAGE];

  const int per_xcd = gridDim.x >> 3;
  const int u = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (u >= (SPLIT ? tp.rem * tp.slices : ntiles)) return;
  const int slice = SPLIT ? u / tp.rem : 0;
  const int tr = SPLIT ? u - slice * tp.rem : 0;
  const int t = SPLIT ? tp.tile0 + tr : u;
  const int tm = t / tiles_n, tn = t - tm * tiles_n;
  const int64_t i0 = (int64_t)tm * TBM, j0 = (int64_t)tn * TBN;
  const int64_t colbytes = g.s8_groups * P * 16;
  const char* __restrict__ Ta = static_cast<const char*>(g.a_s8) + i0 * colbytes;
  const char* __restrict__ Xb = static_cast<const char*>(g.b_s8) + j0 * colbytes;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wi = wave % WGI, wj = wave / WGI;
  const int l32 = lane & 31, h = lane >> 5;

  // Each wave-wide direct load fills 1 KB of the stage: T blocks first (1024
  // / CBT columns each), then the block's (1024 / CBX columns).  A lane
  // fetches the piece whose slot in its column is its position in the
  // column's stretch (lds_slot is an involution in p).
  auto issue = [&](int64_t c) {
    char* base = lds + (int)(c & 1) * STAGE;
#pragma unroll
    for (int e = 0; e < LOADS; ++e) {
      const int blk = wave * LOADS + e;
      const char* src;
      if (blk < TBLK) {
        const int col = blk * (1024 / CBT) + lane / PT;
        const int pc = lds_slot<CBT, PT>(col, lane % PT);
        src = Ta + (int64_t)col * colbytes + c * (GPC * P * 16) + pc * 16;
      } else {
        const int col = (blk - TBLK) * (1024 / CBX) + lane / PXN;
        const int pc = lds_slot<CBX, PXN>(col, lane % PXN);
        const int gq = pc / PX, q = pc - gq * PX;
        src = Xb + (int64_t)col * colbytes + c * (GPC * P * 16) + (gq * P + 2 * q) * 16;
      }
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                       (__attribute__((address_space(3))) void*)(base + blk * 1024),
                                       16, 0, 0);
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

  const int64_t nchunks = g.s8_groups / GPC;
  const int64_t cb = SPLIT ? slice * tp.cps : 0;
  const int64_t ce = SPLIT ? (cb + tp.cps < nchunks ? cb + tp.cps : nchunks) : nchunks;
  issue(cb);
  for (int64_t c = cb; c < ce; ++c) {
    // as in the 16-deep kernel: chunk c has landed, every wave is done with
    // chunk c-1's stage, which chunk c+1 then fills
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0x70);  // vmcnt(0) lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (c + 1 < ce) issue(c + 1);
    const char* st = lds + (int)(c & 1) * STAGE;
    const char* stx = st + TBYTES;
#pragma unroll
    for (int s = 0; s < KC2 / 16; ++s) {
      const int gq = 2 * s + h;  // the lane's 8-row group within the chunk
      u4v tf[2][P], xf[2][PX];
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const int ct = wi * 64 + f * 32 + l32;
        const int cx = wj * 64 + f * 32 + l32;
#pragma unroll
        for (int p = 0; p < P; ++p)
          tf[f][p] = *reinterpret_cast<const u4v*>(st + ct * CBT +
                                                   lds_slot<CBT, PT>(ct, gq * P + p) * 16);
#pragma unroll
        for (int q = 0; q < PX; ++q)
          xf[f][q] = *reinterpret_cast<const u4v*>(stx + cx * CBX +
                                                   lds_slot<CBX, PXN>(cx, gq * PX + q) * 16);
      }
      if constexpr (CPLX) {
#pragma unroll
        for (int fj = 0; fj < 2; ++fj) {
          const u4v nxi = neg_u4(xf[fj][1]);
#pragma unroll
          for (int fi = 0; fi < 2; ++fi) {
            f16v re = acc_re[fi][fj], im = acc_im[fi][fj];
            re = mfma(xf[fj][0], tf[fi][1], re);
            im = mfma(xf[fj][1], tf[fi][1], im);
            re = mfma(nxi, tf[fi][3], re);
            im = mfma(xf[fj][0], tf[fi][3], im);
            re = mfma(xf[fj][0], tf[fi][0], re);
            im = mfma(xf[fj][1], tf[fi][0], im);
            re = mfma(nxi, tf[fi][2], re);
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
            re = mfma(xf[fj][0], tf[fi][1], re);
            re = mfma(xf[fj][0], tf[fi][0], re);
            acc_re[fi][fj] = re;
          }
      }
    }
  }
  if constexpr (SPLIT)
    store_partial<CPLX>(tp.ws + (int64_t)u * (CPLX ? 2 : 1) * (TBM * TBN), acc_re, acc_im, wi, wj,
                        l32, h);
  else
    epilogue<CPLX>(g, acc_re, acc_im, i0, j0, wi, wj, l32, h);
}

// Split-K tail: sum the slices' partial tiles (FP64) and apply the
// Chebyshev-step update, one element per thread, rows fastest.
template <bool CPLX>
__global__ void tail_finish_k(GemmArgs g, int tiles_n, TailPlan tp) {
  constexpr int TE = TBM * TBN;
  const int64_t total = (int64_t)tp.rem * TE;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int tr = (int)(idx / TE);
    const int e = (int)(idx - (int64_t)tr * TE);
    const int jl = e / TBM, il = e - jl * TBM;
    const int t = tp.tile0 + tr;
    const int tm = t / tiles_n, tn = t - tm * tiles_n;
    const int64_t i = (int64_t)tm * TBM + il, j = (int64_t)tn * TBN + jl;
    if (i >= g.M || j >= g.N) continue;
    double vr = 0.0, vi = 0.0;
    for (int sl = 0; sl < tp.slices; ++sl) {
      const float* p = tp.ws + ((int64_t)sl * tp.rem + tr) * (CPLX ? 2 : 1) * TE + e;
      vr += (double)p[0];
      if constexpr (CPLX) vi += (double)p[TE];
    }
    cheb_elem<CPLX>(g, i, j, vr, vi);
  }
}

// ------------------------------------------------------------------ split

// One thread per row of a column (consecutive threads read consecutive
// rows: coalesced), writing its hi and lo halves as 2-byte values into the
// planes of its 8-row group.
template <bool CPLX>
__global__ void split_s8_k(const double* __restrict__ src, int64_t lds, int64_t rows,
                           int64_t cols, int64_t cols_pad, int64_t groups, int conj,
                           char* __restrict__ dst) {
  constexpr int P = CPLX ? 4 : 2;
  const int64_t rows_pad = groups * 8;
  const int64_t total = cols_pad * rows_pad;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = idx / rows_pad, r = idx - c * rows_pad;
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
    unsigned short* out =
        reinterpret_cast<unsigned short*>(dst + (c * groups + (r >> 3)) * P * 16) + (r & 7);
#pragma unroll
    for (int q = 0; q < P / 2; ++q) put_split(out, q, x[q]);
  }
}

}  // namespace

void split_s8(bool cplx, bool conj, const void* src, int64_t lds, int64_t rows, int64_t cols,
              int64_t cols_pad, void* dst, int64_t groups, hipStream_t st) {
  CHASE_REQUIRE(groups * 8 >= rows && groups % (S8_KPAD / 8) == 0 && cols_pad >= cols,
                "split layout too small");
  const int64_t total = cols_pad * groups * 8;
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

int device_cus() {
  static std::atomic<int> cached[16];
  int dev = 0;
  CHASE_HIP(hipGetDevice(&dev));
  if (dev < 16 && cached[dev].load() > 0) return cached[dev].load();
  int n = 0;
  CHASE_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
  if (dev < 16) cached[dev].store(n);
  return n;
}

// 32-deep chunks for the two-term products unless CHASE_BF16_KCHUNK=16 (the
// 16-deep kernel, kept for the three-term products and for comparison).
bool two_term_k32() {
  static const bool on = [] {
    const char* e = std::getenv("CHASE_BF16_KCHUNK");
    return !(e && std::atoi(e) == 16);
  }();
  return on;
}

void gemm_bf16x3(bool cplx, const GemmArgs& g, hipStream_t st, int terms) {
  if (g.M <= 0 || g.N <= 0) return;
  CHASE_REQUIRE(g.a_s8 && g.b_s8 && g.s8_groups > 0 && g.s8_groups % (KC / 8) == 0,
                "split-BF16 operands missing");
  CHASE_REQUIRE(g.s8_groups * 8 >= g.K, "split-BF16 operands shorter than K");
  CHASE_REQUIRE(terms == 2 || terms == 3, "split-BF16 products take two or three terms");
  const bool k32 = terms == 2 && g.s8_groups % (KC2 / 8) == 0 && two_term_k32();
  const int tiles_m = (int)((g.M + TBM - 1) / TBM);
  const int tiles_n = (int)((g.N + TBN - 1) / TBN);
  const int ntiles = tiles_m * tiles_n;
  const int64_t nchunks = g.s8_groups / ((k32 ? KC2 : KC) / 8);
  // One workgroup per CU (LDS-bound), so a launch runs in rounds of `cus`
  // tiles.  A last round filled at most half is run as a split-K tail: its
  // tiles in K slices of at least 256 rows of K on the idle CUs, the FP32
  // partial tiles summed by a second kernel.
  const int64_t min_chunks = 256 / (k32 ? KC2 : KC);
  const int cus = device_cus();
  TailPlan tp{0, 0, 1, nchunks, g.s8_tail};
  if (g.s8_tail && cus > 0) {
    const int rem = ntiles % cus;
    if (rem > 0 && 2 * rem <= cus) {
      const int64_t want = std::min<int64_t>(
          {(int64_t)(cus / rem), (int64_t)(S8_TAIL_SLOTS / rem), nchunks / min_chunks});
      if (want >= 2) {
        tp.cps = (nchunks + want - 1) / want;
        tp.slices = (int)((nchunks + tp.cps - 1) / tp.cps);
        tp.rem = rem;
        tp.tile0 = ntiles - rem;
      }
    }
  }
  const int whole = ntiles - tp.rem;
  if (whole > 0) {
    const int grid_x = (whole + 7) / 8 * 8;
    if (cplx && k32)
      hipLaunchKernelGGL((gemm_bf16x2_k32_kernel<true, false>), dim3(grid_x), dim3(NTHR), 0, st,
                         g, tiles_n, whole, tp);
    else if (k32)
      hipLaunchKernelGGL((gemm_bf16x2_k32_kernel<false, false>), dim3(grid_x), dim3(NTHR), 0, st,
                         g, tiles_n, whole, tp);
    else if (cplx && terms == 3)
      hipLaunchKernelGGL((gemm_bf16x3_kernel<true, false, 3>), dim3(grid_x), dim3(NTHR), 0, st, g,
                         tiles_n, whole, tp);
    else if (cplx)
      hipLaunchKernelGGL((gemm_bf16x3_kernel<true, false, 2>), dim3(grid_x), dim3(NTHR), 0, st, g,
                         tiles_n, whole, tp);
    else if (terms == 3)
      hipLaunchKernelGGL((gemm_bf16x3_kernel<false, false, 3>), dim3(grid_x), dim3(NTHR), 0, st,
                         g, tiles_n, whole, tp);
    else
      hipLaunchKernelGGL((gemm_bf16x3_kernel<false, false, 2>), dim3(grid_x), dim3(NTHR), 0, st,
                         g, tiles_n, whole, tp);
    CHASE_HIP(hipGetLastError());
  }
  if (tp.rem > 0) {
    const int items = tp.rem * tp.slices;
    const int grid_x = (items + 7) / 8 * 8;
    const int64_t elems = (int64_t)tp.rem * TBM * TBN;
    const unsigned fin = (unsigned)std::min<int64_t>((elems + 255) / 256, 8192);
    if (cplx && k32)
      hipLaunchKernelGGL((gemm_bf16x2_k32_kernel<true, true>), dim3(grid_x), dim3(NTHR), 0, st,
                         g, tiles_n, ntiles, tp);
    else if (k32)
      hipLaunchKernelGGL((gemm_bf16x2_k32_kernel<false, true>), dim3(grid_x), dim3(NTHR), 0, st,
                         g, tiles_n, ntiles, tp);
    else if (cplx && terms == 3)
      hipLaunchKernelGGL((gemm_bf16x3_kernel<true, true, 3>), dim3(grid_x), dim3(NTHR), 0, st, g,
                         tiles_n, ntiles, tp);
    else if (cplx)
      hipLaunchKernelGGL((gemm_bf16x3_kernel<true, true, 2>), dim3(grid_x), dim3(NTHR), 0, st, g,
                         tiles_n, ntiles, tp);
    else if (terms == 3)
      hipLaunchKernelGGL((gemm_bf16x3_kernel<false, true, 3>), dim3(grid_x), dim3(NTHR), 0, st,
                         g, tiles_n, ntiles, tp);
    else
      hipLaunchKernelGGL((gemm_bf16x3_kernel<false, true, 2>), dim3(grid_x), dim3(NTHR), 0, st,
                         g, tiles_n, ntiles, tp);
    CHASE_HIP(hipGetLastError());
    if (cplx)
      hipLaunchKernelGGL(tail_finish_k<true>, dim3(fin), dim3(256), 0, st, g, tiles_n, tp);
    else
      hipLaunchKernelGGL(tail_finish_k<false>, dim3(fin), dim3(256), 0, st, g, tiles_n, tp);
    CHASE_HIP(hipGetLastError());
  }
}

}  // namespace chase
