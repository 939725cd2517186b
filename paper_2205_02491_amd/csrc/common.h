// Internal declarations shared by the ChASE HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/chase.h"

namespace chase {

struct Error : std::runtime_error {
  chase_status status;
  Error(chase_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define CHASE_HIP(call)                                                            \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::chase::Error(CHASE_ERR_HIP, std::string(#call) + ": " +              \
                                              hipGetErrorString(e_));              \
  } while (0)

#define CHASE_REQUIRE(cond, msg)                                                   \
  do {                                                                             \
    if (!(cond)) throw ::chase::Error(CHASE_ERR_ARG, msg);                         \
  } while (0)

struct c128 {
  double re, im;
};
struct c64 {
  float re, im;
};

// ------------------------------------------------------------------ GEMM
// Operand forms: N = as stored (column-major), C = conjugate transpose
// (transpose for real data).
enum Op { OP_N = 0, OP_C = 1 };

// Epilogues of the tile GEMM C = op(A) op(B):
//   STORE : C = alpha*AB + beta*C
//   CHEB  : out = alpha*(AB - gamma*Xs) + beta*out   (one Chebyshev step;
//           Xs is the B operand itself, out may hold X_{s-2})
//   SPLITK: partial sums of a K-slice to a workspace (reduced separately)
//   RESID : partial column sums of |AB - lambda_j * V|^2 per row tile
enum Epi { EPI_STORE = 0, EPI_CHEB = 1, EPI_SPLITK = 2, EPI_RESID = 3 };

// Arithmetic of the products: FP64 (double MFMA), FP32 (float MFMA,
// operands rounded to float when staged in LDS, FP32 accumulation) or split
// BF16 (three BF16 MFMAs per real product on hi/lo splits of both operands,
// FP32 accumulation; operands in the s8 layout below).
enum Prec { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16X3 = 2, PREC_BF16X2 = 3 };
inline bool is_split_bf16(Prec p) { return p == PREC_BF16X3 || p == PREC_BF16X2; }

struct GemmArgs {
  int64_t M, N, K;
  const void* A;  // element type: c128/double, or c64/float when a_f32
  int64_t lda;
  const void* B;
  int64_t ldb;
  void* C;  // output (STORE/CHEB: same element type as B; SPLITK: ws)
  int64_t ldc;
  double alpha, beta, gamma;
  const double* lambda;  // RESID: per-column shift (device)
  const void* V;         // RESID: matrix subtracted (ld ldv)
  int64_t ldv;
  double* partial;       // RESID: [row_tiles][N] partial sums
  int splits;            // SPLITK: number of K slices (grid z)
  int64_t kslice;        // SPLITK: K length per slice (multiple of the K tile)
  int a_f32;             // A stored as c64/float (mixed-precision copy of H)
  // CHEB: optional forcing term + colcoef[j] * F(i, j) (defect-correction
  // form of the filter); RESID: optional store of the residual block to F
  const double* colcoef;
  void* F;
  int64_t ldf;
  // PREC_BF16X3: s8 splits of the operands (A: T = conj(H) = H^T, columns
  // padded to S8_COLS_A; B: the block X, columns padded to S8_COLS_B), with
  // s8_groups 8-row groups per column.  B above stays the FP64 block read by
  // the epilogue.
  const void* a_s8;
  const void* b_s8;
  int64_t s8_groups;
  // PREC_BF16X3: workspace (s8_tail_bytes) for the split-K tail of the
  // launch; nullptr runs every tile whole
  float* s8_tail;
  // PREC_BF16X3, optional: the epilogue also writes the s8 split of its
  // output (the next filter step's operand) to s8_next, output column j
  // (>= s8_next_col0) as split column j - s8_next_col0, rows < M only (the
  // zero padding rows of s8_next are left as they are)
  void* s8_next;
  int64_t s8_next_col0;
  // Triangular structure (0: none).  SPLITK, square result: only the tiles
  // on and above the diagonal are computed (Hermitian products; the
  // reduction mirrors them).  STORE with B as stored: column j of B is zero
  // below row tri_row0 + j, so a column tile's K loop stops there.
  int tri;
  int64_t tri_row0;
};

// ------------------------------------------------------------------ split BF16
// s8 layout of a K x C matrix: K padded with zero rows to a multiple of
// S8_KPAD and grouped by 8; group g of column c at byte (c*groups + g)*planes*16
// holding re_hi[8] re_lo[8] im_hi[8] im_lo[8] (real: hi[8] lo[8]),
// hi = bf16(x), lo = bf16(x - hi), round to nearest even.
constexpr int S8_KPAD = 32;  // the two-term kernel's K chunk
constexpr int S8_COLS_A = 256;  // row tile of the split-BF16 GEMM
constexpr int S8_COLS_B = 128;  // column tile of the split-BF16 GEMM
inline int64_t s8_groups(int64_t K) { return (K + S8_KPAD - 1) / S8_KPAD * (S8_KPAD / 8); }
inline int64_t s8_pad(int64_t c, int64_t tile) { return (c + tile - 1) / tile * tile; }
inline size_t s8_bytes(bool cplx, int64_t K, int64_t cols_pad) {
  return (size_t)s8_groups(K) * (cplx ? 64 : 32) * (size_t)cols_pad;
}
// FP32 partial tiles of the split-K tail: at most S8_TAIL_SLOTS (tile, K
// slice) pairs of S8_COLS_A x S8_COLS_B (re and im for complex).
constexpr int S8_TAIL_SLOTS = 256;
inline size_t s8_tail_bytes(bool cplx) {
  return (size_t)S8_TAIL_SLOTS * S8_COLS_A * S8_COLS_B * (cplx ? 2 : 1) * sizeof(float);
}
// Split the rows x cols FP64 block src (ld lds) into dst (s8 layout, groups
// per column, cols_pad columns; columns >= cols and rows >= rows are zero).
// conj: store the conjugate (complex).
void split_s8(bool cplx, bool conj, const void* src, int64_t lds, int64_t rows, int64_t cols,
              int64_t cols_pad, void* dst, int64_t groups, hipStream_t st);
// Filter step C = alpha (A B - gamma B) + beta C [+ colcoef F] with split-BF16
// products (GemmArgs a_s8, b_s8, s8_groups; M = rows of C, K <= 8*s8_groups).
// terms = 3: hi*hi + hi*lo + lo*hi; terms = 2: the block operand as bf16
// only (hi*hi + lo_H*hi).
void gemm_bf16x3(bool cplx, const GemmArgs& g, hipStream_t st, int terms = 3);

// Launch the tile GEMM. cplx selects complex (c128) vs real (double) data.
void gemm(bool cplx, Prec prec, Op opa, Op opb, Epi epi, const GemmArgs& g,
          hipStream_t st);
int gemm_row_tiles(int64_t M);
// Split-K plan for an M x N result with long K: number of slices and the
// per-slice K length; workspace elements needed = splits * M * N.
void splitk_plan(int64_t M, int64_t N, int64_t K, int* splits, int64_t* kslice,
                 bool tri = false);
// Edge of the square tiles of the split-K products (the unit of `tri`).
int splitk_tile();

// ------------------------------------------------------------------ misc kernels
void fill_zero(void* p, int64_t bytes, hipStream_t st);
void copy_cols(bool cplx, const void* src, int64_t lds, void* dst, int64_t ldd, int64_t n,
               int64_t k, hipStream_t st);
void gather_cols(bool cplx, const void* src, int64_t lds, void* dst, int64_t ldd, int64_t n,
                 int64_t k, const int* perm_dev, hipStream_t st);
// sum the split-K slices ws[z][i + j*M] into C (ld ldc); herm: C=(S+S^H)/2.
// tri_tile > 0 (herm, M == N): only the tiles of that edge on and above the
// diagonal were computed; C = S above the diagonal tiles, its conjugate
// transpose below them, (S+S^H)/2 within them.
void splitk_reduce(bool cplx, const void* ws, int splits, int64_t M, int64_t N, void* C,
                   int64_t ldc, bool herm, hipStream_t st, int tri_tile = 0);
// Gram post-processing for Cholesky QR: d_j = 1/sqrt(S_jj); S = D S D + shift*I;
// flags[0] set to 1 if some S_jj <= 0 or is not finite.
void gram_scale(bool cplx, void* S, int64_t lds, int64_t k, double shift, double* d,
                int* flags, hipStream_t st);
// A(i,i) += shift (real) for a k x k matrix
void add_diag(bool cplx, void* A, int64_t lda, int64_t k, double shift, hipStream_t st);
// M = D * triu(Rinv): scale row i by d_i, zero the strictly lower part.
void triu_rowscale(bool cplx, void* R, int64_t ldr, int64_t k, const double* d,
                   hipStream_t st);
void diag_real(bool cplx, const void* A, int64_t lda, int64_t k, double* out,
               hipStream_t st);
// res[j] = sqrt(sum_t partial[t][j]) * inv_scale
void resid_finish(const double* partial, int tiles, int64_t N, double inv_scale, double* res,
                  hipStream_t st);
// V = V * diag(g) (columns scaled by real g)
void scale_cols(bool cplx, void* V, int64_t ldv, int64_t n, int64_t k, const double* g,
                hipStream_t st);
// Y[:, j] = (a ? a[j] : 1) X[:, j] + (b ? b[j] : 0) Y[:, j]   (a, b on the device)
void axpby_cols(bool cplx, const double* a, const void* X, int64_t ldx, const double* b, void* Y,
                int64_t ldy, int64_t n, int64_t k, hipStream_t st);
// Y += a * X for n x k blocks
void axpy_cols(bool cplx, double a, const void* X, int64_t ldx, void* Y, int64_t ldy, int64_t n,
               int64_t k, hipStream_t st);
// Hermitian part in place: A = (A + A^H)/2 (n x n)
void herm_part(bool cplx, void* A, int64_t lda, int64_t n, hipStream_t st);
// c128 -> c64 (or double -> float) conversion of an n x n matrix into ld n
void to_f32(bool cplx, const void* src, int64_t lds, void* dst, int64_t n, hipStream_t st);
// flags[0] |= 1 if any entry of the n x k block is not finite
void check_finite(bool cplx, const void* X, int64_t ldx, int64_t n, int64_t k, int* flags,
                  hipStream_t st);

// Seeded N(0, 1) draws into an n x k block (ld ldx; complex: re and im each
// N(0, 1)) from a counter-based generator, reproducible for (seed, stream_id).
void fill_gaussian(bool cplx, void* X, int64_t ldx, int64_t n, int64_t k, uint64_t seed,
                   uint64_t stream_id, hipStream_t st);
// Debug checks of an n x n matrix: out2[0] = max |A - A^H| (mode 0) or
// max |A - I| (mode 1), out2[1] = max |A| (device doubles).
void max_defect(bool cplx, const void* A, int64_t lda, int64_t n, int mode, double* out2,
                hipStream_t st);
// Batched conjugate gradients (one system per column of an n x k block):
// out[j] = Re(x_j^H y_j)
void col_dots(bool cplx, const void* X, int64_t ldx, const void* Y, int64_t ldy, int64_t n,
              int64_t k, double* out, hipStream_t st);
// Column j is live while rr_j > tol2 rr0_j and pq_j > 0 (converged or
// broken-down columns are frozen).  Live columns: alpha_j = rr_j / pq_j;
// X += alpha P; R -= alpha Q; rr_new_j = |r_j|^2; frozen: rr_new_j = rr_j.
// (all blocks ld `ld`)
void cg_step(bool cplx, void* X, void* R, const void* P, const void* Q, int64_t ld, int64_t n,
             int64_t k, const double* rr, const double* rr0, const double* pq, double tol2,
             double* rr_new, hipStream_t st);
// Live columns (same test, before the step): beta_j = rr_new_j / rr_j;
// P = R + beta P; rr = rr_new
void cg_dir(bool cplx, void* P, const void* R, int64_t ld, int64_t n, int64_t k, double* rr,
            const double* rr0, const double* pq, double tol2, const double* rr_new,
            hipStream_t st);
// E = Hermitian part of the divided-difference matrix M_ij / (lam_j - lam_i)
// (0 on the diagonal and between equal eigenvalues), k x k
void sym_divdiff(bool cplx, const void* M, int64_t ldm, const double* lam, int64_t k, void* E,
                 int64_t lde, hipStream_t st);

// ------------------------------------------------------------------ FP64 products on INT8
// Integer modular emulation of the FP64 filter product (crt.hip).
constexpr int kCrtMaxModuli = 16;
// fewest moduli with which Rayleigh-Ritz's H Q also runs on INT8
constexpr int kCrtMinModuliRR = 14;
struct CrtBasis {
  int n_mod;               // number of moduli (8, 10, 12, 14 or 16)
  int m[kCrtMaxModuli];    // the moduli
  int inv[kCrtMaxModuli];  // (m_0 ... m_{t-1})^{-1} mod m_t
  int pa, pb;              // bits of the integer forms of H's rows and X's columns
};
// Basis for products with inner dimension K.
CrtBasis crt_basis(int n_mod, int64_t K, bool cplx);
// Device bytes: residue planes of H (+ row exponents); per-step planes of a
// block of up to kmax columns, their INT32 products and column exponents.
size_t crt_h_bytes(bool cplx, int64_t n, int n_mod);
size_t crt_x_bytes(bool cplx, int64_t n, int kmax, int n_mod);
// Residue planes of the Hermitian H into hbuf (crt_h_bytes).
void crt_prepare_h(bool cplx, const void* H, int64_t ldh, int64_t n, const CrtBasis& B,
                   void* hbuf, hipStream_t st);
// One filter step with the EPI_CHEB epilogue (GemmArgs as for gemm(); A must
// be the H whose planes hbuf holds), products on the INT8 matrix cores.
void crt_cheb(bool cplx, const GemmArgs& g, const CrtBasis& B, const void* hbuf, void* xbuf,
              int kmax, rocblas_handle rb, hipStream_t st);

// ------------------------------------------------------------------ Cholesky
// A = R^H R for the Hermitian positive definite k x k matrix A (ld lda,
// upper triangle read and overwritten by R; the strict lower triangle is
// left alone).  d_info (device) receives 0, or the 1-based order of the
// first pivot that is not positive (then A holds partial results).
void cholesky_upper(bool cplx, void* A, int64_t lda, int k, int* d_info, hipStream_t st);

// ------------------------------------------------------------------ Jacobi eigensolver
// Device workspace of the block Jacobi eigensolver for orders up to kmax.
size_t jacobi_ws_bytes(bool cplx, int kmax);
// Squared Frobenius norms of a k x k matrix: off2 off the diagonal, dia2 on it
// (synchronises the stream).
void jacobi_norms(bool cplx, const void* G, int64_t ldg, int k, void* ws, int kmax, double* off2,
                  double* dia2, hipStream_t st);
// Eigen-decomposition of the Hermitian k x k G (destroyed) by block-cyclic
// Jacobi until off2 <= tol^2 (off2 + dia2) (the norms of G on entry, from
// jacobi_norms); V (k x k) is scratch, W (may be G) receives the
// eigenvectors and d_evals / evals_host the eigenvalues, ascending; d_perm
// holds k ints.  Returns the sweeps; throws CHASE_ERR_NUMERIC after
// max_sweeps.
int jacobi_heev(bool cplx, void* G, int64_t ldg, int k, void* V, int64_t ldv, void* W,
                int64_t ldw, double* d_evals, int* d_perm, void* ws, int kmax, double* evals_host,
                hipStream_t st, double off2, double dia2, double tol, int max_sweeps);

// ------------------------------------------------------------------ Lanczos
struct LanczosBufs {
  void* q_prev;    // n x nv
  void* q_cur;     // n x nv
  void* w;         // n x nv
  void* wpart;     // splits x nv x n
  double* dotp;    // blocks x nv
  double* nrmp;    // blocks x nv
  double* alpha;   // steps x nv
  double* beta;    // steps x nv
  int max_splits;
  hipEvent_t* gemv_ev = nullptr;  // optional: 2 x steps events around each block GEMV
};
void lanczos_run(bool cplx, const void* H, int64_t ldh, int64_t n, const void* S, int nv,
                 int steps, LanczosBufs& b, hipStream_t st);
size_t lanczos_bytes(bool cplx, int64_t n, int nv, int steps, int* max_splits);

}  // namespace chase
