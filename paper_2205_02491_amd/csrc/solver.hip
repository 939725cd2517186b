// ChASE driver (Algorithm 1) on one MI355X and the C ABI of include/chase.h.
//
// H stays resident and const in HBM for the whole solve; the search block
// V (n x (nev+nex)) and two scratch blocks of the same shape live in the
// handle's workspace, allocated once (the paper pre-allocates its library
// buffers before the main loop).  Per iteration the host only sees a few KB:
// the QR pivots, the Ritz values and the residual norms.
#include <rocblas/rocblas.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "common.h"
#include "hostmath.h"

using namespace chase;

struct chase_handle_s {
  chase_dtype dtype;
  bool cplx;
  int64_t n;
  int nev, nex, ne;
  chase_opts opts;
  size_t esz;  // bytes per element (16 or 8)
  int device;
  // n x ne blocks, ld n
  void *V = nullptr, *W = nullptr, *Z = nullptr;
  // ne x ne matrices
  void *G = nullptr, *R = nullptr;
  void* ws = nullptr;  // split-K workspace
  size_t ws_elems = 0;
  double *d_scale = nullptr, *d_evals = nullptr, *d_res = nullptr, *d_partial = nullptr,
         *d_E = nullptr, *d_g = nullptr;
  int *d_flags = nullptr, *d_info = nullptr, *d_perm = nullptr;
  void* tau = nullptr;
  LanczosBufs lz{};
  void* H32 = nullptr;   // low-precision copy of H for the FP32 filter
  // split-BF16 filter: s8 splits of conj(H) (columns padded to S8_COLS_A)
  // and of the block being multiplied (ne padded to S8_COLS_B columns)
  void* Hs8 = nullptr;
  void* Xs8 = nullptr;
  void* Xs8b = nullptr;     // second block split: step s writes step s+1's operand
  float* s8tail = nullptr;  // FP32 partial tiles of the GEMM's split-K tail
  int64_t s8_groups = 0;
  void* Rres = nullptr;  // residual vectors H v - theta v of the active block (mixed modes)
  double* d_coef = nullptr;  // per-step, per-column coefficients of the filter's defect form
  // filter tape (record_tape)
  void* tape = nullptr;
  size_t tape_bytes = 0;
  void* adj = nullptr;  // eigenvector adjoint: two n x ne blocks (first use; in allocs)
  void* jac_ws = nullptr;  // Jacobi eigensolver workspace (orders up to ne)
  // FP64 filter products on the INT8 matrix cores (opts.fp64_emulation > 0):
  // residue planes of H and the per-step buffers
  void* crt_h = nullptr;
  void* crt_x = nullptr;
  CrtBasis crt{};
  std::vector<int> tape_deg;
  std::vector<Coef> tape_coef;
  int tape_k = 0;
  bool tape_valid = false;
  rocblas_handle rb = nullptr;
  std::vector<hipEvent_t> evs;
  hipEvent_t eig_ev[2] = {nullptr, nullptr};  // around the small eigensolve
  std::vector<void*> allocs;
};

// Work buffers of chase_lanczos_noalloc: a fixed device array (one copy per
// GPU, held until the process ends) instead of a handle's workspace.  Host
// code reaches it only through the address hipGetSymbolAddress returns on
// each device; the array's name is not a device address on the host.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_last_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the no-allocation scratch on the current device, looked
// up once per device.
char* noalloc_scratch() {
  int dev = 0;
  CHASE_HIP(hipGetDevice(&dev));
  CHASE_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    CHASE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    CHASE_REQUIRE(p != nullptr, "scratch symbol has no device address");
    g_scratch_ptr[dev] = p;
  }
  return static_cast<char*>(g_scratch_ptr[dev]);
}

// roctx range around a phase of the solve: named spans on the timeline of
// a profiler that records markers (rocprofv3 --marker-trace); a few hundred
// nanoseconds each otherwise.
struct Range {
  bool open = true;
  explicit Range(const char* name) { roctxRangePushA(name); }
  void end() {
    if (open) roctxRangePop();
    open = false;
  }
  ~Range() { end(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

using clk = std::chrono::steady_clock;
double secs(clk::time_point a, clk::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}

char* off(void* p, int64_t elems, size_t esz) { return static_cast<char*>(p) + elems * (int64_t)esz; }

void* dev_alloc(chase_handle_s* h, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(CHASE_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  h->allocs.push_back(p);
  return p;
}

// Host-to-device copy of a small pageable host array; returns once the copy
// has completed so the host array may go out of scope.
void h2d_sync(void* dst, const void* src, size_t bytes, hipStream_t st) {
  CHASE_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
  CHASE_HIP(hipStreamSynchronize(st));
}

void rb_check(rocblas_status s, const char* what) {
  if (s != rocblas_status_success)
    throw Error(CHASE_ERR_HIP, std::string(what) + " failed: " + rocblas_status_to_string(s));
}

size_t splitk_ws_elems(int ne) {
  size_t mx = 0;
  for (int k = 1; k <= ne; ++k) {
    int s;
    int64_t ks;
    // K is at least ne (the library's projections have K = n >= ne); the
    // Hermitian products computed as triangles have the most slices
    splitk_plan(k, k, INT64_MAX / 4, &s, &ks, true);
    mx = std::max(mx, (size_t)s * k * k);
  }
  return mx;
}

constexpr int kMaxDegree = 1000;  // largest filter degree any entry point accepts

struct Sizes {
  size_t blocks, small, lz, ws, h32, adj, crt, total;
  int lz_splits;
};

Sizes sizes(chase_dtype dt, int64_t n, int nev, int nex, const chase_opts& o) {
  Sizes s{};
  const bool cplx = dt == CHASE_C128;
  const size_t esz = cplx ? 16 : 8;
  const int64_t ne = nev + nex;
  s.blocks = 3 * (size_t)n * ne * esz + 2 * (size_t)ne * ne * esz;
  s.ws = splitk_ws_elems((int)ne) * esz;
  s.small = (size_t)ne * 8 * 5 + (size_t)gemm_row_tiles(n) * ne * 8 + 64 + (size_t)ne * 4 +
            (size_t)ne * esz;
  s.lz = lanczos_bytes(cplx, n, o.lanczos_vecs, o.lanczos_steps, &s.lz_splits);
  if (o.filter_prec == CHASE_PREC_FP32)
    s.h32 = (size_t)n * n * esz / 2 + (size_t)n * ne * esz;
  else if (o.filter_prec == CHASE_PREC_BF16X3 || o.filter_prec == CHASE_PREC_BF16X2)
    s.h32 = s8_bytes(cplx, n, s8_pad(n, S8_COLS_A)) +
            2 * s8_bytes(cplx, n, s8_pad(ne, S8_COLS_B)) + s8_tail_bytes(cplx) +
            (size_t)n * ne * esz;
  s.small += (size_t)(kMaxDegree + 1) * ne * 8;
  s.small += jacobi_ws_bytes(cplx, (int)ne);
  // adjoint buffers reserved up front: the eigenvector adjoint's two blocks
  // and a filter tape of adjoint_reserve steps over ne columns
  if (o.adjoint_reserve > 0)
    s.adj = 2 * (size_t)n * ne * esz + (size_t)(o.adjoint_reserve + 1) * n * ne * esz;
  if (o.fp64_emulation > 0)
    s.crt = crt_h_bytes(cplx, n, o.fp64_emulation) + crt_x_bytes(cplx, n, (int)ne, o.fp64_emulation);
  s.total = s.blocks + s.ws + s.small + s.lz + s.h32 + s.adj + s.crt;
  return s;
}

void validate_opts(const chase_opts& o) {
  CHASE_REQUIRE(o.max_deg >= 2 && o.max_deg <= kMaxDegree, "max_deg out of range [2,1000]");
  CHASE_REQUIRE(o.deg_extra >= 0, "deg_extra < 0");
  CHASE_REQUIRE(o.lanczos_steps >= 1 && o.lanczos_steps <= 200, "lanczos_steps out of range");
  CHASE_REQUIRE(o.lanczos_vecs >= 1 && o.lanczos_vecs <= 8, "lanczos_vecs out of range [1,8]");
  CHASE_REQUIRE(o.adjoint_reserve >= 0 && o.adjoint_reserve <= kMaxDegree,
                "adjoint_reserve out of range [0, 1000]");
  CHASE_REQUIRE(o.max_iter >= 1, "max_iter < 1");
  CHASE_REQUIRE(o.initial_rr == 0 || o.initial_rr == 1, "initial_rr must be 0 or 1");
  CHASE_REQUIRE(o.fp64_tail >= -1 && o.fp64_tail <= kMaxDegree, "fp64_tail out of range [-1,1000]");
  CHASE_REQUIRE(o.fp64_emulation == 0 || o.fp64_emulation == 8 || o.fp64_emulation == 10 ||
                    o.fp64_emulation == 12 || o.fp64_emulation == 14 || o.fp64_emulation == 16,
                "fp64_emulation must be 0, 8, 10, 12, 14 or 16");
  CHASE_REQUIRE(o.eig_solver == CHASE_EIG_AUTO || o.eig_solver == CHASE_EIG_LIBRARY ||
                    o.eig_solver == CHASE_EIG_JACOBI,
                "unknown eig_solver");
  CHASE_REQUIRE(o.filter_prec == CHASE_PREC_FP64 || o.filter_prec == CHASE_PREC_FP32 ||
                    o.filter_prec == CHASE_PREC_BF16X3 || o.filter_prec == CHASE_PREC_BF16X2,
                "unknown filter_prec");
}

// ------------------------------------------------------------------ GEMM helpers
GemmArgs gargs(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
               int64_t ldb, void* C, int64_t ldc) {
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  g.C = C;
  g.ldc = ldc;
  g.alpha = 1.0;
  return g;
}

// C (k1 x k2, ld ldc) = A^H B for tall A (K x k1), B (K x k2).  herm: the
// product is Hermitian (k1 == k2); only the tiles on and above the diagonal
// are computed and the result is made exactly Hermitian (mirrored tiles,
// (S+S^H)/2 within the diagonal ones).
void gram(chase_handle_s* h, const void* A, int64_t lda, const void* B, int64_t ldb, int64_t K,
          int64_t k1, int64_t k2, void* C, int64_t ldc, bool herm, hipStream_t st) {
  const bool tri = herm && k1 == k2;
  int splits;
  int64_t ks;
  splitk_plan(k1, k2, K, &splits, &ks, tri);
  CHASE_REQUIRE((size_t)splits * k1 * k2 <= h->ws_elems, "split-K workspace too small");
  GemmArgs g = gargs(k1, k2, K, A, lda, B, ldb, h->ws, k1);
  g.splits = splits;
  g.kslice = ks;
  g.tri = tri ? 1 : 0;
  gemm(h->cplx, PREC_F64, OP_C, OP_N, EPI_SPLITK, g, st);
  splitk_reduce(h->cplx, h->ws, splits, k1, k2, C, ldc, herm, st, tri ? splitk_tile() : 0);
}

// C = A B; tri_row0 >= 0: column j of B is zero below row tri_row0 + j
// (an upper-triangular factor), which bounds the K loop of each column tile.
void gemm_nn(chase_handle_s* h, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda,
             const void* B, int64_t ldb, void* C, int64_t ldc, hipStream_t st,
             int64_t tri_row0 = -1) {
  GemmArgs g = gargs(M, N, K, A, lda, B, ldb, C, ldc);
  if (tri_row0 >= 0) {
    g.tri = 1;
    g.tri_row0 = tri_row0;
  }
  gemm(h->cplx, PREC_F64, OP_N, OP_N, EPI_STORE, g, st);
}

// ------------------------------------------------------------------ filter
struct FilterTiming {
  int64_t matvecs = 0;
  double ktime = 0.0;  // seconds of filter GEMMs (HIP events)
  int64_t launches = 0;
};

Prec to_prec(int p) {
  return p == CHASE_PREC_BF16X3   ? PREC_BF16X3
         : p == CHASE_PREC_BF16X2 ? PREC_BF16X2
         : p == CHASE_PREC_FP32   ? PREC_F32
                                  : PREC_F64;
}

// Split-BF16 operands of the filter steps.  The split of H is the
// handle's.  The block operand of a step is split by the split kernel on the
// first step of a filter call; every later step finds it already written by
// the previous step's epilogue (which emits the split of its output beside
// the FP64 result), so the block is split once per call, not per step.
// The split kernel runs outside the timed GEMM window.
struct Bf16Steps {
  chase_handle_s* h;
  void* cur;          // split of this step's operand
  void* other;        // where this step's epilogue writes the next operand
  bool ready = false; // cur already holds this step's operand
  explicit Bf16Steps(chase_handle_s* hh) : h(hh), cur(hh->Xs8), other(hh->Xs8b) {
    CHASE_REQUIRE(h->Hs8 && h->Xs8 && h->Xs8b, "split-BF16 products need a handle created with "
                                              "filter_prec = CHASE_PREC_BF16X3 or BF16X2");
  }
  // g: the step's GEMM (B = its FP64 operand, cols columns); next_col0 >= 0:
  // the next step multiplies this step's output columns [next_col0, cols)
  void prepare(GemmArgs& g, int cols, int next_col0, hipStream_t st) {
    if (!ready)
      split_s8(h->cplx, false, g.B, g.ldb, h->n, cols, s8_pad(cols, S8_COLS_B), cur,
               h->s8_groups, st);
    g.a_s8 = h->Hs8;
    g.b_s8 = cur;
    g.s8_groups = h->s8_groups;
    g.s8_tail = h->s8tail;
    g.s8_next = next_col0 >= 0 ? other : nullptr;
    g.s8_next_col0 = next_col0 >= 0 ? next_col0 : 0;
  }
  void advance(const GemmArgs& g) {
    ready = g.s8_next != nullptr;
    if (ready) std::swap(cur, other);
  }
};

// First active column of filter step s (degrees non-decreasing).
int step_first_col(const int* deg, int k, int s) {
  return (int)(std::lower_bound(deg, deg + k, s) - deg);
}

// split of conj(H) = H^T (H Hermitian) for the split-BF16 products
void split_h(chase_handle_s* h, const void* H, int64_t ldh, hipStream_t st) {
  CHASE_REQUIRE(h->Hs8, "split-BF16 products need a handle created with "
                        "filter_prec = CHASE_PREC_BF16X3 or BF16X2");
  split_s8(h->cplx, true, H, ldh, h->n, h->n, s8_pad(h->n, S8_COLS_A), h->Hs8, h->s8_groups, st);
}

// One FP64 filter step (EPI_CHEB): on the FP64 matrix cores, or with the
// handle's fp64_emulation on the INT8 ones (H's residue planes must have been
// prepared from the same H, crt_prepare_h).
void fp64_step(chase_handle_s* h, const GemmArgs& g, hipStream_t st) {
  if (h->crt_h)
    crt_cheb(h->cplx, g, h->crt, h->crt_h, h->crt_x, h->ne, h->rb, st);
  else
    gemm(h->cplx, PREC_F64, OP_N, OP_N, EPI_CHEB, g, st);
}

void prepare_h_products(chase_handle_s* h, const void* H, int64_t ldh, hipStream_t st) {
  if (h->crt_h) crt_prepare_h(h->cplx, H, ldh, h->n, h->crt, h->crt_h, st);
}

// X (n x k, ld ldx) <- p_{m_a}(H) x_a ; Wb (n x k, ld ldw) ping-pong scratch.
// degrees non-decreasing, even, >= 2.  With a low precision `prec`, steps
// s >= fp64_from run with FP64 products instead (timed into *ft64): the
// rounding errors of the earlier low-precision steps are then damped by the
// remaining steps like any other unwanted component.
void run_filter(chase_handle_s* h, const void* H, int64_t ldh, void* X, int64_t ldx, void* Wb,
                int64_t ldw, int k, const int* deg, double b_sup, double mu_1, double mu_ne,
                Prec prec, bool tape, FilterTiming& ft, hipStream_t st, int fp64_from = 0,
                FilterTiming* ft64 = nullptr) {
  if (k <= 0) return;
  const int64_t n = h->n;
  const int mmax = deg[k - 1];
  if (prec == PREC_F64 || fp64_from <= 0 || !ft64) fp64_from = mmax + 1;
  const std::vector<Coef> cf = cheb_coefficients(mmax, b_sup, mu_1, mu_ne);
  const void* Ah = H;
  int64_t lda = ldh;
  int a_f32 = 0;
  if (prec == PREC_F32 && h->H32) {
    Ah = h->H32;
    lda = n;
    a_f32 = 1;
  }
  if (tape) {
    // slot s holds X_s of all k columns (columns not active at step s keep
    // their last value, which the adjoint never reads)
    copy_cols(h->cplx, X, ldx, h->tape, n, n, k, st);
  }
  const size_t need_ev = 2 * (size_t)mmax;
  while (h->evs.size() < need_ev) {
    hipEvent_t e;
    CHASE_HIP(hipEventCreate(&e));
    h->evs.push_back(e);
  }
  std::unique_ptr<Bf16Steps> bsteps;
  if (is_split_bf16(prec)) bsteps.reset(new Bf16Steps(h));
  for (int s = 1; s <= mmax; ++s) {
    const int a0 = step_first_col(deg, k, s);
    const int cols = k - a0;
    if (cols <= 0) continue;
    const bool low = s < fp64_from;
    void* src = (s & 1) ? X : Wb;  // X_{s-1}
    void* dst = (s & 1) ? Wb : X;  // X_s over X_{s-2}
    const int64_t lds = (s & 1) ? ldx : ldw, ldd = (s & 1) ? ldw : ldx;
    GemmArgs g = gargs(n, cols, n, low ? Ah : H, low ? lda : ldh, off(src, a0 * lds, h->esz), lds,
                       off(dst, a0 * ldd, h->esz), ldd);
    g.alpha = cf[s - 1].alpha;
    g.gamma = cf[s - 1].gamma;
    g.beta = cf[s - 1].beta;
    g.a_f32 = low ? a_f32 : 0;
    if (bsteps && low) {
      // the epilogue emits the next step's operand split only if that step
      // also runs on split-BF16 products
      const int a1 = step_first_col(deg, k, s + 1);
      bsteps->prepare(g, cols, (s < mmax && a1 < k && s + 1 < fp64_from) ? a1 - a0 : -1, st);
    }
    CHASE_HIP(hipEventRecord(h->evs[2 * (s - 1)], st));
    if (low && prec != PREC_F64)
      gemm(h->cplx, prec, OP_N, OP_N, EPI_CHEB, g, st);
    else
      fp64_step(h, g, st);
    CHASE_HIP(hipEventRecord(h->evs[2 * (s - 1) + 1], st));
    if (bsteps && low) bsteps->advance(g);
    FilterTiming& fs = low ? ft : *ft64;
    fs.matvecs += cols;
    fs.launches += 1;
    if (tape)
      copy_cols(h->cplx, off(dst, a0 * ldd, h->esz), ldd,
                off(h->tape, ((int64_t)s * k + a0) * n, h->esz), n, n, cols, st);
  }
  CHASE_HIP(hipStreamSynchronize(st));
  for (int s = 1; s <= mmax; ++s) {
    const int a0 = (int)(std::lower_bound(deg, deg + k, s) - deg);
    if (k - a0 <= 0) continue;
    float ms = 0.f;
    CHASE_HIP(hipEventElapsedTime(&ms, h->evs[2 * (s - 1)], h->evs[2 * (s - 1) + 1]));
    (s < fp64_from ? ft : *ft64).ktime += ms * 1e-3;
  }
  if (tape) {
    h->tape_deg.assign(deg, deg + k);
    h->tape_coef = cf;
    h->tape_k = k;
    h->tape_valid = true;
  }
}

// Defect-correction form of the filter for Ritz vectors.  V (n x k, ld ldv)
// holds Ritz vectors v_a with Ritz values theta[a] and residuals
// R (n x k, ld ldr), r_a = H v_a - theta_a v_a.  With T_s the scaled
// Chebyshev polynomials of Eq. (3) (T_0 = 1):
//   p(H) v = T_m(theta) v + D_m,   D_0 = 0,  D_1 = alpha_1 r,
//   D_s = alpha_s (H - gamma I) D_{s-1} + beta_s D_{s-2} + alpha_s T_{s-1}(theta) r,
// which follows from (H - gamma I) v = (theta - gamma) v + r.  The rounding
// error of the products H D is relative to ||D|| ~ ||r|| instead of ||p(H) v||,
// so FP32 products keep the convergence of the FP64 filter down to FP64
// residual levels.  D ping-pongs between W1 (odd s) and W2 (even s), ld n.
void run_filter_defect(chase_handle_s* h, const void* H, int64_t ldh, void* V, int64_t ldv,
                       const void* R, int64_t ldr, void* W1, void* W2, int k, const int* deg,
                       const double* theta, double b_sup, double mu_1, double mu_ne, Prec prec,
                       FilterTiming& ft, hipStream_t st) {
  if (k <= 0) return;
  const int64_t n = h->n;
  const int mmax = deg[k - 1];
  const std::vector<Coef> cf = cheb_coefficients(mmax, b_sup, mu_1, mu_ne);
  // coefficient table: row s (1..mmax) = alpha_s T_{s-1}(theta_a); row 0 = T_{m_a}(theta_a)
  std::vector<double> tab((size_t)(mmax + 1) * k, 0.0);
  for (int a = 0; a < k; ++a) {
    double tp = 0.0, tc = 1.0;
    for (int s = 1; s <= deg[a]; ++s) {
      const Coef& c = cf[s - 1];
      tab[(size_t)s * k + a] = c.alpha * tc;
      const double tn = c.alpha * (theta[a] - c.gamma) * tc + c.beta * tp;
      tp = tc;
      tc = tn;
    }
    tab[a] = tc;
  }
  h2d_sync(h->d_coef, tab.data(), tab.size() * 8, st);
  const void* Ah = H;
  int64_t lda = ldh;
  int a_f32 = 0;
  if (prec == PREC_F32 && h->H32) {
    Ah = h->H32;
    lda = n;
    a_f32 = 1;
  }
  while (h->evs.size() < 2 * (size_t)mmax) {
    hipEvent_t e;
    CHASE_HIP(hipEventCreate(&e));
    h->evs.push_back(e);
  }
  // D_1 = alpha_1 r ; D_0 = 0
  axpby_cols(h->cplx, h->d_coef + k, R, ldr, nullptr, W1, n, n, k, st);
  fill_zero(W2, (int64_t)n * k * (int64_t)h->esz, st);
  std::unique_ptr<Bf16Steps> bsteps;
  if (is_split_bf16(prec)) bsteps.reset(new Bf16Steps(h));
  for (int s = 2; s <= mmax; ++s) {
    const int a0 = step_first_col(deg, k, s);
    const int cols = k - a0;
    if (cols <= 0) continue;
    void* src = (s & 1) ? W2 : W1;  // D_{s-1}
    void* dst = (s & 1) ? W1 : W2;  // D_s over D_{s-2}
    GemmArgs g = gargs(n, cols, n, Ah, lda, off(src, (int64_t)a0 * n, h->esz), n,
                       off(dst, (int64_t)a0 * n, h->esz), n);
    g.alpha = cf[s - 1].alpha;
    g.gamma = cf[s - 1].gamma;
    g.beta = cf[s - 1].beta;
    g.a_f32 = a_f32;
    g.colcoef = h->d_coef + (size_t)s * k + a0;
    g.F = const_cast<char*>(static_cast<const char*>(R)) + (int64_t)a0 * ldr * (int64_t)h->esz;
    g.ldf = ldr;
    if (bsteps) {
      const int a1 = step_first_col(deg, k, s + 1);
      bsteps->prepare(g, cols, (s < mmax && a1 < k) ? a1 - a0 : -1, st);
    }
    CHASE_HIP(hipEventRecord(h->evs[2 * (s - 1)], st));
    if (prec == PREC_F64)
      fp64_step(h, g, st);
    else
      gemm(h->cplx, prec, OP_N, OP_N, EPI_CHEB, g, st);
    CHASE_HIP(hipEventRecord(h->evs[2 * (s - 1) + 1], st));
    if (bsteps) bsteps->advance(g);
    ft.matvecs += cols;
    ft.launches += 1;
  }
  // p(H) v = T_m(theta) v + D_m  (degrees are even: D_m is in W2)
  axpby_cols(h->cplx, nullptr, W2, n, h->d_coef, V, ldv, n, k, st);
  CHASE_HIP(hipStreamSynchronize(st));
  for (int s = 2; s <= mmax; ++s) {
    const int a0 = (int)(std::lower_bound(deg, deg + k, s) - deg);
    if (k - a0 <= 0) continue;
    float ms = 0.f;
    CHASE_HIP(hipEventElapsedTime(&ms, h->evs[2 * (s - 1)], h->evs[2 * (s - 1) + 1]));
    ft.ktime += ms * 1e-3;
  }
}

void ensure_tape(chase_handle_s* h, int k, int mmax) {
  const size_t need = (size_t)(mmax + 1) * h->n * k * h->esz;
  if (h->tape && h->tape_bytes >= need) return;
  if (h->tape) {
    CHASE_HIP(hipFree(h->tape));
    h->tape = nullptr;
    h->tape_bytes = 0;
  }
  size_t fr = 0, tot = 0;
  CHASE_HIP(hipMemGetInfo(&fr, &tot));
  if (need > fr) throw Error(CHASE_ERR_NOMEM, "filter tape does not fit in device memory");
  if (hipMalloc(&h->tape, need) != hipSuccess) {
    (void)hipGetLastError();
    h->tape = nullptr;
    throw Error(CHASE_ERR_NOMEM, "filter tape allocation failed");
  }
  h->tape_bytes = need;
}

// ------------------------------------------------------------------ QR
// Orthonormalise X (n x k, ld ldx) keeping its first L columns.
// Cholesky QR with column scaling (S = D X^H X D = R^H R, X <- X D R^{-1})
// until two consecutive passes are clean (CholeskyQR2).  A pass whose factor
// shows a condition number near 1/sqrt(eps) (smallest pivot of the scaled
// factor below 1e-5, or a failed factorisation) is redone on the shifted Gram
// matrix S + sI, s = 11 (n k + k (k+1)) eps ||XD||_F^2 (shifted Cholesky QR);
// each shifted pass divides the condition number by about 1/sqrt(s/k), so
// even numerically rank-deficient filtered blocks are reduced in a few
// passes.  Householder QR is the last resort.  Scratch: Wb (n x k, ld n),
// R (k x k), G (k x k, copy of the scaled Gram matrix).
void householder_qr(chase_handle_s* h, void* X, int64_t ldx, int k, int L, void* Wb,
                    chase_stats* stats, hipStream_t st) {
  const int64_t n = h->n;
  const bool cplx = h->cplx;
  if (stats) stats->qr_householder++;
  if (L > 0) copy_cols(cplx, X, ldx, Wb, n, n, L, st);
  if (cplx) {
    rb_check(rocsolver_zgeqrf(h->rb, n, k, static_cast<rocblas_double_complex*>(X), ldx,
                              static_cast<rocblas_double_complex*>(h->tau)),
             "zgeqrf");
    rb_check(rocsolver_zungqr(h->rb, n, k, k, static_cast<rocblas_double_complex*>(X), ldx,
                              static_cast<rocblas_double_complex*>(h->tau)),
             "zungqr");
  } else {
    rb_check(rocsolver_dgeqrf(h->rb, n, k, static_cast<double*>(X), ldx,
                              static_cast<double*>(h->tau)),
             "dgeqrf");
    rb_check(rocsolver_dorgqr(h->rb, n, k, k, static_cast<double*>(X), ldx,
                              static_cast<double*>(h->tau)),
             "dorgqr");
  }
  if (L > 0) copy_cols(cplx, Wb, n, X, ldx, n, L, st);
  int bad = 0;
  fill_zero(h->d_flags, sizeof(int), st);
  check_finite(cplx, X, ldx, n, k, h->d_flags, st);
  CHASE_HIP(hipMemcpyAsync(&bad, h->d_flags, sizeof(int), hipMemcpyDeviceToHost, st));
  CHASE_HIP(hipStreamSynchronize(st));
  if (bad) throw Error(CHASE_ERR_NUMERIC, "QR breakdown (non-finite values)");
}

void potrf(chase_handle_s* h, void* R, int64_t ldr, int k, hipStream_t st) {
  cholesky_upper(h->cplx, R, ldr, k, h->d_info, st);
}

void qr_step(chase_handle_s* h, void* X, int64_t ldx, int k, int L, void* Wb, chase_stats* stats,
             hipStream_t st) {
  const int64_t n = h->n;
  const bool cplx = h->cplx;
  void* R = h->R;
  const int64_t ldr = k;
  const double u = 1.1102230246251565e-16;
  const double shift = 11.0 * ((double)n * k + (double)k * (k + 1)) * u * (double)k;
  constexpr int kMaxShifted = 6;
  int clean = 0, shifted = 0;
  std::vector<double> diag(k);
  int hinfo[2];
  auto sync_info = [&](bool want_diag) {
    CHASE_HIP(hipMemcpyAsync(&hinfo[0], h->d_info, sizeof(int), hipMemcpyDeviceToHost, st));
    CHASE_HIP(hipMemcpyAsync(&hinfo[1], h->d_flags, sizeof(int), hipMemcpyDeviceToHost, st));
    if (want_diag) {
      diag_real(cplx, R, ldr, k, h->d_res, st);
      CHASE_HIP(hipMemcpyAsync(diag.data(), h->d_res, k * sizeof(double),
                               hipMemcpyDeviceToHost, st));
    }
    CHASE_HIP(hipStreamSynchronize(st));
  };
  while (clean < 2) {
    gram(h, X, ldx, X, ldx, n, k, k, R, ldr, true, st);
    fill_zero(h->d_flags, 2 * sizeof(int), st);
    gram_scale(cplx, R, ldr, k, 0.0, h->d_scale, h->d_flags, st);
    // keep the scaled Gram matrix in case the pass has to be shifted
    copy_cols(cplx, R, ldr, h->G, ldr, k, k, st);
    potrf(h, R, ldr, k, st);
    sync_info(true);
    if (hinfo[1] != 0) return householder_qr(h, X, ldx, k, L, Wb, stats, st);
    double dmin = INFINITY;
    for (double d : diag) dmin = std::min(dmin, std::fabs(d));
    const bool ok = hinfo[0] == 0 && dmin >= 1e-5;
    if (!ok) {
      if (clean > 0 || shifted >= kMaxShifted)
        return householder_qr(h, X, ldx, k, L, Wb, stats, st);
      // shifted pass on the saved Gram matrix
      copy_cols(cplx, h->G, ldr, R, ldr, k, k, st);
      add_diag(cplx, R, ldr, k, shift, st);
      potrf(h, R, ldr, k, st);
      sync_info(false);
      if (hinfo[0] != 0) return householder_qr(h, X, ldx, k, L, Wb, stats, st);
      ++shifted;
      if (stats) stats->qr_shifted++;
    } else {
      ++clean;
    }
    if (cplx)
      rb_check(rocsolver_ztrtri(h->rb, rocblas_fill_upper, rocblas_diagonal_non_unit, k,
                                static_cast<rocblas_double_complex*>(R), ldr, h->d_info),
               "ztrtri");
    else
      rb_check(rocsolver_dtrtri(h->rb, rocblas_fill_upper, rocblas_diagonal_non_unit, k,
                                static_cast<double*>(R), ldr, h->d_info),
               "dtrtri");
    triu_rowscale(cplx, R, ldr, k, h->d_scale, st);
    // Wb = X * (D R^{-1}); the locked columns keep their values.  Column j
    // of the factor's block [L, k) is zero below row L + j.
    gemm_nn(h, n, k - L, k, X, ldx, off(R, (int64_t)L * ldr, h->esz), ldr, Wb, n, st, L);
    copy_cols(cplx, Wb, n, off(X, (int64_t)L * ldx, h->esz), ldx, n, k - L, st);
  }
}

// ------------------------------------------------------------------ Rayleigh-Ritz + residual
// The automatic choice runs Jacobi when the off-diagonal part of the
// projected matrix has at most this fraction of its Frobenius norm.
constexpr double kAutoJacobiOff = 0.05;
constexpr double kJacobiTol = 1e-14;
constexpr int kJacobiMaxSweeps = 60;

// Dense eigensolve of the Hermitian k x k matrix h->G (ld k): eigenvalues
// ascending to h->d_evals, eigenvectors over h->G.  Returns the Jacobi
// sweeps (-1: the library's divide and conquer ran).
int small_eig(chase_handle_s* h, int k, int method, hipStream_t st) {
  double off2 = 0.0, dia2 = 0.0;
  if (method != CHASE_EIG_LIBRARY) {
    jacobi_norms(h->cplx, h->G, k, k, h->jac_ws, h->ne, &off2, &dia2, st);
    if (method == CHASE_EIG_AUTO)
      method = off2 <= kAutoJacobiOff * kAutoJacobiOff * (off2 + dia2) ? CHASE_EIG_JACOBI
                                                                        : CHASE_EIG_LIBRARY;
  }
  if (method == CHASE_EIG_JACOBI) {
    // callers check the library solver's info word: Jacobi reports by throwing
    fill_zero(h->d_info, sizeof(int), st);
    std::vector<double> ev(k);
    return jacobi_heev(h->cplx, h->G, k, k, h->R, k, h->G, k, h->d_evals, h->d_perm, h->jac_ws,
                       h->ne, ev.data(), st, off2, dia2, kJacobiTol, kJacobiMaxSweeps);
  }
  if (h->cplx)
    rb_check(rocsolver_zheevd(h->rb, rocblas_evect_original, rocblas_fill_upper, k,
                              static_cast<rocblas_double_complex*>(h->G), k, h->d_evals, h->d_E,
                              h->d_info),
             "zheevd");
  else
    rb_check(rocsolver_dsyevd(h->rb, rocblas_evect_original, rocblas_fill_upper, k,
                              static_cast<double*>(h->G), k, h->d_evals, h->d_E, h->d_info),
             "dsyevd");
  return -1;
}

// Q (n x k, ld ldq) orthonormal -> Ritz vectors; ritz/res on the device
// (h->d_evals, h->d_res).  Scratch: P (n x k, ld n), Zb (n x k, ld n).
void rr_step(chase_handle_s* h, const void* H, int64_t ldh, void* Q, int64_t ldq, int k,
             double norm_scale, void* P, void* Zb, double* t_rr, double* t_resid,
             hipStream_t st, void* Rout = nullptr, int64_t ldr = 0, double* t_eig = nullptr,
             chase_stats* stats = nullptr) {
  const int64_t n = h->n;
  const bool cplx = h->cplx;
  auto t0 = clk::now();
  // P = H Q   (the HEMM of the Rayleigh-Ritz step; with fp64_emulation on
  // the INT8 matrix cores, as the filter's FP64 products, if the moduli keep
  // the FP64 accuracy class: the residuals the solve reports come from P,
  // and with 12 moduli (integer forms of ~39 bits at n = 20000) they were
  // off by half the tolerance)
  if (h->crt_h && h->crt.n_mod >= kCrtMinModuliRR) {
    GemmArgs g = gargs(n, k, n, H, ldh, Q, ldq, P, n);
    g.gamma = 0.0;
    g.beta = 0.0;
    fp64_step(h, g, st);
  } else {
    gemm_nn(h, n, k, n, H, ldh, Q, ldq, P, n, st);
  }
  // G = Q^H P, exactly Hermitian
  gram(h, Q, ldq, P, n, n, k, k, h->G, k, true, st);
  if (t_eig) CHASE_HIP(hipEventRecord(h->eig_ev[0], st));
  const int sweeps = small_eig(h, k, h->opts.eig_solver, st);
  if (stats && sweeps >= 0) {
    stats->eig_jacobi_calls++;
    stats->eig_jacobi_sweeps += sweeps;
  }
  if (t_eig) CHASE_HIP(hipEventRecord(h->eig_ev[1], st));
  // Ritz vectors Z = Q W
  gemm_nn(h, n, k, k, Q, ldq, h->G, k, Zb, n, st);
  CHASE_HIP(hipStreamSynchronize(st));
  auto t1 = clk::now();
  // residual: (P W) - Z diag(theta), column norms, without a second HEMM
  GemmArgs g = gargs(n, k, k, P, n, h->G, k, nullptr, 0);
  g.lambda = h->d_evals;
  g.V = Zb;
  g.ldv = n;
  g.partial = h->d_partial;
  g.F = Rout;
  g.ldf = ldr;
  gemm(cplx, PREC_F64, OP_N, OP_N, EPI_RESID, g, st);
  resid_finish(h->d_partial, gemm_row_tiles(n), k, 1.0 / norm_scale, h->d_res, st);
  copy_cols(cplx, Zb, n, Q, ldq, n, k, st);
  CHASE_HIP(hipStreamSynchronize(st));
  auto t2 = clk::now();
  if (t_rr) *t_rr += secs(t0, t1);
  if (t_resid) *t_resid += secs(t1, t2);
  if (t_eig) {
    float ms = 0.f;
    CHASE_HIP(hipEventElapsedTime(&ms, h->eig_ev[0], h->eig_ev[1]));
    *t_eig += ms * 1e-3;
  }
}

void check_info(chase_handle_s* h, hipStream_t st, const char* what) {
  int info = 0;
  CHASE_HIP(hipMemcpyAsync(&info, h->d_info, sizeof(int), hipMemcpyDeviceToHost, st));
  CHASE_HIP(hipStreamSynchronize(st));
  if (info != 0)
    throw Error(CHASE_ERR_NUMERIC, std::string(what) + " did not converge (info=" +
                                       std::to_string(info) + ")");
}

// The Lanczos step on the given buffers: runs, tridiagonals to the host,
// bounds (Zhou-Li b_sup, lowest Ritz value, density-of-states estimate of
// the n_e-th eigenvalue).
Bounds lanczos_on(bool cplx, LanczosBufs& lz, const void* H, int64_t ldh, int64_t n, int ne,
                  const void* S, int nv, int steps, std::vector<double>* a_out,
                  std::vector<double>* b_out, std::vector<int>* lens, hipStream_t st) {
  lanczos_run(cplx, H, ldh, n, S, nv, steps, lz, st);
  std::vector<double> a((size_t)steps * nv), b((size_t)steps * nv);
  CHASE_HIP(hipMemcpyAsync(a.data(), lz.alpha, a.size() * 8, hipMemcpyDeviceToHost, st));
  CHASE_HIP(hipMemcpyAsync(b.data(), lz.beta, b.size() * 8, hipMemcpyDeviceToHost, st));
  CHASE_HIP(hipStreamSynchronize(st));
  for (double x : a)
    if (!std::isfinite(x)) throw Error(CHASE_ERR_NUMERIC, "non-finite Lanczos coefficients");
  Bounds bd = lanczos_bounds(a, b, nv, steps, n, ne, lens);
  if (a_out) *a_out = a;
  if (b_out) *b_out = b;
  return bd;
}

// Lanczos run-major output arrays from the step-major device layout.
void lanczos_outputs(const Bounds& bd, const std::vector<double>& a, const std::vector<double>& b,
                     const std::vector<int>& lens, int nvec, int steps, double* b_sup,
                     double* mu_1, double* mu_ne, double* alpha_host, double* beta_host,
                     int* steps_host) {
  if (b_sup) *b_sup = bd.b_sup;
  if (mu_1) *mu_1 = bd.mu_1;
  if (mu_ne) *mu_ne = bd.mu_ne;
  for (int r = 0; r < nvec; ++r)
    for (int j = 0; j < steps; ++j) {
      if (alpha_host) alpha_host[(size_t)r * steps + j] = a[(size_t)j * nvec + r];
      if (beta_host) beta_host[(size_t)r * steps + j] = b[(size_t)j * nvec + r];
    }
  if (steps_host)
    for (int r = 0; r < nvec; ++r) steps_host[r] = lens[r];
}

Bounds do_lanczos(chase_handle_s* h, const void* H, int64_t ldh, const void* S, int nv, int steps,
                  std::vector<double>* a_out, std::vector<double>* b_out, std::vector<int>* lens,
                  hipStream_t st, double* gemv_s = nullptr) {
  while (h->evs.size() < 2 * (size_t)steps) {
    hipEvent_t e;
    CHASE_HIP(hipEventCreate(&e));
    h->evs.push_back(e);
  }
  h->lz.gemv_ev = gemv_s ? h->evs.data() : nullptr;
  Bounds bd;
  try {
    bd = lanczos_on(h->cplx, h->lz, H, ldh, h->n, h->ne, S, nv, steps, a_out, b_out, lens, st);
  } catch (...) {
    h->lz.gemv_ev = nullptr;
    throw;
  }
  h->lz.gemv_ev = nullptr;
  if (gemv_s) {
    *gemv_s = 0.0;
    for (int j = 0; j < steps; ++j) {
      float ms = 0.f;
      CHASE_HIP(hipEventElapsedTime(&ms, h->evs[2 * j], h->evs[2 * j + 1]));
      *gemv_s += ms * 1e-3;
    }
  }
  return bd;
}

template <typename F>
chase_status guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return CHASE_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return CHASE_ERR_HIP;
  }
}

void set_stream(chase_handle_s* h, hipStream_t st) {
  CHASE_HIP(hipSetDevice(h->device));
  rb_check(rocblas_set_stream(h->rb, st), "rocblas_set_stream");
}

// ------------------------------------------------------------------ solve
void solve_impl(chase_handle_s* h, const void* H, int64_t ldh, double tol, int degree,
                const void* V0, const void* S, double* evals, void* evecs, int64_t ldv,
                double* resid, chase_stats* out_stats, hipStream_t st, bool* noconv) {
  const int64_t n = h->n;
  const int ne = h->ne, nev = h->nev;
  const bool cplx = h->cplx;
  const chase_opts& o = h->opts;
  chase_stats stats{};
  Range r_solve("chase_solve");
  auto T0 = clk::now();
  const int deg0 = degree + (degree & 1);

  if (o.debug) {
    // H Hermitian is a precondition of the method (and of the split-BF16
    // copy, which stores conj(H) as the transpose)
    double d[2];
    max_defect(cplx, H, ldh, n, 0, h->d_res, st);
    CHASE_HIP(hipMemcpyAsync(d, h->d_res, sizeof(d), hipMemcpyDeviceToHost, st));
    CHASE_HIP(hipStreamSynchronize(st));
    stats.debug_herm_defect = d[1] > 0 ? d[0] / d[1] : 0.0;
    if (!std::isfinite(d[0]) || !std::isfinite(d[1]))
      throw Error(CHASE_ERR_NUMERIC, "H holds non-finite values");
    if (d[0] > 1e-12 * d[1])
      throw Error(CHASE_ERR_ARG, "H is not Hermitian: max |H - H^H| = " + std::to_string(d[0]) +
                                     " (max |H| = " + std::to_string(d[1]) + ")");
  }
  // start blocks the caller did not supply: seeded draws into the Lanczos
  // buffer (S) and the search block (V0)
  if (!S) {
    fill_gaussian(cplx, h->lz.w, n, n, o.lanczos_vecs, (uint64_t)(uint32_t)o.seed, 1, st);
    S = h->lz.w;
  }

  // Lanczos spectral bounds
  const int steps = (int)std::min<int64_t>(o.lanczos_steps, n);
  std::vector<double> lz_a, lz_b;
  Range r_lz("lanczos");
  Bounds bd = do_lanczos(h, H, ldh, S, o.lanczos_vecs, steps, &lz_a, &lz_b, nullptr, st,
                         &stats.t_lanczos_gemv);
  r_lz.end();
  stats.lanczos_gemv_launches = steps;
  stats.lanczos_gemv_bytes = (double)steps * (double)n * (double)n * (double)h->esz;
  auto T1 = clk::now();
  stats.t_lanczos = secs(T0, T1);
  const double b_sup = bd.b_sup;
  double mu_1 = bd.mu_1, mu_ne = bd.mu_ne;
  // residuals relative to a lower bound of ||H||_2, so that res <= tol
  // guarantees ||H v - theta v|| <= tol ||H||_2
  const double norm_est = bd.norm_lower > 0 ? bd.norm_lower : std::fabs(bd.b_sup);

  const bool mixed = o.filter_prec != CHASE_PREC_FP64;
  const Prec plow = to_prec(o.filter_prec) == PREC_F64 ? PREC_F32 : to_prec(o.filter_prec);
  // The start block's plain pass carries an absolute rounding floor (about
  // 1e-2 of the result with the block rounded to bf16), the defect-form
  // passes one relative to the residual: the two-term split-BF16 mode runs
  // its start pass with three terms and only the defect-form passes with two.
  const Prec pstart = plow == PREC_BF16X2 ? PREC_BF16X3 : plow;
  const double tau_sw = o.switch_tol > 0 ? o.switch_tol : 0.0;
  // FP64 tail of the start block's low-precision pass: the rounding error of
  // the low-precision products (relative size `floor` after a plain pass)
  // sits in all directions; each later step damps its unwanted part relative
  // to the nev-th wanted vector by rho = |t| + sqrt(t^2 - 1), t = (lambda_nev
  // - c)/e (the growth rate of the degree step), lambda_nev estimated from the
  // Lanczos density of states.  The tail is the number of final FP64 steps
  // that bring floor down to tol; it is used only when it is shorter than the
  // pass (when the spectrum is hard, the defect-correction passes of the
  // later iterations do that work instead).
  int fp64_tail = 0;
  if (mixed && !o.initial_rr) {
    if (o.fp64_tail > 0) {
      fp64_tail = std::min(o.fp64_tail, deg0);
    } else if (o.fp64_tail < 0) {
      const double lam_nev = lanczos_bounds(lz_a, lz_b, o.lanczos_vecs, steps, n, nev, nullptr).mu_ne;
      const double floor = low_precision_floor(pstart == PREC_BF16X3, n);
      fp64_tail = fp64_tail_steps(floor, lam_nev, 0.5 * (b_sup + mu_ne), 0.5 * (b_sup - mu_ne),
                                  tol, deg0);
    }
  }
  stats.fp64_tail = fp64_tail;
  if (plow == PREC_F32 && mixed && h->H32) to_f32(cplx, H, ldh, h->H32, n, st);
  if (is_split_bf16(plow)) split_h(h, H, ldh, st);
  prepare_h_products(h, H, ldh, st);

  if (V0)
    CHASE_HIP(hipMemcpyAsync(h->V, V0, (size_t)n * ne * h->esz, hipMemcpyDeviceToDevice, st));
  else
    fill_gaussian(cplx, h->V, n, n, ne, (uint64_t)(uint32_t)o.seed, 0, st);
  std::vector<int> m(ne, deg0);
  std::vector<double> lam(ne, 0.0), res(ne, INFINITY);
  // Precision policy (mixed mode).  low[j]: column j is filtered with FP32
  // products in the coming iteration: the start block with the plain
  // recurrence, Ritz vectors with the defect-correction form (whose FP32
  // rounding error scales with the residual, so it converges as the FP64
  // filter does).  A Ritz rank (absolute position j after Rayleigh-Ritz)
  // switches to the FP64 filter for good if its residual grows tenfold in an
  // iteration, or once it is below switch_tol when that option is set.
  std::vector<char> low(ne, mixed ? 1 : 0), fp64_rank(ne, mixed ? 0 : 1);
  std::vector<double> res_rank_prev(ne, INFINITY);
  int L = 0;
  bool converged = false;
  std::vector<int> perm(ne);
  FilterTiming ft64, ftlo;
  // After Rayleigh-Ritz on the active block [L, L+ka): residuals, precision
  // switches, locking of the converged prefix, and unless done the bounds,
  // degrees and sort for the next filter.  Returns true when the solve stops.
  auto after_rr = [&](int it, int ka, int n64) -> bool {
    check_info(h, st, "Hermitian eigensolver");
    CHASE_HIP(hipMemcpyAsync(&lam[L], h->d_evals, ka * sizeof(double), hipMemcpyDeviceToHost, st));
    std::vector<double> r_new(ka);
    CHASE_HIP(hipMemcpyAsync(r_new.data(), h->d_res, ka * sizeof(double), hipMemcpyDeviceToHost,
                             st));
    CHASE_HIP(hipStreamSynchronize(st));
    for (int a = 0; a < ka; ++a) {
      if (!std::isfinite(r_new[a]) || !std::isfinite(lam[L + a]))
        throw Error(CHASE_ERR_NUMERIC, "non-finite Ritz value or residual");
    }
    for (int a = 0; a < ka; ++a) {
      const int j = L + a;
      res[j] = r_new[a];
      if (mixed && !fp64_rank[j] && (r_new[a] <= tau_sw || r_new[a] > 10.0 * res_rank_prev[j]))
        fp64_rank[j] = 1;
      res_rank_prev[j] = r_new[a];
    }
    // ---- deflation & locking: longest converged prefix
    int nconv = 0;
    while (L + nconv < ne && res[L + nconv] <= tol) ++nconv;
    L += nconv;
    if (o.verbose) {
      double rmax = 0;
      for (int a = L; a < ne; ++a) rmax = std::max(rmax, res[a]);
      std::fprintf(stderr,
                   "chase it %d: filtered %d (%d low), locked %d, max_res %.3e, mu1 %.6f, "
                   "mune %.6f\n",
                   it + 1, ka, ka - n64, L, rmax, mu_1, mu_ne);
    }
    if (L >= nev) {
      converged = true;
      return true;
    }
    if (it + 1 == o.max_iter) return true;
    // ---- bounds, degrees, precision groups, sort
    mu_1 = *std::min_element(lam.begin(), lam.end());
    mu_ne = *std::max_element(lam.begin(), lam.end());
    const double c = 0.5 * (b_sup + mu_ne), e = 0.5 * (b_sup - mu_ne);
    const int kb = ne - L;
    std::vector<int> grp(kb);
    for (int a = 0; a < kb; ++a) {
      const int j = L + a;
      m[j] = optimal_degree(res[j], lam[j], c, e, tol, o, deg0);
      grp[a] = (mixed && !fp64_rank[j]) ? 1 : 0;
    }
    std::vector<int> idx(kb);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
      if (grp[x] != grp[y]) return grp[x] < grp[y];
      return m[L + x] < m[L + y];
    });
    std::vector<int> m2(kb);
    std::vector<double> lam2(kb), res2(kb);
    std::vector<char> low2(kb);
    for (int a = 0; a < kb; ++a) {
      m2[a] = m[L + idx[a]];
      lam2[a] = lam[L + idx[a]];
      res2[a] = res[L + idx[a]];
      low2[a] = (char)grp[idx[a]];
    }
    for (int a = 0; a < kb; ++a) {
      m[L + a] = m2[a];
      lam[L + a] = lam2[a];
      res[L + a] = res2[a];
      low[L + a] = low2[a];
    }
    h2d_sync(h->d_perm, idx.data(), kb * sizeof(int), st);
    gather_cols(cplx, off(h->V, (int64_t)L * n, h->esz), n, h->W, n, n, kb, h->d_perm, st);
    copy_cols(cplx, h->W, n, off(h->V, (int64_t)L * n, h->esz), n, n, kb, st);
    if (mixed) {
      gather_cols(cplx, off(h->Rres, (int64_t)L * n, h->esz), n, h->W, n, n, kb, h->d_perm, st);
      copy_cols(cplx, h->W, n, off(h->Rres, (int64_t)L * n, h->esz), n, n, kb, st);
    }
    return false;
  };
  // Optional Rayleigh-Ritz on the start block (an extension of Algorithm 1,
  // for warm starts from approximate eigenvectors): already converged pairs
  // lock before any filtering, the first filter uses the degrees optimised
  // from the start block's residuals, and the mixed modes filter its Ritz
  // vectors in the defect-correction form from the first pass on.
  // Debug mode: every phase's output must be finite, and the block must be
  // orthonormal after each QR step (max |V^H V - I| over the whole block).
  auto debug_check = [&](const char* phase, int col0, bool orth) {
    if (!o.debug) return;
    int bad = 0;
    fill_zero(h->d_flags, sizeof(int), st);
    check_finite(cplx, off(h->V, (int64_t)col0 * n, h->esz), n, n, ne - col0, h->d_flags, st);
    CHASE_HIP(hipMemcpyAsync(&bad, h->d_flags, sizeof(int), hipMemcpyDeviceToHost, st));
    CHASE_HIP(hipStreamSynchronize(st));
    if (bad) throw Error(CHASE_ERR_NUMERIC, std::string("non-finite values after ") + phase);
    if (!orth) return;
    double d[2];
    gram(h, h->V, n, h->V, n, n, ne, ne, h->R, ne, true, st);
    max_defect(cplx, h->R, ne, ne, 1, h->d_res, st);
    CHASE_HIP(hipMemcpyAsync(d, h->d_res, sizeof(d), hipMemcpyDeviceToHost, st));
    CHASE_HIP(hipStreamSynchronize(st));
    stats.debug_orth_defect = std::max(stats.debug_orth_defect, d[0]);
    if (!(d[0] <= 1e-8))
      throw Error(CHASE_ERR_NUMERIC, std::string("block not orthonormal after ") + phase +
                                         ": max |Q^H Q - I| = " + std::to_string(d[0]));
  };
  bool have_ritz = false;
  if (o.initial_rr) {
    qr_step(h, h->V, n, ne, 0, h->W, &stats, st);
    debug_check("QR", 0, true);
    rr_step(h, H, ldh, h->V, n, ne, norm_est, h->W, h->Z, &stats.t_rr, &stats.t_resid, st,
            mixed ? h->Rres : nullptr, n, &stats.t_rr_eig, &stats);
    debug_check("Rayleigh-Ritz", 0, false);
    have_ritz = true;
    if (after_rr(-1, ne, 0)) stats.iterations = 0;
  }
  for (int it = 0; it < o.max_iter && !converged; ++it) {
    stats.iterations = it + 1;
    const int ka = ne - L;
    // ---- filter (FP64 group first, then the low-precision group)
    Range r_f("filter");
    auto F0 = clk::now();
    int n64 = 0;
    while (n64 < ka && !low[L + n64]) ++n64;
    if (n64 > 0)
      run_filter(h, H, ldh, off(h->V, (int64_t)L * n, h->esz), n, h->W, n, n64, &m[L], b_sup,
                 mu_1, mu_ne, PREC_F64, false, ft64, st);
    if (ka - n64 > 0) {
      if (it == 0 && !have_ritz)  // start block: no Ritz pairs yet, plain low-precision products
        run_filter(h, H, ldh, off(h->V, (int64_t)(L + n64) * n, h->esz), n, h->W, n, ka - n64,
                   &m[L + n64], b_sup, mu_1, mu_ne, pstart, false, ftlo, st,
                   fp64_tail > 0 ? m[ne - 1] - fp64_tail + 1 : 0, &ft64);
      else  // Ritz vectors: defect-correction form with low-precision products
        run_filter_defect(h, H, ldh, off(h->V, (int64_t)(L + n64) * n, h->esz), n,
                          off(h->Rres, (int64_t)(L + n64) * n, h->esz), n, h->W, h->Z,
                          ka - n64, &m[L + n64], &lam[L + n64], b_sup, mu_1, mu_ne, plow,
                          ftlo, st);
    }
    auto F1 = clk::now();
    r_f.end();
    stats.t_filter += secs(F0, F1);
    debug_check("the filter", L, false);
    // ---- QR of [Y V]
    F1 = clk::now();
    Range r_qr("qr");
    qr_step(h, h->V, n, ne, L, h->W, &stats, st);
    r_qr.end();
    auto Q1 = clk::now();
    stats.t_qr += secs(F1, Q1);
    debug_check("QR", 0, true);
    // ---- Rayleigh-Ritz + residuals on the active part
    Range r_rr("rayleigh_ritz_residual");
    rr_step(h, H, ldh, off(h->V, (int64_t)L * n, h->esz), n, ka, norm_est, h->W, h->Z, &stats.t_rr,
            &stats.t_resid, st, mixed ? off(h->Rres, (int64_t)L * n, h->esz) : nullptr, n,
            &stats.t_rr_eig, &stats);
    r_rr.end();
    debug_check("Rayleigh-Ritz", L, false);
    if (after_rr(it, ka, n64)) break;
  }
  // ---- output: lowest nev of the locked pairs (or of all pairs on NOCONV)
  const int pool = converged ? L : ne;
  std::vector<int> idx(pool);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return lam[x] < lam[y]; });
  idx.resize(nev);
  for (int i = 0; i < nev; ++i) {
    evals[i] = lam[idx[i]];
    if (resid) resid[i] = res[idx[i]];
  }
  h2d_sync(h->d_perm, idx.data(), nev * sizeof(int), st);
  gather_cols(cplx, h->V, n, evecs, ldv, n, nev, h->d_perm, st);
  CHASE_HIP(hipStreamSynchronize(st));
  stats.locked = L;
  stats.matvecs_fp64 = ft64.matvecs;
  stats.matvecs_low = ftlo.matvecs;
  stats.t_filter_kernels = ft64.ktime + ftlo.ktime;
  stats.t_filter_kernels_low = ftlo.ktime;
  stats.filter_launches_low = ftlo.launches;
  stats.filter_launches = ft64.launches + ftlo.launches;
  stats.filter_flops = (cplx ? 8.0 : 2.0) * (double)n * (double)n *
                       (double)(ft64.matvecs + ftlo.matvecs);
  stats.b_sup = b_sup;
  stats.mu_1 = mu_1;
  stats.mu_ne = mu_ne;
  stats.t_all = secs(T0, clk::now());
  if (out_stats) *out_stats = stats;
  *noconv = !converged;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

void chase_default_opts(chase_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_deg = 36;
  o->deg_extra = 2;
  o->optimize_degree = 1;
  o->lanczos_steps = 25;
  o->lanczos_vecs = 4;
  o->max_iter = 50;
  o->filter_prec = CHASE_PREC_FP64;
  o->switch_tol = 0.0;
  o->fp64_tail = -1;
  o->verbose = 0;
}

size_t chase_workspace_bytes(chase_dtype dtype, int64_t n, int nev, int nex, const chase_opts* opts) {
  if (n < 1 || nev < 1 || nex < 1 || (int64_t)nev + nex > n) return 0;
  if (dtype != CHASE_C128 && dtype != CHASE_F64) return 0;
  chase_opts o;
  chase_default_opts(&o);
  if (opts) o = *opts;
  return sizes(dtype, n, nev, nex, o).total;
}

const char* chase_last_error(void) { return g_last_error.c_str(); }

chase_status chase_filter_coefficients(int m, double b_sup, double mu_1, double mu_ne,
                                       double* coef_host) {
  return guarded([&] {
    CHASE_REQUIRE(coef_host != nullptr, "NULL pointer argument");
    CHASE_REQUIRE(m >= 1 && m <= kMaxDegree, "m out of range [1, 1000]");
    CHASE_REQUIRE(std::isfinite(b_sup) && std::isfinite(mu_1) && std::isfinite(mu_ne) &&
                      mu_1 < mu_ne && mu_ne < b_sup,
                  "need mu_1 < mu_ne < b_sup");
    const std::vector<Coef> cf = cheb_coefficients(m, b_sup, mu_1, mu_ne);
    for (int s = 0; s < m; ++s) {
      coef_host[3 * s] = cf[s].alpha;
      coef_host[3 * s + 1] = cf[s].gamma;
      coef_host[3 * s + 2] = cf[s].beta;
    }
  });
}

chase_status chase_spectral_bounds(const double* alpha_host, const double* beta_host, int nvec,
                                   int steps, int64_t n, int n_e, double* b_sup, double* mu_1,
                                   double* mu_ne, int* steps_host) {
  return guarded([&] {
    CHASE_REQUIRE(alpha_host && beta_host && b_sup && mu_1 && mu_ne, "NULL pointer argument");
    CHASE_REQUIRE(nvec >= 1 && steps >= 1, "nvec and steps must be >= 1");
    CHASE_REQUIRE(n_e >= 1 && n_e <= n, "need 1 <= n_e <= n");
    std::vector<double> a((size_t)steps * nvec), b((size_t)steps * nvec);
    for (int r = 0; r < nvec; ++r)
      for (int j = 0; j < steps; ++j) {
        a[(size_t)j * nvec + r] = alpha_host[(size_t)r * steps + j];
        b[(size_t)j * nvec + r] = beta_host[(size_t)r * steps + j];
      }
    for (size_t i = 0; i < a.size(); ++i)
      CHASE_REQUIRE(std::isfinite(a[i]) && std::isfinite(b[i]) && b[i] >= 0.0,
                    "alpha must be finite, beta finite and >= 0");
    std::vector<int> lens;
    const Bounds bd = lanczos_bounds(a, b, nvec, steps, n, n_e, &lens);
    *b_sup = bd.b_sup;
    *mu_1 = bd.mu_1;
    *mu_ne = bd.mu_ne;
    if (steps_host)
      for (int r = 0; r < nvec; ++r) steps_host[r] = lens[r];
  });
}

chase_status chase_degrees(const double* resid_host, const double* ritz_host, int k, double b_sup,
                           double mu_ne, double tol, int degree, const chase_opts* opts,
                           int* degrees_host) {
  return guarded([&] {
    CHASE_REQUIRE(resid_host && ritz_host && degrees_host, "NULL pointer argument");
    CHASE_REQUIRE(k >= 0, "k must be >= 0");
    CHASE_REQUIRE(std::isfinite(b_sup) && std::isfinite(mu_ne) && mu_ne < b_sup,
                  "need mu_ne < b_sup");
    CHASE_REQUIRE(tol > 0.0 && std::isfinite(tol), "tol must be > 0");
    CHASE_REQUIRE(degree >= 2, "degree must be >= 2");
    chase_opts o;
    chase_default_opts(&o);
    if (opts) o = *opts;
    validate_opts(o);
    const double c = 0.5 * (b_sup + mu_ne), e = 0.5 * (b_sup - mu_ne);
    const int deg0 = degree + (degree & 1);
    for (int a = 0; a < k; ++a) {
      CHASE_REQUIRE(resid_host[a] > 0.0 && std::isfinite(resid_host[a]) &&
                        std::isfinite(ritz_host[a]),
                    "residuals must be finite and > 0, Ritz values finite");
      degrees_host[a] = optimal_degree(resid_host[a], ritz_host[a], c, e, tol, o, deg0);
    }
  });
}

chase_status chase_create(chase_handle_t* out, chase_dtype dtype, int64_t n, int nev, int nex,
                          const chase_opts* opts) {
  chase_handle_s* h = nullptr;
  chase_status st = guarded([&] {
    CHASE_REQUIRE(out != nullptr, "handle pointer is NULL");
    *out = nullptr;
    CHASE_REQUIRE(dtype == CHASE_C128 || dtype == CHASE_F64, "unknown dtype");
    CHASE_REQUIRE(n >= 1 && nev >= 1 && nex >= 1, "need n >= 1, nev >= 1, nex >= 1");
    CHASE_REQUIRE((int64_t)nev + nex <= n, "nev + nex must not exceed n");
    chase_opts o;
    chase_default_opts(&o);
    if (opts) o = *opts;
    validate_opts(o);
    h = new chase_handle_s();
    h->dtype = dtype;
    h->cplx = dtype == CHASE_C128;
    h->n = n;
    h->nev = nev;
    h->nex = nex;
    h->ne = nev + nex;
    h->opts = o;
    h->esz = h->cplx ? 16 : 8;
    CHASE_HIP(hipGetDevice(&h->device));
    const Sizes sz = sizes(dtype, n, nev, nex, o);
    size_t fr = 0, tot = 0;
    CHASE_HIP(hipMemGetInfo(&fr, &tot));
    const size_t h32_bytes = (size_t)n * n * h->esz / 2;
    // the FP32 copy of H is optional (without it the FP32 products round H
    // while staging it in LDS); the split-BF16 copies are required
    const size_t need_min = sz.total - (o.filter_prec == CHASE_PREC_FP32 ? h32_bytes : 0);
    if (need_min > fr)
      throw Error(CHASE_ERR_NOMEM, "workspace of " + std::to_string(need_min) +
                                       " bytes exceeds free device memory (" +
                                       std::to_string(fr) + ")");
    // the low-precision copy of H is optional: without it the FP32 products
    // round H's entries while staging them in LDS
    const bool with_h32 = o.filter_prec == CHASE_PREC_FP32 &&
                          sz.total + ((size_t)1 << 30) <= fr;
    const int64_t ne = h->ne;
    h->V = dev_alloc(h, (size_t)n * ne * h->esz);
    h->W = dev_alloc(h, (size_t)n * ne * h->esz);
    h->Z = dev_alloc(h, (size_t)n * ne * h->esz);
    h->G = dev_alloc(h, (size_t)ne * ne * h->esz);
    h->R = dev_alloc(h, (size_t)ne * ne * h->esz);
    h->ws_elems = splitk_ws_elems((int)ne);
    h->ws = dev_alloc(h, h->ws_elems * h->esz);
    h->d_scale = static_cast<double*>(dev_alloc(h, ne * 8));
    h->d_evals = static_cast<double*>(dev_alloc(h, ne * 8));
    h->d_res = static_cast<double*>(dev_alloc(h, ne * 8));
    h->d_E = static_cast<double*>(dev_alloc(h, ne * 8));
    h->d_g = static_cast<double*>(dev_alloc(h, ne * 8));
    h->d_partial = static_cast<double*>(dev_alloc(h, (size_t)gemm_row_tiles(n) * ne * 8));
    h->d_flags = static_cast<int*>(dev_alloc(h, 64));
    h->d_info = static_cast<int*>(dev_alloc(h, 64));
    h->d_perm = static_cast<int*>(dev_alloc(h, ne * 4));
    h->tau = dev_alloc(h, ne * h->esz);
    const int W = h->cplx ? 2 : 1;
    const int nv = o.lanczos_vecs, steps = o.lanczos_steps;
    lanczos_bytes(h->cplx, n, nv, steps, &h->lz.max_splits);
    h->lz.q_prev = dev_alloc(h, (size_t)n * nv * W * 8);
    h->lz.q_cur = dev_alloc(h, (size_t)n * nv * W * 8);
    h->lz.w = dev_alloc(h, (size_t)n * nv * W * 8);
    h->lz.wpart = dev_alloc(h, (size_t)h->lz.max_splits * nv * n * W * 8);
    h->lz.dotp = static_cast<double*>(dev_alloc(h, 128 * nv * 8));
    h->lz.nrmp = static_cast<double*>(dev_alloc(h, 128 * nv * 8));
    h->lz.alpha = static_cast<double*>(dev_alloc(h, (size_t)steps * nv * 8));
    h->lz.beta = static_cast<double*>(dev_alloc(h, (size_t)steps * nv * 8));
    if (o.filter_prec == CHASE_PREC_FP32) {
      if (with_h32) h->H32 = dev_alloc(h, h32_bytes);
      h->Rres = dev_alloc(h, (size_t)n * ne * h->esz);
    } else if (o.filter_prec == CHASE_PREC_BF16X3 || o.filter_prec == CHASE_PREC_BF16X2) {
      h->s8_groups = s8_groups(n);
      h->Hs8 = dev_alloc(h, s8_bytes(h->cplx, n, s8_pad(n, S8_COLS_A)));
      const size_t xb = s8_bytes(h->cplx, n, s8_pad(ne, S8_COLS_B));
      h->Xs8 = dev_alloc(h, xb);
      h->Xs8b = dev_alloc(h, xb);
      // the zero padding rows of both block splits: the split kernel rewrites
      // them, the epilogue that fills the second buffer never touches them
      CHASE_HIP(hipMemset(h->Xs8, 0, xb));
      CHASE_HIP(hipMemset(h->Xs8b, 0, xb));
      h->s8tail = static_cast<float*>(dev_alloc(h, s8_tail_bytes(h->cplx)));
      h->Rres = dev_alloc(h, (size_t)n * ne * h->esz);
    }
    h->d_coef = static_cast<double*>(dev_alloc(h, (size_t)(kMaxDegree + 1) * ne * 8));
    h->jac_ws = dev_alloc(h, jacobi_ws_bytes(h->cplx, (int)ne));
    if (o.fp64_emulation > 0) {
      CHASE_REQUIRE(n <= 65535, "fp64_emulation needs n <= 65535");
      h->crt = crt_basis(o.fp64_emulation, n, h->cplx);
      h->crt_h = dev_alloc(h, crt_h_bytes(h->cplx, n, o.fp64_emulation));
      h->crt_x = dev_alloc(h, crt_x_bytes(h->cplx, n, (int)ne, o.fp64_emulation));
    }
    if (o.adjoint_reserve > 0) {
      h->adj = dev_alloc(h, 2 * (size_t)n * ne * h->esz);
      ensure_tape(h, (int)ne, o.adjoint_reserve);
    }
    rb_check(rocblas_create_handle(&h->rb), "rocblas_create_handle");
    CHASE_HIP(hipEventCreate(&h->eig_ev[0]));
    CHASE_HIP(hipEventCreate(&h->eig_ev[1]));
    if (const char* e = std::getenv("CHASE_DEBUG"))
      if (std::atoi(e) != 0) h->opts.debug = 1;
    *out = h;
  });
  if (st != CHASE_OK && h) chase_destroy(h);
  return st;
}

void chase_destroy(chase_handle_t h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->tape) (void)hipFree(h->tape);
  for (hipEvent_t e : h->evs) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->eig_ev)
    if (e) (void)hipEventDestroy(e);
  if (h->rb) rocblas_destroy_handle(h->rb);
  delete h;
}

chase_status chase_solve(chase_handle_t h, const void* H, int64_t ldh, double tol, int degree,
                         const void* V0, const void* S, double* evals_host, void* evecs_dev,
                         int64_t ldv, double* resid_host, chase_stats* stats, void* stream) {
  bool noconv = false;
  chase_status s = guarded([&] {
    CHASE_REQUIRE(h != nullptr, "handle is NULL");
    CHASE_REQUIRE(H && evals_host && evecs_dev, "NULL pointer argument");
    CHASE_REQUIRE(ldh >= h->n && ldv >= h->n, "leading dimension smaller than n");
    CHASE_REQUIRE(tol > 0 && std::isfinite(tol), "tol must be positive");
    CHASE_REQUIRE(degree >= 2 && degree <= std::min(h->opts.max_deg + 1, kMaxDegree),
                  "degree out of range [2, min(max_deg + 1, 1000)]");
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_stream(h, st);
    solve_impl(h, H, ldh, tol, degree, V0, S, evals_host, evecs_dev, ldv, resid_host, stats, st,
               &noconv);
  });
  if (s == CHASE_OK && noconv) {
    g_last_error = "maximum number of iterations reached";
    return CHASE_ERR_NOCONV;
  }
  return s;
}

chase_status chase_lanczos(chase_handle_t h, const void* H, int64_t ldh, const void* S, int nvec,
                           int steps, double* b_sup, double* mu_1, double* mu_ne,
                           double* alpha_host, double* beta_host, int* steps_host, void* stream) {
  return guarded([&] {
    CHASE_REQUIRE(h != nullptr, "handle is NULL");
    CHASE_REQUIRE(H && S, "NULL pointer argument");
    CHASE_REQUIRE(ldh >= h->n, "ldh < n");
    CHASE_REQUIRE(nvec >= 1 && nvec <= h->opts.lanczos_vecs, "nvec out of range");
    CHASE_REQUIRE(steps >= 1 && steps <= h->opts.lanczos_steps && steps <= h->n,
                  "steps out of range");
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_stream(h, st);
    std::vector<double> a, b;
    std::vector<int> lens;
    Bounds bd = do_lanczos(h, H, ldh, S, nvec, steps, &a, &b, &lens, st);
    lanczos_outputs(bd, a, b, lens, nvec, steps, b_sup, mu_1, mu_ne, alpha_host, beta_host,
                    steps_host);
  });
}

chase_status chase_lanczos_noalloc(chase_dtype dtype, const void* H, int64_t ldh, int64_t n,
                                   int n_e, const void* S, int nvec, int steps, double* b_sup,
                                   double* mu_1, double* mu_ne, double* alpha_host,
                                   double* beta_host, int* steps_host, void* stream) {
  return guarded([&] {
    CHASE_REQUIRE(dtype == CHASE_C128 || dtype == CHASE_F64, "unknown dtype");
    CHASE_REQUIRE(n >= 1 && n_e >= 1 && n_e <= n, "sizes out of range (1 <= n_e <= n)");
    CHASE_REQUIRE(H && S, "NULL pointer argument");
    CHASE_REQUIRE(ldh >= n, "ldh < n");
    CHASE_REQUIRE(nvec >= 1 && nvec <= 8, "nvec out of range [1, 8]");
    CHASE_REQUIRE(steps >= 1 && steps <= 200 && steps <= n, "steps out of range [1, min(200, n)]");
    const bool cplx = dtype == CHASE_C128;
    const int W = cplx ? 2 : 1;
    int splits = 0;
    const size_t need = lanczos_bytes(cplx, n, nvec, steps, &splits) + 8 * 256;
    CHASE_REQUIRE(need <= kNoAllocScratchBytes,
                  "problem needs " + std::to_string(need) +
                      " bytes of Lanczos buffers, more than the no-allocation scratch (" +
                      std::to_string(kNoAllocScratchBytes) + " bytes)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* p = noalloc_scratch();
    auto take = [&p](size_t bytes) {
      char* q = p;
      p += (bytes + 255) / 256 * 256;
      return q;
    };
    LanczosBufs lz{};
    lz.max_splits = splits;
    lz.q_prev = take((size_t)n * nvec * W * 8);
    lz.q_cur = take((size_t)n * nvec * W * 8);
    lz.w = take((size_t)n * nvec * W * 8);
    lz.wpart = take((size_t)splits * nvec * n * W * 8);
    lz.dotp = reinterpret_cast<double*>(take(128 * (size_t)nvec * 8));
    lz.nrmp = reinterpret_cast<double*>(take(128 * (size_t)nvec * 8));
    lz.alpha = reinterpret_cast<double*>(take((size_t)steps * nvec * 8));
    lz.beta = reinterpret_cast<double*>(take((size_t)steps * nvec * 8));
    std::vector<double> a, b;
    std::vector<int> lens;
    Bounds bd = lanczos_on(cplx, lz, H, ldh, n, n_e, S, nvec, steps, &a, &b, &lens, st);
    lanczos_outputs(bd, a, b, lens, nvec, steps, b_sup, mu_1, mu_ne, alpha_host, beta_host,
                    steps_host);
  });
}

chase_status chase_filter(chase_handle_t h, const void* H, int64_t ldh, void* X, int64_t ldx, int k,
                          const int* degrees, double b_sup, double mu_1, double mu_ne, int prec,
                          int record_tape, int64_t* matvecs, void* stream) {
  return guarded([&] {
    CHASE_REQUIRE(h != nullptr, "handle is NULL");
    CHASE_REQUIRE(H && X && degrees, "NULL pointer argument");
    CHASE_REQUIRE(ldh >= h->n && ldx >= h->n, "leading dimension smaller than n");
    CHASE_REQUIRE(k >= 1 && k <= h->ne, "k must be in [1, nev+nex]");
    CHASE_REQUIRE(prec == CHASE_PREC_FP64 || prec == CHASE_PREC_FP32 || prec == CHASE_PREC_BF16X3 ||
                      prec == CHASE_PREC_BF16X2,
                  "unknown precision");
    CHASE_REQUIRE((prec != CHASE_PREC_BF16X3 && prec != CHASE_PREC_BF16X2) || h->Hs8,
                  "split-BF16 products need a handle created with filter_prec = "
                  "CHASE_PREC_BF16X3 or CHASE_PREC_BF16X2");
    CHASE_REQUIRE(std::isfinite(b_sup) && std::isfinite(mu_1) && std::isfinite(mu_ne) &&
                      mu_1 < mu_ne && mu_ne < b_sup,
                  "need mu_1 < mu_ne < b_sup");
    for (int a = 0; a < k; ++a) {
      CHASE_REQUIRE(degrees[a] >= 2 && degrees[a] % 2 == 0 && degrees[a] <= kMaxDegree,
                    "degrees must be even and in [2, 1000]");
      CHASE_REQUIRE(a == 0 || degrees[a] >= degrees[a - 1], "degrees must be non-decreasing");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_stream(h, st);
    if (record_tape) ensure_tape(h, k, degrees[k - 1]);
    if (prec == CHASE_PREC_FP32 && h->H32) to_f32(h->cplx, H, ldh, h->H32, h->n, st);
    if (prec == CHASE_PREC_BF16X3 || prec == CHASE_PREC_BF16X2) split_h(h, H, ldh, st);
    prepare_h_products(h, H, ldh, st);
    FilterTiming ft;
    h->tape_valid = false;
    run_filter(h, H, ldh, X, ldx, h->W, h->n, k, degrees, b_sup, mu_1, mu_ne, to_prec(prec),
               record_tape != 0, ft, st);
    if (matvecs) *matvecs = ft.matvecs;
  });
}

chase_status chase_filter_ritz(chase_handle_t h, const void* H, int64_t ldh, void* V,
                               int64_t ldv, const void* R, int64_t ldr, const double* theta, int k,
                               const int* degrees, double b_sup, double mu_1, double mu_ne,
                               int prec, int64_t* matvecs, void* stream) {
  return guarded([&] {
    CHASE_REQUIRE(h != nullptr, "handle is NULL");
    CHASE_REQUIRE(H && V && R && theta && degrees, "NULL pointer argument");
    CHASE_REQUIRE(ldh >= h->n && ldv >= h->n && ldr >= h->n, "leading dimension smaller than n");
    CHASE_REQUIRE(k >= 1 && k <= h->ne, "k must be in [1, nev+nex]");
    CHASE_REQUIRE(prec == CHASE_PREC_FP64 || prec == CHASE_PREC_FP32 || prec == CHASE_PREC_BF16X3 ||
                      prec == CHASE_PREC_BF16X2,
                  "unknown precision");
    CHASE_REQUIRE((prec != CHASE_PREC_BF16X3 && prec != CHASE_PREC_BF16X2) || h->Hs8,
                  "split-BF16 products need a handle created with filter_prec = "
                  "CHASE_PREC_BF16X3 or CHASE_PREC_BF16X2");
    CHASE_REQUIRE(std::isfinite(b_sup) && std::isfinite(mu_1) && std::isfinite(mu_ne) &&
                      mu_1 < mu_ne && mu_ne < b_sup,
                  "need mu_1 < mu_ne < b_sup");
    for (int a = 0; a < k; ++a) {
      CHASE_REQUIRE(std::isfinite(theta[a]), "theta must be finite");
      CHASE_REQUIRE(degrees[a] >= 2 && degrees[a] % 2 == 0 && degrees[a] <= kMaxDegree,
                    "degrees must be even and in [2, 1000]");
      CHASE_REQUIRE(a == 0 || degrees[a] >= degrees[a - 1], "degrees must be non-decreasing");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_stream(h, st);
    if (prec == CHASE_PREC_FP32 && h->H32) to_f32(h->cplx, H, ldh, h->H32, h->n, st);
    if (prec == CHASE_PREC_BF16X3 || prec == CHASE_PREC_BF16X2) split_h(h, H, ldh, st);
    prepare_h_products(h, H, ldh, st);
    FilterTiming ft;
    run_filter_defect(h, H, ldh, V, ldv, R, ldr, h->W, h->Z, k, degrees, theta, b_sup, mu_1,
                      mu_ne, to_prec(prec), ft, st);
    if (matvecs) *matvecs = ft.matvecs;
  });
}

chase_status chase_qr(chase_handle_t h, void* X, int64_t ldx, int k, int locked,
                      int* shifted_passes, int* householder, void* stream) {
  return guarded([&] {
    CHASE_REQUIRE(h != nullptr, "handle is NULL");
    CHASE_REQUIRE(X != nullptr, "NULL pointer argument");
    CHASE_REQUIRE(ldx >= h->n, "ldx < n");
    CHASE_REQUIRE(k >= 1 && k <= h->ne && locked >= 0 && locked < k, "bad k / locked");
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_stream(h, st);
    chase_stats qs{};
    qr_step(h, X, ldx, k, locked, h->W, &qs, st);
    CHASE_HIP(hipStreamSynchronize(st));
    if (shifted_passes) *shifted_passes = qs.qr_shifted;
    if (householder) *householder = qs.qr_householder;
  });
}

chase_status chase_rayleigh_ritz(chase_handle_t h, const void* H, int64_t ldh, void* Q, int64_t ldq,
                                 int k, double norm_scale, double* ritz, double* resid,
                                 void* stream) {
  return guarded([&] {
    CHASE_REQUIRE(h != nullptr, "handle is NULL");
    CHASE_REQUIRE(H && Q && ritz, "NULL pointer argument");
    CHASE_REQUIRE(ldh >= h->n && ldq >= h->n, "leading dimension smaller than n");
    CHASE_REQUIRE(k >= 1 && k <= h->ne, "k must be in [1, nev+nex]");
    CHASE_REQUIRE(norm_scale > 0, "norm_scale must be positive");
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_stream(h, st);
    prepare_h_products(h, H, ldh, st);
    rr_step(h, H, ldh, Q, ldq, k, norm_scale, h->W, h->Z, nullptr, nullptr, st);
    check_info(h, st, "Hermitian eigensolver");
    CHASE_HIP(hipMemcpyAsync(ritz, h->d_evals, k * 8, hipMemcpyDeviceToHost, st));
    if (resid) CHASE_HIP(hipMemcpyAsync(resid, h->d_res, k * 8, hipMemcpyDeviceToHost, st));
    CHASE_HIP(hipStreamSynchronize(st));
  });
}

chase_status chase_heev(chase_handle_t h, void* G, int64_t ldg, int k, int method, double* evals,
                        int* sweeps, void* stream) {
  return guarded([&] {
    CHASE_REQUIRE(h != nullptr, "handle is NULL");
    CHASE_REQUIRE(G && evals, "NULL pointer argument");
    CHASE_REQUIRE(k >= 1 && k <= h->ne, "k must be in [1, nev+nex]");
    CHASE_REQUIRE(ldg >= k, "leading dimension smaller than k");
    CHASE_REQUIRE(method == CHASE_EIG_AUTO || method == CHASE_EIG_LIBRARY ||
                      method == CHASE_EIG_JACOBI,
                  "unknown eigensolver");
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_stream(h, st);
    copy_cols(h->cplx, G, ldg, h->G, k, k, k, st);
    const int sw = small_eig(h, k, method, st);
    if (sw < 0) check_info(h, st, "Hermitian eigensolver");
    copy_cols(h->cplx, h->G, k, G, ldg, k, k, st);
    CHASE_HIP(hipMemcpyAsync(evals, h->d_evals, k * 8, hipMemcpyDeviceToHost, st));
    CHASE_HIP(hipStreamSynchronize(st));
    if (sweeps) *sweeps = sw < 0 ? 0 : sw;
  });
}

chase_status chase_cholesky(chase_handle_t h, void* A, int64_t lda, int k, int* info,
                            void* stream) {
  return guarded([&] {
    CHASE_REQUIRE(h != nullptr, "handle is NULL");
    CHASE_REQUIRE(info && (A || k == 0), "NULL pointer argument");
    CHASE_REQUIRE(k >= 0, "k must be non-negative");
    CHASE_REQUIRE(lda >= std::max(1, k), "leading dimension smaller than k");
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_stream(h, st);
    cholesky_upper(h->cplx, A, lda, k, h->d_info, st);
    CHASE_HIP(hipMemcpyAsync(info, h->d_info, sizeof(int), hipMemcpyDeviceToHost, st));
    CHASE_HIP(hipStreamSynchronize(st));
  });
}

chase_status chase_eigval_adjoint(chase_handle_t h, const void* V, int64_t ldv, int m,
                                  const double* g_host, void* dH, int64_t ldd, void* stream) {
  return guarded([&] {
    CHASE_REQUIRE(h != nullptr, "handle is NULL");
    CHASE_REQUIRE(V && g_host && dH, "NULL pointer argument");
    CHASE_REQUIRE(ldv >= h->n && ldd >= h->n, "leading dimension smaller than n");
    CHASE_REQUIRE(m >= 1 && m <= h->ne, "m must be in [1, nev+nex]");
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_stream(h, st);
    const int64_t n = h->n;
    // Z = V diag(g); dH += Z V^H
    copy_cols(h->cplx, V, ldv, h->Z, n, n, m, st);
    h2d_sync(h->d_g, g_host, m * 8, st);
    scale_cols(h->cplx, h->Z, n, n, m, h->d_g, st);
    GemmArgs g = gargs(n, n, m, h->Z, n, V, ldv, dH, ldd);
    g.beta = 1.0;
    gemm(h->cplx, PREC_F64, OP_N, OP_C, EPI_STORE, g, st);
    CHASE_HIP(hipStreamSynchronize(st));
  });
}

chase_status chase_eigvec_adjoint(chase_handle_t h, const void* H, int64_t ldh, const void* V,
                                  int64_t ldv, int m, const double* lambda_host, const void* G,
                                  int64_t ldg, void* dH, int64_t ldd, double tol, int max_iter,
                                  int* iterations, void* stream) {
  return guarded([&] {
    CHASE_REQUIRE(h != nullptr, "handle is NULL");
    CHASE_REQUIRE(H && V && lambda_host && G && dH, "NULL pointer argument");
    CHASE_REQUIRE(ldh >= h->n && ldv >= h->n && ldg >= h->n && ldd >= h->n,
                  "leading dimension smaller than n");
    CHASE_REQUIRE(m >= 1 && m <= h->ne && m < h->n, "m must be in [1, nev+nex] and below n");
    CHASE_REQUIRE(tol > 0 && std::isfinite(tol) && max_iter >= 1, "need tol > 0, max_iter >= 1");
    for (int i = 0; i < m; ++i)
      CHASE_REQUIRE(std::isfinite(lambda_host[i]), "eigenvalues must be finite");
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_stream(h, st);
    const bool cplx = h->cplx;
    const int64_t n = h->n, ne = h->ne;
    const size_t esz = h->esz;
    if (!h->adj) h->adj = dev_alloc(h, 2 * (size_t)n * ne * esz);
    // blocks (n x m, ld n): X solution, R residual, P direction, Q = P_perp (H - Lambda) P
    void* X = h->adj;
    void* R = off(h->adj, n * ne, esz);
    void* P = h->W;
    void* Q = h->Z;
    double* lam = h->d_evals;
    double* rr = h->d_coef;
    double* rr_new = rr + ne;
    double* pq = rr + 2 * ne;
    double* rr0 = rr + 3 * ne;
    h2d_sync(lam, lambda_host, m * 8, st);
    // M = V^H G (m x m, in G, ld ne)
    gram(h, V, ldv, G, ldg, n, m, m, h->G, ne, false, st);
    // Complement: (H - lambda_j) x_j = b_j = -(I - V V^H) g_j with x_j orthogonal
    // to V.  On that complement H - lambda_j is positive definite (V holds
    // the lowest eigenvectors), so each column is a conjugate-gradient solve;
    // the products are one GEMM with the per-column shift in its epilogue,
    // projected back onto the complement every step.
    copy_cols(cplx, G, ldg, R, n, n, m, st);
    {
      GemmArgs g = gargs(n, m, m, V, ldv, h->G, ne, R, n);  // R = V M - G
      g.beta = -1.0;
      gemm(cplx, PREC_F64, OP_N, OP_N, EPI_STORE, g, st);
    }
    fill_zero(X, n * m * (int64_t)esz, st);
    copy_cols(cplx, R, n, P, n, n, m, st);
    col_dots(cplx, R, n, R, n, n, m, rr, st);
    CHASE_HIP(hipMemcpyAsync(rr0, rr, m * 8, hipMemcpyDeviceToDevice, st));
    std::vector<double> hr(m), hr0(m);
    CHASE_HIP(hipMemcpyAsync(hr0.data(), rr0, m * 8, hipMemcpyDeviceToHost, st));
    CHASE_HIP(hipStreamSynchronize(st));
    bool done = true;
    for (int j = 0; j < m; ++j) done = done && hr0[j] == 0.0;
    int it = 0;
    while (!done && it < max_iter) {
      ++it;
      {  // Q = (H - Lambda) P
        GemmArgs g = gargs(n, m, n, H, ldh, P, n, nullptr, n);
        g.lambda = lam;
        g.V = P;
        g.ldv = n;
        g.partial = h->d_partial;
        g.F = Q;
        g.ldf = n;
        gemm(cplx, PREC_F64, OP_N, OP_N, EPI_RESID, g, st);
      }
      // Q -= V (V^H Q)
      gram(h, V, ldv, Q, n, n, m, m, h->R, ne, false, st);
      {
        GemmArgs g = gargs(n, m, m, V, ldv, h->R, ne, Q, n);
        g.alpha = -1.0;
        g.beta = 1.0;
        gemm(cplx, PREC_F64, OP_N, OP_N, EPI_STORE, g, st);
      }
      col_dots(cplx, P, n, Q, n, n, m, pq, st);
      cg_step(cplx, X, R, P, Q, n, n, m, rr, rr0, pq, tol * tol, rr_new, st);
      cg_dir(cplx, P, R, n, n, m, rr, rr0, pq, tol * tol, rr_new, st);
      if (it % 10 == 0 || it == max_iter) {
        CHASE_HIP(hipMemcpyAsync(hr.data(), rr, m * 8, hipMemcpyDeviceToHost, st));
        CHASE_HIP(hipStreamSynchronize(st));
        double worst = 0.0;
        for (int j = 0; j < m; ++j) {
          if (!std::isfinite(hr[j])) throw Error(CHASE_ERR_NUMERIC, "non-finite CG residual");
          if (hr0[j] > 0) worst = std::max(worst, std::sqrt(hr[j] / hr0[j]));
        }
        done = worst <= tol;
      }
    }
    if (iterations) *iterations = it;
    if (!done) throw Error(CHASE_ERR_NOCONV, "eigenvector adjoint: CG did not reach tol");
    // X -= V (V^H X) (exactly on the complement)
    gram(h, V, ldv, X, n, n, m, m, h->R, ne, false, st);
    {
      GemmArgs g = gargs(n, m, m, V, ldv, h->R, ne, X, n);
      g.alpha = -1.0;
      g.beta = 1.0;
      gemm(cplx, PREC_F64, OP_N, OP_N, EPI_STORE, g, st);
    }
    // dH += (X V^H + V X^H) / 2
    {
      GemmArgs g = gargs(n, n, m, X, n, V, ldv, dH, ldd);
      g.alpha = 0.5;
      g.beta = 1.0;
      gemm(cplx, PREC_F64, OP_N, OP_C, EPI_STORE, g, st);
      GemmArgs g2 = gargs(n, n, m, V, ldv, X, n, dH, ldd);
      g2.alpha = 0.5;
      g2.beta = 1.0;
      gemm(cplx, PREC_F64, OP_N, OP_C, EPI_STORE, g2, st);
    }
    // Within the block: dH += V E V^H, E = Hermitian part of M_ij / (lambda_j - lambda_i)
    sym_divdiff(cplx, h->G, ne, lam, m, h->R, ne, st);
    {
      GemmArgs g = gargs(n, m, m, V, ldv, h->R, ne, Q, n);  // Q = V E
      gemm(cplx, PREC_F64, OP_N, OP_N, EPI_STORE, g, st);
      GemmArgs g2 = gargs(n, n, m, Q, n, V, ldv, dH, ldd);  // dH += Q V^H
      g2.beta = 1.0;
      gemm(cplx, PREC_F64, OP_N, OP_C, EPI_STORE, g2, st);
    }
    CHASE_HIP(hipStreamSynchronize(st));
  });
}

chase_status chase_filter_adjoint(chase_handle_t h, const void* H, int64_t ldh, const void* gY,
                                  int64_t ldg, void* dH, int64_t ldd, void* gX, void* stream) {
  return guarded([&] {
    CHASE_REQUIRE(h != nullptr, "handle is NULL");
    CHASE_REQUIRE(H && gY && dH, "NULL pointer argument");
    CHASE_REQUIRE(h->tape_valid, "no recorded filter tape (call chase_filter with record_tape=1)");
    CHASE_REQUIRE(ldh >= h->n && ldg >= h->n && ldd >= h->n, "leading dimension smaller than n");
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_stream(h, st);
    const int64_t n = h->n;
    const int k = h->tape_k;
    const std::vector<int>& deg = h->tape_deg;
    const int mmax = deg[k - 1];
    const std::vector<Coef>& cf = h->tape_coef;
    // Reverse sweep of X_s = a_s (H - c) X_{s-1} + b_s X_{s-2}, s = 1..m_a:
    //   Gb_{s-1} += a_s (H - c) Gb_s ; Gb_{s-2} += b_s Gb_s ; dH += a_s Gb_s X_{s-1}^H
    // Column a enters the sweep at s = m_a with Gb = gY.  Buffers (n x k):
    //   G1 = Gb_s, G0 = Gb_{s-1}, with G2 accumulating Gb_{s-2} and rotated.
    void* G1 = h->V;
    void* G0 = h->W;
    void* G2 = h->Z;
    const size_t bytes = (size_t)n * k * h->esz;
    fill_zero(G1, bytes, st);
    fill_zero(G0, bytes, st);
    fill_zero(G2, bytes, st);
    // columns with m_a == mmax start at s = mmax
    auto first_col = [&](int s) { return (int)(std::lower_bound(deg.begin(), deg.end(), s) - deg.begin()); };
    for (int s = mmax; s >= 1; --s) {
      // inject gY for columns whose degree is exactly s: they start here
      const int a_lo = first_col(s), a_hi = first_col(s + 1);
      if (a_hi > a_lo)
        copy_cols(h->cplx, off(const_cast<void*>(gY), (int64_t)a_lo * ldg, h->esz), ldg,
                  off(G1, (int64_t)a_lo * n, h->esz), n, n, a_hi - a_lo, st);
      const int a0 = a_lo;  // active columns at step s: degree >= s
      const int cols = k - a0;
      if (cols <= 0) continue;
      const Coef c = cf[s - 1];
      void* g1 = off(G1, (int64_t)a0 * n, h->esz);
      // dH += a_s Gb_s X_{s-1}^H  (X_{s-1} from tape slot s-1)
      {
        GemmArgs g = gargs(n, n, cols, g1, n, off(h->tape, ((int64_t)(s - 1) * k + a0) * n, h->esz),
                           n, dH, ldd);
        g.alpha = c.alpha;
        g.beta = 1.0;
        gemm(h->cplx, PREC_F64, OP_N, OP_C, EPI_STORE, g, st);
      }
      // Gb_{s-1} += a_s (H - c) Gb_s   (EPI_CHEB with beta = 1 accumulates)
      {
        GemmArgs g = gargs(n, cols, n, H, ldh, g1, n, off(G0, (int64_t)a0 * n, h->esz), n);
        g.alpha = c.alpha;
        g.gamma = c.gamma;
        g.beta = 1.0;
        gemm(h->cplx, PREC_F64, OP_N, OP_N, EPI_CHEB, g, st);
      }
      // Gb_{s-2} += b_s Gb_s
      if (c.beta != 0.0)
        axpy_cols(h->cplx, c.beta, g1, n, off(G2, (int64_t)a0 * n, h->esz), n, n, cols, st);
      // rotate: Gb_{s-1} becomes the current, Gb_{s-2} the next accumulator
      std::swap(G1, G0);  // G1 = Gb_{s-1}
      std::swap(G0, G2);  // G0 = Gb_{s-2}, G2 = old Gb_s (to be cleared)
      fill_zero(off(G2, (int64_t)a0 * n, h->esz), (size_t)n * cols * h->esz, st);
    }
    // G1 now holds Gb_0 = dL/dX_0
    if (gX) copy_cols(h->cplx, G1, n, gX, ldg, n, k, st);
    herm_part(h->cplx, dH, ldd, n, st);
    CHASE_HIP(hipStreamSynchronize(st));
  });
}

}  // extern "C"
