// Internal declarations of the tensor-train solver library (not installed).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/tt_fde.h"

namespace ttf {

using zc = double2;  // complex double, interleaved (re, im)

// Split-K partial sums of one GEMM never take more than this many complex
// doubles (64 MiB): the split count is lowered to fit, so one workspace of
// this size serves every GEMM of a context.
constexpr size_t SPLITK_WS_ELEMS = size_t(1) << 22;

// panel width of the fast QR form
constexpr int WIDE_NB = 64;

// ------------------------------------------------------------------ errors
struct Error {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define TTF_HIP(call) ::ttf::hip_check((call), #call)

// Local (one-axis) operators of the grid discretisation, stored row by row
// as taps (column, weight) in compressed rows: the non-zeros of row i of
// operator o are taps tap_ptr[o n + i] .. tap_ptr[o n + i + 1] - 1.  The
// finite-difference operators have at most four per row; the cumulative
// (trapezoid) integral of the CDF equation is lower triangular.
//   I identity, X multiply by the coordinate, G first derivative, L2 second
//   derivative, XG = X G, XL2 = X L2, SG = diag(sin(pi u)) G, K = X - J with
//   J the cumulative trapezoid integral from the lower end of the axis.
enum LocalOp { OP_I = 0, OP_X = 1, OP_G = 2, OP_L2 = 3, OP_XG = 4, OP_XL2 = 5, OP_SG = 6, OP_K = 7, NOPS = 8 };

// Automaton transition (TT-matrix entry) at one site.
struct Entry {
  int alpha, beta, lop;
  double cre, cim;
};

// Packed device form of a transition list grouped by one channel index.
struct DevEntry {
  int other;  // the channel on the other side of the site
  int lop;
  double cre, cim;
};

struct DevBlock {  // exact apply: one (alpha, beta) block and its op list
  int alpha, beta, first, count;
};
struct DevBlockOp {
  int lop, pad;
  double cre, cim;
};

}  // namespace ttf

// ------------------------------------------------------------ opaque types
namespace ttf {
// where a block of device memory goes back to: the allocator of the
// context that made it (kept by value, so an object may be destroyed after
// its context) or hipFree
struct DevFree {
  tt_allocator a{};
  bool has = false;
  hipStream_t stream = nullptr;
  void operator()(void* p) const {
    if (!p) return;
    if (has)
      a.free(p, (void*)stream, a.user);
    else
      (void)hipFree(p);
  }
};
}  // namespace ttf

struct tt_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string last_error;
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> ws;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  // profiling
  bool profiling = false;
  bool profile_shapes = false;  // also key GEMM timings by shape
  long long qr_fallbacks = 0;   // QRs redone in the robust form
  // blocked Jacobi SVDs: count, sweeps launched, sweeps up to convergence,
  // and how many ended on the all-pairs rotation test
  long long jacobi_svds = 0, jacobi_sweeps_launched = 0, jacobi_sweeps_needed = 0, jacobi_check_passed = 0;
  std::string profile_only;     // when set, only this kernel class is timed
  int profile_every = 1;        // time one in this many launches of it
  long long profile_seen = 0;
  struct Stat {
    double ms = 0, flops = 0, bytes = 0;
    long long n = 0;
  };
  std::map<std::string, Stat> stats;
  struct Pending {
    std::string name;
    hipEvent_t a, b;
    double flops, bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;
  // sweeps the last Jacobi SVD of each size (m, k) needed: the next one of
  // that size launches as many before its first convergence check
  std::map<std::pair<int, int>, int> jacobi_sweeps_seen;
  int jacobi_max_sweeps = 60;   // sweep limit of every Jacobi SVD (tt_ctx_set_option)
  int qr_min_level = 0;         // most economical QR form allowed (tt_ctx_set_option)
  int sketch_mixed_passes = 1;  // reduced precision in the power passes but the last (tt_ctx_set_option)
  int qr_wide = 0;              // 64-column panels in the fast QR form (tt_ctx_set_option)
  int jacobi_fused = 1;         // sweeps of a Jacobi SVD in one launch per batch (tt_ctx_set_option)
  long jacobi_wait_limit = 1L << 20;  // polls of a fused-sweep barrier before it gives up

  // device memory: through the caller's allocator when one was given at
  // creation, else hipMalloc / hipFree; dev_alloc returns null on failure
  tt_allocator allocator{};
  bool has_allocator = false;
  void* dev_alloc(size_t bytes);
  void dev_free(void* p);
  ttf::DevFree releaser() const {
    ttf::DevFree r;
    r.a = allocator;
    r.has = has_allocator;
    r.stream = stream;
    return r;
  }

  void* get_ws(const std::string& name, size_t bytes);
  void* host_scratch(size_t bytes);
  void sync();
  void resolve_stats();
};


struct tt_tensor {
  tt_ctx* ctx = nullptr;
  ttf::DevFree release;          // returns the cores' memory
  int d = 0;
  int n = 0;                     // the common mode size; 0 when the sizes differ
  int dtype = TT_C128;           // storage of the cores (TT_C64: complex float)
  std::vector<int> nk;           // mode sizes n_1..n_d
  std::vector<int> cap, rank;
  std::vector<ttf::zc*> core;    // complex double, or complex float for TT_C64
  int orth = TT_ORTH_NONE;
  size_t cap_elems(int k) const { return (size_t)cap[k] * nk[k] * cap[k + 1]; }
  size_t elems(int k) const { return (size_t)rank[k] * nk[k] * rank[k + 1]; }
  size_t esize() const { return dtype == TT_C64 ? 8 : 16; }
};

struct tt_op {
  int d = 0, n = 0;
  double L = 0, nu = 0, adv = 1.0;
  double diff = 0.0;                  // numerical-diffusion coefficient kappa
  double ident = 0.0;                 // coefficient of an identity term
  std::vector<double> B, D;           // host coefficients
  std::vector<double> grid;           // a_i
  int kind = 0;                       // 0 Burgers-Hopf characteristic function, 1 CDF equation
  double gamma = 0.0, alpha = 0.0;    // CDF equation: viscosity and reaction amplitude
  std::vector<int> tap_ptr;           // NOPS n + 1 row starts
  std::vector<int> tap_col;           // columns of the taps
  std::vector<double> tap_w;          // weights of the taps
  std::vector<int> R;                 // bond dimensions, d+1
  std::vector<std::vector<ttf::Entry>> site;
  // device copies (when created with a context)
  tt_ctx* ctx = nullptr;
  ttf::DevFree release;
  int* d_tap_ptr = nullptr;
  int* d_tap_col = nullptr;
  double* d_tap_w = nullptr;
  struct SiteDev {
    int* in_ptr = nullptr;   // CSR over beta: incoming (alpha, op, coef)
    ttf::DevEntry* in_ent = nullptr;
    int* out_ptr = nullptr;  // CSR over alpha: outgoing (beta, op, coef)
    ttf::DevEntry* out_ent = nullptr;
    ttf::DevBlock* blocks = nullptr;
    ttf::DevBlockOp* bops = nullptr;
    int nblocks = 0;
  };
  std::vector<SiteDev> dev;
};

namespace ttf {

// ---------------------------------------------------------- host builder
void build_burgers_hopf(tt_op* op);  // fills everything but device data
void build_cdf_burgers(tt_op* op);   // the CDF equation (kind 1), likewise

// --------------------------------------------------------------- profiling
struct KTimer {
  tt_ctx* ctx;
  const char* name;
  double flops, bytes;
  hipEvent_t a = nullptr, b = nullptr;
  bool kernel = false;  // the events are taken by one kernel dispatch itself
  // kernel_events: the timed region is exactly one launch made with
  // TTF_LAUNCH, whose dispatch records the start and stop events (kernel
  // execution time, without the dispatch gap a stream event would include)
  KTimer(tt_ctx* c, const char* nm, double fl, double by, bool kernel_events = false);
  ~KTimer();
};

// hipLaunchKernelGGL, or hipExtLaunchKernelGGL with the events of an active
// kernel-event timer
#define TTF_LAUNCH(kt, kfn, grid, block, shmem, stream, ...)                                    \
  do {                                                                                          \
    if ((kt).a && (kt).kernel)                                                                  \
      hipExtLaunchKernelGGL(kfn, grid, block, shmem, stream, (kt).a, (kt).b, 0, __VA_ARGS__);   \
    else                                                                                        \
      hipLaunchKernelGGL(kfn, grid, block, shmem, stream, __VA_ARGS__);                         \
  } while (0)

// ---------------------------------------------------- rank predictor MLP
struct MlpDev {
  int n_in = 0, width = 0, nparams = 0, bcap = 0, step = 0;
  float* p = nullptr;       // FP32 master parameters
  _Float16* ph = nullptr;   // FP16 parameters used by the forward pass
  float* g = nullptr;       // gradients
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  float* act = nullptr;     // activations and deltas for bcap samples
  float* loss = nullptr;    // one float
};
void mlp_forward(tt_ctx* ctx, const MlpDev& m, const float* X, int B, float* h1, float* h2, float* y);
void mlp_gradients(tt_ctx* ctx, const MlpDev& m, const float* X, const float* T, int B, float* loss_dev);
void mlp_adam_step(tt_ctx* ctx, MlpDev& m, float lr);
void mlp_refresh_half(tt_ctx* ctx, MlpDev& m);
void mlp_half_values(tt_ctx* ctx, const MlpDev& m, float* out_dev);

// ------------------------------------------------------- kernel launchers
// op codes for GEMM operands
enum { OPN = 0, OPT = 1, OPC = 2 };

// C[M x N] = alpha op(A) op(B) + beta C, column major, batched with strides.
void zgemm(tt_ctx* ctx, int opA, int opB, int M, int N, int K, zc alpha, const zc* A,
           long lda, long strideA, const zc* B, long ldb, long strideB, zc beta, zc* C,
           long ldc, long strideC, int batch = 1);
// The same product in the arithmetic `fmt` (TT_PREC_*): FP64, or a split
// 16-bit form on the matrix cores (FP32 accumulation, FP64 operands and
// result; zgemm_split, k_mixed.hip).
void zgemm_prec(int fmt, tt_ctx* ctx, int opA, int opB, int M, int N, int K, zc alpha, const zc* A,
                long lda, long strideA, const zc* B, long ldb, long strideB, zc beta, zc* C,
                long ldc, long strideC, int batch);
void zgemm_split(int fmt, tt_ctx* ctx, int opA, int opB, int M, int N, int K, zc alpha, const zc* A, long lda,
                 long strideA, const zc* B, long ldb, long strideB, zc beta, zc* C, long ldc, long strideC,
                 int batch);
// C = alpha sum_s ws[s] + beta C over nsplit split-K partials
// ws[s][batch][N][M] (fixed summation order)
// Tuned GEMM launch shapes (the autotuner's table, process-wide): for a
// GEMM of the given form and shape, the workgroup tile (a, b: BM x BN of the
// FP64/FP32 kernel, or TI x TJ 32-blocks of the split 16-bit kernel) and the
// split-K factor.  A forced choice (set by the tuner on its own thread)
// takes precedence over the table.
struct GemmChoice {
  int a = 0, b = 0, nsplit = 0;
};
bool gemm_choice(int fmt, int opA, int opB, int M, int N, int K, int batch, GemmChoice* out);
void gemm_force(const GemmChoice* c);  // nullptr: none (calling thread only)
// table entries as 10 ints: fmt, opA, opB, M, N, K, batch, a, b, nsplit
void gemm_table_put(const int* e);
int gemm_table_count();
bool gemm_table_entry(int index, int* e);
void gemm_table_clear();
void splitk_finish(tt_ctx* ctx, int M, int N, int batch, int nsplit, zc* ws, zc alpha, zc beta, zc* C, long ldc,
                   long strideC);

// LDS Householder leaves for panels of at most 32 columns: P balanced row
// blocks of 32..256 rows, see k_qr.hip
void pt_leaves(tt_ctx* ctx, zc* Q, long ldq, int nleaves, int m, int k, zc* R, long ldr, long strideR);
void pt_assemble(tt_ctx* ctx, zc* Q, long ldq, int m, int k, int nleaves, const zc* S, long lds);
int pt_max_rows();
int pt_max_cols();
// block Gram-Schmidt helpers (k_qr.hip)
void bcgs_flag(tt_ctx* ctx, const zc* Y, long ldy, int m, int nb, const zc* W, long ldw, int p0, int* flags,
               double* part);
int bcgs_flag_groups(int m);  // partial sums used by bcgs_flag (part holds groups * nb)
void bcgs_pip(tt_ctx* ctx, const zc* W2, int p0, int nb, const zc* R1, zc* Ro, zc* Rd, long ldr, const int* flags,
              zc* R2inv, int* bad);
void chol_solve(tt_ctx* ctx, zc* Y, long ldy, int m, int nb, const zc* G, double tau, const zc* Rprev, zc* Rout,
                int* bad);
void panel_trmm(tt_ctx* ctx, zc* Z, long ldz, int m, int nb, const zc* Rinv);
// the same for panels of up to 64 columns, and the Cholesky factor and
// inverse of an up to 64 x 64 Gram matrix in one workgroup
void panel_trmm_wide(tt_ctx* ctx, zc* Z, long ldz, int m, int nb, const zc* Rinv);
void chol_factor_wide(tt_ctx* ctx, const zc* G, long ldg, int nb, double tau, bool absolute, const zc* Rprev,
                      zc* Rout, long ldo, const int* flags, zc* Rinv, int* bad);
void zero_ints(tt_ctx* ctx, int* x, int n);
void bcgs_random(tt_ctx* ctx, zc* Qp, long ldq, int m, int nb, const int* flags, uint64_t seed, int tag);
void bcgs_masked_add(tt_ctx* ctx, zc* Rd, long ldr, const zc* W, long ldw, int rows, int nb, const int* flags);
void bcgs_put_diag(tt_ctx* ctx, zc* Rd, long ldr, const zc* Rp, int nb, const int* flags);
void fill_zero(tt_ctx* ctx, zc* x, long n);
// dst (k x m, ld ldd) = src (m x k, ld lds)^H
void conj_transpose(tt_ctx* ctx, const zc* src, long lds, zc* dst, long ldd, int m, int k);
// One-sided Jacobi SVD of B (m x k, ld m) in place: on exit the columns of B
// are U * Sigma, sorted by decreasing norm; sigma[k] holds the norms and B
// is scratch; U (m x k, ld m) receives the normalised columns (zero where
// sigma = 0).  Writes the
// number of sweeps used to *sweeps (device int).
void jacobi_svd(tt_ctx* ctx, int m, int k, zc* B, zc* U, double* sigma, int* sweeps);
// the same with its counters in the per-device static scratch (allocates
// nothing; *sweeps_host is a host int, the call synchronises)
void jacobi_svd_noalloc(tt_ctx* ctx, int m, int k, zc* B, zc* U, double* sigma, int* sweeps_host);
void noalloc_scratch_init(int device);  // once per device, that device current

// Elementwise / small helpers.
void set_identity(tt_ctx* ctx, zc* A, int m, int k, long lda);  // A = I (m x k)
void copy_matrix(tt_ctx* ctx, const zc* src, long lds, zc* dst, long ldd, int m, int k);
void frob_norm2(tt_ctx* ctx, const zc* x, long n, double* out_dev);  // single value

// TT kernels
void concat_core(tt_ctx* ctx, int nterms, const zc* const* src, const int* r0s, const int* r1s,
                 const zc* coefs, int kind, int n, zc* dst, int R0, int R1);
void widen_c64(tt_ctx* ctx, const void* src, zc* dst, long n);      // complex float -> double
void narrow_c128(tt_ctx* ctx, const zc* src, void* dst, long n);    // complex double -> float
void tt_eval_kernel(tt_ctx* ctx, int d, const int* nk, const zc* const* cores, const int* ranks,
                    const int32_t* idx, int64_t npts, zc* out);
void gaussian_factor(tt_ctx* ctx, zc* core, int n, double L, double mu, double sigma);
void nn_gaussian_core(tt_ctx* ctx, zc* core, int r0, int n, int r1, int nprev, double L, double mu, double sigma,
                      double c);
void cdf_gaussian_factor(tt_ctx* ctx, zc* core, int n, double box, double sigma);
void identity_core(tt_ctx* ctx, zc* core, int n, int r1);  // (n r1) x n x r1, I
void apply_exact_core(tt_ctx* ctx, const tt_op* op, int site, const zc* x, int r0, int r1,
                      zc* y);
// left-sketch gather:  W[j,i,b,beta] = sum_in(beta) c * (O V[j,alpha,:,b])[i]
void gather_left(tt_ctx* ctx, const tt_op* op, int site, const zc* V, zc* W, int l, int r1);
// right gather: Z[a,alpha,i,q] = sum_out(alpha) c * (O V2[a,:,beta,q])[i]
void gather_right(tt_ctx* ctx, const tt_op* op, int site, const zc* V2, zc* Z, int r0, int s);
// Gaussian sketch core (counter-based Philox4x32-10 + Box-Muller)
void sketch_core(tt_ctx* ctx, zc* w, long count, uint64_t seed, int site, double scale);
// x <- 2^-e x with e the largest exponent in x (e[0]); with accumulate,
// e[1] += e.  pow2_restore: x <- 2^e[1] x.  e: two device ints.
void pow2_normalize(tt_ctx* ctx, zc* x, long n, int* e, bool accumulate);
void pow2_restore(tt_ctx* ctx, zc* x, long n, const int* e);

}  // namespace ttf
