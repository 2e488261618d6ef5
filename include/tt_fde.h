/*
 * tt_fde.h - C ABI of the MI355X tensor-train solver for the Burgers-Hopf
 * characteristic-function PDE.
 *
 * The method (Rodgers & Venturi, "Tensor approximation of functional
 * differential equations"):
 *   - Sec. 3, eq. (hyper1): projecting the Hopf FDE of Burgers' equation
 *     (Sec. 5, eq. (eqn:BHfde), no reaction term) onto d Fourier modes gives
 *     the linear PDE
 *         dphi/dt = sum_k a_k [ (i/2) sum_jl B_kjl d2phi/da_j da_l
 *                               + nu sum_j D_kj dphi/da_j ].
 *   - Sec. 4, eq. (tt)/(eqn:ode): phi is held on an n^d tensor-product grid
 *     (second-order finite differences) as a tensor train.
 *   - Sec. 4.1, eq. (eqn:discrete-flow-trunc-intro): step-truncation; an
 *     explicit Runge-Kutta step off the TT manifold followed by truncation.
 *   - App. A.1: TT format, sum by concatenation, scaling, orthogonalisation
 *     (Alg. 1, mirrored) and truncation by rounding (Alg. 2, mirrored).
 *
 * Conventions shared by every entry point
 *   - All floating-point data are complex double, stored interleaved
 *     (re, im) as pairs of doubles.
 *   - A TT core C_k has shape r_{k-1} x n x r_k and is stored column major
 *     with the left rank index fastest: C[a, i, b] at a + r_{k-1}(i + n b)
 *     (the vertical / horizontal flattenings of App. A.1 are then zero-copy).
 *   - Every call is enqueued asynchronously on the context's HIP stream
 *     unless stated otherwise.  Device pointers passed in must stay valid
 *     until the enqueued work completes.
 *   - Every call returns TT_OK (0) or a negative TT_E* code; no exception
 *     crosses the ABI.  tt_last_error() gives a text for the last failure on
 *     that context.  After TT_EHIP the context should be destroyed.
 *   - A null context, tensor, operator or network handle (the destroy calls
 *     included) or a null required output pointer gives TT_EINVAL before any
 *     HIP call.  Exceptions: tt_last_error(NULL) returns "null context",
 *     tt_ctx_stream(NULL) returns NULL, and tt_step_batch with count 0 is
 *     an empty batch (TT_OK).
 *   - Tensors own cap-sized device buffers allocated at creation; no call in
 *     the stepping path allocates tensor storage.  Contexts own workspaces,
 *     grown on first use to the largest size a call needs.
 */
#ifndef TT_FDE_H
#define TT_FDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TT_MAX_D 128

enum {
  TT_OK = 0,
  TT_EINVAL = -1,      /* invalid argument (null pointer, bad option)         */
  TT_ESHAPE = -2,      /* d / n / rank mismatch between arguments             */
  TT_ECAPACITY = -3,   /* a result rank exceeds the output tensor's capacity  */
  TT_ENOMEM = -4,      /* device or host allocation failed                    */
  TT_EHIP = -5,        /* a HIP runtime call failed                           */
  TT_ENOCONV = -6,     /* Jacobi SVD or TT-GMRES did not converge in its limit */
  TT_ENONFINITE = -7   /* a non-finite value was detected                     */
};

/* Orthogonality state of a tensor (App. A.1 definitions). */
enum { TT_ORTH_NONE = 0, TT_ORTH_RIGHT = 1, TT_ORTH_LEFT = 2 };

/* Operator application modes. */
enum {
  TT_APPLY_EXACT = 0,  /* operator in TT-matrix form times x: ranks multiply   */
  TT_APPLY_SKETCH = 1  /* fused apply + randomised range compression           */
};

/* Step-truncation schemes of tt_step (Sec. 4.1). */
enum {
  TT_STEP_RK4 = 0,      /* classical RK4, four stages (default)                  */
  TT_STEP_EULER = 1,    /* truncated explicit Euler, eq. (adaptive-euler-method) */
  TT_STEP_MIDPOINT = 2, /* truncated explicit midpoint,
                           eq. (adaptive-midpoint-method_2)                      */
  TT_STEP_IMPLICIT_EULER = 3,    /* implicit step-truncation Euler,
                                    eq. (EB-linear), TT-GMRES                    */
  TT_STEP_IMPLICIT_MIDPOINT = 4  /* implicit step-truncation midpoint,
                                    eq. (MP-linear), TT-GMRES                    */
};

/* Arithmetic of the operator application's contractions. */
enum {
  TT_PREC_FP64 = 0,    /* plain complex FP64                                   */
  TT_PREC_BF16X3 = 1,  /* split-BF16x3 on the bf16 matrix cores, FP32
                          accumulation (about 17 significant bits; see
                          tt_zgemm_mixed)                                      */
  TT_PREC_FP16X3 = 2,  /* split-FP16x3 on the fp16 matrix cores with a
                          power-of-two scale per K stage, FP32 accumulation
                          (about 22 significant bits)                          */
  TT_PREC_FP32 = 3     /* operands rounded to FP32 on the fp32 matrix cores,
                          FP32 accumulation within each K step of 16 and FP64
                          across them (the FP32 form)                          */
};

typedef struct tt_ctx tt_ctx;
typedef struct tt_tensor tt_tensor;
typedef struct tt_op tt_op;

/* Storage precision of a tensor's cores. */
typedef enum {
  TT_C128 = 0,  /* complex double (interleaved pairs of doubles) */
  TT_C64 = 1    /* complex float: half the memory at rest; every call works
                   on complex-double copies of the C64 tensors it touches
                   (held in context workspaces) and rounds results back */
} tt_dtype;

/* Device-memory provider of a context (for example a bridge to a caching
 * allocator).  alloc returns `bytes` of device memory usable on `stream`
 * (a hipStream_t), or NULL when it cannot (the library call then fails
 * with TT_ENOMEM); free returns a block alloc gave.  `user` is passed
 * back unchanged.  Both are called from the thread that makes the library
 * call, possibly several at once from tt_step_batch. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* p, void* stream, void* user);
  void* user;
} tt_allocator;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  hip_stream is a hipStream_t or
 * NULL (the context then creates its own default-priority stream).  alloc
 * (may be NULL: hipMalloc / hipFree) provides every device allocation made
 * for this context: tensor cores, operator tables, workspaces, the
 * predictor network; the struct is copied.  Workspaces grow to the largest
 * size a call needed and are kept: after one call at the largest shapes
 * (tt_step_reserve), later calls at those or smaller shapes allocate
 * nothing.  Destroy tensors, operators and networks before their context. */
int tt_ctx_create(int device, void* hip_stream, const tt_allocator* alloc, tt_ctx** out);
int tt_ctx_destroy(tt_ctx* ctx);
/* Wait for all work enqueued on the context's stream. */
int tt_ctx_sync(tt_ctx* ctx);
const char* tt_last_error(const tt_ctx* ctx);
/* The hipStream_t all work is enqueued on. */
void* tt_ctx_stream(const tt_ctx* ctx);

/* Per-kernel timing with HIP events on the context stream (off by default).
 * on = 0 off, 1 on, 2 on and every GEMM also recorded under the key
 * "zgemm:<opA><opB>:MxNxKxbatch".  Kernel classes (one kernel each unless
 * noted): "zgemm" (the GEMM proper), "zgemm_reduce" (its split-K
 * reduction), "pt_leaf" (LDS panel Householder QR leaves), "pt_assemble",
 * "bcgs_pip", "panel_trmm", "jacobi_svd" (a whole small SVD: several
 * kernels and one host synchronisation), "gather_left", "gather_right",
 * "apply_exact", "concat", "eval".  flops / bytes are the algorithmic counts
 * of the launches recorded; times are summed event durations.  Every call
 * syncs the context stream. */
int tt_ctx_set_profiling(tt_ctx* ctx, int on);
/* Restrict event timing to one kernel class (NULL or "" = all classes), so
 * that a timed run pays the event overhead of that class only. */
int tt_ctx_set_profile_filter(tt_ctx* ctx, const char* kernel);

/* With a profile filter set, time only one in `every` launches of the
 * filtered class (a uniform sample: its statistics report the sampled
 * launches, so averages stay unbiased while the event overhead falls).
 * every >= 1; 1 (the default) times every launch. */
int tt_ctx_set_profile_sampling(tt_ctx* ctx, int every);
int tt_ctx_reset_stats(tt_ctx* ctx);

/* Context options.  TT_OPT_JACOBI_MAX_SWEEPS (1..60, default 60): sweep
 * limit of every Jacobi SVD on this context (the truncation SVD of App. A.4
 * inside tt_round / tt_step, and tt_svd_small).  An SVD that has not
 * converged at its limit is an error: the call fails with TT_ENOCONV and
 * takes no truncation from it.  A small limit forces that path, so callers
 * can test their handling of it.  TT_OPT_QR_MIN_LEVEL (0..2, default 0):
 * the first form every orthogonalisation tries (0: Cholesky QR twice per
 * panel with the checked fast second pass, 1: Householder panels with the
 * fast second pass, 2: Householder panels twice); each form falls back to
 * the next when its checks fail, so results agree to rounding.
 * TT_OPT_JACOBI_FUSED (0 or 1, default 1): 1 runs each batch of Jacobi
 * sweeps as one launch whose workgroups meet at grid barriers between the
 * rounds of a sweep (SVDs up to 1024 columns), 0 launches every round on
 * its own; both apply the same rotations in the same order, so the results
 * are bitwise the same.  TT_OPT_JACOBI_WAIT_LIMIT (0 .. 2^40, default
 * 2^20): polls a workgroup of the fused form makes at one barrier before it
 * gives up; every workgroup then returns and the call fails with
 * TT_ENOCONV (0 forces that path for tests).  TT_OPT_QR_WIDE_PANELS (0 or
 * 1, default 0): the Cholesky form of the orthogonalisations takes panels
 * of 64 columns (1: the factor and its inverse formed once per pass, then
 * a triangular update) or 32 (0); results agree to rounding.
 * TT_OPT_SKETCH_MIXED_PASSES (0 or 1, default 1): with power passes, the
 * reduced precision of a sketched apply covers the Gaussian sketch pass
 * only (0) or every pass but the last (1); the last pass, the projection
 * whose result is truncated, is FP64.  TT_EINVAL for an
 * unknown option or a value out of range. */
enum {
  TT_OPT_JACOBI_MAX_SWEEPS = 1,
  TT_OPT_QR_MIN_LEVEL = 2,
  TT_OPT_JACOBI_FUSED = 3,
  TT_OPT_JACOBI_WAIT_LIMIT = 4,
  TT_OPT_QR_WIDE_PANELS = 5,
  TT_OPT_SKETCH_MIXED_PASSES = 6
};
int tt_ctx_set_option(tt_ctx* ctx, int option, long long value);
int tt_ctx_get_stats(tt_ctx* ctx, const char* kernel, double* total_ms,
                     double* flops, double* bytes, long long* launches);
/* All recorded keys as text, one line each: "key launches total_ms flops
 * bytes", NUL-terminated in buf (cap bytes, caller-owned); the first line,
 * "qr_fallbacks N 0 0 0", counts the QR factorisations since the last reset
 * whose fast second pass was unsafe and that were redone in the robust form
 * (counted whether or not profiling is on).  Returns TT_ECAPACITY when the
 * text was cut. */
int tt_ctx_dump_stats(tt_ctx* ctx, char* buf, long cap);

/* ---------------------------------------------------------------- tensors */

/* Tensor with d modes of sizes n[0..d-1] (each >= 4) and rank capacities
 * rank_cap[0..d] (rank_cap[0] and rank_cap[d] must be 1), cores stored as
 * `dtype`.  Cores are allocated at capacity (through the context's
 * allocator).  Initial ranks are all 1 with zero cores.  Tensors whose mode
 * sizes differ serve the TT arithmetic (tt_round, tt_axpy, tt_sum, tt_dot,
 * tt_norm, tt_eval, copies); the operator calls need every size equal to
 * the operator's n (TT_ESHAPE otherwise). */
int tt_tensor_create(tt_ctx* ctx, int d, const int* n, const int* rank_cap, tt_dtype dtype, tt_tensor** out);
/* Mode sizes (d ints) and storage type of a tensor. */
int tt_tensor_get_modes(const tt_tensor* t, int* n, int* dtype);
int tt_tensor_destroy(tt_tensor* t);
/* Copy host cores in (synchronous).  ranks[0..d]; cores[k] points to
 * 2*ranks[k]*n_k*ranks[k+1] doubles in the layout above (complex double on
 * the host whatever the storage type; C64 storage rounds them). */
int tt_tensor_set_cores(tt_tensor* t, const int* ranks, const double* const* cores);
/* Current ranks (host copy; reflects all completed work - call after
 * tt_ctx_sync for work still in flight). */
int tt_tensor_get_ranks(const tt_tensor* t, int* ranks);
/* Copy cores out to host buffers sized by the current ranks, as complex
 * double (synchronous). */
int tt_tensor_get_cores(const tt_tensor* t, double* const* cores);
int tt_tensor_get_orth(const tt_tensor* t);
/* dst <- src (same d and mode sizes; dst capacities must hold src's ranks;
 * storage types may differ: the copy converts). */
int tt_tensor_copy(tt_ctx* ctx, const tt_tensor* src, tt_tensor* dst);
/* Rank-one Gaussian characteristic function on the grid a_i = -L + 2Li/(n-1):
 * phi0(a) = prod_k exp(i mu_k a_k - sigma_k^2 a_k^2 / 2)
 * (characteristic function of independent N(mu_k, sigma_k^2) amplitudes). */
int tt_tensor_set_gaussian(tt_ctx* ctx, tt_tensor* t, const double* mu,
                           const double* sigma, double L);

/* -------------------------------------------------------------- operator */

/* Build the Burgers-Hopf operator for d Fourier modes (mode k = 1..d has
 * wavenumber ceil(k/2), cosine for odd k, sine for even k) on n grid points
 * per axis over [-L, L] with viscosity nu.  Finite differences: centred
 * second order, one-sided second-order boundary rows.  The operator is held
 * as a TT-matrix (finite-state automaton over the local operators I, X, G,
 * L2, XG) whose bond dimension is at most 2d + 2.  ctx may be NULL: the
 * operator is then host-only (usable with the export calls below). */
int tt_op_create_burgers_hopf(tt_ctx* ctx, int d, int n, double L, double nu, tt_op** out);
/* Same with the advective (B) term multiplied by `advection` (1 gives the
 * Burgers-Hopf operator, 0 the viscous-only operator whose exact
 * semi-discrete solution is known in closed form). */
int tt_op_create_burgers_hopf_scaled(tt_ctx* ctx, int d, int n, double L, double nu,
                                     double advection, tt_op** out);
/* The general form: advection scales the B term as above; diffusion >= 0
 * adds the numerical-diffusion stabilisation kappa sum_k d^2/da_k^2 of the
 * explicit runs of Sec. 5.2 (kappa = diffusion, chosen by the caller
 * proportional to dt; 0 gives the plain operator). */
typedef struct {
  int size;              /* sizeof(tt_op_opts) */
  int pad;
  double advection;      /* 1: Burgers-Hopf */
  double diffusion;      /* kappa >= 0 */
} tt_op_opts;
int tt_op_create_burgers_hopf_ex(tt_ctx* ctx, int d, int n, double L, double nu, const tt_op_opts* opts,
                                 tt_op** out);
/* The CDF equation (Sec. 5, eq. (eqn:cdf-burgers)): the joint cumulative
 * distribution F(u_1..u_d, t) of the stochastic Burgers equation with
 * reaction alpha sin(pi u) and viscosity gamma (eq. (eqn:burgers-rxn)) at d
 * evenly spaced points of the circle, periodic second-order differences in
 * x.  With D1, D2 those difference matrices (spacing 2 pi / d):
 *   dF/dt = sum_i [-gamma D2_ii u_i - alpha sin(pi u_i)] dF/du_i
 *         + sum_{i != j} [D1_ij u_i - gamma D2_ij] (u_j - J_j) dF/du_i
 * (J_j the cumulative integral along u_j from the lower end; the reaction
 * enters once).  Phase space [-box, box]^d with n points per axis, centred
 * second-order differences with outflow boundaries (dF/du = 0 there),
 * trapezoid rule for J.  Real coefficients; tensors stay complex (imaginary
 * parts zero).  TT-matrix form over the local operators of
 * tt_op_export_local_ops; bond dimension at most 10.  ctx may be NULL
 * (host-only operator).  *out is owned by the caller (tt_op_destroy).
 * TT_EINVAL for d outside 1..128, n < 4, a size mismatch of opts, box <= 0,
 * gamma < 0 or diffusion < 0, or when no term remains (d = 1 with gamma,
 * alpha and diffusion all zero). */
typedef struct {
  int size;              /* sizeof(tt_cdf_opts) */
  int pad;
  double box;            /* half-width of the phase-space box (> 0) */
  double gamma;          /* viscosity (>= 0) */
  double alpha;          /* reaction amplitude */
  double diffusion;      /* kappa >= 0: kappa sum_k d2F/du_k^2 (numerical diffusion) */
} tt_cdf_opts;
int tt_op_create_cdf_burgers(tt_ctx* ctx, int d, int n, const tt_cdf_opts* opts, tt_op** out);
/* The CDF equation's initial condition (Sec. 5, the paper's product of
 * zero-mean Gaussian CDFs): 0.5 (1 + erf(u_k / (sigma sqrt 2))) on the grid
 * u_i = -box + 2 box i / (n-1) of every axis; t becomes rank one (any
 * capacity suffices).  Asynchronous on the context's stream; TT_EINVAL for
 * box <= 0 or sigma <= 0. */
int tt_tensor_set_cdf_gaussian(tt_ctx* ctx, tt_tensor* t, double sigma, double box);
int tt_op_destroy(tt_op* op);
/* Bond dimensions R[0..d] of the operator's TT-matrix form. */
int tt_op_get_ranks(const tt_op* op, int* R);
/* Host-side export for inspection and tests (no device work):
 *   coefficients: B (d*d*d, index (k*d + j)*d + l) and D (d*d, k*d + j);
 *   local operators: nops*n*n doubles, op-major, row-major n x n matrices,
 *     in the order I, X, G, L2, XG, XL2, SG = diag(sin(pi u)) G,
 *     K = X - J (J the cumulative trapezoid integral; the last two used by
 *     the CDF equation) (returns nops via *nops);
 *   site entries: for site m (0-based) the transitions
 *     (alpha, beta, local op, coefficient re/im) of the automaton.
 *     Call with NULL arrays to query the count. */
int tt_op_export_coefficients(const tt_op* op, double* B, double* D);
int tt_op_export_local_ops(const tt_op* op, int* nops, double* mats);
int tt_op_export_site(const tt_op* op, int site, int* count, int* alpha, int* beta,
                      int* lop, double* coef);

/* ----------------------------------------------------------- arithmetic */

typedef struct {
  int size;              /* sizeof(tt_apply_opts) */
  int mode;              /* TT_APPLY_EXACT or TT_APPLY_SKETCH */
  int sketch_rank;       /* sketch width l for TT_APPLY_SKETCH (>= 1) */
  int precision;         /* TT_PREC_FP64, or TT_PREC_BF16X3 / TT_PREC_FP16X3 /
                            TT_PREC_FP32:
                            the sketch contractions in that split 16-bit
                            form (mixed form; the exact product and
                            everything else stay FP64).  With power > 0
                            the last sweep (the projection) is FP64 and
                            the earlier ones use it, or only the Gaussian
                            sketch sweep with TT_OPT_SKETCH_MIXED_PASSES 0 */
  uint64_t seed;         /* counter-based RNG key for the Gaussian sketch */
  int power;             /* SKETCH: subspace-iteration passes after the
                            first sweep, 0..8 */
  int pad;
} tt_apply_opts;

/* y <- L x.  EXACT: the TT-matrix product (Sec. 3 operator applied core by
 * core; ranks R_k r_k; y needs that capacity).  SKETCH: y is the projection
 * of L x onto bases found by a randomised range finder in TT form of width
 * l: left Gaussian TT sketches of L x, then a right-to-left sweep of LQ
 * factorisations giving right-orthonormal cores; each of `power` further
 * sweeps runs the other way with the previous sweep's interface chains in
 * place of the sketch (a subspace-iteration step per bond).  For an odd
 * `power` the Gaussian sketches are drawn from the right and the first
 * sweep runs left to right, so the last sweep always runs right to left
 * and y is right-orthonormal.  Ranks <= l (bounded by n^k and n^(d-k)); exact whenever l
 * reaches the ranks of L x.  The projection of L x onto a truncation of
 * it is, at Sec. 4.1's truncation T, an approximation of T[L x]: its error
 * against the exact T[L x] falls with l and with the passes. */
int tt_apply(tt_ctx* ctx, const tt_op* op, const tt_tensor* x, tt_tensor* y,
             const tt_apply_opts* opts);

/* z <- alpha x + beta y by concatenation (App. A.1).  Scalars are complex
 * (re, im).  z must not alias x or y. */
int tt_axpy(tt_ctx* ctx, double alpha_re, double alpha_im, const tt_tensor* x,
            double beta_re, double beta_im, const tt_tensor* y, tt_tensor* z);
/* z <- sum_t coef[t] x_t (coef: 2*nterms doubles), one concatenation. */
int tt_sum(tt_ctx* ctx, int nterms, const double* coef, const tt_tensor* const* xs,
           tt_tensor* z);

typedef struct {
  int d;
  int ranks[TT_MAX_D + 1];     /* output ranks */
  double tail[TT_MAX_D];       /* discarded Frobenius tail per bond */
  double sigma_min_kept[TT_MAX_D];
  double norm;                 /* ||x|| before truncation */
  int jacobi_sweeps_max;
  int pad;
  double sv_last[TT_MAX_D][8]; /* per bond the 8 smallest kept singular values,
                                  decreasing, zeros in front when fewer */
  double sigma_first_cut[TT_MAX_D]; /* per bond the largest discarded singular
                                  value (0 when none is discarded): with
                                  sigma_min_kept it gives the gap at the cut,
                                  near 1 where the truncation is ill-determined */
} tt_round_report;

/* TT rounding (App. A.1, Alg. 2 mirrored): right-to-left orthogonalisation
 * (skipped when x is already right-orthogonal), then a left-to-right sweep
 * of truncated SVDs.  Per bond the smallest rank k >= 1 whose discarded tail
 * is <= eps_rel * ||x|| / sqrt(d - 1) is kept, then k <= rmax[b] (rmax:
 * NULL for no cap, or d+1 ints whose entry b caps bond b, <= 0 meaning no
 * cap there; the end entries are ignored) and k <= the capacity of x.
 * Output cores 1..d-1 are left-orthonormal.  rep may be NULL; when given
 * it is filled on return (the call then synchronises).  TT_ENOCONV when a
 * truncation SVD stops at its sweep limit (x then holds the rounding up to
 * that bond, a valid TT of the same tensor up to the tails cut so far). */
int tt_round(tt_ctx* ctx, tt_tensor* x, double eps_rel, const int* rmax, tt_round_report* rep);

/* Gaussian characteristic function with tridiagonal covariance (amplitudes
 * u ~ N(mu, Sigma), Sigma_kk = sigma_k^2, Sigma_k,k+1 = rho_k sigma_k
 * sigma_k+1): phi0(a) = prod_k exp(i mu_k a_k - sigma_k^2 a_k^2 / 2)
 * prod_k exp(-rho_k sigma_k sigma_k+1 a_k a_k+1) on the grid a_i = -L + 2Li/(n-1).  The
 * exact nearest-neighbour product has bond ranks n; t receives its
 * rounding (eps_rel, rmax and rep as in tt_round; t's capacities must hold
 * the rounded ranks, TT_ECAPACITY otherwise).  rho: d-1 values in
 * (-1/2, 1/2), which keeps Sigma positive definite. */
int tt_tensor_set_gaussian_tridiag(tt_ctx* ctx, tt_tensor* t, const double* mu, const double* sigma,
                                   const double* rho, double L, double eps_rel, const int* rmax,
                                   tt_round_report* rep);

typedef struct {
  int size;              /* sizeof(tt_step_opts) */
  int rmax;              /* rank cap of every truncation */
  double eps;            /* relative tolerance of every truncation */
  int apply_mode;        /* TT_APPLY_EXACT or TT_APPLY_SKETCH */
  int sketch_rank;
  uint64_t seed;
  int precision;         /* a TT_PREC_* value (the operator
                            applications' contractions; QR, SVD, truncation
                            test and sums always FP64) */
  int scheme;            /* a TT_STEP_* value */
  double gmres_tol;      /* implicit schemes: relative residual target of
                            TT-GMRES (> 0) */
  int gmres_max_iter;    /* implicit schemes: Krylov dimension, 1..40 */
  int krylov_rmax;       /* implicit schemes: rank cap of the Krylov vectors
                            (0: 2 rmax), at most 256 */
  const int* learned_widths; /* learned form (RK4): NULL, or d+1 per-bond sketch
                            widths (entries 1..512; the end entries are
                            ignored). Every truncation of a sum in the step
                            (the stage inputs and the final combination) is
                            then a randomised rounding to these widths
                            (tt_round_randomized), accepted when its a
                            posteriori relative error is at most
                            learned_tol and finished by the deterministic
                            rounding of its small result; otherwise the
                            deterministic rounding of the sum is used */
  double learned_tol;    /* relative error accepted from a randomised rounding */
  const int* learned_apply_widths; /* learned form (RK4, sketched apply): NULL,
                            or d+1 per-bond sketch widths (1..512, the end
                            entries ignored, capped at sketch_rank) for the
                            stage applications; a stage whose rounded
                            derivative reaches its width at a bond (the
                            width may have cut it) is applied again at
                            sketch_rank (fallback) */
  int sketch_power;      /* subspace-iteration passes of every sketched
                            apply (tt_apply_opts.power), 0..8 */
  int pad2;
} tt_step_opts;

typedef struct {
  int stages;
  int max_rank;          /* largest rank of any truncated tensor in the step */
  int ranks[TT_MAX_D + 1];
  int learned_used;      /* randomised truncations tried (learned form) */
  int learned_fallback;  /* ... of which missed learned_tol (deterministic used) */
  double learned_err;    /* the largest a posteriori relative error among them */
  double final_norm;     /* norm of the final combination (explicit schemes) */
  double final_sv[TT_MAX_D][8]; /* sv_last of the final rounding */
  int k_ranks[TT_MAX_D + 1];  /* per bond, the largest rank of the rounded
                                 stage derivatives (explicit schemes) */
  int learned_apply_fallback; /* stages applied again at sketch_rank */
} tt_step_report;

/* One step-truncation step of df/dt = L f, in place, T = tt_round(eps,
 * rmax).  TT_STEP_RK4 (classical RK4 with a truncation after every
 * operator application and every stage combination):
 *   k1 = T[L f],  y2 = T[f + dt/2 k1],  k2 = T[L y2],  y3 = T[f + dt/2 k2],
 *   k3 = T[L y3], y4 = T[f + dt k3],    k4 = T[L y4],
 *   f <- T[f + dt/6 (k1 + 2 k2 + 2 k3 + k4)]
 * Each of the four stages is one operator application, its truncation, one
 * combination and its truncation (the last stage's combination is the
 * final one).  TT_STEP_EULER: f <- T[f + dt T[L f]] (one stage).
 * TT_STEP_MIDPOINT: f <- T[f + dt T[L(f + dt/2 T[L f])]] (two stages; the
 * stage input f + dt/2 T[L f] is not truncated, as in Sec. 4.1).
 * rep->stages is 4, 1 or 2.
 * TT_STEP_IMPLICIT_EULER / TT_STEP_IMPLICIT_MIDPOINT (Sec. 4.1): solve
 * (I - dt L) x = f, resp. (I - dt/2 L) x = T[f + dt/2 T[L f]], by TT-GMRES
 * (tt_solve_shifted) started from the explicit Euler / midpoint step, then
 * f <- T[x]; rep->stages counts the operator applications.  TT_ENOCONV if
 * GMRES does not reach gmres_tol within gmres_max_iter iterations (f is
 * then left unchanged).  TT_EINVAL for an unknown scheme. */
int tt_step(tt_ctx* ctx, const tt_op* op, tt_tensor* f, double dt,
            const tt_step_opts* opts, tt_step_report* rep);

/* Sizes every workspace and temporary tt_step needs for f's capacities:
 * one step (opts, dt) of a copy of f's shape with every interior rank at
 * its capacity (seeded random cores); f is not read or changed.  After it,
 * tt_step on tensors of that shape with these options allocates nothing
 * (synchronous; it allocates). */
int tt_step_reserve(tt_ctx* ctx, const tt_op* op, const tt_tensor* f, double dt, const tt_step_opts* opts);

/* Batched form: `count` independent instances, instance i being one
 * tt_step(ctxs[i], ops[i], fs[i], dts[i], &opts[i], &reps[i]) (reps may be
 * NULL).  Instances with the same context run in order on one host thread
 * and that context's stream; distinct contexts run on their own threads,
 * so their kernels overlap on the GPU (each instance alone leaves most of
 * the chip idle: its kernels are small and latency-bound).  Every context
 * must be used by this call only.  status[i] receives instance i's return
 * code (an instance that fails leaves the others running); the call
 * returns TT_OK or the first nonzero status.  Synchronous. */
int tt_step_batch(int count, tt_ctx* const* ctxs, const tt_op* const* ops, tt_tensor* const* fs,
                  const double* dts, const tt_step_opts* opts, tt_step_report* reps, int* status);

/* out[p] = x[idx[p, 0], ..., idx[p, d-1]] (iterated matrix product,
 * App. A.1).  idx: device int32 array npts x d (row p contiguous);
 * out: device array of npts complex values. */
int tt_eval(tt_ctx* ctx, const tt_tensor* x, const int32_t* idx, int64_t npts, double* out);

/* Building block exposed for testing and benchmarking: complex double GEMM
 * on the context stream, C = alpha op(A) op(B) + beta C, column major, with
 * op 0 = none, 1 = transpose, 2 = conjugate transpose, and `batch` strided
 * batches.  A, B, C are device pointers to interleaved complex doubles;
 * leading dimensions and strides count complex elements. */
int tt_zgemm(tt_ctx* ctx, int opA, int opB, int M, int N, int K, double alpha_re, double alpha_im,
             const double* A, int64_t lda, int64_t strideA, const double* B, int64_t ldb,
             int64_t strideB, double beta_re, double beta_im, double* C, int64_t ldc,
             int64_t strideC, int batch);

/* The same product in a split 16-bit arithmetic on the matrix cores: the
 * core contractions of the mixed-precision form.  Every real operand is
 * split as hi + lo in the 16-bit format and each real product taken as
 * hi*hi + hi*lo + lo*hi with FP32 accumulation, summed into FP64.
 * precision TT_PREC_BF16X3: bfloat16 halves, error about 1e-5 of
 * |op(A)| |op(B)| per entry.  TT_PREC_FP16X3: half-precision halves with a
 * power-of-two scale per 32-wide K stage of each operand tile, error about
 * 5e-7 of the same.  TT_PREC_FP32 (not split): operands rounded to FP32
 * on the fp32 matrix cores, FP32 sums over K steps of 16 added in FP64,
 * error about 1e-6 of the same.  Other arguments and layout as tt_zgemm;
 * TT_EINVAL for any other precision. */
int tt_zgemm_mixed(tt_ctx* ctx, int precision, int opA, int opB, int M, int N, int K, double alpha_re,
                   double alpha_im, const double* A, int64_t lda, int64_t strideA, const double* B,
                   int64_t ldb, int64_t strideB, double beta_re, double beta_im, double* C, int64_t ldc,
                   int64_t strideC, int batch);

/* GEMM launch-shape autotuner (process-wide table).  Every GEMM of the
 * library picks its workgroup tile and split-K factor by a rule of the
 * output shape; an entry of this table replaces the rule for one exact
 * (precision, opA, opB, M, N, K, batch).  tt_gemm_autotune times every
 * candidate tile (FP64/FP32: 64x64, 128x32, 64x32, 32x32, 32x64; split
 * 16-bit: 64x64, 32x64, 64x32, 32x32 as TI x TJ blocks of 32) with every
 * power-of-two split-K factor up to half the K steps, on random operands it
 * allocates (and frees) itself, three timed runs each after one warm-up on
 * the context's stream, and stores the fastest; choice (3 ints, may be
 * NULL): tile a, b and the split factor; best_us (may be NULL): its time.
 * Synchronous; it allocates device memory, so it is a set-up step, not for
 * code under graph capture.  Different split factors sum in different
 * groupings: results differ at rounding level from the untuned rule, and
 * are deterministic for a given table.  Table entries are 10 ints:
 * precision, opA, opB, M, N, K, batch, a, b, split; get/set copy one entry
 * (TT_EINVAL for an index out of range or an invalid entry). */
int tt_gemm_autotune(tt_ctx* ctx, int precision, int opA, int opB, int M, int N, int K, int batch, int* choice,
                     double* best_us);
int tt_gemm_table_count(void);
int tt_gemm_table_get(int index, int* entry);
int tt_gemm_table_set(const int* entry);
int tt_gemm_table_clear(void);

/* Complex inner product <x, y> = sum over all entries of conj(x) y
 * (synchronous): left-to-right contraction of the cores, two GEMMs per
 * core (App. A.1 arithmetic).  out: host array of 2 doubles (re, im). */
int tt_dot(tt_ctx* ctx, const tt_tensor* x, const tt_tensor* y, double* out);

/* TT-GMRES for the shifted system (I - c L) x = b of the implicit
 * step-truncation schemes (Sec. 4.1, eq. (EB-linear) / (MP-linear); the
 * method of the reference cited there): Krylov vectors are TTs truncated to
 * krylov_eps (relative) and krylov_rmax after every operator application
 * and orthogonalisation (two classical Gram-Schmidt passes with TT inner
 * products), the small Hessenberg least-squares problem is solved by Givens
 * rotations on the host, and the solution x0 + V y is truncated to (eps,
 * rmax).  x: on entry the initial guess when use_guess (else zero), on exit
 * the truncated solution (its capacities must hold rmax).  Synchronous. */
typedef struct {
  int size;              /* sizeof(tt_solve_opts) */
  int max_iter;          /* Krylov dimension, 1..40 (no restart) */
  double tol;            /* relative residual target ||r|| <= tol ||b|| */
  double krylov_eps;     /* relative truncation of Krylov vectors (> 0) */
  int krylov_rmax;       /* rank cap of Krylov vectors, 1..256 */
  int rmax;              /* rank cap of the returned solution */
  double eps;            /* relative truncation of the returned solution */
  int apply_mode;        /* TT_APPLY_EXACT or TT_APPLY_SKETCH */
  int sketch_rank;
  uint64_t seed;
  int precision;         /* TT_PREC_* of the operator applications */
  int use_guess;         /* 1: x holds the initial guess */
} tt_solve_opts;

typedef struct {
  int iterations;        /* Krylov vectors generated */
  int converged;         /* residual estimate <= tol */
  double residual;       /* final relative residual estimate |g_{k+1}| / ||b|| */
  int max_rank;          /* largest rank of a Krylov vector */
  int pad;
} tt_solve_report;

int tt_solve_shifted(tt_ctx* ctx, const tt_op* op, double c, const tt_tensor* b, tt_tensor* x,
                     const tt_solve_opts* opts, tt_solve_report* rep);

/* Randomised rounding with per-bond sketch widths (the randomised tt_round
 * of the learned form): y = the sketched product of x with the identity
 * operator, i.e. left Gaussian TT sketches of widths[k] (Philox key seed)
 * and a right-to-left sweep of LQ factorisations; y is right-orthonormal
 * with rank k <= widths[k] (widths: d+1 ints, ends ignored, each within
 * y's capacity).  *rel_err (may be NULL) receives an estimate of
 * ||x - y|| / ||x|| by an independent Gaussian TT sketch Omega of 64 rows
 * (bond rank 64, its own Philox key): ||Omega x - Omega y|| / ||Omega x||,
 * from chain contractions only (no factorisation, no cancellation of
 * squares); the a posteriori check that decides whether the deterministic
 * rounding is needed.  Synchronous. */
int tt_round_randomized(tt_ctx* ctx, const tt_tensor* x, const int* widths, uint64_t seed, tt_tensor* y,
                        double* rel_err);

/* ---------------------------------------------------- rank predictor MLP */
/* The learned form's per-bond rank predictor: n_in -> width -> width -> 1
 * with ReLU hidden layers, FP16 parameters widened to FP32 for products
 * on the FP32 matrix cores with FP32 activations, deltas and sums, FP32
 * master parameters and Adam (beta 0.9, 0.999, eps 1e-8) for
 * training on the loss L = (1 / 2B) sum_b (y_b - t_b)^2.  Parameter vector
 * (host float32, tt_mlp_param_count of them): W1 (width x n_in, row-major),
 * b1 (width), W2 (width x width), b2 (width), W3 (1 x width), b3 (1).
 * Samples: a device float32 matrix B x n_in (row-major), targets and
 * outputs device float32 vectors of B; B at most max_batch.  Every sum runs
 * in a fixed order: results are deterministic.  All calls are on the
 * context's stream; the ones returning host values synchronise. */
typedef struct tt_mlp tt_mlp;
int tt_mlp_create(tt_ctx* ctx, int n_in, int width, int max_batch, tt_mlp** out);
int tt_mlp_destroy(tt_mlp* m);
int tt_mlp_param_count(const tt_mlp* m);
/* set the FP32 master parameters (their FP16 copy follows; Adam restarts) */
int tt_mlp_set_params(tt_ctx* ctx, tt_mlp* m, const float* host);
/* as_used = 0: the master parameters; 1: the FP16 values the forward uses */
int tt_mlp_get_params(tt_ctx* ctx, const tt_mlp* m, float* host, int as_used);
int tt_mlp_forward(tt_ctx* ctx, tt_mlp* m, const float* x, int B, float* y);
/* loss and gradient (host, nparams floats; either may be NULL) at the
 * FP16 parameters */
int tt_mlp_gradients(tt_ctx* ctx, tt_mlp* m, const float* x, const float* t, int B, float* loss, float* grad);
/* `iters` full-batch Adam steps at learning rate lr; *loss (may be NULL)
 * receives the loss after them */
int tt_mlp_train(tt_ctx* ctx, tt_mlp* m, const float* x, const float* t, int B, int iters, float lr, float* loss);

/* Frobenius norm of x (synchronous; computed by orthogonalisation). */
int tt_norm(tt_ctx* ctx, const tt_tensor* x, double* out);

/* Building block exposed for testing: the QR factorisation used by every
 * orthogonalisation of the TT sweeps (the QR of V(C) and the LQ of H(C),
 * App. A.1, Alg. 1-2).  A (m x k, ld lda >= m, m >= k >= 1) = Q R with Q
 * (m x k, ld m) orthonormal and R (k x k, ld k) upper triangular, also for
 * rank-deficient A: a column whose residual after projection onto the
 * earlier ones is below 1e-13 of its own norm is dependent; its R column is
 * zero below the projection coefficients and its Q column a random
 * direction orthogonal to the others.  Device pointers to
 * interleaved complex doubles; A is not modified; synchronous (one host
 * synchronisation per attempt of the checked fast path). */
int tt_qr(tt_ctx* ctx, int m, int k, const double* A, int64_t lda, double* Q, double* R);

/* Building block exposed for testing: one-sided Jacobi SVD of the small
 * factor of a TT truncation (App. A.4): B (m x k, ld m, m <= 1536 and
 * k <= 1536, overwritten) has left singular vectors U (m x k, ld m; columns
 * in order of decreasing singular value, a zero column for a zero singular
 * value) and singular values sigma (k doubles, decreasing).  sweeps
 * (host int, may be null) receives the number of sweeps.  Device pointers;
 * synchronous.  TT_ENOCONV when 60 sweeps did not converge. */
int tt_svd_small(tt_ctx* ctx, int m, int k, double* B, double* U, double* sigma, int* sweeps);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): tt_svd_small with the
 * same arguments, layout and results, allocating nothing.  Its sweep
 * counters live in a per-GPU static device array of 1 KiB (held until the
 * process ends), set up when a context is created on that GPU; the call
 * synchronises the context's stream to read the sweep count.  Calls that
 * overlap on one GPU (two streams or threads) share that array and race:
 * serialise them.  TT_EINVAL for sizes outside 1..1536 or while profiling
 * is on (event timing allocates events); TT_ENOCONV as tt_svd_small. */
int tt_svd_small_noalloc(tt_ctx* ctx, int m, int k, double* B, double* U, double* sigma, int* sweeps);

#ifdef __cplusplus
}
#endif
#endif /* TT_FDE_H */
