// C ABI and host orchestration: tensors, operator upload, TT rounding
// sweeps, exact and sketched operator application, RK4 step-truncation.
#include <algorithm>
#include <cmath>
#include <complex>
#include <mutex>
#include <thread>
#include <cstring>
#include <new>
#include <tuple>

#include "common.hpp"

namespace ttf {

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(TT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

KTimer::KTimer(tt_ctx* c, const char* nm, double fl, double by, bool kernel_events)
    : ctx(c), name(nm), flops(fl), bytes(by), kernel(kernel_events) {
  if (!ctx || !ctx->profiling) return;
  if (!ctx->profile_only.empty() && ctx->profile_only != nm) return;
  if (ctx->profile_every > 1 && (ctx->profile_seen++ % ctx->profile_every) != 0) return;
  auto take = [&]() {
    hipEvent_t e;
    if (!ctx->free_events.empty()) {
      e = ctx->free_events.back();
      ctx->free_events.pop_back();
    } else {
      TTF_HIP(hipEventCreate(&e));
    }
    return e;
  };
  a = take();
  b = take();
  if (!kernel) TTF_HIP(hipEventRecord(a, ctx->stream));
}

KTimer::~KTimer() {
  if (!a) return;
  if (!kernel) (void)hipEventRecord(b, ctx->stream);
  ctx->pending.push_back({name, a, b, flops, bytes});
}

}  // namespace ttf

using namespace ttf;

void* tt_ctx::dev_alloc(size_t bytes) {
  if (has_allocator) return allocator.alloc(bytes, (void*)stream, allocator.user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void tt_ctx::dev_free(void* p) {
  if (!p) return;
  if (has_allocator)
    allocator.free(p, (void*)stream, allocator.user);
  else
    (void)hipFree(p);
}

void* tt_ctx::get_ws(const std::string& name, size_t bytes) {
  Buf& b = ws[name];
  if (b.bytes >= bytes && b.p) return b.p;
  if (b.p) {
    TTF_HIP(hipStreamSynchronize(stream));
    dev_free(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  const size_t want = std::max<size_t>(bytes + bytes / 8, 4096);
  b.p = dev_alloc(want);
  if (!b.p) fail(TT_ENOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed (" + name + ")");
  b.bytes = want;
  return b.p;
}

void* tt_ctx::host_scratch(size_t bytes) {
  if (pinned_bytes >= bytes) return pinned;
  if (pinned) {
    TTF_HIP(hipStreamSynchronize(stream));
    TTF_HIP(hipHostFree(pinned));
    pinned = nullptr;
    pinned_bytes = 0;
  }
  const size_t want = std::max<size_t>(bytes, 1 << 16);
  TTF_HIP(hipHostMalloc(&pinned, want, hipHostMallocDefault));
  pinned_bytes = want;
  return pinned;
}

void tt_ctx::resolve_stats() {
  for (auto& p : pending) {
    float ms = 0;
    TTF_HIP(hipEventSynchronize(p.b));
    if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) {
      // a timed launch that did not happen (an error path): nothing to add
      (void)hipGetLastError();
      free_events.push_back(p.a);
      free_events.push_back(p.b);
      continue;
    }
    Stat& s = stats[p.name];
    s.ms += ms;
    s.flops += p.flops;
    s.bytes += p.bytes;
    s.n += 1;
    free_events.push_back(p.a);
    free_events.push_back(p.b);
  }
  pending.clear();
}

void tt_ctx::sync() {
  TTF_HIP(hipStreamSynchronize(stream));
  resolve_stats();
}

namespace {

#define ABI_TRY try {
#define ABI_CATCH(ctxp)                                   \
  }                                                       \
  catch (const ttf::Error& e) {                           \
    if (ctxp) (ctxp)->last_error = e.msg;                 \
    return e.code;                                        \
  }                                                       \
  catch (const std::bad_alloc&) {                         \
    if (ctxp) (ctxp)->last_error = "host allocation failed"; \
    return TT_ENOMEM;                                     \
  }                                                       \
  catch (const std::exception& e) {                       \
    if (ctxp) (ctxp)->last_error = e.what();              \
    return TT_EINVAL;                                     \
  }                                                       \
  catch (...) {                                           \
    if (ctxp) (ctxp)->last_error = "unknown error";       \
    return TT_EINVAL;                                     \
  }

inline zc Z(double re, double im = 0.0) { return make_double2(re, im); }

void require(bool c, int code, const char* msg) {
  if (!c) fail(code, msg);
}

void copy_d2d(tt_ctx* ctx, zc* dst, const zc* src, size_t elems) {
  if (elems == 0 || dst == src) return;
  TTF_HIP(hipMemcpyAsync(dst, src, elems * sizeof(zc), hipMemcpyDeviceToDevice, ctx->stream));
}

// ------------------------------------------------------------- QR
// Householder TSQR of a panel of k <= 32 columns held in q (m x k, ld ldq),
// in place: q becomes Q, r (ld ldr) the k x k R factor.  P balanced row
// blocks of at most 256 rows are factored in LDS; their stacked R factors
// (P k x k, ld P k) are factored recursively and each block of Q is then
// multiplied by its k x k block of the stacked Q.
void ptsqr_inplace(tt_ctx* ctx, int m, int k, zc* q, long ldq, zc* r, long ldr, int level) {
  require(m >= k && k >= 1 && k <= pt_max_cols(), TT_EINVAL, "panel tsqr: bad shape");
  const int bmax = pt_max_rows();
  if (m <= bmax) {
    pt_leaves(ctx, q, ldq, 1, m, k, r, ldr, 0);
    return;
  }
  const int P = (m + bmax - 1) / bmax;  // every block has floor(m / P) > bmax / 2 >= k rows
  const long Sm = (long)P * k;
  zc* S = (zc*)ctx->get_ws("ptsqr_S" + std::to_string(level), sizeof(zc) * Sm * k);
  pt_leaves(ctx, q, ldq, P, m, k, S, Sm, k);
  ptsqr_inplace(ctx, (int)Sm, k, S, Sm, r, ldr, level + 1);
  pt_assemble(ctx, q, ldq, m, k, P, S, Sm);
}

// QR of A (m x k, m >= k) by block classical Gram-Schmidt with
// reorthogonalisation over panels of 32 columns: Q (m x k, ld m)
// orthonormal, R (k x k, ld k) upper triangular, A = Q R.  The matrix is
// factored in place: q holds A on entry and Q on exit.
// Per panel: project out the earlier columns (W = Q^H A_p, A_p -= Q W);
// replace every column whose residual is below 1e-13 of its norm (a column
// dependent on the earlier ones to working accuracy, or zero) by a Gaussian
// vector, to be left out of R; factor the panel (Q1 R1); then project once
// more.
// level 0 factors the panel by Cholesky QR twice (panels of 32 columns, or
// of 64 with TT_OPT_QR_WIDE_PANELS 1), levels 1 and 2 by the Householder
// TSQR (panels of 32); levels 0 and 1 finish with the Pythagorean shortcut
// (Cholesky of I - W2^H W2, see bcgs_pip), level 2 factors the reprojected
// panel again with the TSQR and projects and factors it a third time.  Shortcuts raise *bad when they are not safe
// for the data (bad may be null at level 2).
void bcgs_qr_inplace(tt_ctx* ctx, int m, int k, zc* q, zc* r, int level, int* bad) {
  require(m >= k && k >= 1, TT_EINVAL, "qr: need m >= k >= 1");
  // level 0 takes panels of 64 columns (Cholesky factor and inverse in one
  // workgroup, then a triangular update), levels 1 and 2 panels of 32
  // (the Householder leaves' width)
  const bool wide = level == 0 && ctx->qr_wide;
  const int NB = wide ? WIDE_NB : pt_max_cols();
  fill_zero(ctx, r, (long)k * k);
  // small work: W2, T (k x NB), R1, R2, Rpp, Gm, Ra, Rinv (NB x NB), flags,
  // norm partials; sized for the widest panel
  const size_t kb = (size_t)k * WIDE_NB, bb = (size_t)WIDE_NB * WIDE_NB;
  const int G = bcgs_flag_groups(m);
  zc* W2 = (zc*)ctx->get_ws("bcgs_small", sizeof(zc) * (2 * kb + 6 * bb) + sizeof(double) * ((size_t)(G + 1) * WIDE_NB));
  zc* T = W2 + kb;
  zc* R1 = T + kb;
  zc* R2 = R1 + bb;
  zc* Rpp = R2 + bb;
  zc* Gm = Rpp + bb;
  zc* Ra = Gm + bb;
  zc* Rinv = Ra + bb;
  int* flags = (int*)(Rinv + bb);
  double* part = (double*)(Rinv + bb) + WIDE_NB;  // WIDE_NB ints fit in WIDE_NB doubles
  const uint64_t rseed = 0x243F6A8885A308D3ull;
  for (int p0 = 0; p0 < k; p0 += NB) {
    const int nb = std::min(NB, k - p0);
    zc* Ap = q + (long)m * p0;
    zc* Rp = r + (long)k * p0;  // R[0:p0, p0:p0+nb]
    if (p0 > 0) {
      zgemm(ctx, OPC, OPN, p0, nb, m, Z(1), q, m, 0, Ap, m, 0, Z(0), Rp, k, 0);
      zgemm(ctx, OPN, OPN, m, nb, p0, Z(-1), q, m, 0, Rp, k, 0, Z(1), Ap, m, 0);
    }
    bcgs_flag(ctx, Ap, m, m, nb, Rp, k, p0, flags, part);
    bcgs_random(ctx, Ap, m, m, nb, flags, rseed, p0);
    if (wide) {
      // Cholesky QR twice, the factor and its inverse formed once per pass;
      // then, past the first panel, the second projection and the
      // Pythagorean factor of I - W2^H W2 (as bcgs_pip, absolute pivot test)
      zgemm(ctx, OPC, OPN, nb, nb, m, Z(1), Ap, m, 0, Ap, m, 0, Z(0), Gm, nb, 0);
      chol_factor_wide(ctx, Gm, nb, nb, 1e-12, false, nullptr, Ra, nb, nullptr, Rinv, bad);
      panel_trmm_wide(ctx, Ap, m, m, nb, Rinv);
      zgemm(ctx, OPC, OPN, nb, nb, m, Z(1), Ap, m, 0, Ap, m, 0, Z(0), Gm, nb, 0);
      chol_factor_wide(ctx, Gm, nb, nb, 0.5, false, Ra, R1, nb, nullptr, Rinv, bad);
      panel_trmm_wide(ctx, Ap, m, m, nb, Rinv);
      if (p0 == 0) {
        bcgs_put_diag(ctx, r, k, R1, nb, flags);
        continue;
      }
      zgemm(ctx, OPC, OPN, p0, nb, m, Z(1), q, m, 0, Ap, m, 0, Z(0), W2, p0, 0);
      zgemm(ctx, OPN, OPN, m, nb, p0, Z(-1), q, m, 0, W2, p0, 0, Z(1), Ap, m, 0);
      set_identity(ctx, Gm, nb, nb, nb);
      zgemm(ctx, OPC, OPN, nb, nb, p0, Z(-1), W2, p0, 0, W2, p0, 0, Z(1), Gm, nb, 0);
      chol_factor_wide(ctx, Gm, nb, nb, 1e-2, true, R1, r + (long)k * p0 + p0, k, flags, Rinv, bad);
      zgemm(ctx, OPN, OPN, p0, nb, nb, Z(1), W2, p0, 0, R1, nb, 0, Z(0), T, p0, 0);
      bcgs_masked_add(ctx, Rp, k, T, p0, p0, nb, flags);
      panel_trmm_wide(ctx, Ap, m, m, nb, Rinv);
      continue;
    }
    if (level == 0) {
      // Cholesky QR twice: Y = Y Ra^{-1}, then again with Rb; R1 = Rb Ra
      // (a column dependent within the panel makes a pivot fail the test)
      zgemm(ctx, OPC, OPN, nb, nb, m, Z(1), Ap, m, 0, Ap, m, 0, Z(0), Gm, nb, 0);
      chol_solve(ctx, Ap, m, m, nb, Gm, 1e-12, nullptr, Ra, bad);
      zgemm(ctx, OPC, OPN, nb, nb, m, Z(1), Ap, m, 0, Ap, m, 0, Z(0), Gm, nb, 0);
      chol_solve(ctx, Ap, m, m, nb, Gm, 0.5, Ra, R1, bad);
    } else {
      ptsqr_inplace(ctx, m, nb, Ap, m, R1, nb, 0);
    }
    if (p0 == 0) {
      bcgs_put_diag(ctx, r, k, R1, nb, flags);
      continue;
    }
    zgemm(ctx, OPC, OPN, p0, nb, m, Z(1), q, m, 0, Ap, m, 0, Z(0), W2, p0, 0);
    zgemm(ctx, OPN, OPN, m, nb, p0, Z(-1), q, m, 0, W2, p0, 0, Z(1), Ap, m, 0);
    if (level == 2) {
      // Householder factor of the reprojected panel, then a third projection
      // and factorisation: a column that the second projection left with
      // little more than rounding error (nearly in the span of the earlier
      // columns) is normalised by the factorisation, and only one more pass
      // makes it orthogonal to them to working accuracy
      ptsqr_inplace(ctx, m, nb, Ap, m, R2, nb, 0);
      zgemm(ctx, OPN, OPN, nb, nb, nb, Z(1), R2, nb, 0, R1, nb, 0, Z(0), Rpp, nb, 0);
      zgemm(ctx, OPN, OPN, p0, nb, nb, Z(1), W2, p0, 0, R1, nb, 0, Z(0), T, p0, 0);
      bcgs_masked_add(ctx, Rp, k, T, p0, p0, nb, flags);
      zgemm(ctx, OPC, OPN, p0, nb, m, Z(1), q, m, 0, Ap, m, 0, Z(0), W2, p0, 0);
      zgemm(ctx, OPN, OPN, m, nb, p0, Z(-1), q, m, 0, W2, p0, 0, Z(1), Ap, m, 0);
      ptsqr_inplace(ctx, m, nb, Ap, m, R2, nb, 0);
      zgemm(ctx, OPN, OPN, nb, nb, nb, Z(1), R2, nb, 0, Rpp, nb, 0, Z(0), Gm, nb, 0);
      zgemm(ctx, OPN, OPN, p0, nb, nb, Z(1), W2, p0, 0, Rpp, nb, 0, Z(0), T, p0, 0);
      bcgs_masked_add(ctx, Rp, k, T, p0, p0, nb, flags);
      bcgs_put_diag(ctx, r + (long)k * p0 + p0, k, Gm, nb, flags);
    } else {
      bcgs_pip(ctx, W2, p0, nb, R1, Rp, r + (long)k * p0 + p0, k, flags, R2, bad);
      panel_trmm(ctx, Ap, m, m, nb, R2);
    }
  }
}

// Runs the fastest form and checks its flag (one host synchronisation per
// attempt); when a shortcut was unsafe for some panel, `load` refills q and
// the next, more robust form runs: level 0 factors each projected panel by
// Cholesky QR twice, level 1 by the Householder TSQR, both finishing with
// the Pythagorean second pass; level 2 uses the Householder TSQR for both
// passes and cannot fail.
// With deferred_bad, only the fast form runs and its flag is or-ed into
// *deferred_bad (device) without a host synchronisation: the caller reads
// it at its next synchronisation and redoes the work from start_level 1.
template <class Load>
void qr_checked(tt_ctx* ctx, int m, int k, zc* q, zc* r, Load load, int* deferred_bad = nullptr,
                int start_level = 0) {
  start_level = std::max(start_level, ctx->qr_min_level);
  if (deferred_bad && start_level == 0) {
    load();
    bcgs_qr_inplace(ctx, m, k, q, r, 0, deferred_bad);
    return;
  }
  int* bad = (int*)ctx->get_ws("qr_bad", 64);
  int* h = (int*)ctx->host_scratch(64);
  for (int level = start_level; level < 2; ++level) {
    zero_ints(ctx, bad, 1);
    load();
    bcgs_qr_inplace(ctx, m, k, q, r, level, bad);
    TTF_HIP(hipMemcpyAsync(h, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    TTF_HIP(hipStreamSynchronize(ctx->stream));
    if (h[0] == 0) return;
    ctx->qr_fallbacks += 1;
  }
  load();
  bcgs_qr_inplace(ctx, m, k, q, r, 2, nullptr);
}

// QR of A (m x k, ld lda, m >= k): Q (m x k, ld m), R (k x k, ld k).
void tsqr(tt_ctx* ctx, int m, int k, const zc* a, long lda, zc* q, zc* r, int* deferred_bad = nullptr,
          int start_level = 0) {
  qr_checked(ctx, m, k, q, r, [&]() { copy_matrix(ctx, a, lda, q, m, m, k); }, deferred_bad, start_level);
}

// LQ of A (k x m, ld lda, k <= m): A = R^H Qt^H with Qt (m x k, ld m) having
// orthonormal columns; returns Qt and R (k x k upper).
void tsqr_lq(tt_ctx* ctx, int k, int m, const zc* a, long lda, zc* qt, zc* r, int* deferred_bad = nullptr,
             int start_level = 0) {
  qr_checked(ctx, m, k, qt, r, [&]() { conj_transpose(ctx, a, lda, qt, m, k, m); }, deferred_bad, start_level);
}

int bounded_pow(int n, int e, int cap) {
  long v = 1;
  for (int i = 0; i < e && v < cap; ++i) v *= n;
  return (int)std::min<long>(v, cap);
}

// ------------------------------------------------------- TT rounding
void phase1_right_orth(tt_ctx* ctx, tt_tensor* x) {
  const int d = x->d;
  auto& r = x->rank;
  for (int c = d - 1; c >= 1; --c) {
    const int n = x->nk[c], nl = x->nk[c - 1];
    const int p0 = r[c], p1 = r[c + 1];
    const int N = n * p1;
    const int rl = r[c - 1];
    // the new C_{c-1} has N columns when H(C_c) is taller than wide, else p0
    zc* tmp = (zc*)ctx->get_ws("ph1_tmp", sizeof(zc) * (size_t)rl * nl * (p0 > N ? N : p0));
    if (p0 > N) {
      // H(C_c) is taller than wide: C_c <- I, C_{c-1} <- C_{c-1} H(C_c)
      zgemm(ctx, OPN, OPN, rl * nl, N, p0, Z(1), x->core[c - 1], (long)rl * nl, 0, x->core[c], p0, 0, Z(0), tmp,
            (long)rl * nl, 0);
      copy_d2d(ctx, x->core[c - 1], tmp, (size_t)rl * nl * N);
      identity_core(ctx, x->core[c], n, p1);
      r[c] = N;
    } else {
      zc* qt = (zc*)ctx->get_ws("ph1_q", sizeof(zc) * (size_t)p0 * N);
      zc* R = (zc*)ctx->get_ws("ph1_r", sizeof(zc) * (size_t)p0 * p0);
      tsqr_lq(ctx, p0, N, x->core[c], p0, qt, R);
      conj_transpose(ctx, qt, N, x->core[c], p0, N, p0);  // C_c <- Qt^H
      // C_{c-1} <- C_{c-1} L, L = R^H
      zgemm(ctx, OPN, OPC, rl * nl, p0, p0, Z(1), x->core[c - 1], (long)rl * nl, 0, R, p0, 0, Z(0), tmp,
            (long)rl * nl, 0);
      copy_d2d(ctx, x->core[c - 1], tmp, (size_t)rl * nl * p0);
    }
  }
  x->orth = TT_ORTH_RIGHT;
}

double core_norm(tt_ctx* ctx, const tt_tensor* x, int k) {
  double* dv = (double*)ctx->get_ws("norm_out", 64);
  frob_norm2(ctx, x->core[k], (long)x->elems(k), dv);
  double* h = (double*)ctx->host_scratch(64);
  TTF_HIP(hipMemcpyAsync(h, dv, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  TTF_HIP(hipStreamSynchronize(ctx->stream));
  return std::sqrt(std::max(0.0, h[0]));
}

int truncation_rank(const std::vector<double>& s, double delta, int cap, double* tail_out) {
  const int k = (int)s.size();
  std::vector<double> tail(k + 1, 0.0);
  for (int i = k - 1; i >= 0; --i) tail[i] = tail[i + 1] + s[i] * s[i];
  int kk = k;
  for (int j = 1; j <= k; ++j)
    if (std::sqrt(tail[j]) <= delta) {
      kk = j;
      break;
    }
  // singular values at roundoff level (sigma^2 <= 4e-30 sum sigma^2) are
  // zero: the Jacobi SVD does not rotate such columns, so their left
  // vectors are not orthogonal to the others and U_k U_k^H would stop being
  // a projector if they were kept (only reachable with eps = 0)
  int nz = 0;
  while (nz < k && s[nz] * s[nz] > 4e-30 * tail[0]) ++nz;
  kk = std::min(kk, std::max(nz, 1));
  if (cap > 0) kk = std::min(kk, cap);
  kk = std::max(kk, 1);
  if (tail_out) *tail_out = std::sqrt(tail[kk]);
  return kk;
}

// caps: per-bond rank caps (d+1 ints, <= 0: none), or null with rmax for
// every bond (rmax <= 0: none)
void round_tensor(tt_ctx* ctx, tt_tensor* x, double eps, int rmax, tt_round_report* rep,
                  const int* caps = nullptr) {
  require(x->dtype == TT_C128, TT_EINVAL, "internal: rounding needs complex-double storage");
  const int d = x->d;
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->d = d;
  }
  if (d == 1) {
    if (rep) {
      rep->ranks[0] = rep->ranks[1] = 1;
      rep->norm = core_norm(ctx, x, 0);
    }
    return;
  }
  if (x->orth != TT_ORTH_RIGHT) phase1_right_orth(ctx, x);
  auto& r = x->rank;
  const double norm = core_norm(ctx, x, 0);
  const double delta = eps * norm / std::sqrt((double)(d - 1));
  int sweeps_max = 0;
  for (int c = 0; c < d - 1; ++c) {
    const int n = x->nk[c], n1 = x->nk[c + 1];
    const int m = r[c] * n, k = r[c + 1];
    const int rr = r[c + 2];
    const int sq = std::min(m, k);  // size of the square factor
    zc* Q = (zc*)ctx->get_ws("p2_q", sizeof(zc) * (size_t)m * k);
    zc* R = (zc*)ctx->get_ws("p2_r", sizeof(zc) * (size_t)sq * sq);
    zc* B = (zc*)ctx->get_ws("p2_b", sizeof(zc) * (size_t)sq * sq);
    zc* U = (zc*)ctx->get_ws("p2_u", sizeof(zc) * (size_t)sq * sq);
    double* sig = (double*)ctx->get_ws("p2_sig", sizeof(double) * (sq + 8));
    int* sw = (int*)(sig + sq + 2);
    zc* carry = (zc*)ctx->get_ws("p2_carry", sizeof(zc) * (size_t)sq * k);
    zc* tmp = (zc*)ctx->get_ws("p2_tmp", sizeof(zc) * (size_t)sq * n1 * rr);
    const zc* V = x->core[c];
    int* qbad = (int*)(sig + sq + 4);  // fast-form QR flag, read with sigma
    // the factorisations only read the core, so a failed fast form is
    // redone from the start (deferred: no synchronisation of its own)
    auto factor = [&](bool fast) {
      int* db = fast ? qbad : nullptr;
      const int lvl = fast ? 0 : 1;
      if (fast) zero_ints(ctx, qbad, 1);
      if (m >= k) {
        // V = Q R and R = R2^H Q2^H: R and B = R2^H share their left
        // singular vectors; one-sided Jacobi converges in far fewer sweeps
        // on the lower-triangular B than on R itself
        tsqr(ctx, m, k, V, m, Q, R, db, lvl);
        zc* Q2 = (zc*)ctx->get_ws("p2_q2", sizeof(zc) * (size_t)k * k);
        zc* R2 = (zc*)ctx->get_ws("p2_r2", sizeof(zc) * (size_t)k * k);
        tsqr_lq(ctx, k, k, R, k, Q2, R2, db, lvl);
        conj_transpose(ctx, R2, k, B, k, k, k);
      } else {
        // V^H (k x m) = Q' R' ; SVD of R'^H gives the left vectors of V
        tsqr_lq(ctx, m, k, V, m, Q, R, db, lvl);
        conj_transpose(ctx, R, m, B, m, m, m);  // B = R'^H
      }
      jacobi_svd(ctx, sq, sq, B, U, sig, sw);
    };
    double* h = (double*)ctx->host_scratch(sizeof(double) * (sq + 8));
    factor(true);
    TTF_HIP(hipMemcpyAsync(h, sig, sizeof(double) * (sq + 8), hipMemcpyDeviceToHost, ctx->stream));
    TTF_HIP(hipStreamSynchronize(ctx->stream));
    int qb = 0;
    std::memcpy(&qb, (char*)(h + sq + 4), sizeof(int));
    if (qb) {
      ctx->qr_fallbacks += 1;
      factor(false);
      TTF_HIP(hipMemcpyAsync(h, sig, sizeof(double) * (sq + 8), hipMemcpyDeviceToHost, ctx->stream));
      TTF_HIP(hipStreamSynchronize(ctx->stream));
    }
    std::vector<double> s(h, h + sq);
    for (double v : s)
      if (!std::isfinite(v)) fail(TT_ENONFINITE, "non-finite singular value in tt_round");
    int swp = 0;
    std::memcpy(&swp, (char*)(h + sq + 2), sizeof(int));
    // an SVD stopped at its sweep limit leaves U unorthogonal: no truncation
    // may be taken from it
    require(swp > 0, TT_ENOCONV, "tt_round: Jacobi SVD did not converge within its sweep limit");
    sweeps_max = std::max(sweeps_max, swp);
    int capk = x->cap[c + 1];
    const int cb = caps ? caps[c + 1] : rmax;
    if (cb > 0) capk = std::min(capk, cb);
    double tail = 0;
    const int kk = truncation_rank(s, delta, capk, &tail);
    if (m >= k) {
      // C_c <- Q U_k ; carry = U_k^H R
      zgemm(ctx, OPN, OPN, m, kk, k, Z(1), Q, m, 0, U, k, 0, Z(0), x->core[c], m, 0);
      zgemm(ctx, OPC, OPN, kk, k, k, Z(1), U, k, 0, R, k, 0, Z(0), carry, kk, 0);
    } else {
      // C_c <- U_k ; carry = U_k^H V
      zgemm(ctx, OPC, OPN, kk, k, m, Z(1), U, m, 0, V, m, 0, Z(0), carry, kk, 0);
      copy_d2d(ctx, x->core[c], U, (size_t)m * kk);
    }
    // C_{c+1} <- carry H(C_{c+1})
    zgemm(ctx, OPN, OPN, kk, n1 * rr, k, Z(1), carry, kk, 0, x->core[c + 1], k, 0, Z(0), tmp, kk, 0);
    copy_d2d(ctx, x->core[c + 1], tmp, (size_t)kk * n1 * rr);
    r[c + 1] = kk;
    if (rep) {
      rep->tail[c] = tail;
      rep->sigma_min_kept[c] = s[kk - 1];
      rep->sigma_first_cut[c] = kk < sq ? s[kk] : 0.0;
      for (int j = 0; j < 8; ++j) {
        const int idx = kk - 8 + j;
        rep->sv_last[c][j] = idx >= 0 ? s[idx] : 0.0;
      }
    }
  }
  x->orth = TT_ORTH_LEFT;
  if (rep) {
    for (int c = 0; c <= d; ++c) rep->ranks[c] = r[c];
    rep->norm = norm;
    rep->jacobi_sweeps_max = sweeps_max;
  }
}

// --------------------------------------------------------- operator apply
void check_same_shape(const tt_op* op, const tt_tensor* x) {
  require(op->d == x->d && op->n == x->n, TT_ESHAPE, "operator and tensor shapes differ");
  require(x->dtype == TT_C128, TT_EINVAL, "internal: operator calls need complex-double storage");
}

void apply_exact(tt_ctx* ctx, const tt_op* op, const tt_tensor* x, tt_tensor* y) {
  const int d = x->d;
  for (int k = 0; k <= d; ++k)
    require((long)op->R[k] * x->rank[k] <= y->cap[k], TT_ECAPACITY, "tt_apply: output capacity too small");
  for (int k = 0; k < d; ++k) apply_exact_core(ctx, op, k, x->core[k], x->rank[k], x->rank[k + 1], y->core[k]);
  for (int k = 0; k <= d; ++k) y->rank[k] = op->R[k] * x->rank[k];
  y->orth = TT_ORTH_NONE;
}

// Sketched operator application: y = the projection of L x onto bases found
// by a randomised range finder in TT form.  Pass 0 draws Gaussian TT
// sketches and contracts them with the left parts of L x (left chains S_m);
// pass 1 sweeps right to left: at site m the contraction M = S_m Z_m of the
// left chain with the right part of L x (already projected onto the bases
// found to its right) is factored by LQ, whose orthonormal rows are the new
// right-orthonormal core, and the right chain P_m = Z_m Q carries the
// projection one site on.  Each of the `power` further passes sweeps the
// other way with the previous pass's chains in place of the sketch (a
// subspace-iteration step: the bases of a bond become the range of L x
// restricted to the other side's bases).  For an odd count the sketches
// are drawn from the right instead (right chains, first pass left to
// right), so that the last pass always runs right to left and y ends
// right-orthonormal.  Exact whenever the widths reach the ranks of L x.
void apply_sketch(tt_ctx* ctx, const tt_op* op, const tt_tensor* x, tt_tensor* y, int l, uint64_t seed,
                  int precision, const int* widths = nullptr, int power = 0) {
  // the sketch contractions in plain FP64 or a split 16-bit form (mixed).
  // With power passes the last pass, the projection whose result the
  // truncation takes, is FP64: its arithmetic error enters the projection
  // itself, which cap-limited cuts amplify (split-FP16x3 there puts stage
  // outputs 2e-5 from FP64 at d = 50), while the earlier passes only find
  // the bases (with them in split-FP16x3, 4e-8)
  int prec = precision;
  auto gemm = [ctx, &prec](tt_ctx*, int opA, int opB, int M, int N, int K, zc alpha, const zc* A, long lda, long sA,
                           const zc* B, long ldb, long sB, zc beta, zc* C, long ldc, long sC, int batch) {
    zgemm_prec(prec, ctx, opA, opB, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch);
  };
  const int d = x->d, n = x->n;
  const auto& r = x->rank;
  const auto& R = op->R;
  require(l >= 1, TT_EINVAL, "tt_apply: sketch rank must be >= 1");
  require(power >= 0 && power <= 8, TT_EINVAL, "tt_apply: power passes must be 0..8");
  std::vector<int> ll(d + 1);
  // sketch width per bond (uniform l, or the given widths)
  for (int m = 0; m <= d; ++m) {
    const int w = widths ? std::max(1, widths[m]) : l;
    ll[m] = std::min(bounded_pow(n, m, w), bounded_pow(n, d - m, w));
  }
  for (int m = 0; m <= d; ++m) require(ll[m] <= y->cap[m], TT_ECAPACITY, "tt_apply: output capacity below sketch rank");
  if (d == 1) {
    apply_exact_core(ctx, op, 0, x->core[0], 1, 1, y->core[0]);
    y->rank[0] = y->rank[1] = 1;
    y->orth = TT_ORTH_NONE;
    return;
  }
  // workspace sizes
  size_t big0 = 0, big1 = 0, sk_total = 0, p_total = 0, om = 0;
  std::vector<size_t> sk_off(d + 1, 0), p_off(d + 1, 0);
  for (int m = 0; m < d; ++m) {
    big0 = std::max(big0, (size_t)ll[m] * R[m] * n * r[m + 1]);          // V
    big1 = std::max(big1, (size_t)ll[m] * n * r[m + 1] * R[m + 1]);      // W
    big0 = std::max(big0, (size_t)r[m] * n * R[m + 1] * ll[m + 1]);      // V2
    big1 = std::max(big1, (size_t)r[m] * R[m] * n * ll[m + 1]);          // Z
    om = std::max(om, (size_t)ll[m] * n * ll[m + 1]);
  }
  for (int m = 0; m <= d; ++m) {
    sk_off[m] = sk_total;
    sk_total += (size_t)ll[m] * r[m] * R[m];
    p_off[m] = p_total;
    p_total += (size_t)r[m] * R[m] * ll[m];
  }
  zc* V = (zc*)ctx->get_ws("sk_big0", sizeof(zc) * big0);
  zc* W = (zc*)ctx->get_ws("sk_big1", sizeof(zc) * big1);
  zc* S = (zc*)ctx->get_ws("sk_S", sizeof(zc) * sk_total);   // left chains
  zc* P = (zc*)ctx->get_ws("sk_P", sizeof(zc) * p_total);    // right chains
  zc* omega = (zc*)ctx->get_ws("sk_omega", sizeof(zc) * om);
  size_t mmax = 0;
  for (int m = 0; m < d; ++m) mmax = std::max(mmax, (size_t)ll[m] * n * ll[m + 1]);
  zc* M = (zc*)ctx->get_ws("sk_M", sizeof(zc) * std::max<size_t>(mmax, 1));
  zc* Qm = (zc*)ctx->get_ws("sk_Q", sizeof(zc) * std::max<size_t>(mmax, 1));
  int lmax = 1;
  for (int m = 0; m <= d; ++m) lmax = std::max(lmax, ll[m]);
  zc* Rm = (zc*)ctx->get_ws("sk_R", sizeof(zc) * (size_t)lmax * lmax);
  // power-of-two scales of the chains: [0] current exponent, [1] the sum of
  // the exponents taken out of the chain that carries the projection
  // (restored in the pass's last core); [8] the deferred flag of the fast QR
  // form, read once after the whole application
  int* pexp = (int*)ctx->get_ws("sk_pow2", 64);
  int* qr_flag = pexp + 8;
  const int qr_level = 0;
  const zc one = Z(1);
  // ---- pass 0: Gaussian left sketches S_{m+1} = omega_m^T (Y_m contracted with S_m), S_0 = 1
  auto sketch_pass = [&]() {
    TTF_HIP(hipMemcpyAsync(S + sk_off[0], &one, sizeof(zc), hipMemcpyHostToDevice, ctx->stream));
    for (int m = 0; m + 1 < d; ++m) {
      const int lm = ll[m], lp = ll[m + 1], r0 = r[m], r1 = r[m + 1], R0 = R[m], R1 = R[m + 1];
      const zc* Sm = S + sk_off[m];
      // V[j, alpha, i', b] = sum_a S_m[j, a, alpha] C_m[a, i', b]  (batched over alpha)
      gemm(ctx, OPN, OPN, lm, n * r1, r0, Z(1), Sm, lm, (long)lm * r0, x->core[m], r0, 0, Z(0), V, (long)lm * R0,
            lm, R0);
      gather_left(ctx, op, m, V, W, lm, r1);
      sketch_core(ctx, omega, (long)lm * n * lp, seed, m, 1.0 / std::sqrt((double)lp));
      gemm(ctx, OPT, OPN, lp, r1 * R1, lm * n, Z(1), omega, (long)lm * n, 0, W, (long)lm * n, 0, Z(0),
            S + sk_off[m + 1], lp, 0, 1);
      // the range found does not depend on the scale of S
      pow2_normalize(ctx, S + sk_off[m + 1], (long)lp * r1 * R1, pexp, false);
    }
  };
  // ---- Gaussian right sketches P_m = (Z_m contracted with P_{m+1}) omega_m,
  // P_d = 1 (the mirror of pass 0, for an odd number of power passes)
  auto right_sketch_pass = [&]() {
    TTF_HIP(hipMemcpyAsync(P + p_off[d], &one, sizeof(zc), hipMemcpyHostToDevice, ctx->stream));
    int sp = 1;
    for (int m = d - 1; m >= 1; --m) {
      const int r0 = r[m], r1 = r[m + 1], R0 = R[m], R1 = R[m + 1];
      gemm(ctx, OPN, OPN, r0 * n, R1 * sp, r1, Z(1), x->core[m], (long)r0 * n, 0, P + p_off[m + 1], r1, 0, Z(0),
           V, (long)r0 * n, 0, 1);
      gather_right(ctx, op, m, V, W, r0, sp);  // Z: (r0 R0) x (n s_{m+1})
      const int lm = ll[m];
      sketch_core(ctx, omega, (long)n * sp * lm, seed ^ 0x5851F42D4C957F2Dull, m, 1.0 / std::sqrt((double)lm));
      gemm(ctx, OPN, OPN, r0 * R0, lm, n * sp, Z(1), W, (long)r0 * R0, 0, omega, (long)n * sp, 0, Z(0),
           P + p_off[m], (long)r0 * R0, 0, 1);
      pow2_normalize(ctx, P + p_off[m], (long)r0 * R0 * lm, pexp, false);
      sp = lm;
    }
  };
  // ---- right-to-left pass with the left chains S: right-orthonormal y and
  // the right chains P_m = Z_m Q_m ((r_m R_m) x l_m, layout [a, alpha, q])
  auto right_to_left = [&]() {
    zero_ints(ctx, pexp, 2);
    TTF_HIP(hipMemcpyAsync(P + p_off[d], &one, sizeof(zc), hipMemcpyHostToDevice, ctx->stream));
    int sp = 1;
    for (int m = d - 1; m >= 0; --m) {
      const int r0 = r[m], r1 = r[m + 1], R0 = R[m], R1 = R[m + 1];
      // V2[a, i', beta, q] = V(C_m) P_{m+1}
      gemm(ctx, OPN, OPN, r0 * n, R1 * sp, r1, Z(1), x->core[m], (long)r0 * n, 0, P + p_off[m + 1], r1, 0, Z(0),
            V, (long)r0 * n, 0, 1);
      if (m == 0) {
        gather_right(ctx, op, 0, V, y->core[0], 1, sp);
        pow2_restore(ctx, y->core[0], (long)n * sp, pexp);
        break;
      }
      gather_right(ctx, op, m, V, W, r0, sp);  // Z in W
      const int lm = ll[m];
      const int N = n * sp;
      // M = S_m Z  (l_m x n s_{m+1})
      gemm(ctx, OPN, OPN, lm, N, r0 * R0, Z(1), S + sk_off[m], lm, 0, W, (long)r0 * R0, 0, Z(0), M, lm, 0, 1);
      // M = R^H Qt^H: the new core is Qt^H (right-orthonormal rows)
      tsqr_lq(ctx, lm, N, M, lm, Qm, Rm, qr_flag, qr_level);
      conj_transpose(ctx, Qm, N, y->core[m], lm, N, lm);
      y->rank[m] = lm;
      // P_m = Z Q^H = Z Qt  ((r0 R0) x l_m)
      gemm(ctx, OPN, OPN, r0 * R0, lm, N, Z(1), W, (long)r0 * R0, 0, Qm, N, 0, Z(0), P + p_off[m], (long)r0 * R0, 0,
            1);
      pow2_normalize(ctx, P + p_off[m], (long)r0 * R0 * lm, pexp, true);
      sp = lm;
    }
    y->rank[0] = y->rank[d] = 1;
    y->orth = TT_ORTH_RIGHT;
  };
  // ---- left-to-right pass with the right chains P: left-orthonormal y and
  // the left chains S_{m+1} = U_m^H W_m (layout [j, a, alpha], as the sketch's)
  auto left_to_right = [&]() {
    zero_ints(ctx, pexp, 2);
    TTF_HIP(hipMemcpyAsync(S + sk_off[0], &one, sizeof(zc), hipMemcpyHostToDevice, ctx->stream));
    int sm = 1;
    for (int m = 0; m < d; ++m) {
      const int r0 = r[m], r1 = r[m + 1], R0 = R[m], R1 = R[m + 1];
      gemm(ctx, OPN, OPN, sm, n * r1, r0, Z(1), S + sk_off[m], sm, (long)sm * r0, x->core[m], r0, 0, Z(0), V,
            (long)sm * R0, sm, R0);
      if (m == d - 1) {
        gather_left(ctx, op, m, V, y->core[m], sm, 1);
        pow2_restore(ctx, y->core[m], (long)sm * n, pexp);
        break;
      }
      gather_left(ctx, op, m, V, W, sm, r1);  // W: (s_m n) x (r1 R1)
      const int lp = ll[m + 1];
      const int rows = sm * n;
      // M = W P_{m+1}  ((s_m n) x l_{m+1}); M = U R, U the new left-orthonormal core
      gemm(ctx, OPN, OPN, rows, lp, r1 * R1, Z(1), W, rows, 0, P + p_off[m + 1], (long)r1 * R1, 0, Z(0), M, rows, 0,
            1);
      tsqr(ctx, rows, lp, M, rows, y->core[m], Rm, qr_flag, qr_level);
      y->rank[m + 1] = lp;
      // S_{m+1} = U^H W  (l_{m+1} x (r1 R1))
      gemm(ctx, OPC, OPN, lp, r1 * R1, rows, Z(1), y->core[m], rows, 0, W, rows, 0, Z(0), S + sk_off[m + 1], lp, 0,
            1);
      pow2_normalize(ctx, S + sk_off[m + 1], (long)lp * r1 * R1, pexp, true);
      sm = lp;
    }
    y->rank[0] = y->rank[d] = 1;
    y->orth = TT_ORTH_LEFT;
  };
  // the factorisations of every sweep take the fast form with one deferred
  // check; when it was unsafe for some panel, the sweeps run again with
  // every factorisation checked (and redone robustly) on its own
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (attempt == 0) zero_ints(ctx, qr_flag, 1);
    else qr_flag = nullptr;  // every factorisation checked on its own
    // the passes alternate and the last one runs right to left (y right-
    // orthonormal, so a rounding of y skips its orthogonalisation sweep):
    // an even count of power passes starts from left sketches, an odd one
    // from right sketches
    prec = precision;
    const bool from_right = (power & 1) != 0;
    if (from_right)
      right_sketch_pass();
    else
      sketch_pass();
    for (int p = 0; p <= power; ++p) {
      // reduced precision in the Gaussian pass, and with
      // TT_OPT_SKETCH_MIXED_PASSES 1 in every power pass but the last; the
      // last pass (the projection itself) always in the requested
      // precision when there are no power passes, else FP64
      prec = (power == 0 || (ctx->sketch_mixed_passes && p < power)) ? precision : TT_PREC_FP64;
      if (((p & 1) != 0) != from_right)
        left_to_right();
      else
        right_to_left();
    }
    if (attempt == 1) break;
    int* h = (int*)ctx->host_scratch(64);
    TTF_HIP(hipMemcpyAsync(h, qr_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    TTF_HIP(hipStreamSynchronize(ctx->stream));
    if (h[0] == 0) break;
    ctx->qr_fallbacks += 1;
  }
}

void apply_any(tt_ctx* ctx, const tt_op* op, const tt_tensor* x, tt_tensor* y, int mode, int l, uint64_t seed,
               int precision, int power = 0) {
  require(precision == TT_PREC_FP64 || precision == TT_PREC_BF16X3 || precision == TT_PREC_FP16X3 ||
              precision == TT_PREC_FP32,
          TT_EINVAL,
          "tt_apply: unknown precision");
  check_same_shape(op, x);
  require(x->d == y->d && x->n == y->n, TT_ESHAPE, "tt_apply: x and y shapes differ");
  require(x != y, TT_EINVAL, "tt_apply: y must not alias x");
  require(op->ctx == ctx, TT_EINVAL, "tt_apply: operator was created on another context");
  if (mode == TT_APPLY_EXACT)
    apply_exact(ctx, op, x, y);
  else if (mode == TT_APPLY_SKETCH)
    apply_sketch(ctx, op, x, y, l, seed, precision, nullptr, power);
  else
    fail(TT_EINVAL, "tt_apply: unknown mode");
}

// ------------------------------------------------------------------ sums
void sum_tensors(tt_ctx* ctx, int nterms, const zc* coef, const tt_tensor* const* xs, tt_tensor* z) {
  require(nterms >= 1 && nterms <= 8, TT_EINVAL, "tt_sum: 1..8 terms supported");
  const int d = z->d;
  require(z->dtype == TT_C128, TT_EINVAL, "internal: sums need complex-double storage");
  std::vector<int> rk(d + 1, 0);
  for (int t = 0; t < nterms; ++t) {
    require(xs[t] && xs[t]->d == d && xs[t]->nk == z->nk, TT_ESHAPE, "tt_sum: shape mismatch");
    require(xs[t]->dtype == TT_C128, TT_EINVAL, "internal: sums need complex-double storage");
    require(xs[t] != z, TT_EINVAL, "tt_sum: output aliases an input");
  }
  rk[0] = rk[d] = 1;
  for (int k = 1; k < d; ++k) {
    for (int t = 0; t < nterms; ++t) rk[k] += xs[t]->rank[k];
    require(rk[k] <= z->cap[k], TT_ECAPACITY, "tt_sum: output capacity too small");
  }
  std::vector<const zc*> src(nterms);
  std::vector<int> r0s(nterms), r1s(nterms);
  for (int k = 0; k < d; ++k) {
    for (int t = 0; t < nterms; ++t) {
      src[t] = xs[t]->core[k];
      r0s[t] = xs[t]->rank[k];
      r1s[t] = xs[t]->rank[k + 1];
    }
    const int kind = (d == 1) ? 3 : (k == 0 ? 0 : (k == d - 1 ? 2 : 1));
    concat_core(ctx, nterms, src.data(), r0s.data(), r1s.data(), coef, kind, z->nk[k], z->core[k], rk[k], rk[k + 1]);
  }
  z->rank = rk;
  z->orth = TT_ORTH_NONE;
}

tt_tensor* make_tensor_nk(tt_ctx* ctx, int d, const std::vector<int>& nk, const std::vector<int>& cap,
                          int dtype = TT_C128) {
  require(d >= 1 && d <= TT_MAX_D, TT_EINVAL, "tensor dimension must be in 1..128");
  require((int)nk.size() == d, TT_EINVAL, "one mode size per mode");
  for (int v : nk) require(v >= 4, TT_EINVAL, "mode size must be at least 4");
  require(dtype == TT_C128 || dtype == TT_C64, TT_EINVAL, "unknown storage type");
  require((int)cap.size() == d + 1 && cap[0] == 1 && cap[d] == 1, TT_EINVAL, "rank capacities must start and end with 1");
  for (int c : cap) require(c >= 1, TT_EINVAL, "rank capacities must be positive");
  tt_tensor* t = new tt_tensor;
  t->ctx = ctx;
  t->release = ctx->releaser();
  t->d = d;
  t->nk = nk;
  t->n = nk[0];
  for (int v : nk)
    if (v != nk[0]) t->n = 0;
  t->dtype = dtype;
  t->cap = cap;
  t->rank.assign(d + 1, 1);
  t->core.assign(d, nullptr);
  for (int k = 0; k < d; ++k) {
    // whole complex doubles (a complex-float core of odd length gets one
    // spare entry), so the clear below stays inside the block
    const size_t bytes = (t->esize() * t->cap_elems(k) + sizeof(zc) - 1) / sizeof(zc) * sizeof(zc);
    t->core[k] = (zc*)ctx->dev_alloc(bytes);
    if (!t->core[k]) {
      for (int j = 0; j < k; ++j) ctx->dev_free(t->core[j]);
      delete t;
      fail(TT_ENOMEM, "tensor core allocation failed");
    }
    fill_zero(ctx, t->core[k], (long)(bytes / sizeof(zc)));
  }
  return t;
}

tt_tensor* make_tensor(tt_ctx* ctx, int d, int n, const std::vector<int>& cap) {
  return make_tensor_nk(ctx, d, std::vector<int>(std::max(d, 0), n), cap);
}

void free_tensor(tt_tensor* t) {
  if (!t) return;
  for (auto p : t->core) t->release(p);
  delete t;
}

void copy_tensor(tt_ctx* ctx, const tt_tensor* src, tt_tensor* dst) {
  require(src->d == dst->d && src->nk == dst->nk, TT_ESHAPE, "tt_tensor_copy: shape mismatch");
  for (int k = 0; k <= src->d; ++k) require(src->rank[k] <= dst->cap[k], TT_ECAPACITY, "tt_tensor_copy: capacity too small");
  if (src == dst) return;
  for (int k = 0; k < src->d; ++k) {
    const long e = (long)src->elems(k);
    if (src->dtype == dst->dtype) {
      if (e > 0 && dst->core[k] != src->core[k])
        TTF_HIP(hipMemcpyAsync(dst->core[k], src->core[k], src->esize() * e, hipMemcpyDeviceToDevice, ctx->stream));
    } else if (src->dtype == TT_C64) {
      widen_c64(ctx, src->core[k], dst->core[k], e);
    } else {
      narrow_c128(ctx, src->core[k], dst->core[k], e);
    }
  }
  dst->rank = src->rank;
  dst->orth = src->orth;
}

// temporaries used by tt_step / tt_norm, cached per context and shape
struct StepTemps {
  tt_tensor* k[4] = {nullptr, nullptr, nullptr, nullptr};
  tt_tensor* ysum = nullptr;
  tt_tensor* y = nullptr;
  tt_tensor* fsum = nullptr;
};
// the temporaries caches are shared by every context; contexts may step on
// different host threads (tt_step_batch), so lookups and inserts are
// serialised (map references stay valid across inserts)
std::mutex& cache_mutex() {
  static std::mutex m;
  return m;
}

std::map<std::pair<tt_ctx*, std::string>, StepTemps>& step_cache() {
  static std::map<std::pair<tt_ctx*, std::string>, StepTemps> c;
  return c;
}
std::map<std::pair<tt_ctx*, std::string>, tt_tensor*>& norm_cache() {
  static std::map<std::pair<tt_ctx*, std::string>, tt_tensor*> c;
  return c;
}

std::string shape_key(int d, int n, const std::vector<int>& cap, int extra) {
  std::string s = std::to_string(d) + ":" + std::to_string(n) + ":" + std::to_string(extra);
  for (int c : cap) s += "," + std::to_string(c);
  return s;
}

// named temporaries (TT-GMRES and friends), reused while their capacities
// suffice
std::map<std::pair<tt_ctx*, std::string>, tt_tensor*>& pool_cache() {
  static std::map<std::pair<tt_ctx*, std::string>, tt_tensor*> c;
  return c;
}

tt_tensor* pooled_nk(tt_ctx* ctx, const std::string& name, int d, const std::vector<int>& nk,
                     const std::vector<int>& cap, int dtype = TT_C128) {
  tt_tensor*& t = [&]() -> tt_tensor*& {
    std::lock_guard<std::mutex> lock(cache_mutex());
    return pool_cache()[{ctx, name}];
  }();
  bool ok = t && t->d == d && t->nk == nk && t->dtype == dtype;
  for (int k = 0; ok && k <= d; ++k) ok = t->cap[k] >= cap[k];
  if (!ok) {
    if (t) {
      TTF_HIP(hipStreamSynchronize(ctx->stream));
      free_tensor(t);
    }
    t = nullptr;
    t = make_tensor_nk(ctx, d, nk, cap, dtype);
  }
  return t;
}

tt_tensor* pooled(tt_ctx* ctx, const std::string& name, int d, int n, const std::vector<int>& cap) {
  return pooled_nk(ctx, name, d, std::vector<int>(d, n), cap);
}

// A complex-double working copy of a C64 tensor for the length of one call
// (the tensor itself when it is stored as complex double); `load` copies
// its content in.  `narrow_back` stores a working copy's result into the
// C64 tensor it stands for.
tt_tensor* widened(tt_ctx* ctx, const tt_tensor* x, const char* slot, bool load = true) {
  if (x->dtype == TT_C128) return const_cast<tt_tensor*>(x);
  tt_tensor* w = pooled_nk(ctx, std::string("c64:") + slot, x->d, x->nk, x->cap);
  if (load) {
    copy_tensor(ctx, x, w);
    w->rank = x->rank;
    w->orth = x->orth;
  }
  return w;
}

void narrow_back(tt_ctx* ctx, const tt_tensor* w, tt_tensor* x) {
  if (w == x) return;
  copy_tensor(ctx, w, x);
  x->rank = w->rank;
  x->orth = w->orth;
}

// identity operators (randomised rounding), built once per context and shape
std::map<std::tuple<tt_ctx*, int, int>, tt_op*>& identity_ops() {
  static std::map<std::tuple<tt_ctx*, int, int>, tt_op*> c;
  return c;
}

void free_op(tt_op* op);

void drop_ctx_caches(tt_ctx* ctx) {
  std::lock_guard<std::mutex> lock(cache_mutex());
  {
    auto& io = identity_ops();
    for (auto it = io.begin(); it != io.end();) {
      if (std::get<0>(it->first) == ctx) {
        free_op(it->second);
        it = io.erase(it);
      } else {
        ++it;
      }
    }
  }
  auto& pc = pool_cache();
  for (auto it = pc.begin(); it != pc.end();) {
    if (it->first.first == ctx) {
      free_tensor(it->second);
      it = pc.erase(it);
    } else {
      ++it;
    }
  }
  auto& sc = step_cache();
  for (auto it = sc.begin(); it != sc.end();) {
    if (it->first.first == ctx) {
      for (auto* t : it->second.k) free_tensor(t);
      free_tensor(it->second.ysum);
      free_tensor(it->second.y);
      free_tensor(it->second.fsum);
      it = sc.erase(it);
    } else {
      ++it;
    }
  }
  auto& nc = norm_cache();
  for (auto it = nc.begin(); it != nc.end();) {
    if (it->first.first == ctx) {
      free_tensor(it->second);
      it = nc.erase(it);
    } else {
      ++it;
    }
  }
}

void upload_op(tt_ctx* ctx, tt_op* op) {
  const int d = op->d, n = op->n;
  op->ctx = ctx;
  op->release = ctx->releaser();
  auto dalloc = [ctx](void** dst, size_t bytes) {
    *dst = ctx->dev_alloc(bytes);
    if (!*dst) fail(TT_ENOMEM, "operator upload: device allocation failed");
  };
  dalloc((void**)&op->d_tap_ptr, sizeof(int) * op->tap_ptr.size());
  dalloc((void**)&op->d_tap_col, sizeof(int) * std::max<size_t>(1, op->tap_col.size()));
  dalloc((void**)&op->d_tap_w, sizeof(double) * std::max<size_t>(1, op->tap_w.size()));
  TTF_HIP(hipMemcpy(op->d_tap_ptr, op->tap_ptr.data(), sizeof(int) * op->tap_ptr.size(), hipMemcpyHostToDevice));
  TTF_HIP(hipMemcpy(op->d_tap_col, op->tap_col.data(), sizeof(int) * op->tap_col.size(), hipMemcpyHostToDevice));
  TTF_HIP(hipMemcpy(op->d_tap_w, op->tap_w.data(), sizeof(double) * op->tap_w.size(), hipMemcpyHostToDevice));
  (void)n;
  op->dev.assign(d, {});
  for (int s = 0; s < d; ++s) {
    const auto& ent = op->site[s];
    const int R0 = op->R[s], R1 = op->R[s + 1];
    // CSR by beta (incoming) and by alpha (outgoing)
    std::vector<int> inp(R1 + 1, 0), outp(R0 + 1, 0);
    for (const Entry& e : ent) {
      inp[e.beta + 1]++;
      outp[e.alpha + 1]++;
    }
    for (int i = 0; i < R1; ++i) inp[i + 1] += inp[i];
    for (int i = 0; i < R0; ++i) outp[i + 1] += outp[i];
    std::vector<DevEntry> ine(ent.size()), oute(ent.size());
    std::vector<int> fi(inp.begin(), inp.end() - 1), fo(outp.begin(), outp.end() - 1);
    for (const Entry& e : ent) {
      ine[fi[e.beta]++] = DevEntry{e.alpha, e.lop, e.cre, e.cim};
      oute[fo[e.alpha]++] = DevEntry{e.beta, e.lop, e.cre, e.cim};
    }
    // exact-apply blocks
    std::map<std::pair<int, int>, std::vector<DevBlockOp>> blk;
    for (const Entry& e : ent) blk[{e.alpha, e.beta}].push_back(DevBlockOp{e.lop, 0, e.cre, e.cim});
    std::vector<DevBlock> blocks;
    std::vector<DevBlockOp> bops;
    for (auto& kv : blk) {
      blocks.push_back(DevBlock{kv.first.first, kv.first.second, (int)bops.size(), (int)kv.second.size()});
      for (auto& b : kv.second) bops.push_back(b);
    }
    auto& sd = op->dev[s];
    sd.nblocks = (int)blocks.size();
    auto up = [&](void** dst, const void* src, size_t bytes) {
      dalloc(dst, std::max<size_t>(bytes, 16));
      if (bytes) TTF_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    };
    up((void**)&sd.in_ptr, inp.data(), sizeof(int) * inp.size());
    up((void**)&sd.out_ptr, outp.data(), sizeof(int) * outp.size());
    up((void**)&sd.in_ent, ine.data(), sizeof(DevEntry) * ine.size());
    up((void**)&sd.out_ent, oute.data(), sizeof(DevEntry) * oute.size());
    up((void**)&sd.blocks, blocks.data(), sizeof(DevBlock) * blocks.size());
    up((void**)&sd.bops, bops.data(), sizeof(DevBlockOp) * bops.size());
  }
}

void free_op(tt_op* op) {
  if (!op) return;
  if (op->ctx) {
    const ttf::DevFree& f = op->release;
    f(op->d_tap_ptr);
    f(op->d_tap_col);
    f(op->d_tap_w);
    for (auto& sd : op->dev) {
      f(sd.in_ptr);
      f(sd.out_ptr);
      f(sd.in_ent);
      f(sd.out_ent);
      f(sd.blocks);
      f(sd.bops);
    }
  }
  delete op;
}

}  // namespace

// =================================================================== ABI
extern "C" {

int tt_ctx_create(int device, void* hip_stream, const tt_allocator* alloc, tt_ctx** out) {
  tt_ctx* ctx = nullptr;
  ABI_TRY
  require(out != nullptr, TT_EINVAL, "tt_ctx_create: out is NULL");
  *out = nullptr;
  require(!alloc || (alloc->alloc && alloc->free), TT_EINVAL, "tt_ctx_create: allocator without alloc or free");
  int ndev = 0;
  TTF_HIP(hipGetDeviceCount(&ndev));
  require(device >= 0 && device < ndev, TT_EINVAL, "tt_ctx_create: no such device");
  TTF_HIP(hipSetDevice(device));
  noalloc_scratch_init(device);
  ctx = new tt_ctx;
  ctx->device = device;
  if (alloc) {
    ctx->allocator = *alloc;
    ctx->has_allocator = true;
  }
  if (hip_stream) {
    ctx->stream = (hipStream_t)hip_stream;
  } else {
    TTF_HIP(hipStreamCreate(&ctx->stream));
    ctx->own_stream = true;
  }
  *out = ctx;
  return TT_OK;
  }
  catch (const ttf::Error& e) {
    delete ctx;
    return e.code;
  }
  catch (...) {
    delete ctx;
    return TT_EINVAL;
  }
}

int tt_ctx_destroy(tt_ctx* ctx) {
  if (!ctx) return TT_EINVAL;
  (void)hipStreamSynchronize(ctx->stream);
  drop_ctx_caches(ctx);
  for (auto& kv : ctx->ws) ctx->dev_free(kv.second.p);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  for (auto& p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : ctx->free_events) (void)hipEventDestroy(e);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return TT_OK;
}

int tt_ctx_sync(tt_ctx* ctx) {
  if (!ctx) return TT_EINVAL;
  ABI_TRY
  ctx->sync();
  return TT_OK;
  ABI_CATCH(ctx)
}

const char* tt_last_error(const tt_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

void* tt_ctx_stream(const tt_ctx* ctx) { return ctx ? (void*)ctx->stream : nullptr; }

int tt_ctx_set_profiling(tt_ctx* ctx, int on) {
  if (!ctx) return TT_EINVAL;
  ABI_TRY
  ctx->sync();
  ctx->profiling = on != 0;
  ctx->profile_shapes = on == 2;
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_ctx_set_profile_filter(tt_ctx* ctx, const char* kernel) {
  if (!ctx) return TT_EINVAL;
  ABI_TRY
  ctx->sync();
  ctx->profile_only = kernel ? kernel : "";
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_ctx_set_profile_sampling(tt_ctx* ctx, int every) {
  if (!ctx || every < 1) return TT_EINVAL;
  ABI_TRY
  ctx->sync();
  ctx->profile_every = every;
  ctx->profile_seen = 0;
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_ctx_set_option(tt_ctx* ctx, int option, long long value) {
  if (!ctx) return TT_EINVAL;
  ABI_TRY
  if (option == TT_OPT_QR_MIN_LEVEL) {
    require(value >= 0 && value <= 2, TT_EINVAL, "tt_ctx_set_option: QR level must be 0..2");
    ctx->qr_min_level = (int)value;
    return TT_OK;
  }
  if (option == TT_OPT_JACOBI_MAX_SWEEPS) {
    require(value >= 1 && value <= 60, TT_EINVAL, "tt_ctx_set_option: Jacobi sweep limit must be 1..60");
    ctx->jacobi_max_sweeps = (int)value;
    return TT_OK;
  }
  if (option == TT_OPT_SKETCH_MIXED_PASSES) {
    require(value == 0 || value == 1, TT_EINVAL, "tt_ctx_set_option: the mixed-passes switch is 0 or 1");
    ctx->sketch_mixed_passes = (int)value;
    return TT_OK;
  }
  if (option == TT_OPT_QR_WIDE_PANELS) {
    require(value == 0 || value == 1, TT_EINVAL, "tt_ctx_set_option: the wide-panel switch is 0 or 1");
    ctx->qr_wide = (int)value;
    return TT_OK;
  }
  if (option == TT_OPT_JACOBI_FUSED) {
    require(value == 0 || value == 1, TT_EINVAL, "tt_ctx_set_option: the fused Jacobi switch is 0 or 1");
    ctx->jacobi_fused = (int)value;
    return TT_OK;
  }
  if (option == TT_OPT_JACOBI_WAIT_LIMIT) {
    require(value >= 0 && value <= (1LL << 40), TT_EINVAL, "tt_ctx_set_option: wait limit must be 0..2^40");
    ctx->jacobi_wait_limit = (long)value;
    return TT_OK;
  }
  fail(TT_EINVAL, "tt_ctx_set_option: unknown option");
  ABI_CATCH(ctx)
}

int tt_ctx_reset_stats(tt_ctx* ctx) {
  if (!ctx) return TT_EINVAL;
  ABI_TRY
  ctx->sync();
  ctx->stats.clear();
  ctx->qr_fallbacks = 0;
  ctx->jacobi_svds = ctx->jacobi_sweeps_launched = ctx->jacobi_sweeps_needed = ctx->jacobi_check_passed = 0;
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_ctx_get_stats(tt_ctx* ctx, const char* kernel, double* total_ms, double* flops, double* bytes,
                     long long* launches) {
  if (!ctx || !kernel) return TT_EINVAL;
  ABI_TRY
  ctx->sync();
  auto it = ctx->stats.find(kernel);
  tt_ctx::Stat s;
  if (it != ctx->stats.end()) s = it->second;
  if (total_ms) *total_ms = s.ms;
  if (flops) *flops = s.flops;
  if (bytes) *bytes = s.bytes;
  if (launches) *launches = s.n;
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_ctx_dump_stats(tt_ctx* ctx, char* buf, long cap) {
  if (!ctx || !buf || cap <= 0) return TT_EINVAL;
  ABI_TRY
  ctx->sync();
  std::string out;
  char line[512];
  std::snprintf(line, sizeof(line), "qr_fallbacks %lld 0 0 0\n", ctx->qr_fallbacks);
  out += line;
  const std::pair<const char*, long long> counters[] = {{"jacobi_svds", ctx->jacobi_svds},
                                                        {"jacobi_sweeps_launched", ctx->jacobi_sweeps_launched},
                                                        {"jacobi_sweeps_needed", ctx->jacobi_sweeps_needed},
                                                        {"jacobi_check_passed", ctx->jacobi_check_passed}};
  for (const auto& c : counters) {
    std::snprintf(line, sizeof(line), "%s %lld 0 0 0\n", c.first, c.second);
    out += line;
  }
  for (const auto& kv : ctx->stats) {
    std::snprintf(line, sizeof(line), "%s %lld %.6f %.6g %.6g\n", kv.first.c_str(), kv.second.n, kv.second.ms,
                  kv.second.flops, kv.second.bytes);
    out += line;
  }
  const long n = std::min<long>((long)out.size(), cap - 1);
  std::memcpy(buf, out.data(), (size_t)n);
  buf[n] = 0;
  return (long)out.size() < cap ? TT_OK : TT_ECAPACITY;
  ABI_CATCH(ctx)
}

int tt_tensor_create(tt_ctx* ctx, int d, const int* n, const int* rank_cap, tt_dtype dtype, tt_tensor** out) {
  if (!ctx || !n || !rank_cap || !out) return TT_EINVAL;
  ABI_TRY
  *out = nullptr;
  require(d >= 1 && d <= TT_MAX_D, TT_EINVAL, "tensor dimension must be in 1..128");
  *out = make_tensor_nk(ctx, d, std::vector<int>(n, n + d), std::vector<int>(rank_cap, rank_cap + d + 1), (int)dtype);
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_tensor_get_modes(const tt_tensor* t, int* n, int* dtype) {
  if (!t) return TT_EINVAL;
  if (n)
    for (int k = 0; k < t->d; ++k) n[k] = t->nk[k];
  if (dtype) *dtype = t->dtype;
  return TT_OK;
}

int tt_tensor_destroy(tt_tensor* t) {
  if (!t) return TT_EINVAL;
  (void)hipStreamSynchronize(t->ctx->stream);
  free_tensor(t);
  return TT_OK;
}

int tt_tensor_set_cores(tt_tensor* t, const int* ranks, const double* const* cores) {
  if (!t || !ranks || !cores) return TT_EINVAL;
  tt_ctx* ctx = t->ctx;
  ABI_TRY
  require(ranks[0] == 1 && ranks[t->d] == 1, TT_EINVAL, "boundary ranks must be 1");
  for (int k = 0; k <= t->d; ++k) require(ranks[k] >= 1 && ranks[k] <= t->cap[k], TT_ECAPACITY, "rank exceeds capacity");
  TTF_HIP(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < t->d; ++k) {
    require(cores[k] != nullptr, TT_EINVAL, "null core pointer");
    const size_t elems = (size_t)ranks[k] * t->nk[k] * ranks[k + 1];
    if (t->dtype == TT_C128) {
      TTF_HIP(hipMemcpy(t->core[k], cores[k], sizeof(zc) * elems, hipMemcpyHostToDevice));
    } else {
      zc* stage = (zc*)ctx->get_ws("c64_stage", sizeof(zc) * elems);
      TTF_HIP(hipMemcpy(stage, cores[k], sizeof(zc) * elems, hipMemcpyHostToDevice));
      narrow_c128(ctx, stage, t->core[k], (long)elems);
      TTF_HIP(hipStreamSynchronize(ctx->stream));
    }
  }
  t->rank.assign(ranks, ranks + t->d + 1);
  t->orth = TT_ORTH_NONE;
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_tensor_get_ranks(const tt_tensor* t, int* ranks) {
  if (!t || !ranks) return TT_EINVAL;
  for (int k = 0; k <= t->d; ++k) ranks[k] = t->rank[k];
  return TT_OK;
}

int tt_tensor_get_cores(const tt_tensor* t, double* const* cores) {
  if (!t || !cores) return TT_EINVAL;
  tt_ctx* ctx = t->ctx;
  ABI_TRY
  TTF_HIP(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < t->d; ++k) {
    require(cores[k] != nullptr, TT_EINVAL, "null core pointer");
    if (t->dtype == TT_C128) {
      TTF_HIP(hipMemcpy(cores[k], t->core[k], sizeof(zc) * t->elems(k), hipMemcpyDeviceToHost));
    } else {
      zc* stage = (zc*)ctx->get_ws("c64_stage", sizeof(zc) * t->elems(k));
      widen_c64(ctx, t->core[k], stage, (long)t->elems(k));
      TTF_HIP(hipStreamSynchronize(ctx->stream));
      TTF_HIP(hipMemcpy(cores[k], stage, sizeof(zc) * t->elems(k), hipMemcpyDeviceToHost));
    }
  }
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_tensor_get_orth(const tt_tensor* t) { return t ? t->orth : TT_EINVAL; }

int tt_tensor_copy(tt_ctx* ctx, const tt_tensor* src, tt_tensor* dst) {
  if (!ctx || !src || !dst) return TT_EINVAL;
  ABI_TRY
  copy_tensor(ctx, src, dst);
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_tensor_set_gaussian(tt_ctx* ctx, tt_tensor* t, const double* mu, const double* sigma, double L) {
  if (!ctx || !t || !mu || !sigma) return TT_EINVAL;
  ABI_TRY
  require(L > 0, TT_EINVAL, "L must be positive");
  tt_tensor* w = widened(ctx, t, "t", false);
  for (int k = 0; k < t->d; ++k) gaussian_factor(ctx, w->core[k], t->nk[k], L, mu[k], sigma[k]);
  w->rank.assign(t->d + 1, 1);
  w->orth = TT_ORTH_NONE;
  narrow_back(ctx, w, t);
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_tensor_set_gaussian_tridiag(tt_ctx* ctx, tt_tensor* t, const double* mu, const double* sigma,
                                   const double* rho, double L, double eps_rel, const int* rmax,
                                   tt_round_report* rep) {
  if (!ctx || !t || !mu || !sigma || (t->d > 1 && !rho)) return TT_EINVAL;
  ABI_TRY
  require(L > 0, TT_EINVAL, "L must be positive");
  require(eps_rel >= 0, TT_EINVAL, "eps must be >= 0");
  const int d = t->d;
  for (int k = 0; k + 1 < d; ++k)
    require(std::fabs(rho[k]) < 0.5, TT_EINVAL, "correlations must lie in (-1/2, 1/2)");
  // the exact nearest-neighbour product (bond k has the rank of mode k)
  std::vector<int> cap(d + 1, 1);
  for (int k = 1; k < d; ++k) cap[k] = t->nk[k - 1];
  tt_tensor* e = pooled_nk(ctx, "nn_ic", d, t->nk, cap);
  for (int k = 0; k < d; ++k) {
    const double c = k > 0 ? rho[k - 1] * sigma[k - 1] * sigma[k] : 0.0;
    nn_gaussian_core(ctx, e->core[k], cap[k], t->nk[k], cap[k + 1], k > 0 ? t->nk[k - 1] : 1, L, mu[k], sigma[k], c);
  }
  e->rank = cap;
  e->orth = TT_ORTH_NONE;
  round_tensor(ctx, e, eps_rel, 0, rep, rmax);
  copy_tensor(ctx, e, t);
  t->rank = e->rank;
  t->orth = e->orth;
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_tensor_set_cdf_gaussian(tt_ctx* ctx, tt_tensor* t, double sigma, double box) {
  if (!ctx || !t) return TT_EINVAL;
  ABI_TRY
  require(box > 0 && sigma > 0, TT_EINVAL, "need box > 0 and sigma > 0");
  tt_tensor* w = widened(ctx, t, "t", false);
  for (int k = 0; k < t->d; ++k) cdf_gaussian_factor(ctx, w->core[k], t->nk[k], box, sigma);
  w->rank.assign(t->d + 1, 1);
  w->orth = TT_ORTH_NONE;
  narrow_back(ctx, w, t);
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_op_create_cdf_burgers(tt_ctx* ctx, int d, int n, const tt_cdf_opts* opts, tt_op** out) {
  if (!out) return TT_EINVAL;
  if (!opts || opts->size != (int)sizeof(tt_cdf_opts)) {
    if (ctx) ctx->last_error = "tt_cdf_opts.size mismatch";
    return TT_EINVAL;
  }
  tt_op* op = nullptr;
  ABI_TRY
  *out = nullptr;
  require(d >= 1 && d <= TT_MAX_D, TT_EINVAL, "d must be in 1..128");
  require(n >= 4, TT_EINVAL, "n must be at least 4");
  require(opts->box > 0 && opts->gamma >= 0 && opts->diffusion >= 0, TT_EINVAL,
          "need box > 0, gamma >= 0 and diffusion >= 0");
  op = new tt_op;
  op->kind = 1;
  op->d = d;
  op->n = n;
  op->L = opts->box;
  op->gamma = opts->gamma;
  op->alpha = opts->alpha;
  op->diff = opts->diffusion;
  build_cdf_burgers(op);
  if (ctx) upload_op(ctx, op);
  *out = op;
  return TT_OK;
  }
  catch (const ttf::Error& e) {
    if (ctx) ctx->last_error = e.msg;
    free_op(op);
    return e.code;
  }
  catch (...) {
    free_op(op);
    return TT_EINVAL;
  }
}

int tt_op_create_burgers_hopf(tt_ctx* ctx, int d, int n, double L, double nu, tt_op** out) {
  return tt_op_create_burgers_hopf_scaled(ctx, d, n, L, nu, 1.0, out);
}

static int create_op(tt_ctx* ctx, int d, int n, double L, double nu, double advection, double diffusion,
                     tt_op** out) {
  if (!out) return TT_EINVAL;
  tt_op* op = nullptr;
  ABI_TRY
  *out = nullptr;
  require(d >= 1 && d <= TT_MAX_D, TT_EINVAL, "d must be in 1..128");
  require(n >= 4, TT_EINVAL, "n must be at least 4");
  require(L > 0 && nu >= 0, TT_EINVAL, "need L > 0 and nu >= 0");
  require(diffusion >= 0, TT_EINVAL, "numerical diffusion must be >= 0");
  op = new tt_op;
  op->d = d;
  op->n = n;
  op->L = L;
  op->nu = nu;
  op->adv = advection;
  op->diff = diffusion;
  build_burgers_hopf(op);
  if (ctx) upload_op(ctx, op);
  *out = op;
  return TT_OK;
  }
  catch (const ttf::Error& e) {
    if (ctx) ctx->last_error = e.msg;
    free_op(op);
    return e.code;
  }
  catch (...) {
    free_op(op);
    return TT_EINVAL;
  }
}

int tt_op_create_burgers_hopf_scaled(tt_ctx* ctx, int d, int n, double L, double nu, double advection,
                                     tt_op** out) {
  return create_op(ctx, d, n, L, nu, advection, 0.0, out);
}

int tt_op_create_burgers_hopf_ex(tt_ctx* ctx, int d, int n, double L, double nu, const tt_op_opts* opts,
                                 tt_op** out) {
  if (!opts || opts->size != (int)sizeof(tt_op_opts)) {
    if (ctx) ctx->last_error = "tt_op_opts.size mismatch";
    return TT_EINVAL;
  }
  return create_op(ctx, d, n, L, nu, opts->advection, opts->diffusion, out);
}

int tt_op_destroy(tt_op* op) {
  if (!op) return TT_EINVAL;
  if (op->ctx) (void)hipStreamSynchronize(op->ctx->stream);
  free_op(op);
  return TT_OK;
}

int tt_op_get_ranks(const tt_op* op, int* R) {
  if (!op || !R) return TT_EINVAL;
  for (int k = 0; k <= op->d; ++k) R[k] = op->R[k];
  return TT_OK;
}

int tt_op_export_coefficients(const tt_op* op, double* B, double* D) {
  if (!op) return TT_EINVAL;
  if (B) std::memcpy(B, op->B.data(), sizeof(double) * op->B.size());
  if (D) std::memcpy(D, op->D.data(), sizeof(double) * op->D.size());
  return TT_OK;
}

int tt_op_export_local_ops(const tt_op* op, int* nops, double* mats) {
  if (!op) return TT_EINVAL;
  const int n = op->n;
  if (nops) *nops = NOPS;
  if (mats) {
    std::memset(mats, 0, sizeof(double) * NOPS * n * n);
    for (int o = 0; o < NOPS; ++o)
      for (int i = 0; i < n; ++i) {
        const int row = o * n + i;
        for (int ti = op->tap_ptr[row]; ti < op->tap_ptr[row + 1]; ++ti)
          mats[(size_t)row * n + op->tap_col[ti]] += op->tap_w[ti];
      }
  }
  return TT_OK;
}

int tt_op_export_site(const tt_op* op, int site, int* count, int* alpha, int* beta, int* lop, double* coef) {
  if (!op || !count || site < 0 || site >= op->d) return TT_EINVAL;
  const auto& ent = op->site[site];
  *count = (int)ent.size();
  if (alpha && beta && lop && coef) {
    for (size_t i = 0; i < ent.size(); ++i) {
      alpha[i] = ent[i].alpha;
      beta[i] = ent[i].beta;
      lop[i] = ent[i].lop;
      coef[2 * i] = ent[i].cre;
      coef[2 * i + 1] = ent[i].cim;
    }
  }
  return TT_OK;
}

int tt_apply(tt_ctx* ctx, const tt_op* op, const tt_tensor* x, tt_tensor* y, const tt_apply_opts* opts) {
  if (!ctx || !op || !x || !y || !opts) return TT_EINVAL;
  ABI_TRY
  require(opts->size == (int)sizeof(tt_apply_opts), TT_EINVAL, "tt_apply_opts.size mismatch");
  require(x != y, TT_EINVAL, "tt_apply: y must not alias x");
  tt_tensor* xw = widened(ctx, x, "x");
  tt_tensor* yw = widened(ctx, y, "y", false);
  apply_any(ctx, op, xw, yw, opts->mode, opts->sketch_rank, opts->seed, opts->precision, opts->power);
  narrow_back(ctx, yw, y);
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_axpy(tt_ctx* ctx, double ar, double ai, const tt_tensor* x, double br, double bi, const tt_tensor* y,
            tt_tensor* z) {
  if (!ctx || !x || !y || !z) return TT_EINVAL;
  ABI_TRY
  require(z != x && z != y, TT_EINVAL, "tt_axpy: z aliases an input");
  const tt_tensor* xs[2] = {widened(ctx, x, "s0"), widened(ctx, y, "s1")};
  const zc coef[2] = {Z(ar, ai), Z(br, bi)};
  tt_tensor* zw = widened(ctx, z, "z", false);
  sum_tensors(ctx, 2, coef, xs, zw);
  narrow_back(ctx, zw, z);
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_sum(tt_ctx* ctx, int nterms, const double* coef, const tt_tensor* const* xs, tt_tensor* z) {
  if (!ctx || !coef || !xs || !z) return TT_EINVAL;
  ABI_TRY
  require(nterms >= 1 && nterms <= 8, TT_EINVAL, "tt_sum: 1..8 terms");
  std::vector<zc> c(nterms);
  std::vector<const tt_tensor*> xw(nterms);
  for (int t = 0; t < nterms; ++t) {
    c[t] = Z(coef[2 * t], coef[2 * t + 1]);
    require(xs[t] && xs[t] != z, TT_EINVAL, "tt_sum: null input or output aliasing an input");
    xw[t] = widened(ctx, xs[t], ("s" + std::to_string(t)).c_str());
  }
  tt_tensor* zw = widened(ctx, z, "z", false);
  sum_tensors(ctx, nterms, c.data(), xw.data(), zw);
  narrow_back(ctx, zw, z);
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_round(tt_ctx* ctx, tt_tensor* x, double eps_rel, const int* rmax, tt_round_report* rep) {
  if (!ctx || !x) return TT_EINVAL;
  ABI_TRY
  require(eps_rel >= 0, TT_EINVAL, "tt_round: eps must be >= 0");
  tt_tensor* xw = widened(ctx, x, "x");
  round_tensor(ctx, xw, eps_rel, 0, rep, rmax);
  narrow_back(ctx, xw, x);
  return TT_OK;
  ABI_CATCH(ctx)
}

}  // extern "C"

namespace {

// <x, y> = sum conj(x) y by left-to-right contraction:
// W_{k+1} = V(X_k)^H (W_k H(Y_k)), W_0 = 1 (App. A.1 arithmetic)
zc dot_tensors(tt_ctx* ctx, const tt_tensor* x, const tt_tensor* y) {
  require(x->d == y->d && x->nk == y->nk, TT_ESHAPE, "tt_dot: shape mismatch");
  require(x->dtype == TT_C128 && y->dtype == TT_C128, TT_EINVAL, "internal: dot needs complex-double storage");
  const int d = x->d;
  size_t wmax = 1, tmax = 1;
  for (int k = 0; k < d; ++k) {
    wmax = std::max(wmax, (size_t)x->rank[k + 1] * y->rank[k + 1]);
    tmax = std::max(tmax, (size_t)x->rank[k] * x->nk[k] * y->rank[k + 1]);
  }
  zc* W = (zc*)ctx->get_ws("dot_W", sizeof(zc) * wmax);
  zc* W2 = (zc*)ctx->get_ws("dot_W2", sizeof(zc) * wmax);
  zc* T = (zc*)ctx->get_ws("dot_T", sizeof(zc) * tmax);
  zc* h = (zc*)ctx->host_scratch(sizeof(zc));
  *h = Z(1);
  TTF_HIP(hipMemcpyAsync(W, h, sizeof(zc), hipMemcpyHostToDevice, ctx->stream));
  for (int k = 0; k < d; ++k) {
    const int rx0 = x->rank[k], ry0 = y->rank[k], rx1 = x->rank[k + 1], ry1 = y->rank[k + 1];
    const int n = x->nk[k];
    // T (rx0 x n ry1) = W (rx0 x ry0) H(Y_k)
    zgemm(ctx, OPN, OPN, rx0, n * ry1, ry0, Z(1), W, rx0, 0, y->core[k], ry0, 0, Z(0), T, rx0, 0);
    // W' (rx1 x ry1) = V(X_k)^H T, T read as (rx0 n) x ry1
    zgemm(ctx, OPC, OPN, rx1, ry1, rx0 * n, Z(1), x->core[k], (long)rx0 * n, 0, T, (long)rx0 * n, 0, Z(0), W2, rx1,
          0);
    std::swap(W, W2);
  }
  TTF_HIP(hipMemcpyAsync(h, W, sizeof(zc), hipMemcpyDeviceToHost, ctx->stream));
  TTF_HIP(hipStreamSynchronize(ctx->stream));
  return *h;
}

// ||x|| of a tensor the last rounding left left-orthogonal: the norm of
// its last core; otherwise orthogonalise a copy first
double tensor_norm(tt_ctx* ctx, const tt_tensor* x) {
  if (x->orth == TT_ORTH_LEFT) return core_norm(ctx, x, x->d - 1);
  if (x->orth == TT_ORTH_RIGHT || x->d == 1) return core_norm(ctx, x, 0);
  tt_tensor* tmp = pooled_nk(ctx, "norm_tmp", x->d, x->nk, x->rank);
  copy_tensor(ctx, x, tmp);
  phase1_right_orth(ctx, tmp);
  return core_norm(ctx, tmp, 0);
}

std::vector<int> interior_caps(int d, int c) {
  std::vector<int> cap(d + 1, c);
  cap[0] = cap[d] = 1;
  return cap;
}

// t <- the zero tensor (all ranks 1)
void set_zero(tt_ctx* ctx, tt_tensor* t) {
  for (int k = 0; k < t->d; ++k) fill_zero(ctx, t->core[k], t->nk[k]);
  t->rank.assign(t->d + 1, 1);
  t->orth = TT_ORTH_NONE;
}

// out <- T[sum_t coef_t xs_t] for any number of terms: chunks of at most
// `chunk` terms are summed and truncated in turn (relative tolerance eps,
// cap rmax), the running sum being the first term of every later chunk.
// `acc` holds each partial sum; out may be any tensor not among xs.
void sum_round(tt_ctx* ctx, const std::vector<zc>& coef, const std::vector<const tt_tensor*>& xs, tt_tensor* out,
               double eps, int rmax, const std::string& tag) {
  const int d = out->d, n = out->n;
  const int nt = (int)xs.size();
  int maxr = 1;
  for (auto* t : xs)
    for (int k = 0; k <= d; ++k) maxr = std::max(maxr, t->rank[k]);
  maxr = std::max(maxr, rmax);
  // keep every partial sum within the SVD size limit (512)
  const int chunk = std::max(1, std::min(7, 512 / maxr - 1));
  tt_tensor* acc = pooled(ctx, tag + "_acc", d, n, interior_caps(d, std::min(512, maxr * (chunk + 1))));
  tt_tensor* run = pooled(ctx, tag + "_run", d, n, interior_caps(d, maxr));
  bool have = false;
  for (int t0 = 0; t0 < nt; t0 += chunk) {
    const int t1 = std::min(nt, t0 + chunk);
    std::vector<zc> c;
    std::vector<const tt_tensor*> x;
    if (have) {
      c.push_back(Z(1));
      x.push_back(run);
    }
    for (int t = t0; t < t1; ++t) {
      c.push_back(coef[t]);
      x.push_back(xs[t]);
    }
    sum_tensors(ctx, (int)x.size(), c.data(), x.data(), acc);
    round_tensor(ctx, acc, eps, rmax, nullptr);
    copy_tensor(ctx, acc, run);
    have = true;
  }
  copy_tensor(ctx, run, out);
}

struct GmresResult {
  int iterations = 0, converged = 0, max_rank = 0, applications = 0;
  double residual = 0.0;
};

// TT-GMRES for (I - c L) x = b; x holds the guess (use_guess) and receives
// the truncated solution.  Returns the report; the caller decides what a
// missed tolerance means.
GmresResult gmres_shifted(tt_ctx* ctx, const tt_op* op, double c, const tt_tensor* b, tt_tensor* x,
                          const tt_solve_opts& o) {
  const int d = b->d, n = b->n, m = o.max_iter, kr = o.krylov_rmax;
  GmresResult res;
  const auto capk = interior_caps(d, kr);
  // operator application output capacity
  std::vector<int> capa(d + 1, 1);
  for (int k = 1; k < d; ++k)
    capa[k] = o.apply_mode == TT_APPLY_EXACT ? op->R[k] * std::max(kr, o.rmax) : std::max(o.sketch_rank, kr);
  tt_tensor* ab = pooled(ctx, "gm_apply", d, n, capa);
  tt_tensor* w = pooled(ctx, "gm_w", d, n, capk);
  tt_tensor* x0 = pooled(ctx, "gm_x0", d, n, interior_caps(d, std::max(kr, o.rmax)));
  std::vector<tt_tensor*> V(m + 1);
  for (int j = 0; j <= m; ++j) V[j] = pooled(ctx, "gm_V" + std::to_string(j), d, n, capk);
  uint64_t seed = o.seed;
  auto apply_shift = [&](const tt_tensor* v, tt_tensor* out) {
    // out <- T[v - c L v]
    apply_any(ctx, op, v, ab, o.apply_mode, o.sketch_rank, seed, o.precision);
    seed += 0x9E3779B97F4A7C15ull;
    ++res.applications;
    sum_round(ctx, {Z(1), Z(-c)}, {v, ab}, out, o.krylov_eps, kr, "gm_s");
  };
  const double bnorm = tensor_norm(ctx, b);
  if (bnorm == 0.0) {
    set_zero(ctx, x);  // the solution is zero
    res.converged = 1;
    return res;
  }
  // r0 = b - (x0 - c L x0), or b for a zero guess
  if (o.use_guess) {
    copy_tensor(ctx, x, x0);
    apply_shift(x0, w);
    sum_round(ctx, {Z(1), Z(-1)}, {b, w}, V[0], o.krylov_eps, kr, "gm_s");
  } else {
    set_zero(ctx, x0);
    sum_round(ctx, {Z(1)}, {b}, V[0], o.krylov_eps, kr, "gm_s");
  }
  const double beta = tensor_norm(ctx, V[0]);
  std::vector<std::vector<std::complex<double>>> H(m + 1, std::vector<std::complex<double>>(m, 0.0));
  std::vector<double> cs(m, 0.0);
  std::vector<std::complex<double>> sn(m, 0.0), g(m + 1, 0.0);
  g[0] = beta;
  int k = 0;
  res.residual = beta / bnorm;
  if (res.residual <= o.tol) {
    res.converged = 1;
  } else {
    {
      const zc inv = Z(1.0 / beta);
      tt_tensor* t = pooled(ctx, "gm_tmp", d, n, capk);
      copy_tensor(ctx, V[0], t);
      sum_tensors(ctx, 1, &inv, std::vector<const tt_tensor*>{t}.data(), V[0]);
    }
    for (int j = 0; j < m; ++j) {
      apply_shift(V[j], w);
      // two classical Gram-Schmidt passes against V_0..V_j
      std::vector<std::complex<double>> h(j + 1, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<zc> coef{Z(1)};
        std::vector<const tt_tensor*> xs{w};
        for (int i = 0; i <= j; ++i) {
          const zc p = dot_tensors(ctx, V[i], w);
          h[i] += std::complex<double>(p.x, p.y);
          coef.push_back(Z(-p.x, -p.y));
          xs.push_back(V[i]);
        }
        tt_tensor* t = pooled(ctx, "gm_tmp", d, n, capk);
        copy_tensor(ctx, w, t);
        xs[0] = t;
        sum_round(ctx, coef, xs, w, o.krylov_eps, kr, "gm_s");
      }
      const double hn = tensor_norm(ctx, w);
      for (int i = 0; i <= j; ++i) H[i][j] = h[i];
      H[j + 1][j] = hn;
      for (int q = 0; q <= d; ++q) res.max_rank = std::max(res.max_rank, w->rank[q]);
      // previous rotations, then a new one that zeroes H[j+1][j]
      for (int i = 0; i < j; ++i) {
        const std::complex<double> a = H[i][j], bb = H[i + 1][j];
        H[i][j] = cs[i] * a + sn[i] * bb;
        H[i + 1][j] = -std::conj(sn[i]) * a + cs[i] * bb;
      }
      {
        const std::complex<double> a = H[j][j];
        const double t = std::abs(a), r = std::hypot(t, hn);
        if (t == 0.0) {
          cs[j] = 0.0;
          sn[j] = 1.0;
          H[j][j] = hn;
        } else {
          cs[j] = t / r;
          sn[j] = (a / t) * hn / r;
          H[j][j] = (a / t) * r;
        }
        H[j + 1][j] = 0.0;
        g[j + 1] = -std::conj(sn[j]) * g[j];
        g[j] = cs[j] * g[j];
      }
      k = j + 1;
      res.residual = std::abs(g[j + 1]) / bnorm;
      if (res.residual <= o.tol || hn <= 1e-300) {
        res.converged = res.residual <= o.tol;
        if (hn <= 1e-300) res.converged = 1;  // exact breakdown: the Krylov space holds the solution
        break;
      }
      const zc inv = Z(1.0 / hn);
      sum_tensors(ctx, 1, &inv, std::vector<const tt_tensor*>{w}.data(), V[j + 1]);
    }
  }
  res.iterations = k;
  // y = H^-1 g (upper triangular k x k); x = x0 + V y
  std::vector<std::complex<double>> y(k, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    std::complex<double> acc = g[i];
    for (int j = i + 1; j < k; ++j) acc -= H[i][j] * y[j];
    y[i] = acc / H[i][i];
  }
  std::vector<zc> coef{Z(1)};
  std::vector<const tt_tensor*> xs{x0};
  for (int i = 0; i < k; ++i) {
    coef.push_back(Z(y[i].real(), y[i].imag()));
    xs.push_back(V[i]);
  }
  tt_tensor* xs_out = pooled(ctx, "gm_xout", d, n, interior_caps(d, std::max(kr, o.rmax)));
  sum_round(ctx, coef, xs, xs_out, std::min(o.krylov_eps, o.eps), std::max(kr, o.rmax), "gm_x");
  round_tensor(ctx, xs_out, o.eps, o.rmax, nullptr);
  copy_tensor(ctx, xs_out, x);
  return res;
}

void check_solve_opts(const tt_solve_opts& o) {
  require(o.max_iter >= 1 && o.max_iter <= 40, TT_EINVAL, "TT-GMRES: max_iter must be in 1..40");
  require(o.tol > 0.0, TT_EINVAL, "TT-GMRES: tol must be > 0");
  require(o.krylov_eps > 0.0, TT_EINVAL, "TT-GMRES: krylov_eps must be > 0");
  require(o.krylov_rmax >= 1 && o.krylov_rmax <= 256, TT_EINVAL, "TT-GMRES: krylov_rmax must be in 1..256");
  require(o.rmax >= 1 && o.eps >= 0.0, TT_EINVAL, "TT-GMRES: bad rmax or eps");
  require(o.apply_mode == TT_APPLY_EXACT || (o.apply_mode == TT_APPLY_SKETCH && o.sketch_rank >= 1), TT_EINVAL,
          "TT-GMRES: bad apply mode");
  require(o.precision == TT_PREC_FP64 || o.precision == TT_PREC_BF16X3 || o.precision == TT_PREC_FP16X3 ||
              o.precision == TT_PREC_FP32,
          TT_EINVAL,
          "TT-GMRES: unknown precision");
}

void randomized_into(tt_ctx* ctx, const tt_tensor* x, const int* widths, uint64_t seed, tt_tensor* y);
double sketch_rel_error(tt_ctx* ctx, int npieces, const zc* coef, const tt_tensor* const* pieces,
                        const tt_tensor* y, uint64_t seed);

}  // namespace

extern "C" {

int tt_step(tt_ctx* ctx, const tt_op* op, tt_tensor* f, double dt, const tt_step_opts* opts, tt_step_report* rep) {
  if (!ctx || !op || !f || !opts) return TT_EINVAL;
  ABI_TRY
  if (f->dtype != TT_C128) {
    tt_tensor* fw = widened(ctx, f, "f");
    const int rc = tt_step(ctx, op, fw, dt, opts, rep);
    if (rc == TT_OK) narrow_back(ctx, fw, f);
    return rc;
  }
  require(opts->size == (int)sizeof(tt_step_opts), TT_EINVAL, "tt_step_opts.size mismatch");
  require(opts->rmax >= 1, TT_EINVAL, "tt_step: rmax must be >= 1");
  require(opts->precision == TT_PREC_FP64 || opts->precision == TT_PREC_BF16X3 || opts->precision == TT_PREC_FP16X3 ||
              opts->precision == TT_PREC_FP32,
          TT_EINVAL, "tt_step: unknown precision");
  const int scheme = opts->scheme;
  require(scheme >= TT_STEP_RK4 && scheme <= TT_STEP_IMPLICIT_MIDPOINT, TT_EINVAL, "tt_step: unknown scheme");
  const bool implicit = scheme == TT_STEP_IMPLICIT_EULER || scheme == TT_STEP_IMPLICIT_MIDPOINT;
  if (opts->learned_apply_widths) {
    require(scheme == TT_STEP_RK4 && opts->apply_mode == TT_APPLY_SKETCH, TT_EINVAL,
            "tt_step: learned_apply_widths needs the RK4 scheme and the sketched apply");
    for (int k = 0; k <= f->d; ++k)
      require(opts->learned_apply_widths[k] >= 1 && opts->learned_apply_widths[k] <= 512, TT_EINVAL,
              "tt_step: learned_apply_widths outside [1, 512]");
  }
  if (opts->learned_widths) {
    require(scheme == TT_STEP_RK4, TT_EINVAL, "tt_step: learned_widths needs the RK4 scheme");
    require(opts->learned_tol >= 0.0, TT_EINVAL, "tt_step: learned_tol must be >= 0");
    for (int k = 0; k <= f->d; ++k)
      require(opts->learned_widths[k] >= 1 && opts->learned_widths[k] <= 512, TT_EINVAL,
              "tt_step: learned_widths outside [1, 512]");
  }
  tt_solve_opts so{};
  if (implicit) {
    so.size = sizeof(so);
    so.max_iter = opts->gmres_max_iter;
    so.tol = opts->gmres_tol;
    so.krylov_eps = 0.1 * std::min(opts->gmres_tol, opts->eps > 0.0 ? opts->eps : opts->gmres_tol);
    so.krylov_rmax = opts->krylov_rmax > 0 ? opts->krylov_rmax : std::min(256, 2 * opts->rmax);
    so.rmax = opts->rmax;
    so.eps = opts->eps;
    so.apply_mode = opts->apply_mode;
    so.sketch_rank = opts->sketch_rank;
    so.seed = opts->seed ^ 0x5DEECE66Dull;
    so.precision = opts->precision;
    so.use_guess = 1;
    check_solve_opts(so);
  }
  check_same_shape(op, f);
  const int d = f->d, n = f->n, rmax = opts->rmax;
  // capacities of the temporaries: stage derivatives k (apply outputs),
  // stage inputs y (f + c k) and the final combination.  Every rounded
  // tensor has rank at most base = min(rmax, n^k, n^(d-k)) at bond k; f has
  // at most its capacity.
  std::vector<int> capk(d + 1), capy(d + 1), capf(d + 1);
  const int big = 1 << 30;
  for (int k = 0; k <= d; ++k) {
    const bool end = k == 0 || k == d;
    const int bound = std::min(bounded_pow(n, k, big), bounded_pow(n, d - k, big));
    const int fr = end ? 1 : f->cap[k];
    const int base = end ? 1 : std::min(rmax, bound);
    // the midpoint stage input f + dt/2 k is applied untruncated
    const bool mid = scheme == TT_STEP_MIDPOINT || scheme == TT_STEP_IMPLICIT_MIDPOINT;
    const int rin = (mid && !end) ? fr + base : std::max(fr, base);
    if (opts->apply_mode == TT_APPLY_EXACT)
      capk[k] = op->R[k] * rin;
    else
      capk[k] = end ? 1 : std::max(std::min(opts->sketch_rank, bound), base);
    capy[k] = end ? 1 : fr + base;
    capf[k] = end ? 1 : fr + 4 * base;
  }
  // the operator's bond dimensions set the exact apply's capacities
  std::string key = shape_key(d, n, f->cap, rmax) + ":" + std::to_string(scheme) + ":" +
                    std::to_string(opts->apply_mode) + ":" + std::to_string(opts->sketch_rank) + ":R";
  for (int k = 0; k <= d; ++k) key += "," + std::to_string(op->R[k]);
  StepTemps& T = [&]() -> StepTemps& {
    std::lock_guard<std::mutex> lock(cache_mutex());
    return step_cache()[{ctx, key}];
  }();
  if (!T.ysum) {
    const int nk = scheme == TT_STEP_RK4                                                   ? 4
                   : (scheme == TT_STEP_MIDPOINT || scheme == TT_STEP_IMPLICIT_MIDPOINT) ? 2
                                                                                         : 1;
    for (int s = 0; s < nk; ++s) T.k[s] = make_tensor(ctx, d, n, capk);
    T.ysum = make_tensor(ctx, d, n, capy);
    T.fsum = make_tensor(ctx, d, n, capf);
  }
  const double eps = opts->eps;
  const int mode = opts->apply_mode, l = opts->sketch_rank;
  int maxr = 0;
  auto track = [&](const tt_tensor* t) {
    for (int k = 0; k <= d; ++k) maxr = std::max(maxr, t->rank[k]);
  };
  // T[x] of a sum x = sum_i coef_i pieces_i: the deterministic rounding, or
  // (learned form, given widths) the randomised rounding to those widths
  // followed by the deterministic rounding of its small result when the a
  // posteriori error is within learned_tol, else the deterministic rounding
  // of x itself (fallback). Returns the tensor holding the result.
  int learned_used = 0, learned_fallback = 0;
  double learned_err = 0.0;
  std::vector<const tt_tensor*> final_pieces;
  std::vector<zc> final_coef;
  auto truncate = [&](tt_tensor* x, int npieces, const zc* coef, const tt_tensor* const* pieces, const char* slot,
                      uint64_t salt, tt_round_report* rrep) -> tt_tensor* {
    if (!opts->learned_widths || npieces == 0) {
      round_tensor(ctx, x, eps, rmax, rrep);
      return x;
    }
    std::vector<int> w(d + 1, 1);
    int wmax = 1;
    for (int k = 1; k < d; ++k) {
      w[k] = std::max(1, std::min(opts->learned_widths[k], x->rank[k]));
      wmax = std::max(wmax, w[k]);
    }
    tt_tensor* y = pooled(ctx, slot, d, n, interior_caps(d, std::max(wmax, rmax)));
    randomized_into(ctx, x, w.data(), opts->seed ^ (0xA5A5A5A5ull * salt), y);
    const double err = sketch_rel_error(ctx, npieces, coef, pieces, y, opts->seed ^ (0x5BD1E995ull * salt));
    ++learned_used;
    learned_err = std::max(learned_err, err);
    if (err <= opts->learned_tol) {
      round_tensor(ctx, y, eps, rmax, rrep);
      return y;
    }
    ++learned_fallback;
    round_tensor(ctx, x, eps, rmax, rrep);
    return x;
  };
  // stage s: k_s = T[L y_s] with its own sketch seed
  std::vector<int> kr(d + 1, 0);
  int apply_fallback = 0;
  // learned form: per-bond sketch widths for the stage applications
  std::vector<int> aw;
  if (opts->learned_apply_widths && mode == TT_APPLY_SKETCH) {
    aw.assign(d + 1, 1);
    for (int k = 1; k < d; ++k) aw[k] = std::max(1, std::min(opts->learned_apply_widths[k], l));
  }
  auto stage = [&](int s, const tt_tensor* in) {
    const uint64_t seed = opts->seed + 0x9E3779B97F4A7C15ull * (uint64_t)(s + 1);
    bool done = false;
    if (!aw.empty()) {
      int lw = 1;
      for (int k = 0; k <= d; ++k) lw = std::max(lw, aw[k]);
      apply_sketch(ctx, op, in, T.k[s], lw, seed, opts->precision, aw.data(), opts->sketch_power);
      round_tensor(ctx, T.k[s], eps, rmax, nullptr);
      // a bond whose rounded rank reaches a width below the plain one may
      // have been cut by the sketch: apply the stage again at full width
      done = true;
      for (int k = 1; k < d && done; ++k)
        if (aw[k] < l && T.k[s]->rank[k] >= aw[k]) done = false;
      if (!done) ++apply_fallback;
    }
    if (!done) {
      apply_any(ctx, op, in, T.k[s], mode, l, seed, opts->precision, opts->sketch_power);
      round_tensor(ctx, T.k[s], eps, rmax, nullptr);
    }
    for (int k = 0; k <= d; ++k) kr[k] = std::max(kr[k], T.k[s]->rank[k]);
    track(T.k[s]);
  };
  int stages = 0;
  if (scheme == TT_STEP_RK4) {
    const tt_tensor* stage_in = f;
    const double cst[3] = {0.5 * dt, 0.5 * dt, dt};
    for (int s = 0; s < 4; ++s) {
      stage(s, stage_in);
      if (s < 3) {
        const tt_tensor* xs[2] = {f, T.k[s]};
        const zc coef[2] = {Z(1), Z(cst[s])};
        sum_tensors(ctx, 2, coef, xs, T.ysum);
        stage_in = truncate(T.ysum, 2, coef, xs, "learned_ys", (uint64_t)s + 1, nullptr);
        track(stage_in);
      }
    }
    const tt_tensor* xs[5] = {f, T.k[0], T.k[1], T.k[2], T.k[3]};
    const zc coef[5] = {Z(1), Z(dt / 6), Z(dt / 3), Z(dt / 3), Z(dt / 6)};
    sum_tensors(ctx, 5, coef, xs, T.fsum);
    final_pieces.assign(xs, xs + 5);
    final_coef.assign(coef, coef + 5);
    stages = 4;
  } else if (scheme == TT_STEP_EULER) {
    stage(0, f);
    const tt_tensor* xs[2] = {f, T.k[0]};
    const zc coef[2] = {Z(1), Z(dt)};
    sum_tensors(ctx, 2, coef, xs, T.fsum);
    stages = 1;
  } else if (scheme == TT_STEP_MIDPOINT) {
    stage(0, f);
    const tt_tensor* ys[2] = {f, T.k[0]};
    const zc ycoef[2] = {Z(1), Z(0.5 * dt)};
    sum_tensors(ctx, 2, ycoef, ys, T.ysum);  // not truncated
    track(T.ysum);
    stage(1, T.ysum);
    const tt_tensor* xs[2] = {f, T.k[1]};
    const zc coef[2] = {Z(1), Z(dt)};
    sum_tensors(ctx, 2, coef, xs, T.fsum);
    stages = 2;
  } else {
    // implicit: the explicit step of the same kind is the initial guess
    // (Sec. 4.1: the iteration starts from Psi_dt(G, f))
    stage(0, f);
    const tt_tensor* rhs = f;
    double shift = dt;
    if (scheme == TT_STEP_IMPLICIT_EULER) {
      const tt_tensor* xs[2] = {f, T.k[0]};
      const zc coef[2] = {Z(1), Z(dt)};
      sum_tensors(ctx, 2, coef, xs, T.fsum);
      stages = 1;
    } else {
      const tt_tensor* ys[2] = {f, T.k[0]};
      const zc ycoef[2] = {Z(1), Z(0.5 * dt)};
      sum_tensors(ctx, 2, ycoef, ys, T.ysum);
      stage(1, T.ysum);
      const tt_tensor* xs[2] = {f, T.k[1]};
      const zc coef[2] = {Z(1), Z(dt)};
      sum_tensors(ctx, 2, coef, xs, T.fsum);
      // right-hand side T[f + dt/2 T[L f]]
      round_tensor(ctx, T.ysum, eps, rmax, nullptr);
      track(T.ysum);
      rhs = T.ysum;
      shift = 0.5 * dt;
      stages = 2;
    }
    round_tensor(ctx, T.fsum, eps, rmax, nullptr);
    const GmresResult gr = gmres_shifted(ctx, op, shift, rhs, T.fsum, so);
    stages += gr.applications;
    maxr = std::max(maxr, gr.max_rank);
    if (!gr.converged)
      fail(TT_ENOCONV, "tt_step: TT-GMRES reached relative residual " + std::to_string(gr.residual) + " after " +
                           std::to_string(gr.iterations) + " iterations (tolerance " + std::to_string(so.tol) + ")");
  }
  tt_round_report frep;
  std::memset(&frep, 0, sizeof(frep));
  const tt_tensor* result = T.fsum;
  if (!implicit)  // (the implicit solver's output is truncated already)
    result = truncate(T.fsum, (int)final_pieces.size(), final_coef.data(), final_pieces.data(), "learned_yf", 5,
                      &frep);
  if (rep) {
    rep->learned_used = learned_used;
    rep->learned_fallback = learned_fallback;
    rep->learned_err = learned_err;
    rep->learned_apply_fallback = apply_fallback;
    for (int k = 0; k <= d; ++k) rep->k_ranks[k] = kr[k];
  }
  track(result);
  copy_tensor(ctx, result, f);
  if (rep) {
    rep->final_norm = frep.norm;
    std::memcpy(rep->final_sv, frep.sv_last, sizeof(frep.sv_last));
  }
  if (rep) {
    rep->stages = stages;
    rep->max_rank = maxr;
    for (int k = 0; k <= d; ++k) rep->ranks[k] = f->rank[k];
  }
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_dot(tt_ctx* ctx, const tt_tensor* x, const tt_tensor* y, double* out) {
  if (!ctx || !x || !y || !out) return TT_EINVAL;
  ABI_TRY
  const zc v = dot_tensors(ctx, widened(ctx, x, "x"), widened(ctx, y, "y"));
  out[0] = v.x;
  out[1] = v.y;
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_solve_shifted(tt_ctx* ctx, const tt_op* op, double c, const tt_tensor* b, tt_tensor* x,
                     const tt_solve_opts* opts, tt_solve_report* rep) {
  if (!ctx || !op || !b || !x || !opts) return TT_EINVAL;
  ABI_TRY
  require(opts->size == (int)sizeof(tt_solve_opts), TT_EINVAL, "tt_solve_opts.size mismatch");
  require(b != x, TT_EINVAL, "tt_solve_shifted: x aliases b");
  if (b->dtype != TT_C128 || x->dtype != TT_C128) {
    tt_tensor* bw = widened(ctx, b, "b");
    tt_tensor* xw = widened(ctx, x, "x");
    const int rc = tt_solve_shifted(ctx, op, c, bw, xw, opts, rep);
    if (rc == TT_OK) narrow_back(ctx, xw, x);
    return rc;
  }
  check_solve_opts(*opts);
  check_same_shape(op, b);
  check_same_shape(op, x);
  tt_solve_opts o = *opts;
  // the returned solution must fit x
  for (int k = 1; k < x->d; ++k) o.rmax = std::min(o.rmax, x->cap[k]);
  const GmresResult gr = gmres_shifted(ctx, op, c, b, x, o);
  if (rep) {
    rep->iterations = gr.iterations;
    rep->converged = gr.converged;
    rep->residual = gr.residual;
    rep->max_rank = gr.max_rank;
    rep->pad = 0;
  }
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_step_reserve(tt_ctx* ctx, const tt_op* op, const tt_tensor* f, double dt, const tt_step_opts* opts) {
  if (!ctx || !op || !f || !opts) return TT_EINVAL;
  ABI_TRY
  check_same_shape(op, f->dtype == TT_C128 ? f : widened(ctx, f, "f"));
  // steps on a tensor of f's shape and storage with every interior rank at
  // its capacity (random cores): the largest shapes a step can meet.  One
  // step per starting form of the QR factorisations (the later forms are
  // fallbacks that a step takes only on ill-conditioned input, with
  // workspaces of their own), and the largest split-K workspace.
  ctx->get_ws("gemm_splitk", sizeof(zc) * SPLITK_WS_ELEMS);
  tt_tensor* g = pooled_nk(ctx, "reserve", f->d, f->nk, f->cap);
  tt_tensor* gs = f->dtype == TT_C128 ? g : pooled_nk(ctx, "reserve_c64", f->d, f->nk, f->cap, f->dtype);
  const int saved_level = ctx->qr_min_level;
  int rc = TT_OK;
  try {
    for (int level = saved_level; level <= 2 && rc == TT_OK; ++level) {
      for (int k = 0; k < f->d; ++k) {
        g->rank[k] = f->cap[k];
        sketch_core(ctx, g->core[k], (long)g->cap_elems(k), 0x5EEDu + (uint64_t)k, k,
                    1.0 / std::sqrt(2.0 * f->nk[k] * f->cap[k]));
      }
      g->rank[f->d] = 1;
      g->orth = TT_ORTH_NONE;
      if (gs != g) narrow_back(ctx, g, gs);
      ctx->qr_min_level = level;
      tt_step_report rep;
      rc = tt_step(ctx, op, gs, dt, opts, &rep);
    }
  } catch (...) {
    ctx->qr_min_level = saved_level;
    throw;
  }
  ctx->qr_min_level = saved_level;
  ctx->sync();
  return rc;
  ABI_CATCH(ctx)
}

int tt_step_batch(int count, tt_ctx* const* ctxs, const tt_op* const* ops, tt_tensor* const* fs, const double* dts,
                  const tt_step_opts* opts, tt_step_report* reps, int* status) {
  if (count < 0 || (count > 0 && (!ctxs || !ops || !fs || !dts || !opts || !status))) return TT_EINVAL;
  // one host thread per distinct context, running its instances in order on
  // the context's stream: the instances of different contexts overlap on
  // the GPU
  std::vector<tt_ctx*> order;
  std::map<tt_ctx*, std::vector<int>> work;
  for (int i = 0; i < count; ++i) {
    if (!ctxs[i]) return TT_EINVAL;
    if (!work.count(ctxs[i])) order.push_back(ctxs[i]);
    work[ctxs[i]].push_back(i);
  }
  auto run = [&](tt_ctx* ctx) {
    if (hipSetDevice(ctx->device) != hipSuccess) {
      for (int i : work[ctx]) status[i] = TT_EHIP;
      return;
    }
    for (int i : work[ctx]) status[i] = tt_step(ctx, ops[i], fs[i], dts[i], &opts[i], reps ? &reps[i] : nullptr);
  };
  std::vector<std::thread> threads;
  threads.reserve(order.size());
  for (size_t t = 1; t < order.size(); ++t) threads.emplace_back(run, order[t]);
  if (!order.empty()) run(order[0]);
  for (auto& th : threads) th.join();
  for (int i = 0; i < count; ++i)
    if (status[i] != TT_OK) return status[i];
  return TT_OK;
}

}  // extern "C"

namespace {

const tt_op* identity_op(tt_ctx* ctx, int d, int n) {
  std::lock_guard<std::mutex> lock(cache_mutex());
  tt_op*& op = identity_ops()[{ctx, d, n}];
  if (!op) {
    tt_op* o = new tt_op;
    o->d = d;
    o->n = n;
    o->L = 1.0;
    o->nu = 0.0;
    o->adv = 0.0;
    o->ident = 1.0;
    build_burgers_hopf(o);
    upload_op(ctx, o);
    op = o;
  }
  return op;
}

// Randomised rounding with per-bond sketch widths: the sketched product with
// the identity operator (left Gaussian TT sketches, right-to-left sweep of
// LQ factorisations; right-orthonormal result of ranks <= widths), and its
// relative error ||x - y|| / ||x|| from exact TT inner products.
void randomized_into(tt_ctx* ctx, const tt_tensor* x, const int* widths, uint64_t seed, tt_tensor* y) {
  const tt_op* op = identity_op(ctx, x->d, x->n);
  int l = 1;
  for (int k = 0; k <= x->d; ++k) l = std::max(l, widths[k]);
  apply_sketch(ctx, op, x, y, l, seed, TT_PREC_FP64, widths);
}

// A posteriori error of a randomised rounding y of x = sum_i coef_i p_i by
// an independent Gaussian TT sketch: Omega maps a TT to LSK_WIDTH numbers
// through random cores of bond rank LSK_WIDTH (Philox, its own key), and the
// estimate is ||Omega x - Omega y|| / ||Omega x||, Omega x = sum_i coef_i
// Omega p_i.  Only chain contractions (GEMMs, no factorisation), piece by
// piece, so no product touches the wide concatenated sum, and the
// difference is formed between two vectors: no cancellation of squares.
// For a fixed TT z, ||Omega z||^2 / LSK_WIDTH estimates ||z||^2 without
// bias; the ratio's spread is measured against the exact difference norm.
constexpr int LSK_WIDTH = 64;

void sketch_vector(tt_ctx* ctx, const tt_tensor* x, uint64_t seed, zc alpha, zc* acc, bool first) {
  const int d = x->d, s = LSK_WIDTH;
  int rmax = 1;
  for (int k = 0; k <= d; ++k) rmax = std::max(rmax, x->rank[k]);
  size_t vmax = 1, omax = 1;
  for (int k = 0; k < d; ++k) {
    const int sp = k == 0 ? 1 : s;
    vmax = std::max(vmax, (size_t)sp * x->nk[k] * x->rank[k + 1]);
    omax = std::max(omax, (size_t)sp * x->nk[k] * s);
  }
  zc* C = (zc*)ctx->get_ws("lsk_C", sizeof(zc) * (size_t)s * rmax);
  zc* C2 = (zc*)ctx->get_ws("lsk_C2", sizeof(zc) * (size_t)s * rmax);
  zc* V = (zc*)ctx->get_ws("lsk_V", sizeof(zc) * vmax);
  zc* Om = (zc*)ctx->get_ws("lsk_Om", sizeof(zc) * omax);
  const zc one = Z(1);
  TTF_HIP(hipMemcpyAsync(C, &one, sizeof(zc), hipMemcpyHostToDevice, ctx->stream));
  for (int k = 0; k < d; ++k) {
    const int sp = k == 0 ? 1 : s, r0 = x->rank[k], r1 = x->rank[k + 1], n = x->nk[k];
    // V = C (sp x r0) times the core (r0 x n r1): (sp n) x r1
    zgemm(ctx, OPN, OPN, sp, n * r1, r0, Z(1), C, sp, 0, x->core[k], r0, 0, Z(0), V, sp, 0);
    sketch_core(ctx, Om, (long)sp * n * s, seed, k, 1.0 / std::sqrt((double)s));
    // C' = Omega_k^T V: s x r1 (at the last site r1 = 1: the sketch vector)
    const bool last = k == d - 1;
    zgemm(ctx, OPT, OPN, s, r1, sp * n, last ? alpha : Z(1), Om, (long)sp * n, 0, V, (long)sp * n, 0,
          last && !first ? Z(1) : Z(0), last ? acc : C2, s, 0);
    std::swap(C, C2);
  }
}

double sketch_rel_error(tt_ctx* ctx, int npieces, const zc* coef, const tt_tensor* const* pieces,
                        const tt_tensor* y, uint64_t seed) {
  const int s = LSK_WIDTH;
  zc* acc = (zc*)ctx->get_ws("lsk_acc", sizeof(zc) * 2 * s);
  const uint64_t key = seed ^ 0xD1B54A32D192ED03ull;  // independent of the rounding's sketch
  for (int i = 0; i < npieces; ++i) sketch_vector(ctx, pieces[i], key, coef[i], acc, i == 0);
  sketch_vector(ctx, y, key, Z(1), acc + s, true);
  zc* h = (zc*)ctx->host_scratch(sizeof(zc) * 2 * s);
  TTF_HIP(hipMemcpyAsync(h, acc, sizeof(zc) * 2 * s, hipMemcpyDeviceToHost, ctx->stream));
  TTF_HIP(hipStreamSynchronize(ctx->stream));
  double num = 0.0, den = 0.0;
  for (int j = 0; j < s; ++j) {
    const double dr = h[j].x - h[s + j].x, di = h[j].y - h[s + j].y;
    num += dr * dr + di * di;
    den += h[j].x * h[j].x + h[j].y * h[j].y;
  }
  return den > 0.0 ? std::sqrt(num / den) : 0.0;
}

double round_randomized(tt_ctx* ctx, const tt_tensor* x, const int* widths, uint64_t seed, tt_tensor* y) {
  randomized_into(ctx, x, widths, seed, y);
  const zc one = Z(1);
  const tt_tensor* px = x;
  return sketch_rel_error(ctx, 1, &one, &px, y, seed);
}

}  // namespace

extern "C" {

int tt_round_randomized(tt_ctx* ctx, const tt_tensor* x, const int* widths, uint64_t seed, tt_tensor* y,
                        double* rel_err) {
  if (!ctx || !x || !y || !widths) return TT_EINVAL;
  ABI_TRY
  require(x->d == y->d && x->nk == y->nk && x->n > 0, TT_ESHAPE,
          "tt_round_randomized: shape mismatch (equal mode sizes needed)");
  require(x != y, TT_EINVAL, "tt_round_randomized: y aliases x");
  for (int k = 1; k < x->d; ++k)
    require(widths[k] >= 1 && widths[k] <= y->cap[k], TT_ECAPACITY, "tt_round_randomized: width beyond capacity");
  tt_tensor* yw = widened(ctx, y, "y", false);
  const double e = round_randomized(ctx, widened(ctx, x, "x"), widths, seed, yw);
  narrow_back(ctx, yw, y);
  if (rel_err) *rel_err = e;
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_eval(tt_ctx* ctx, const tt_tensor* x, const int32_t* idx, int64_t npts, double* out) {
  if (!ctx || !x || (npts > 0 && (!idx || !out))) return TT_EINVAL;
  ABI_TRY
  for (int k = 0; k <= x->d; ++k) require(x->rank[k] <= 512, TT_EINVAL, "tt_eval: ranks above 512 unsupported");
  const tt_tensor* xw = widened(ctx, x, "x");
  // the core table travels as kernel arguments: nothing to copy or wait for
  tt_eval_kernel(ctx, xw->d, xw->nk.data(), xw->core.data(), xw->rank.data(), idx, npts, (zc*)out);
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_zgemm(tt_ctx* ctx, int opA, int opB, int M, int N, int K, double alpha_re, double alpha_im, const double* A,
             int64_t lda, int64_t strideA, const double* B, int64_t ldb, int64_t strideB, double beta_re,
             double beta_im, double* C, int64_t ldc, int64_t strideC, int batch) {
  if (!ctx) return TT_EINVAL;
  ABI_TRY
  require(opA >= 0 && opA <= 2 && opB >= 0 && opB <= 2, TT_EINVAL, "tt_zgemm: op must be 0, 1 or 2");
  require(M >= 0 && N >= 0 && K >= 0 && batch >= 1, TT_EINVAL, "tt_zgemm: negative size");
  require(C && ((A && B) || K == 0), TT_EINVAL, "tt_zgemm: null pointer");
  require(lda >= std::max(1, opA == OPN ? M : K) && ldb >= std::max(1, opB == OPN ? K : N) && ldc >= std::max(1, M),
          TT_EINVAL, "tt_zgemm: leading dimension too small");
  zgemm(ctx, opA, opB, M, N, K, Z(alpha_re, alpha_im), (const zc*)A, lda, strideA, (const zc*)B, ldb, strideB,
        Z(beta_re, beta_im), (zc*)C, ldc, strideC, batch);
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_zgemm_mixed(tt_ctx* ctx, int precision, int opA, int opB, int M, int N, int K, double alpha_re,
                   double alpha_im, const double* A, int64_t lda, int64_t strideA, const double* B, int64_t ldb,
                   int64_t strideB, double beta_re, double beta_im, double* C, int64_t ldc, int64_t strideC,
                   int batch) {
  if (!ctx) return TT_EINVAL;
  ABI_TRY
  require(precision == TT_PREC_BF16X3 || precision == TT_PREC_FP16X3 || precision == TT_PREC_FP32, TT_EINVAL,
          "tt_zgemm_mixed: precision must be TT_PREC_BF16X3, TT_PREC_FP16X3 or TT_PREC_FP32");
  require(opA >= 0 && opA <= 2 && opB >= 0 && opB <= 2, TT_EINVAL, "tt_zgemm_mixed: op must be 0, 1 or 2");
  require(M >= 0 && N >= 0 && K >= 0 && batch >= 1, TT_EINVAL, "tt_zgemm_mixed: negative size");
  require(C && ((A && B) || K == 0), TT_EINVAL, "tt_zgemm_mixed: null pointer");
  require(lda >= std::max(1, opA == OPN ? M : K) && ldb >= std::max(1, opB == OPN ? K : N) && ldc >= std::max(1, M),
          TT_EINVAL, "tt_zgemm_mixed: leading dimension too small");
  zgemm_prec(precision, ctx, opA, opB, M, N, K, Z(alpha_re, alpha_im), (const zc*)A, lda, strideA, (const zc*)B, ldb,
             strideB, Z(beta_re, beta_im), (zc*)C, ldc, strideC, batch);
  return TT_OK;
  ABI_CATCH(ctx)
}

}  // extern "C"

// ------------------------------------------------------------ autotuner
namespace {
// the launch shapes a GEMM of this form may take (tile codes as in GemmChoice)
std::vector<std::pair<int, int>> gemm_tiles(int precision) {
  if (precision == TT_PREC_FP64 || precision == TT_PREC_FP32) return {{64, 64}, {128, 32}, {64, 32}, {32, 32}, {32, 64}};
  return {{2, 2}, {1, 2}, {2, 1}, {1, 1}};
}
bool gemm_choice_valid(int precision, int a, int b, int nsplit) {
  if (nsplit < 1 || nsplit > 128) return false;
  for (const auto& t : gemm_tiles(precision))
    if (t.first == a && t.second == b) return true;
  return false;
}
struct ForceGuard {
  ~ForceGuard() { ttf::gemm_force(nullptr); }
};
}  // namespace

extern "C" {


int tt_gemm_autotune(tt_ctx* ctx, int precision, int opA, int opB, int M, int N, int K, int batch, int* choice,
                     double* best_us) {
  if (!ctx) return TT_EINVAL;
  zc* bufs[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  auto release = [&]() {
    (void)hipStreamSynchronize(ctx->stream);
    for (zc*& b : bufs)
      if (b) ctx->dev_free(b), b = nullptr;
    for (hipEvent_t& e : ev)
      if (e) (void)hipEventDestroy(e), e = nullptr;
  };
  try {
    require(precision >= TT_PREC_FP64 && precision <= TT_PREC_FP32, TT_EINVAL, "tt_gemm_autotune: unknown precision");
    require(opA >= 0 && opA <= 2 && opB >= 0 && opB <= 2, TT_EINVAL, "tt_gemm_autotune: op must be 0, 1 or 2");
    require(M >= 1 && N >= 1 && K >= 1 && batch >= 1, TT_EINVAL, "tt_gemm_autotune: sizes must be positive");
    const size_t na = (size_t)M * K * batch, nb = (size_t)K * N * batch, nc = (size_t)M * N * batch;
    require(na <= (1ull << 28) && nb <= (1ull << 28) && nc <= (1ull << 28), TT_EINVAL,
            "tt_gemm_autotune: operands above 2^28 elements");
    const size_t ns[3] = {na, nb, nc};
    for (int i = 0; i < 3; ++i) {
      bufs[i] = (zc*)ctx->dev_alloc(sizeof(zc) * ns[i]);
      if (!bufs[i]) fail(TT_ENOMEM, "tt_gemm_autotune: allocation failed");
    }
    sketch_core(ctx, bufs[0], (long)na, 0x5EEDull, 1, 1.0);
    sketch_core(ctx, bufs[1], (long)nb, 0x5EEDull, 2, 1.0);
    fill_zero(ctx, bufs[2], (long)nc);
    const int lda = opA == OPN ? M : K, ldb = opB == OPN ? K : N;
    TTF_HIP(hipEventCreate(&ev[0]));
    TTF_HIP(hipEventCreate(&ev[1]));
    const int kstep = (precision == TT_PREC_FP64 || precision == TT_PREC_FP32) ? 16 : 32;
    const int kblocks = (K + kstep - 1) / kstep;
    ForceGuard guard;
    double best = 1e300;
    GemmChoice bestc;
    for (const auto& t : gemm_tiles(precision))
      for (int sp = 1; sp <= 128; sp *= 2) {
        if (sp > 1 && sp > kblocks / 2) break;
        GemmChoice c;
        c.a = t.first;
        c.b = t.second;
        c.nsplit = sp;
        gemm_force(&c);
        auto run = [&]() {
          zgemm_prec(precision, ctx, opA, opB, M, N, K, Z(1), bufs[0], lda, (long)M * K, bufs[1], ldb, (long)K * N,
                     Z(0), bufs[2], M, (long)M * N, batch);
        };
        try {
          run();
        } catch (const ttf::Error&) {  // a shape this candidate cannot launch (grid limits)
          gemm_force(nullptr);
          continue;
        }
        double tmin = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
          TTF_HIP(hipEventRecord(ev[0], ctx->stream));
          run();
          TTF_HIP(hipEventRecord(ev[1], ctx->stream));
          TTF_HIP(hipEventSynchronize(ev[1]));
          float ms = 0.f;
          TTF_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
          tmin = std::min(tmin, (double)ms * 1e3);
        }
        gemm_force(nullptr);
        if (tmin < best) {
          best = tmin;
          bestc = c;
        }
      }
    require(best < 1e300, TT_EINVAL, "tt_gemm_autotune: no candidate could be launched");
    const int e[10] = {precision, opA, opB, M, N, K, batch, bestc.a, bestc.b, bestc.nsplit};
    gemm_table_put(e);
    if (choice) {
      choice[0] = bestc.a;
      choice[1] = bestc.b;
      choice[2] = bestc.nsplit;
    }
    if (best_us) *best_us = best;
    release();
    return TT_OK;
  } catch (const ttf::Error& e) {
    release();
    ctx->last_error = e.msg;
    return e.code;
  } catch (...) {
    release();
    return TT_EINVAL;
  }
}

int tt_gemm_table_count(void) { return gemm_table_count(); }

int tt_gemm_table_get(int index, int* entry) {
  if (!entry) return TT_EINVAL;
  return gemm_table_entry(index, entry) ? TT_OK : TT_EINVAL;
}

int tt_gemm_table_set(const int* entry) {
  if (!entry) return TT_EINVAL;
  const int p = entry[0];
  if (p < TT_PREC_FP64 || p > TT_PREC_FP32) return TT_EINVAL;
  if (entry[1] < 0 || entry[1] > 2 || entry[2] < 0 || entry[2] > 2) return TT_EINVAL;
  if (entry[3] < 0 || entry[4] < 0 || entry[5] < 0 || entry[6] < 1) return TT_EINVAL;
  if (!gemm_choice_valid(p, entry[7], entry[8], entry[9])) return TT_EINVAL;
  gemm_table_put(entry);
  return TT_OK;
}

int tt_gemm_table_clear(void) {
  gemm_table_clear();
  return TT_OK;
}

int tt_norm(tt_ctx* ctx, const tt_tensor* x, double* out) {
  if (!ctx || !x || !out) return TT_EINVAL;
  ABI_TRY
  std::string key = shape_key(x->d, x->n, x->cap, -1);
  for (int v : x->nk) key += ";" + std::to_string(v);
  tt_tensor*& tmp = [&]() -> tt_tensor*& {
    std::lock_guard<std::mutex> lock(cache_mutex());
    return norm_cache()[{ctx, key}];
  }();
  if (!tmp) tmp = make_tensor_nk(ctx, x->d, x->nk, x->cap);
  copy_tensor(ctx, x, tmp);
  if (tmp->orth != TT_ORTH_RIGHT && x->d > 1) phase1_right_orth(ctx, tmp);
  *out = core_norm(ctx, tmp, 0);
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_qr(tt_ctx* ctx, int m, int k, const double* A, int64_t lda, double* Q, double* R) {
  if (!ctx) return TT_EINVAL;
  ABI_TRY
  require(m >= k && k >= 1, TT_EINVAL, "tt_qr: need m >= k >= 1");
  require(A && Q && R, TT_EINVAL, "tt_qr: null pointer");
  require(lda >= m, TT_EINVAL, "tt_qr: leading dimension too small");
  tsqr(ctx, m, k, (const zc*)A, lda, (zc*)Q, (zc*)R);
  ctx->sync();
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_svd_small(tt_ctx* ctx, int m, int k, double* B, double* U, double* sigma, int* sweeps) {
  if (!ctx) return TT_EINVAL;
  ABI_TRY
  require(m >= 1 && k >= 1 && m <= 1536 && k <= 1536, TT_EINVAL, "tt_svd_small: need 1 <= m, k <= 1536");
  require(B && U && sigma, TT_EINVAL, "tt_svd_small: null pointer");
  int* sw = (int*)ctx->get_ws("svd_small_sweeps", 64);
  jacobi_svd(ctx, m, k, (zc*)B, (zc*)U, sigma, sw);
  int* h = (int*)ctx->host_scratch(64);
  TTF_HIP(hipMemcpyAsync(h, sw, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  ctx->sync();
  if (sweeps) *sweeps = h[0];
  require(h[0] > 0, TT_ENOCONV, "tt_svd_small: Jacobi did not converge within its sweep limit");
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_svd_small_noalloc(tt_ctx* ctx, int m, int k, double* B, double* U, double* sigma, int* sweeps) {
  if (!ctx) return TT_EINVAL;
  ABI_TRY
  require(B && U && sigma, TT_EINVAL, "tt_svd_small_noalloc: null pointer");
  require(!ctx->profiling, TT_EINVAL, "tt_svd_small_noalloc: profiling records events (allocates); turn it off");
  int h = 0;
  jacobi_svd_noalloc(ctx, m, k, (zc*)B, (zc*)U, sigma, &h);
  if (sweeps) *sweeps = h;
  require(h > 0, TT_ENOCONV, "tt_svd_small_noalloc: Jacobi did not converge within its sweep limit");
  return TT_OK;
  ABI_CATCH(ctx)
}

}  // extern "C"

// ------------------------------------------------------ rank predictor MLP
struct tt_mlp {
  ttf::MlpDev d;
  ttf::DevFree release;  // returns its device memory
};

namespace {
void mlp_free(tt_mlp* m) {
  if (!m) return;
  for (void* ptr : {(void*)m->d.p, (void*)m->d.ph, (void*)m->d.g, (void*)m->d.m, (void*)m->d.v, (void*)m->d.act,
                    (void*)m->d.loss})
    m->release(ptr);
  delete m;
}
}  // namespace

extern "C" {

int tt_mlp_create(tt_ctx* ctx, int n_in, int width, int max_batch, tt_mlp** out) {
  if (!ctx || !out) return TT_EINVAL;
  tt_mlp* m = nullptr;
  ABI_TRY
  *out = nullptr;
  require(n_in >= 1 && n_in <= 1024 && width >= 1 && width <= 1024 && max_batch >= 1, TT_EINVAL,
          "tt_mlp_create: n_in, width in 1..1024, max_batch >= 1");
  m = new tt_mlp;
  m->release = ctx->releaser();
  auto& d = m->d;
  d.n_in = n_in;
  d.width = width;
  d.bcap = max_batch;
  d.nparams = width * n_in + width + width * width + width + width + 1;
  auto alloc = [&](void** p, size_t bytes) {
    *p = ctx->dev_alloc(bytes);
    if (!*p) fail(TT_ENOMEM, "tt_mlp_create: allocation failed");
  };
  // float arrays padded to whole complex values: they are cleared with
  // fill_zero, which writes 16-byte elements
  const size_t padded = 4 * (((size_t)d.nparams + 3) / 4);
  alloc((void**)&d.p, sizeof(float) * padded);
  alloc((void**)&d.ph, sizeof(_Float16) * d.nparams);
  alloc((void**)&d.g, sizeof(float) * d.nparams);
  alloc((void**)&d.m, sizeof(float) * padded);
  alloc((void**)&d.v, sizeof(float) * padded);
  alloc((void**)&d.act, sizeof(float) * ((size_t)max_batch * (4 * (size_t)width + 3)));
  alloc((void**)&d.loss, sizeof(float) * 4);
  fill_zero(ctx, (zc*)d.p, (d.nparams + 3) / 4);
  fill_zero(ctx, (zc*)d.m, (d.nparams + 3) / 4);
  fill_zero(ctx, (zc*)d.v, (d.nparams + 3) / 4);
  ttf::mlp_refresh_half(ctx, d);
  *out = m;
  return TT_OK;
  }
  catch (const ttf::Error& e) {
    ctx->last_error = e.msg;
    mlp_free(m);
    return e.code;
  }
  catch (...) {
    mlp_free(m);
    return TT_EINVAL;
  }
}

int tt_mlp_destroy(tt_mlp* m) {
  if (!m) return TT_EINVAL;
  mlp_free(m);
  return TT_OK;
}

int tt_mlp_param_count(const tt_mlp* m) { return m ? m->d.nparams : TT_EINVAL; }

int tt_mlp_set_params(tt_ctx* ctx, tt_mlp* m, const float* host) {
  if (!ctx || !m || !host) return TT_EINVAL;
  ABI_TRY
  auto& d = m->d;
  TTF_HIP(hipMemcpyAsync(d.p, host, sizeof(float) * d.nparams, hipMemcpyHostToDevice, ctx->stream));
  fill_zero(ctx, (zc*)d.m, (d.nparams + 3) / 4);
  fill_zero(ctx, (zc*)d.v, (d.nparams + 3) / 4);
  d.step = 0;
  ttf::mlp_refresh_half(ctx, d);
  ctx->sync();
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_mlp_get_params(tt_ctx* ctx, const tt_mlp* m, float* host, int as_used) {
  if (!ctx || !m || !host) return TT_EINVAL;
  ABI_TRY
  const auto& d = m->d;
  const float* src = d.p;
  if (as_used) {
    float* tmp = (float*)ctx->get_ws("mlp_tmp", sizeof(float) * d.nparams);
    ttf::mlp_half_values(ctx, d, tmp);
    src = tmp;
  }
  TTF_HIP(hipMemcpyAsync(host, src, sizeof(float) * d.nparams, hipMemcpyDeviceToHost, ctx->stream));
  ctx->sync();
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_mlp_forward(tt_ctx* ctx, tt_mlp* m, const float* x, int B, float* y) {
  if (!ctx || !m || !x || !y) return TT_EINVAL;
  ABI_TRY
  auto& d = m->d;
  require(B >= 1 && B <= d.bcap, TT_EINVAL, "tt_mlp_forward: batch above the capacity given at creation");
  float* h1 = d.act;
  float* h2 = h1 + (long)d.bcap * d.width;
  ttf::mlp_forward(ctx, d, x, B, h1, h2, y);
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_mlp_gradients(tt_ctx* ctx, tt_mlp* m, const float* x, const float* t, int B, float* loss, float* grad) {
  if (!ctx || !m || !x || !t) return TT_EINVAL;
  ABI_TRY
  auto& d = m->d;
  require(B >= 1 && B <= d.bcap, TT_EINVAL, "tt_mlp_gradients: batch above the capacity given at creation");
  ttf::mlp_gradients(ctx, d, x, t, B, d.loss);
  if (loss) TTF_HIP(hipMemcpyAsync(loss, d.loss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
  if (grad) TTF_HIP(hipMemcpyAsync(grad, d.g, sizeof(float) * d.nparams, hipMemcpyDeviceToHost, ctx->stream));
  ctx->sync();
  return TT_OK;
  ABI_CATCH(ctx)
}

int tt_mlp_train(tt_ctx* ctx, tt_mlp* m, const float* x, const float* t, int B, int iters, float lr, float* loss) {
  if (!ctx || !m || !x || !t) return TT_EINVAL;
  ABI_TRY
  auto& d = m->d;
  require(B >= 1 && B <= d.bcap && iters >= 0 && lr > 0.0f, TT_EINVAL, "tt_mlp_train: bad batch, iters or lr");
  for (int it = 0; it < iters; ++it) {
    ttf::mlp_gradients(ctx, d, x, t, B, d.loss);
    ttf::mlp_adam_step(ctx, d, lr);
  }
  if (loss) {
    ttf::mlp_gradients(ctx, d, x, t, B, d.loss);
    TTF_HIP(hipMemcpyAsync(loss, d.loss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
  }
  ctx->sync();
  return TT_OK;
  ABI_CATCH(ctx)
}

}  // extern "C"
