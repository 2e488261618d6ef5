// TT-format kernels: concatenation (sums), pointwise evaluation, initial
// condition, exact operator application, the MPO gathers of the sketched
// application, and the Gaussian sketch generator.
#include "common.hpp"
#include "rng.hpp"

namespace ttf {

// ---------------------------------------------------------------- concat
// Sum by concatenation (App. A.1): first cores side by side (scaled by the
// term coefficients), middle cores block diagonal, last cores stacked.
constexpr int MAX_TERMS = 8;
struct ConcatArgs {
  const zc* src[MAX_TERMS];
  int r0[MAX_TERMS], r1[MAX_TERMS];
  int off0[MAX_TERMS + 1], off1[MAX_TERMS + 1];
  zc coef[MAX_TERMS];
  int nterms, kind, n, R0, R1;
};

__global__ void concat_kernel(ConcatArgs a, zc* dst) {
  const long total = (long)a.R0 * a.n * a.R1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int p = (int)(e % a.R0);
    const long rest = e / a.R0;
    const int i = (int)(rest % a.n), q = (int)(rest / a.n);
    int tp = 0, tq = 0;
    while (tp + 1 < a.nterms && p >= a.off0[tp + 1]) ++tp;
    while (tq + 1 < a.nterms && q >= a.off1[tq + 1]) ++tq;
    zc v = make_double2(0.0, 0.0);
    int t = -1;
    if (a.kind == 0) t = tq;            // first core: 1 x n x sum r1
    else if (a.kind == 2) t = tp;       // last core: sum r0 x n x 1
    else if (a.kind == 1) t = (tp == tq) ? tp : -1;  // block diagonal
    else t = -2;                        // d == 1: plain weighted sum
    if (t >= 0) {
      const int pa = (a.kind == 0) ? 0 : p - a.off0[t];
      const int qb = (a.kind == 2) ? 0 : q - a.off1[t];
      const zc x = a.src[t][pa + (long)a.r0[t] * (i + (long)a.n * qb)];
      if (a.kind == 0) {
        const zc c = a.coef[t];
        v = make_double2(c.x * x.x - c.y * x.y, c.x * x.y + c.y * x.x);
      } else {
        v = x;
      }
    } else if (t == -2) {
      for (int s = 0; s < a.nterms; ++s) {
        const zc x = a.src[s][i];
        const zc c = a.coef[s];
        v.x += c.x * x.x - c.y * x.y;
        v.y += c.x * x.y + c.y * x.x;
      }
    }
    dst[e] = v;
  }
}

void concat_core(tt_ctx* ctx, int nterms, const zc* const* src, const int* r0s, const int* r1s,
                 const zc* coefs, int kind, int n, zc* dst, int R0, int R1) {
  if (nterms > MAX_TERMS) fail(TT_EINVAL, "concat: too many terms");
  ConcatArgs a;
  a.nterms = nterms;
  a.kind = kind;
  a.n = n;
  a.R0 = R0;
  a.R1 = R1;
  a.off0[0] = a.off1[0] = 0;
  for (int t = 0; t < nterms; ++t) {
    a.src[t] = src[t];
    a.r0[t] = r0s[t];
    a.r1[t] = r1s[t];
    a.coef[t] = coefs[t];
    a.off0[t + 1] = a.off0[t] + ((kind == 0 || kind == 3) ? 0 : r0s[t]);
    a.off1[t + 1] = a.off1[t] + ((kind == 2 || kind == 3) ? 0 : r1s[t]);
  }
  if (kind == 0 || kind == 3)
    for (int t = 0; t <= nterms; ++t) a.off0[t] = 0;
  if (kind == 2 || kind == 3)
    for (int t = 0; t <= nterms; ++t) a.off1[t] = 0;
  const long total = (long)R0 * n * R1;
  const int blocks = (int)std::min<long>((total + 255) / 256, 16384);
  KTimer kt(ctx, "concat", 0.0, 32.0 * total);
  hipLaunchKernelGGL(concat_kernel, dim3(blocks), dim3(256), 0, ctx->stream, a, dst);
  TTF_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ eval
// f[i_1..i_d] = C_1[0,i_1,:] C_2[:,i_2,:] ... C_d[:,i_d,0] (App. A.1), one
// wavefront per point, the running row vector in LDS.
constexpr int EVAL_RMAX = 512;
// passed by value (about 2 KB of kernel arguments): no device copy of the
// core table, so the read-out needs no synchronisation
struct EvalArgs {
  const zc* cores[TT_MAX_D];
  int ranks[TT_MAX_D + 1];
  int nk[TT_MAX_D];
  const int32_t* idx;
  long npts;
  int d;
  zc* out;
};

__global__ __launch_bounds__(256) void eval_kernel(EvalArgs a) {
  __shared__ zc buf[4][2][EVAL_RMAX];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (long pt = blockIdx.x * 4L + wave; pt < a.npts; pt += gridDim.x * 4L) {
    zc* cur = buf[wave][0];
    zc* nxt = buf[wave][1];
    if (lane == 0) cur[0] = make_double2(1.0, 0.0);
    __builtin_amdgcn_wave_barrier();
    bool bad = false;
    for (int k = 0; k < a.d; ++k) {
      const int r0 = a.ranks[k], r1 = a.ranks[k + 1];
      const int nk = a.nk[k];
      int i = a.idx[pt * a.d + k];
      if (i < 0 || i >= nk) {  // out-of-range index: result is NaN
        bad = true;
        i = 0;
      }
      const zc* C = a.cores[k] + (long)r0 * i;
      for (int b = lane; b < r1; b += 64) {
        double sr = 0, si = 0;
        const zc* col = C + (long)r0 * nk * b;
        for (int q = 0; q < r0; ++q) {
          const zc v = cur[q], c = col[q];
          sr += v.x * c.x - v.y * c.y;
          si += v.x * c.y + v.y * c.x;
        }
        nxt[b] = make_double2(sr, si);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      zc* tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
    if (lane == 0) a.out[pt] = bad ? make_double2(__builtin_nan(""), __builtin_nan("")) : cur[0];
    __builtin_amdgcn_wave_barrier();
  }
}

void tt_eval_kernel(tt_ctx* ctx, int d, const int* nk, const zc* const* cores, const int* ranks,
                    const int32_t* idx, int64_t npts, zc* out) {
  if (npts <= 0) return;
  EvalArgs a{};
  for (int k = 0; k < d; ++k) {
    a.cores[k] = cores[k];
    a.nk[k] = nk[k];
  }
  for (int k = 0; k <= d; ++k) a.ranks[k] = ranks[k];
  a.idx = idx;
  a.npts = (long)npts;
  a.d = d;
  a.out = out;
  const int blocks = (int)std::min<long>((npts + 3) / 4, 65536);
  KTimer kt(ctx, "eval", 0.0, 0.0);
  hipLaunchKernelGGL(eval_kernel, dim3(blocks), dim3(256), 0, ctx->stream, a);
  TTF_HIP(hipGetLastError());
}

// ------------------------------------------------- storage conversion
__global__ void widen_kernel(const float2* __restrict__ src, zc* __restrict__ dst, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const float2 v = src[e];
    dst[e] = make_double2((double)v.x, (double)v.y);
  }
}

__global__ void narrow_kernel(const zc* __restrict__ src, float2* __restrict__ dst, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const zc v = src[e];
    dst[e] = make_float2((float)v.x, (float)v.y);
  }
}

void widen_c64(tt_ctx* ctx, const void* src, zc* dst, long n) {
  if (n <= 0) return;
  const int blocks = (int)std::min<long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(widen_kernel, dim3(blocks), dim3(256), 0, ctx->stream, (const float2*)src, dst, n);
  TTF_HIP(hipGetLastError());
}

void narrow_c128(tt_ctx* ctx, const zc* src, void* dst, long n) {
  if (n <= 0) return;
  const int blocks = (int)std::min<long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(narrow_kernel, dim3(blocks), dim3(256), 0, ctx->stream, src, (float2*)dst, n);
  TTF_HIP(hipGetLastError());
}

// ---------------------------------------------------------- init helpers
__global__ void gaussian_factor_kernel(zc* core, int n, double L, double mu, double sigma) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = -L + 2.0 * L * i / (n - 1);
  const double mag = exp(-0.5 * sigma * sigma * a * a);
  double s, c;
  sincos(mu * a, &s, &c);
  core[i] = make_double2(mag * c, mag * s);
}

// one rank-one factor of the CDF equation's initial condition: the
// Gaussian CDF 0.5 (1 + erf(u / (sigma sqrt 2))) on u_i = -box + 2 box i/(n-1)
__global__ void cdf_gaussian_factor_kernel(zc* core, int n, double box, double sigma) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double u = -box + 2.0 * box * i / (n - 1);
  core[i] = make_double2(0.5 * (1.0 + erf(u / (sigma * sqrt(2.0)))), 0.0);
}

void cdf_gaussian_factor(tt_ctx* ctx, zc* core, int n, double box, double sigma) {
  hipLaunchKernelGGL(cdf_gaussian_factor_kernel, dim3((n + 127) / 128), dim3(128), 0, ctx->stream, core, n, box,
                     sigma);
  TTF_HIP(hipGetLastError());
}

// core k of the nearest-neighbour product TT of a Gaussian characteristic
// function with tridiagonal covariance: entry (p, i, q) of the r0 x n x r1
// core (layout p + r0 (i + n q)) is
//   exp(-c a_p a_i) exp(i mu a_i - sigma^2 a_i^2 / 2) [i == q]
// where the left index p carries the previous coordinate (r0 = its n, or 1
// with c = 0 at the first core) and the right index repeats the current one
// (r1 = n, or 1 at the last core); a_i = -L + 2 L i / (n - 1) on every axis.
__global__ void nn_gaussian_core_kernel(zc* core, int r0, int n, int r1, int nprev, double L, double mu,
                                        double sigma, double c) {
  const long total = (long)r0 * n * r1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int p = (int)(e % r0), i = (int)((e / r0) % n), q = (int)(e / ((long)r0 * n));
    if (r1 > 1 && q != i) {
      core[e] = make_double2(0.0, 0.0);
      continue;
    }
    const double a = -L + 2.0 * L * i / (n - 1);
    const double ap = (r0 > 1) ? -L + 2.0 * L * p / (nprev - 1) : 0.0;
    const double mag = exp(-0.5 * sigma * sigma * a * a - c * ap * a);
    double s, co;
    sincos(mu * a, &s, &co);
    core[e] = make_double2(mag * co, mag * s);
  }
}

void nn_gaussian_core(tt_ctx* ctx, zc* core, int r0, int n, int r1, int nprev, double L, double mu, double sigma,
                      double c) {
  const long total = (long)r0 * n * r1;
  const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(nn_gaussian_core_kernel, dim3(blocks), dim3(256), 0, ctx->stream, core, r0, n, r1, nprev, L,
                     mu, sigma, c);
  TTF_HIP(hipGetLastError());
}

void gaussian_factor(tt_ctx* ctx, zc* core, int n, double L, double mu, double sigma) {
  hipLaunchKernelGGL(gaussian_factor_kernel, dim3((n + 127) / 128), dim3(128), 0, ctx->stream, core, n, L, mu,
                     sigma);
  TTF_HIP(hipGetLastError());
}

__global__ void identity_core_kernel(zc* core, int n, int r1) {
  const long R0 = (long)n * r1;
  const long total = R0 * n * r1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long p = e % R0;
    const long rest = e / R0;
    const int i = (int)(rest % n), b = (int)(rest / n);
    core[e] = make_double2(p == i + (long)n * b ? 1.0 : 0.0, 0.0);
  }
}

void identity_core(tt_ctx* ctx, zc* core, int n, int r1) {
  const long total = (long)n * r1 * n * r1;
  const int blocks = (int)std::min<long>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(identity_core_kernel, dim3(blocks), dim3(256), 0, ctx->stream, core, n, r1);
  TTF_HIP(hipGetLastError());
}

// ------------------------------------------------------- exact apply
// Y[(a + r0 alpha), i, (b + r1 beta)] = sum_{ops of block} c (O C[a,:,b])[i]
__global__ void zero_kernel(zc* y, long total) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
    y[e] = make_double2(0.0, 0.0);
}

__global__ void apply_exact_kernel(const DevBlock* __restrict__ blocks, const DevBlockOp* __restrict__ bops,
                                   int nblocks, const int* __restrict__ tptr, const int* __restrict__ tcol,
                                   const double* __restrict__ tw,
                                   const zc* __restrict__ x, int n, int r0, int r1, int R0, int R1,
                                   zc* __restrict__ y) {
  const long per = (long)r0 * n * r1;
  const long total = per * nblocks;
  const long ld0 = (long)R0 * r0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int bk = (int)(e / per);
    const long loc = e - bk * per;
    const int a = (int)(loc % r0);
    const long rest = loc / r0;
    const int i = (int)(rest % n), b = (int)(rest / n);
    const DevBlock blk = blocks[bk];
    double sr = 0, si = 0;
    for (int o = 0; o < blk.count; ++o) {
      const DevBlockOp bo = bops[blk.first + o];
      double vr = 0, vi = 0;
      const int row = bo.lop * n + i;
      for (int ti = tptr[row]; ti < tptr[row + 1]; ++ti) {
        const double w = tw[ti];
        const zc xv = x[a + (long)r0 * (tcol[ti] + (long)n * b)];
        vr += w * xv.x;
        vi += w * xv.y;
      }
      sr += bo.cre * vr - bo.cim * vi;
      si += bo.cre * vi + bo.cim * vr;
    }
    const long p = a + (long)r0 * blk.alpha;
    const long q = b + (long)r1 * blk.beta;
    y[p + ld0 * (i + (long)n * q)] = make_double2(sr, si);
  }
}

void apply_exact_core(tt_ctx* ctx, const tt_op* op, int site, const zc* x, int r0, int r1, zc* y) {
  const int n = op->n, R0 = op->R[site], R1 = op->R[site + 1];
  const auto& sd = op->dev[site];
  const long total_out = (long)R0 * r0 * n * R1 * r1;
  int blocks = (int)std::min<long>((total_out + 255) / 256, 16384);
  KTimer kt(ctx, "apply_exact", 0.0, 16.0 * total_out);
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, ctx->stream, y, total_out);
  const long total = (long)r0 * n * r1 * sd.nblocks;
  blocks = (int)std::min<long>((total + 255) / 256, 16384);
  if (total > 0)
    hipLaunchKernelGGL(apply_exact_kernel, dim3(blocks), dim3(256), 0, ctx->stream, sd.blocks, sd.bops, sd.nblocks,
                       op->d_tap_ptr, op->d_tap_col, op->d_tap_w, x, n, r0, r1, R0, R1, y);
  TTF_HIP(hipGetLastError());
}

// --------------------------------------------------- sketched-apply gathers
// Left:  W[j, i, b, beta] = sum_{(alpha, o, c) -> beta} c * sum_t w_t V[j, alpha, col_t, b]
//        V layout j + l (alpha + R0 (i' + n b)); W layout j + l (i + n (b + r1 beta)).
// One workgroup per (chunk of 256 consecutive output rows, automaton index,
// outer index): the automaton entries of a workgroup are uniform (scalar
// loads, no divergence), the per-element index arithmetic is 32-bit, and
// consecutive workgroups run through every automaton index of one outer
// index before the next, so the input slice of that outer index is reused
// from the caches.  Workgroups loop over (chunk, index, outer) triples when
// there are more than the grid holds.
constexpr int GATHER_WG = 256;
constexpr long GATHER_MAX_GRID = 1L << 20;

__global__ __launch_bounds__(GATHER_WG) void gather_left_kernel(
    const int* __restrict__ ptr, const DevEntry* __restrict__ ent, const int* __restrict__ tptr,
    const int* __restrict__ tcol, const double* __restrict__ tw, const zc* __restrict__ V, zc* __restrict__ W, int l,
    int n, int r1, int R0, int R1) {
  const int rows = l * n;  // (j, i) pairs, j fastest: W is contiguous over them
  const int nchunk = (rows + GATHER_WG - 1) / GATHER_WG;
  const long nwg = (long)nchunk * R1 * r1;
  for (long wg = blockIdx.x; wg < nwg; wg += gridDim.x) {
    const int chunk = (int)(wg % nchunk);
    const long rest = wg / nchunk;
    const int beta = (int)(rest % R1), b = (int)(rest / R1);
    const int idx = chunk * GATHER_WG + (int)threadIdx.x;
    if (idx >= rows) continue;
    const int j = idx % l, i = idx / l;
    double sr = 0, si = 0;
    for (int q = ptr[beta]; q < ptr[beta + 1]; ++q) {
      const DevEntry en = ent[q];
      double vr = 0, vi = 0;
      const int row = en.lop * n + i;
      for (int ti = tptr[row]; ti < tptr[row + 1]; ++ti) {
        const double w = tw[ti];
        const zc v = V[j + (long)l * (en.other + R0 * (tcol[ti] + n * b))];
        vr += w * v.x;
        vi += w * v.y;
      }
      sr += en.cre * vr - en.cim * vi;
      si += en.cre * vi + en.cim * vr;
    }
    W[idx + (long)rows * (b + (long)r1 * beta)] = make_double2(sr, si);
  }
}

void gather_left(tt_ctx* ctx, const tt_op* op, int site, const zc* V, zc* W, int l, int r1) {
  const int n = op->n, R0 = op->R[site], R1 = op->R[site + 1];
  const long total = (long)l * n * r1 * R1;
  const long nwg = (long)((l * n + GATHER_WG - 1) / GATHER_WG) * R1 * r1;
  if (nwg == 0) return;
  KTimer kt(ctx, "gather_left", 0.0, 32.0 * total);
  hipLaunchKernelGGL(gather_left_kernel, dim3((unsigned)std::min(nwg, GATHER_MAX_GRID)), dim3(GATHER_WG), 0,
                     ctx->stream, op->dev[site].in_ptr, op->dev[site].in_ent, op->d_tap_ptr, op->d_tap_col,
                     op->d_tap_w, V, W, l, n, r1, R0, R1);
  TTF_HIP(hipGetLastError());
}

// Right: Z[a, alpha, i, q] = sum_{alpha -> (beta, o, c)} c * sum_t w_t V2[a, col_t, beta, q]
//        V2 layout a + r0 (i' + n (beta + R1 q)); Z layout a + r0 (alpha + R0 (i + n q)).
//        Workgroups as on the left, over (chunk of (a, i) pairs, alpha, q).
__global__ __launch_bounds__(GATHER_WG) void gather_right_kernel(
    const int* __restrict__ ptr, const DevEntry* __restrict__ ent, const int* __restrict__ tptr,
    const int* __restrict__ tcol, const double* __restrict__ tw, const zc* __restrict__ V2, zc* __restrict__ Z,
    int r0, int n, int s, int R0, int R1) {
  const int rows = r0 * n;  // (a, i) pairs, a fastest
  const int nchunk = (rows + GATHER_WG - 1) / GATHER_WG;
  const long nwg = (long)nchunk * R0 * s;
  for (long wg = blockIdx.x; wg < nwg; wg += gridDim.x) {
    const int chunk = (int)(wg % nchunk);
    const long rest = wg / nchunk;
    const int alpha = (int)(rest % R0), q = (int)(rest / R0);
    const int idx = chunk * GATHER_WG + (int)threadIdx.x;
    if (idx >= rows) continue;
    const int a = idx % r0, i = idx / r0;
    double sr = 0, si = 0;
    for (int p = ptr[alpha]; p < ptr[alpha + 1]; ++p) {
      const DevEntry en = ent[p];
      double vr = 0, vi = 0;
      const int row = en.lop * n + i;
      for (int ti = tptr[row]; ti < tptr[row + 1]; ++ti) {
        const double w = tw[ti];
        const zc v = V2[a + (long)r0 * (tcol[ti] + (long)n * (en.other + (long)R1 * q))];
        vr += w * v.x;
        vi += w * v.y;
      }
      sr += en.cre * vr - en.cim * vi;
      si += en.cre * vi + en.cim * vr;
    }
    Z[a + (long)r0 * (alpha + (long)R0 * (i + (long)n * q))] = make_double2(sr, si);
  }
}

void gather_right(tt_ctx* ctx, const tt_op* op, int site, const zc* V2, zc* Z, int r0, int s) {
  const int n = op->n, R0 = op->R[site], R1 = op->R[site + 1];
  const long total = (long)r0 * R0 * n * s;
  const long nwg = (long)((r0 * n + GATHER_WG - 1) / GATHER_WG) * R0 * s;
  if (nwg == 0) return;
  KTimer kt(ctx, "gather_right", 0.0, 32.0 * total);
  hipLaunchKernelGGL(gather_right_kernel, dim3((unsigned)std::min(nwg, GATHER_MAX_GRID)), dim3(GATHER_WG), 0,
                     ctx->stream, op->dev[site].out_ptr, op->dev[site].out_ent, op->d_tap_ptr, op->d_tap_col,
                     op->d_tap_w, V2, Z, r0, n, s, R0, R1);
  TTF_HIP(hipGetLastError());
}

// ------------------------------------------------------ Gaussian sketch
__global__ void sketch_kernel(zc* w, long count, uint32_t k0, uint32_t k1, uint32_t site, double scale) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) {
    const zc z = philox_gaussian((uint64_t)e, site, k0, k1);
    w[e] = make_double2(z.x * scale, z.y * scale);
  }
}

void sketch_core(tt_ctx* ctx, zc* w, long count, uint64_t seed, int site, double scale) {
  const int blocks = (int)std::min<long>((count + 255) / 256, 8192);
  hipLaunchKernelGGL(sketch_kernel, dim3(blocks), dim3(256), 0, ctx->stream, w, count, (uint32_t)seed,
                     (uint32_t)(seed >> 32), (uint32_t)site, scale);
  TTF_HIP(hipGetLastError());
}

// ------------------------------------------- power-of-two normalisation
// The sketch chains of the sketched apply multiply by operator and core
// factors site after site; their magnitude drifts geometrically along the
// train.  Rescaling by a power of two (exact in floating point) keeps them
// near 1, which the FP32 accumulation of the mixed-precision contractions
// needs; e[0] receives the exponent and, with accumulate, e[1] sums them.
__global__ void pow2_init_kernel(int* e) { e[0] = -1100; }

__global__ void pow2_maxexp_kernel(const zc* __restrict__ x, long n, int* __restrict__ e) {
  int mx = -1100;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double a = fmax(fabs(x[i].x), fabs(x[i].y));
    if (a > 0.0 && a <= 1.7976931348623157e308) mx = max(mx, ilogb(a));
  }
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(e, mx);
}

__global__ void pow2_scale_kernel(zc* __restrict__ x, long n, int* __restrict__ e, int accumulate) {
  const int ex = e[0];
  if (ex <= -1100) return;  // all zero
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const zc v = x[i];
    x[i] = make_double2(ldexp(v.x, -ex), ldexp(v.y, -ex));
  }
  if (accumulate && blockIdx.x == 0 && threadIdx.x == 0) e[1] += ex;
}

__global__ void pow2_apply_kernel(zc* __restrict__ x, long n, const int* __restrict__ e) {
  const int ex = e[1];
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const zc v = x[i];
    x[i] = make_double2(ldexp(v.x, ex), ldexp(v.y, ex));
  }
}

void pow2_normalize(tt_ctx* ctx, zc* x, long n, int* e, bool accumulate) {
  if (n <= 0) return;
  const int blocks = (int)std::min<long>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(pow2_init_kernel, dim3(1), dim3(1), 0, ctx->stream, e);
  hipLaunchKernelGGL(pow2_maxexp_kernel, dim3(blocks), dim3(256), 0, ctx->stream, x, n, e);
  hipLaunchKernelGGL(pow2_scale_kernel, dim3(blocks), dim3(256), 0, ctx->stream, x, n, e, accumulate ? 1 : 0);
  TTF_HIP(hipGetLastError());
}

void pow2_restore(tt_ctx* ctx, zc* x, long n, const int* e) {
  if (n <= 0) return;
  const int blocks = (int)std::min<long>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(pow2_apply_kernel, dim3(blocks), dim3(256), 0, ctx->stream, x, n, e);
  TTF_HIP(hipGetLastError());
}

}  // namespace ttf
