// Small dense factorisation used once per TT bond, one workgroup each.
//
// * jacobi_svd: one-sided (Hestenes) Jacobi SVD of the small square factor
//   R (the "SVD of the R factor" of App. A.4): columns are rotated pairwise
//   until orthogonal; their norms are the singular values and the
//   normalised columns the left singular vectors.  Parallel round-robin
//   ordering, one wavefront per column pair, matrix in LDS when it fits.
#include "common.hpp"
#include "dpp.hpp"

namespace ttf {

constexpr int CHOL_KMAX = 512;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// ------------------------------------------------------------ Jacobi SVD
constexpr int JAC_THREADS = 1024;
constexpr int JAC_GROUPS = JAC_THREADS / 16;
constexpr int JAC_LDS_ELEMS = 9216;  // 144 KiB of complex doubles
constexpr int JAC_MAX_SWEEPS = 60;

// round-robin pairing of players 0..P-1 (P even) in round r
__device__ inline void rr_pair(int P, int r, int i, int& a, int& b) {
  const int M = P - 1;
  if (i == 0) {
    a = 0;
    b = 1 + (r % M);
  } else {
    a = 1 + ((r + i) % M);
    b = 1 + ((r - i + M) % M);
  }
}

// One-sided Jacobi: one 16-lane group per column pair (64 pairs in flight),
// 16-lane DPP reductions; the pairs of a round are disjoint, rounds are
// separated by a barrier.
template <bool IN_LDS>
__global__ __launch_bounds__(JAC_THREADS) void jacobi_kernel(int m, int k, zc* __restrict__ Bg,
                                                             zc* __restrict__ U, double* __restrict__ sigma,
                                                             int* __restrict__ sweeps_out) {
  extern __shared__ double2 lds[];
  __shared__ int rotated;
  __shared__ double norms[CHOL_KMAX];
  zc* B = IN_LDS ? lds : Bg;
  const int t = threadIdx.x, g = t >> 4, l16 = t & 15;
  if (IN_LDS)
    for (long e = t; e < (long)m * k; e += blockDim.x) B[e] = Bg[e];
  __syncthreads();
  const int P = (k + 1) & ~1;
  const double tol = 1e-15 * sqrt((double)m);
  int sweep = 0;
  for (; sweep < JAC_MAX_SWEEPS; ++sweep) {
    if (t == 0) rotated = 0;
    __syncthreads();
    int any = 0;
    for (int r = 0; r < P - 1; ++r) {
      for (int i = g; i < P / 2; i += JAC_GROUPS) {
        int p, q;
        rr_pair(P, r, i, p, q);
        if (p >= k || q >= k) continue;
        zc* x = B + (long)m * p;
        zc* y = B + (long)m * q;
        double al = 0, be = 0, gr = 0, gi = 0;
        for (int row = l16; row < m; row += 16) {
          const zc a = x[row], c = y[row];
          al += a.x * a.x + a.y * a.y;
          be += c.x * c.x + c.y * c.y;
          gr += a.x * c.x + a.y * c.y;  // conj(x) * y
          gi += a.x * c.y - a.y * c.x;
        }
        al = row16_sum(al);
        be = row16_sum(be);
        gr = row16_sum(gr);
        gi = row16_sum(gi);
        const double gg = sqrt(gr * gr + gi * gi);
        if (gg <= tol * sqrt(al * be) || gg == 0.0) continue;
        any = 1;
        // complex rotation orthogonalising columns p and q
        const double zeta = (be - al) / (2.0 * gg);
        const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
        const double er = gr / gg, ei = gi / gg;  // e^{i phi}
        for (int row = l16; row < m; row += 16) {
          const zc a = x[row], c = y[row];
          // x' = cs x - sn e^{-i phi} y ; y' = sn e^{i phi} x + cs y
          zc xn, yn;
          xn.x = cs * a.x - sn * (er * c.x + ei * c.y);
          xn.y = cs * a.y - sn * (er * c.y - ei * c.x);
          yn.x = sn * (er * a.x - ei * a.y) + cs * c.x;
          yn.y = sn * (er * a.y + ei * a.x) + cs * c.y;
          x[row] = xn;
          y[row] = yn;
        }
      }
      __syncthreads();
    }
    if (any) atomicOr(&rotated, 1);
    __syncthreads();
    if (!rotated) break;
  }
  // singular values = column norms
  for (int c = g; c < k; c += JAC_GROUPS) {
    double sq = 0;
    for (int row = l16; row < m; row += 16) {
      const zc a = B[row + (long)m * c];
      sq += a.x * a.x + a.y * a.y;
    }
    sq = row16_sum(sq);
    if (l16 == 0) norms[c] = sqrt(sq);
  }
  __syncthreads();
  // sort by decreasing norm (ties by index) and normalise into U
  for (int c = g; c < k; c += JAC_GROUPS) {
    const double v = norms[c];
    int pos = 0;
    for (int o = 0; o < k; ++o) {
      const double w = norms[o];
      pos += (w > v) || (w == v && o < c);
    }
    const double inv = v > 0 ? 1.0 / v : 0.0;
    for (int row = l16; row < m; row += 16) {
      const zc a = B[row + (long)m * c];
      U[row + (long)m * pos] = make_double2(a.x * inv, a.y * inv);
    }
    if (l16 == 0) sigma[pos] = v;
  }
  if (t == 0) *sweeps_out = sweep + 1;
}

void jacobi_svd(tt_ctx* ctx, int m, int k, zc* B, zc* U, double* sigma, int* sweeps) {
  if (k <= 0) return;
  if (k > CHOL_KMAX) fail(TT_EINVAL, "jacobi_svd: rank above the supported maximum of 512");
  static int lds_limit = -1;
  if (lds_limit < 0) {
    int dev = 0, v = 0;
    TTF_HIP(hipGetDevice(&dev));
    TTF_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    lds_limit = v;
  }
  // per sweep: k(k-1)/2 pairs x (16 m for the inner products + 28 m for the rotation)
  KTimer kt(ctx, "jacobi", 0.0, 0.0);
  const long need = (long)sizeof(zc) * m * k + 8 * CHOL_KMAX + 64;
  if ((long)m * k <= JAC_LDS_ELEMS && need <= lds_limit) {
    const size_t lds = sizeof(zc) * (size_t)m * k;
    hipLaunchKernelGGL(jacobi_kernel<true>, dim3(1), dim3(JAC_THREADS), lds, ctx->stream, m, k, B, U, sigma,
                       sweeps);
  } else {
    hipLaunchKernelGGL(jacobi_kernel<false>, dim3(1), dim3(JAC_THREADS), 0, ctx->stream, m, k, B, U, sigma,
                       sweeps);
  }
  TTF_HIP(hipGetLastError());
}

// ------------------------------------------------------------- helpers
__global__ void set_identity_kernel(zc* A, int m, int k, long lda) {
  const long total = (long)m * k;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e % m), c = (int)(e / m);
    A[r + lda * c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
}

void set_identity(tt_ctx* ctx, zc* A, int m, int k, long lda) {
  const long total = (long)m * k;
  if (total <= 0) return;
  const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(set_identity_kernel, dim3(blocks), dim3(256), 0, ctx->stream, A, m, k, lda);
  TTF_HIP(hipGetLastError());
}

__global__ void copy_matrix_kernel(const zc* src, long lds_, zc* dst, long ldd, int m, int k) {
  const long total = (long)m * k;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e % m), c = (int)(e / m);
    dst[r + ldd * c] = src[r + lds_ * c];
  }
}

void copy_matrix(tt_ctx* ctx, const zc* src, long lds_, zc* dst, long ldd, int m, int k) {
  const long total = (long)m * k;
  if (total <= 0) return;
  const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(copy_matrix_kernel, dim3(blocks), dim3(256), 0, ctx->stream, src, lds_, dst, ldd, m, k);
  TTF_HIP(hipGetLastError());
}

__global__ __launch_bounds__(1024) void frob_norm2_kernel(const zc* x, long n, double* out) {
  __shared__ double red[16];
  double s = 0;
  for (long e = threadIdx.x; e < n; e += blockDim.x) s += x[e].x * x[e].x + x[e].y * x[e].y;
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s;
}

void frob_norm2(tt_ctx* ctx, const zc* x, long n, double* out_dev) {
  hipLaunchKernelGGL(frob_norm2_kernel, dim3(1), dim3(1024), 0, ctx->stream, x, n, out_dev);
  TTF_HIP(hipGetLastError());
}

}  // namespace ttf
