// QR factorisations for the orthogonalisations of the TT sweeps: the QR of
// V(C) and the LQ of H(C) (App. A.1, Alg. 1 and Alg. 2).
//
// * Panel Householder QR (pt_leaves / pt_assemble): tall blocks of at most
//   32 columns, tree-reduced as in the paper's TSQR (App. A.3) but inside
//   one GPU: leaves of at most 256 rows are factored by separate
//   workgroups, their stacked R factors are factored again, and Q is
//   assembled top-down.  Householder reflections keep Q orthonormal to
//   working precision whatever the rank of the panel.
// * Helpers of the block Gram-Schmidt QR that orthogonalises wide matrices
//   panel by panel (the host loop is in capi.cpp).
#include "common.hpp"
#include "dpp.hpp"
#include "rng.hpp"

namespace ttf {

constexpr int PT_ROWS = 256;
constexpr int PT_COLS = 32;

// sum over a 32-lane half of a wavefront, bitwise identical in every lane
__device__ inline double hw_sum(double x) {
  x = row16_sum(x);
  x += __shfl_xor(x, 16, 64);
  return x;
}

// Householder QR of one row block per workgroup.  Leaf i owns rows
// [i m / P, (i+1) m / P) of the m x k matrix at Qbase (ld ldq), k <= 32 and
// every leaf 32..256 rows; it leaves the explicit Q factor in place and
// writes R_i (k x k upper) at Rbase + i strideR (ld ldr).
// Column c lives in the registers of half-wavefront c (8 rows per lane).
// Step j: the owner of column j forms reflector j (LAPACK zlarfg
// convention, H = I - tau v v^H with v_j = 1) and publishes v and tau in
// LDS; after one barrier every later column applies H^H.  The explicit Q
// is then built column by column, q_c = H_0 ... H_c e_c, with no further
// synchronisation.
__global__ __launch_bounds__(1024) void pt_leaf_kernel(zc* __restrict__ Qbase, long ldq, int nleaves, int m, int k,
                                                       zc* __restrict__ Rbase, long ldr, long strideR) {
  constexpr int RPL = PT_ROWS / 32;
  __shared__ zc V[PT_COLS][PT_ROWS];
  __shared__ zc tau[PT_COLS];
  const int leaf = blockIdx.x;
  const long r0 = (long)leaf * m / nleaves, r1 = (long)(leaf + 1) * m / nleaves;
  const int b = (int)(r1 - r0);
  zc* G = Qbase + r0;
  zc* R = Rbase + strideR * leaf;
  const int h = threadIdx.x >> 5, l = threadIdx.x & 31;
  const bool active = h < k;
  zc x[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = l + 32 * i;
    x[i] = (active && row < b) ? G[row + ldq * h] : make_double2(0.0, 0.0);
  }
  for (int j = 0; j < k; ++j) {
    if (h == j) {
      double xs = 0, ar = 0, ai = 0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = l + 32 * i;
        if (row > j) xs += x[i].x * x[i].x + x[i].y * x[i].y;
        if (row == j) {
          ar = x[i].x;
          ai = x[i].y;
        }
      }
      xs = hw_sum(xs);
      ar = hw_sum(ar);
      ai = hw_sum(ai);
      zc tj, sc;
      double be;
      if (xs == 0.0 && ai == 0.0) {
        tj = make_double2(0.0, 0.0);
        be = ar;
        sc = make_double2(0.0, 0.0);
      } else {
        const double nrm = sqrt(ar * ar + ai * ai + xs);
        be = (ar >= 0.0) ? -nrm : nrm;
        tj = make_double2((be - ar) / be, -ai / be);
        const double dr = ar - be, di = ai;
        const double den = dr * dr + di * di;
        sc = make_double2(dr / den, -di / den);
      }
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = l + 32 * i;
        zc v;
        if (row < j) {
          v = make_double2(0.0, 0.0);
        } else if (row == j) {
          v = make_double2(1.0, 0.0);
          x[i] = make_double2(be, 0.0);
        } else {
          v = make_double2(x[i].x * sc.x - x[i].y * sc.y, x[i].x * sc.y + x[i].y * sc.x);
        }
        V[j][row] = v;
      }
      if (l == 0) tau[j] = tj;
    }
    __syncthreads();
    if (h > j && active) {
      const zc t = make_double2(tau[j].x, -tau[j].y);
      if (t.x != 0.0 || t.y != 0.0) {
        double dr = 0, di = 0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const zc w = V[j][l + 32 * i];
          dr += w.x * x[i].x + w.y * x[i].y;
          di += w.x * x[i].y - w.y * x[i].x;
        }
        dr = hw_sum(dr);
        di = hw_sum(di);
        const double sr = t.x * dr - t.y * di, si = t.x * di + t.y * dr;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const zc w = V[j][l + 32 * i];
          x[i].x -= w.x * sr - w.y * si;
          x[i].y -= w.x * si + w.y * sr;
        }
      }
    }
  }
  if (!active) return;
  // R: rows 0..h of column h (k <= 32, so row l sits in x[0])
  if (l < k) R[l + ldr * h] = (l <= h) ? x[0] : make_double2(0.0, 0.0);
  // q_h = H_0 ... H_h e_h
#pragma unroll
  for (int i = 0; i < RPL; ++i) x[i] = make_double2((l + 32 * i == h) ? 1.0 : 0.0, 0.0);
  for (int j = h; j >= 0; --j) {
    const zc t = tau[j];
    if (t.x == 0.0 && t.y == 0.0) continue;
    double dr = 0, di = 0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const zc w = V[j][l + 32 * i];
      dr += w.x * x[i].x + w.y * x[i].y;
      di += w.x * x[i].y - w.y * x[i].x;
    }
    dr = hw_sum(dr);
    di = hw_sum(di);
    const double sr = t.x * dr - t.y * di, si = t.x * di + t.y * dr;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const zc w = V[j][l + 32 * i];
      x[i].x -= w.x * sr - w.y * si;
      x[i].y -= w.x * si + w.y * sr;
    }
  }
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int row = l + 32 * i;
    if (row < b) G[row + ldq * h] = x[i];
  }
}

void pt_leaves(tt_ctx* ctx, zc* Q, long ldq, int nleaves, int m, int k, zc* R, long ldr, long strideR) {
  // leaf sizes are floor(m / P) or ceil(m / P)
  if (k < 1 || k > PT_COLS || nleaves < 1 || m / nleaves < k || (m + nleaves - 1) / nleaves > PT_ROWS)
    fail(TT_EINVAL, "panel QR: bad block shape");
  // Householder factorisation and explicit Q of each leaf (b x k):
  // 2 x (8 b k^2 - 8 k^3 / 3) real flops; the block is read and written once
  const double flops = 16.0 * (double)m * k * k - 16.0 / 3.0 * (double)k * k * k * nleaves;
  KTimer kt(ctx, "pt_leaf", flops, 32.0 * (double)m * k);
  hipLaunchKernelGGL(pt_leaf_kernel, dim3(nleaves), dim3(1024), 0, ctx->stream, Q, ldq, nleaves, m, k, R, ldr,
                     strideR);
  TTF_HIP(hipGetLastError());
}

// Q_i <- Q_i S_i for the leaves of pt_leaves (rows [i m / P, (i+1) m / P)),
// S_i the k x k block at S + i k (ld lds); in place, 64 rows per workgroup.
__global__ __launch_bounds__(256) void pt_assemble_kernel(zc* __restrict__ Q, long ldq, int m, int k, int nleaves,
                                                          const zc* __restrict__ S, long lds_) {
  __shared__ zc tile[PT_COLS][65];
  const long row0 = (long)blockIdx.x * 64;
  const int t = threadIdx.x;
  const int rows = (m - row0 < 64) ? (int)(m - row0) : 64;
  for (int e = t; e < rows * k; e += 256) {
    const int r = e % rows, c = e / rows;
    tile[c][r] = Q[row0 + r + ldq * c];
  }
  __syncthreads();
  for (int e = t; e < rows * k; e += 256) {
    const int r = e % rows, c = e / rows;
    const long gr = row0 + r;
    const int leaf = (int)(((gr + 1) * nleaves - 1) / m);
    const zc* Sl = S + (long)leaf * k + lds_ * c;
    double ar = 0, ai = 0;
    for (int q = 0; q < k; ++q) {
      const zc a = tile[q][r], b = Sl[q];
      ar += a.x * b.x - a.y * b.y;
      ai += a.x * b.y + a.y * b.x;
    }
    Q[gr + ldq * c] = make_double2(ar, ai);
  }
}

void pt_assemble(tt_ctx* ctx, zc* Q, long ldq, int m, int k, int nleaves, const zc* S, long lds_) {
  if (k < 1 || k > PT_COLS) fail(TT_EINVAL, "panel QR: bad assembly shape");
  KTimer kt(ctx, "pt_assemble", 8.0 * (double)m * k * k, 32.0 * (double)m * k);
  hipLaunchKernelGGL(pt_assemble_kernel, dim3((m + 63) / 64), dim3(256), 0, ctx->stream, Q, ldq, m, k, nleaves, S,
                     lds_);
  TTF_HIP(hipGetLastError());
}

int pt_max_rows() { return PT_ROWS; }
int pt_max_cols() { return PT_COLS; }

// ------------------------------------------------------- conj transpose
__global__ void conj_transpose_kernel(const zc* __restrict__ src, long lds_, zc* __restrict__ dst, long ldd, int m,
                                      int k) {
  // dst (k x m) = src (m x k)^H, 32 x 32 tiles through LDS
  __shared__ zc tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;  // bx over m (src rows), by over k (src cols)
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: ty 0..7
  for (int j = ty; j < 32; j += 8) {
    const int r = bx + tx, c = by + j;
    if (r < m && c < k) tile[j][tx] = src[r + lds_ * c];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int r = by + tx, c = bx + j;  // dst row = src col, dst col = src row
    if (r < k && c < m) {
      const zc v = tile[tx][j];
      dst[r + ldd * c] = make_double2(v.x, -v.y);
    }
  }
}

void conj_transpose(tt_ctx* ctx, const zc* src, long lds_, zc* dst, long ldd, int m, int k) {
  if (m <= 0 || k <= 0) return;
  dim3 grid((m + 31) / 32, (k + 31) / 32);
  hipLaunchKernelGGL(conj_transpose_kernel, grid, dim3(256), 0, ctx->stream, src, lds_, dst, ldd, m, k);
  TTF_HIP(hipGetLastError());
}



// ------------------------------------------ block Gram-Schmidt helpers
__device__ inline double wave_sum64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// part[g nb + c] = squared norm of rows [g m / G, (g+1) m / G) of column c
// of Y (m x nb, ld ldy); one wavefront per column, G workgroups
__global__ __launch_bounds__(256) void colnorm_partial_kernel(const zc* __restrict__ Y, long ldy, int m, int nb,
                                                              double* __restrict__ part) {
  const int g = blockIdx.x, G = gridDim.x;
  const long r0 = (long)g * m / G, r1 = (long)(g + 1) * m / G;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = w; c < nb; c += 4) {
    double s = 0;
    for (long r = r0 + lane; r < r1; r += 64) {
      const zc v = Y[r + ldy * c];
      s += v.x * v.x + v.y * v.y;
    }
    s = wave_sum64(s);
    if (lane == 0) part[(long)g * nb + c] = s;
  }
}

// flag[c] = 1 when the residual of panel column c after projection is below
// 1e-13 of the column's norm: the squared residual is the sum of the G
// partial norms (fixed order), the projected part the squared norm of the
// coefficients W (p0 rows, leading dimension ldw).  The test is relative to
// the column alone: the columns of one factorisation may differ in scale by
// many orders (the cores of a sum of TTs carry the norms of its terms).
__global__ __launch_bounds__(1024) void bcgs_flag_kernel(const double* __restrict__ part, int G, int nb,
                                                         const zc* __restrict__ W, long ldw, int p0,
                                                         int* __restrict__ flags) {
  // 16 lanes (one DPP row) per column, up to 64 columns, fixed summation order
  const int c = threadIdx.x >> 4, l = threadIdx.x & 15;
  if (c >= nb) return;
  double res2 = 0, w2 = 0;
  for (int g = l; g < G; g += 16) res2 += part[(long)g * nb + c];
  for (int i = l; i < p0; i += 16) {
    const zc w = W[i + ldw * c];
    w2 += w.x * w.x + w.y * w.y;
  }
  res2 = row16_sum(res2);
  w2 = row16_sum(w2);
  const double tot = res2 + w2;
  if (l == 0) flags[c] = (!(res2 > 1e-26 * tot) || !(res2 > 0.0)) ? 1 : 0;
}



// flagged columns are replaced by standard complex Gaussian vectors
__global__ void bcgs_random_kernel(zc* __restrict__ Qp, long ldq, int m, int nb, const int* __restrict__ flags,
                                   uint32_t k0, uint32_t k1, uint32_t tag) {
  const long total = (long)m * nb;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e % m), c = (int)(e / m);
    if (!flags[c]) continue;
    Qp[r + ldq * c] = philox_gaussian((uint64_t)e, tag, k0, k1);
  }
}

__global__ void bcgs_masked_add_kernel(zc* __restrict__ Rd, long ldr, const zc* __restrict__ W, long ldw, int rows,
                                       int nb, const int* __restrict__ flags) {
  const int total = rows * nb;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int i = e % rows, c = e / rows;
    if (flags[c]) continue;
    zc v = Rd[i + ldr * c];
    const zc w = W[i + ldw * c];
    v.x += w.x;
    v.y += w.y;
    Rd[i + ldr * c] = v;
  }
}

// R[0:nb, 0:nb] (ld ldr) <- Rp (ld nb) with flagged columns zeroed
__global__ void bcgs_put_diag_kernel(zc* __restrict__ Rd, long ldr, const zc* __restrict__ Rp, int nb,
                                     const int* __restrict__ flags) {
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int i = e % nb, c = e / nb;
    Rd[i + ldr * c] = flags[c] ? make_double2(0.0, 0.0) : Rp[i + (long)nb * c];
  }
}

void bcgs_flag(tt_ctx* ctx, const zc* Y, long ldy, int m, int nb, const zc* W, long ldw, int p0, int* flags,
               double* part) {
  const int G = bcgs_flag_groups(m);
  hipLaunchKernelGGL(colnorm_partial_kernel, dim3(G), dim3(256), 0, ctx->stream, Y, ldy, m, nb, part);
  hipLaunchKernelGGL(bcgs_flag_kernel, dim3(1), dim3(1024), 0, ctx->stream, part, G, nb, W, ldw, p0, flags);
  TTF_HIP(hipGetLastError());
}

int bcgs_flag_groups(int m) { return std::max(1, std::min(512, m / 256)); }

void bcgs_random(tt_ctx* ctx, zc* Qp, long ldq, int m, int nb, const int* flags, uint64_t seed, int tag) {
  const long total = (long)m * nb;
  const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(bcgs_random_kernel, dim3(blocks), dim3(256), 0, ctx->stream, Qp, ldq, m, nb, flags,
                     (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)tag);
  TTF_HIP(hipGetLastError());
}

void bcgs_masked_add(tt_ctx* ctx, zc* Rd, long ldr, const zc* W, long ldw, int rows, int nb, const int* flags) {
  if (rows <= 0) return;
  const int total = rows * nb;
  hipLaunchKernelGGL(bcgs_masked_add_kernel, dim3((total + 255) / 256), dim3(256), 0, ctx->stream, Rd, ldr, W, ldw,
                     rows, nb, flags);
  TTF_HIP(hipGetLastError());
}

void bcgs_put_diag(tt_ctx* ctx, zc* Rd, long ldr, const zc* Rp, int nb, const int* flags) {
  hipLaunchKernelGGL(bcgs_put_diag_kernel, dim3(1), dim3(256), 0, ctx->stream, Rd, ldr, Rp, nb, flags);
  TTF_HIP(hipGetLastError());
}

// Cholesky factor and inverse of the nb x nb Hermitian matrix in Gs (LDS),
// G = R^H R with R upper triangular, by a workgroup of 1024 threads (thread
// (i, j) = (t % 32, t / 32) owns entry (i, j)); nb <= 32.
// Factor: step r subtracts conj(G[r][a]) G[r][b] / G[r][r] from the
// trailing entries and stores row r of R, one barrier per step.  Inverse:
// recursive doubling on diagonal blocks of size h = 1, 2, 4, 8, 16: the
// off-diagonal block of [A B; 0 C]^{-1} is -A^{-1} (B C^{-1}).
// Near the identity, G = I + E with every |E_ij| <= 1e-10 (the Gram matrix
// of an already orthonormalised panel), the factor is taken in closed form:
// R = I + U with U the upper part of E and U_ii = E_ii / 2, so that
// R^H R = G + U^H U, and R^{-1} = I - U + U^2 - ..., both truncated after
// the first-order term: the neglected terms are below (32e-10)^2 ~ 1e-17.
// On return Rs holds R (zero below the diagonal and beyond nb), Ri its
// inverse, dinv the reciprocal diagonal; dg holds the original diagonal and
// *bad = 1 when a pivot falls below tau times it (bad may be null).  Gs and
// T are overwritten.
__device__ void block_chol_inv(zc (*Gs)[PT_COLS + 1], zc (*Rs)[PT_COLS + 1], zc (*Ri)[PT_COLS + 1],
                               zc (*T)[PT_COLS + 1], const double* dg, int nb, double tau, int* bad,
                               double* dinv) {
  __shared__ double piv[PT_COLS][2];  // 1 / d and 1 / sqrt(d) of step r
  __shared__ double emax[16];
  const int t = threadIdx.x, i = t & 31, j = t >> 5;
  {
    // largest entry of G - I, over the workgroup
    double e = 0.0;
    if (i < nb && j < nb) {
      const zc g = Gs[i][j];
      e = fmax(fabs(g.x - (i == j ? 1.0 : 0.0)), fabs(g.y));
    }
    for (int off = 32; off > 0; off >>= 1) e = fmax(e, __shfl_xor(e, off, 64));
    if ((t & 63) == 0) emax[t >> 6] = e;
    __syncthreads();
    double em = 0.0;
    for (int w = 0; w < 16; ++w) em = fmax(em, emax[w]);
    if (em <= 1e-10) {
      zc rv = make_double2(0.0, 0.0), iv = make_double2(0.0, 0.0);
      if (i < nb && j < nb) {
        const zc g = Gs[i][j];
        if (i < j) {
          rv = g;
          iv = make_double2(-g.x, -g.y);
        } else if (i == j) {
          const double h = 0.5 * (g.x - 1.0);
          rv = make_double2(1.0 + h, 0.0);
          iv = make_double2(1.0 - h, 0.0);
        }
      } else if (i == j) {  // identity beyond nb
        rv = make_double2(1.0, 0.0);
        iv = rv;
      }
      Rs[i][j] = rv;
      Ri[i][j] = iv;
      if (t < PT_COLS) dinv[t] = (t < nb) ? 1.0 - 0.5 * (Gs[t][t].x - 1.0) : 1.0;
      // pivots are within 1e-10 of 1: the pivot test passes for tau <= 0.5
      __syncthreads();
      return;
    }
  }
  Rs[i][j] = make_double2(0.0, 0.0);
  // the pivot of step r is prepared by the thread that last updated it
  auto pivot = [&](int r, double d) {
    const bool ok = d > tau * dg[r] && d > 0.0;
    if (!ok && bad) *bad = 1;
    const double dd = ok ? d : 1.0;
    const double is = 1.0 / sqrt(dd);
    piv[r][0] = is * is;
    piv[r][1] = is;
    dinv[r] = is;
  };
  if (t == 0 && nb > 0) pivot(0, Gs[0][0].x);
  __syncthreads();
  for (int r = 0; r < nb; ++r) {
    const double id = piv[r][0], is = piv[r][1];
    if (i == r && j >= r && j < nb) {
      const zc g = Gs[r][j];
      Rs[r][j] = (j == r) ? make_double2(1.0 / is, 0.0) : make_double2(g.x * is, g.y * is);
    }
    if (i > r && j >= i && j < nb) {
      const zc x = Gs[r][i], y = Gs[r][j];
      zc g = Gs[i][j];
      g.x -= (x.x * y.x + x.y * y.y) * id;  // conj(x) y / d
      g.y -= (x.x * y.y - x.y * y.x) * id;
      Gs[i][j] = g;
      if (i == r + 1 && j == r + 1) pivot(r + 1, g.x);
    }
    __syncthreads();
  }
  // identity beyond nb keeps the padded factor invertible
  if (i == j && i >= nb) Rs[i][j] = make_double2(1.0, 0.0);
  if (t >= nb && t < PT_COLS) dinv[t] = 1.0;
  __syncthreads();
  Ri[i][j] = (i == j) ? make_double2(dinv[i], 0.0) : make_double2(0.0, 0.0);
  __syncthreads();
  for (int h = 1; h < PT_COLS; h *= 2) {
    const int s0 = (i / (2 * h)) * (2 * h);
    const bool blk = i < s0 + h && j >= s0 + h && j < s0 + 2 * h;
    if (blk) {  // T = B C^{-1}
      double sr = 0, si = 0;
      for (int u = s0 + h; u <= j; ++u) {
        const zc a = Rs[i][u], b = Ri[u][j];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
      }
      T[i][j] = make_double2(sr, si);
    }
    __syncthreads();
    if (blk) {  // X = -A^{-1} T
      double sr = 0, si = 0;
      for (int u = i; u < s0 + h; ++u) {
        const zc a = Ri[i][u], b = T[u][j];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
      }
      Ri[i][j] = make_double2(-sr, -si);
    }
    __syncthreads();
  }
}

// Second pass of the block Gram-Schmidt step for one panel (one workgroup,
// nb <= 32): with Q1 orthonormal and W2 = Q^H Q1 (p0 x nb, ld p0), the
// reorthogonalised panel Z = Q1 - Q W2 has Gram matrix I - W2^H W2, so its
// Cholesky factor R2 comes without another pass over the panel.  Outputs:
// R2^{-1} (nb x nb, ld nb) for Q2 = Z R2^{-1}; the diagonal block R2 R1 of R
// at Rd (ld ldr) and W2 R1 added to the off-diagonal block Ro (p0 x nb, ld
// ldr), both with flagged columns left out; *bad = 1 when a pivot of the
// Cholesky factorisation falls below 0.1 (Z too far from orthonormal for
// this shortcut), in which case the caller redoes the factorisation.
__global__ __launch_bounds__(1024) void bcgs_pip_kernel(const zc* __restrict__ W2, int p0, int nb,
                                                        const zc* __restrict__ R1, zc* __restrict__ Ro,
                                                        zc* __restrict__ Rd, long ldr, const int* __restrict__ flags,
                                                        zc* __restrict__ R2inv, int* __restrict__ bad) {
  __shared__ zc Gs[PT_COLS][PT_COLS + 1];
  __shared__ zc R1s[PT_COLS][PT_COLS + 1];
  __shared__ zc Ri[PT_COLS][PT_COLS + 1];
  __shared__ zc Rs[PT_COLS][PT_COLS + 1];
  __shared__ zc Tt[PT_COLS][PT_COLS + 1];
  __shared__ int fl[PT_COLS];
  __shared__ double dg[PT_COLS], dinv[PT_COLS];
  __shared__ zc Wc[PT_COLS][65];  // 64-row chunks of W2
  const int t = threadIdx.x;
  const int i = t & 31, j = t >> 5;
  if (i < nb && j < nb) R1s[i][j] = R1[i + (long)nb * j];
  if (t < nb) fl[t] = flags[t];
  double gr = (i == j) ? 1.0 : 0.0, gi = 0.0;
  for (int q0 = 0; q0 < p0; q0 += 64) {
    const int rows = min(64, p0 - q0);
    __syncthreads();
    for (int e = t; e < rows * nb; e += 1024) {
      const int r = e % rows, c = e / rows;
      Wc[c][r] = W2[q0 + r + (long)p0 * c];
    }
    __syncthreads();
    if (i < nb && j < nb)
#pragma unroll 8
      for (int r = 0; r < rows; ++r) {
        const zc a = Wc[i][r], b = Wc[j][r];
        gr -= a.x * b.x + a.y * b.y;  // conj(a) b
        gi -= a.x * b.y - a.y * b.x;
      }
    // Ro += W2 R1 on these rows, unflagged columns
    for (int e = t; e < rows * nb; e += 1024) {
      const int r = e % rows, c = e / rows;
      if (fl[c]) continue;
      double sr = 0, si = 0;
#pragma unroll 8
      for (int q = 0; q <= c; ++q) {
        const zc a = Wc[q][r], b = R1s[q][c];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
      }
      zc v = Ro[q0 + r + ldr * c];
      v.x += sr;
      v.y += si;
      Ro[q0 + r + ldr * c] = v;
    }
  }
  if (i < nb && j < nb) Gs[i][j] = make_double2(gr, gi);
  if (t < PT_COLS) dg[t] = 1.0;  // absolute pivot test: Z is near orthonormal
  __syncthreads();
  block_chol_inv(Gs, Rs, Ri, Tt, dg, nb, 1e-2, bad, dinv);
  if (i < nb && j < nb) {
    R2inv[i + (long)nb * j] = Ri[i][j];
    // (R2 R1)[i][j], both upper
    double sr = 0, si = 0;
    for (int q = i; q <= j; ++q) {
      const zc a = Rs[i][q], b = R1s[q][j];
      sr += a.x * b.x - a.y * b.y;
      si += a.x * b.y + a.y * b.x;
    }
    Rd[i + ldr * j] = (i <= j && !fl[j]) ? make_double2(sr, si) : make_double2(0.0, 0.0);
  }
}

// One Cholesky QR pass on the m x nb panel Y given its Gram matrix G
// (ld nb): every workgroup factors G = R^H R and inverts R itself (nb <= 32,
// cheap) and replaces its rpw <= 256 rows by Y R^{-1}; workgroup 0 also
// writes Rout = R Rprev (R without Rprev) and raises *bad when a pivot falls
// below tau times its diagonal entry.  The rows are fetched into registers
// before the factorisation and multiplied in 128-row tiles through LDS.
__global__ __launch_bounds__(1024) void chol_solve_kernel(zc* __restrict__ Y, long ldy, int m, int nb,
                                                         const zc* __restrict__ G, double tau,
                                                         const zc* __restrict__ Rprev, zc* __restrict__ Rout,
                                                         int* __restrict__ bad, int rpw) {
  __shared__ zc Gs[PT_COLS][PT_COLS + 1];
  __shared__ zc Rs[PT_COLS][PT_COLS + 1];
  __shared__ zc Ri[PT_COLS][PT_COLS + 1];
  __shared__ zc Tt[PT_COLS][PT_COLS + 1];
  __shared__ zc tile[PT_COLS][129];
  __shared__ double dg[PT_COLS], dinv[PT_COLS];
  const int t = threadIdx.x;
  const int i = t & 31, j = t >> 5;
  const long row0 = (long)blockIdx.x * rpw;
  const int rows = (m - row0 < rpw) ? (int)(m - row0) : rpw;
  // thread t holds row t % 256 of the block, columns t / 256 + 4 u
  const int rr = t & 255, cg = t >> 8;
  zc y[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int c = cg + 4 * u;
    y[u] = (rr < rows && c < nb) ? Y[row0 + rr + ldy * c] : make_double2(0.0, 0.0);
  }
  if (i < nb && j < nb) Gs[i][j] = G[i + (long)nb * j];
  if (t < nb) dg[t] = G[t + (long)nb * t].x;
  __syncthreads();
  block_chol_inv(Gs, Rs, Ri, Tt, dg, nb, tau, blockIdx.x == 0 ? bad : nullptr, dinv);
  if (blockIdx.x == 0 && i < nb && j < nb) {
    zc v = make_double2(0.0, 0.0);
    if (i <= j) {
      if (Rprev) {
        double sr = 0, si = 0;
        for (int q = i; q <= j; ++q) {
          const zc a = Rs[i][q], b = Rprev[q + (long)nb * j];
          sr += a.x * b.x - a.y * b.y;
          si += a.x * b.y + a.y * b.x;
        }
        v = make_double2(sr, si);
      } else {
        v = Rs[i][j];
      }
    }
    Rout[i + (long)nb * j] = v;
  }
  for (int half = 0; half < 2; ++half) {
    const int lo = 128 * half;
    if (lo >= rows) break;
    __syncthreads();
    if (rr >= lo && rr < lo + 128) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = cg + 4 * u;
        if (c < PT_COLS) tile[c][rr - lo] = y[u];
      }
    }
    __syncthreads();
    const int nrow = (rows - lo < 128) ? rows - lo : 128;
    for (int e = t; e < nrow * nb; e += 1024) {
      const int r = e % nrow, c = e / nrow;
      double sr = 0, si = 0;
#pragma unroll 8
      for (int q = 0; q <= c; ++q) {
        const zc a = tile[q][r], b = Ri[q][c];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
      }
      Y[row0 + lo + r + ldy * c] = make_double2(sr, si);
    }
  }
}

void chol_solve(tt_ctx* ctx, zc* Y, long ldy, int m, int nb, const zc* G, double tau, const zc* Rprev, zc* Rout,
                int* bad) {
  if (nb > PT_COLS) fail(TT_EINVAL, "chol_solve: panel too wide");
  KTimer kt(ctx, "chol_solve", 4.0 * (double)m * nb * nb, 32.0 * (double)m * nb, true);
  // rows per workgroup: 64 .. 256 in steps of 64, so that the launch fills
  // the chip in one wave (every workgroup factors G itself)
  const int rpw = (int)std::min<long>(256, 64 * ((m + 64L * 256 - 1) / (64L * 256)));
  TTF_LAUNCH(kt, chol_solve_kernel, dim3((m + rpw - 1) / rpw), dim3(1024), 0, ctx->stream, Y, ldy, m, nb, G, tau,
             Rprev, Rout, bad, rpw);
  TTF_HIP(hipGetLastError());
}

// Z <- Z Rinv for the m x nb panel Z (ld ldz), Rinv upper nb x nb (ld nb);
// 64 rows per workgroup staged in LDS, in place
__global__ __launch_bounds__(256) void panel_trmm_kernel(zc* __restrict__ Z, long ldz, int m, int nb,
                                                         const zc* __restrict__ Rinv) {
  __shared__ zc tile[PT_COLS][65];
  __shared__ zc Rs[PT_COLS][PT_COLS + 1];
  const long row0 = (long)blockIdx.x * 64;
  const int t = threadIdx.x;
  const int rows = (m - row0 < 64) ? (int)(m - row0) : 64;
  for (int e = t; e < nb * nb; e += 256) Rs[e % nb][e / nb] = Rinv[e];
  for (int e = t; e < rows * nb; e += 256) {
    const int r = e % rows, c = e / rows;
    tile[c][r] = Z[row0 + r + ldz * c];
  }
  __syncthreads();
  for (int e = t; e < rows * nb; e += 256) {
    const int r = e % rows, c = e / rows;
    double sr = 0, si = 0;
#pragma unroll 8
    for (int q = 0; q <= c; ++q) {
      const zc a = tile[q][r], b = Rs[q][c];
      sr += a.x * b.x - a.y * b.y;
      si += a.x * b.y + a.y * b.x;
    }
    Z[row0 + r + ldz * c] = make_double2(sr, si);
  }
}

void bcgs_pip(tt_ctx* ctx, const zc* W2, int p0, int nb, const zc* R1, zc* Ro, zc* Rd, long ldr, const int* flags,
              zc* R2inv, int* bad) {
  if (nb > PT_COLS) fail(TT_EINVAL, "bcgs_pip: panel too wide");
  KTimer kt(ctx, "bcgs_pip", 8.0 * ((double)p0 * nb * nb * 1.5), 16.0 * (double)p0 * nb);
  hipLaunchKernelGGL(bcgs_pip_kernel, dim3(1), dim3(1024), 0, ctx->stream, W2, p0, nb, R1, Ro, Rd, ldr, flags, R2inv,
                     bad);
  TTF_HIP(hipGetLastError());
}

void panel_trmm(tt_ctx* ctx, zc* Z, long ldz, int m, int nb, const zc* Rinv) {
  if (nb > PT_COLS) fail(TT_EINVAL, "panel_trmm: panel too wide");
  KTimer kt(ctx, "panel_trmm", 4.0 * (double)m * nb * nb, 32.0 * (double)m * nb);
  hipLaunchKernelGGL(panel_trmm_kernel, dim3((m + 63) / 64), dim3(256), 0, ctx->stream, Z, ldz, m, nb, Rinv);
  TTF_HIP(hipGetLastError());
}

// ----------------------------------------------- 64-column panels
// Cholesky factor and inverse of an nb x nb Hermitian matrix G (ld ldg,
// nb <= 64) by one workgroup of 1024 threads, each owning the entries
// (i, j) with i = t % 64 and j = t / 64 + 16 u, u < 4.  G = R^H R, R upper
// triangular: step r subtracts conj(G[r][a]) G[r][b] / G[r][r] from the
// trailing upper triangle (one barrier per step; the pivot of the next step
// is prepared by the thread that last updated it) and row r of R is the
// untouched row r of G scaled by 1/sqrt(pivot).  The inverse is built by
// recursive doubling on diagonal blocks of size h = 1 .. 32 (the
// off-diagonal block of [A B; 0 C]^{-1} is -A^{-1} (B C^{-1})), B C^{-1}
// kept in the free lower triangle.  Near the identity (every |G - I| <=
// 1e-10) R = I + U and R^{-1} = I - U to first order (U the upper part of
// G - I with half its diagonal), the neglected terms below (64e-10)^2.
// A pivot d of step r fails when d <= tau dg_r or d <= 0, dg_r the
// original diagonal (or 1 with `absolute`); *bad is then set (bad may be
// null) and 1 taken in its place.  Outputs: Rinv (ld nb) and Rout (ld ldo)
// = R Rprev (or R without Rprev), both upper, with the columns flagged in
// `flags` (may be null) zeroed in Rout.
__global__ __launch_bounds__(1024) void chol_factor_wide_kernel(const zc* __restrict__ G, long ldg, int nb, double tau,
                                                                int absolute, const zc* __restrict__ Rprev,
                                                                zc* __restrict__ Rout, long ldo,
                                                                const int* __restrict__ flags, zc* __restrict__ Rinv,
                                                                int* __restrict__ bad) {
  extern __shared__ double2 wide_lds[];
  zc (*A)[65] = reinterpret_cast<zc (*)[65]>(wide_lds);             // G, then R (upper) and B C^{-1} (lower)
  zc (*Ri)[65] = reinterpret_cast<zc (*)[65]>(wide_lds + 64 * 65);  // R^{-1}
  __shared__ double piv[64][2];
  __shared__ double dg[64], rs[64];
  __shared__ double emax[16];
  const int t = threadIdx.x, i = t & 63, j0 = t >> 6;
  for (int u = 0; u < 4; ++u) {
    const int j = j0 + 16 * u;
    A[i][j] = (i < nb && j < nb) ? G[i + ldg * j] : make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  if (t < 64) dg[t] = (t < nb && !absolute) ? G[t + ldg * t].x : 1.0;
  double e = 0.0;
  for (int u = 0; u < 4; ++u) {
    const int j = j0 + 16 * u;
    if (i < nb && j < nb) {
      const zc g = G[i + ldg * j];
      e = fmax(e, fmax(fabs(g.x - (i == j ? 1.0 : 0.0)), fabs(g.y)));
    }
  }
  for (int off = 32; off > 0; off >>= 1) e = fmax(e, __shfl_xor(e, off, 64));
  if ((t & 63) == 0) emax[t >> 6] = e;
  __syncthreads();
  double em = 0.0;
  for (int w = 0; w < 16; ++w) em = fmax(em, emax[w]);
  if (em <= 1e-10) {
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + 16 * u;
      zc rv = make_double2(0.0, 0.0), iv = make_double2(0.0, 0.0);
      const zc g = A[i][j];
      if (i < j && j < nb) {
        rv = g;
        iv = make_double2(-g.x, -g.y);
      } else if (i == j) {
        const double h = (i < nb) ? 0.5 * (g.x - 1.0) : 0.0;
        rv = make_double2(1.0 + h, 0.0);
        iv = make_double2(1.0 - h, 0.0);
      }
      Ri[i][j] = iv;
      A[i][j] = rv;  // each thread reads and writes only its own entries here
    }
  } else {
    auto pivot = [&](int r, double d) {
      const bool ok = d > tau * dg[r] && d > 0.0;
      if (!ok && bad) *bad = 1;
      const double is = 1.0 / sqrt(ok ? d : 1.0);
      piv[r][0] = is * is;
      piv[r][1] = is;
    };
    if (t == 0 && nb > 0) pivot(0, A[0][0].x);
    __syncthreads();
    for (int r = 0; r < nb; ++r) {
      const double id = piv[r][0];
      if (i > r && i < nb) {
        const zc x = A[r][i];
        for (int u = 0; u < 4; ++u) {
          const int j = j0 + 16 * u;
          if (j >= i && j < nb) {
            const zc y = A[r][j];
            zc g = A[i][j];
            g.x -= (x.x * y.x + x.y * y.y) * id;  // conj(x) y / d
            g.y -= (x.x * y.y - x.y * y.x) * id;
            A[i][j] = g;
            if (i == r + 1 && j == r + 1) pivot(r + 1, g.x);
          }
        }
      }
      __syncthreads();
    }
    // R from the untouched rows; identity beyond nb
    if (t < 64) rs[t] = (t < nb) ? piv[t][1] : 1.0;
    __syncthreads();
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + 16 * u;
      zc v = make_double2(0.0, 0.0);
      if (i == j)
        v = make_double2(1.0 / rs[i], 0.0);
      else if (i < j && j < nb)
        v = make_double2(A[i][j].x * rs[i], A[i][j].y * rs[i]);
      if (i <= j) A[i][j] = v;
      Ri[i][j] = (i == j) ? make_double2(rs[i], 0.0) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int h = 1; h < 64; h *= 2) {
      bool blk[4];
      for (int u = 0; u < 4; ++u) {  // T = B C^{-1}, stored transposed in the lower triangle
        const int j = j0 + 16 * u;
        const int s0 = (i / (2 * h)) * (2 * h);
        blk[u] = i < s0 + h && j >= s0 + h && j < s0 + 2 * h;
        if (blk[u]) {
          double sr = 0, si = 0;
          for (int q = s0 + h; q <= j; ++q) {
            const zc a = A[i][q], b = Ri[q][j];
            sr += a.x * b.x - a.y * b.y;
            si += a.x * b.y + a.y * b.x;
          }
          A[j][i] = make_double2(sr, si);
        }
      }
      __syncthreads();
      for (int u = 0; u < 4; ++u) {  // X = -A^{-1} T
        const int j = j0 + 16 * u;
        if (blk[u]) {
          const int s0 = (i / (2 * h)) * (2 * h);
          double sr = 0, si = 0;
          for (int q = i; q < s0 + h; ++q) {
            const zc a = Ri[i][q], b = A[j][q];
            sr += a.x * b.x - a.y * b.y;
            si += a.x * b.y + a.y * b.x;
          }
          Ri[i][j] = make_double2(-sr, -si);
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int u = 0; u < 4; ++u) {
    const int j = j0 + 16 * u;
    if (i < nb && j < nb) Rinv[i + (long)nb * j] = Ri[i][j];
  }
  if (Rprev) {  // Rprev into the inverse's place
    __syncthreads();
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + 16 * u;
      Ri[i][j] = (i < nb && j < nb) ? Rprev[i + (long)nb * j] : make_double2(0.0, 0.0);
    }
    __syncthreads();
  }
  for (int u = 0; u < 4; ++u) {
    const int j = j0 + 16 * u;
    if (i >= nb || j >= nb) continue;
    zc v = make_double2(0.0, 0.0);
    if (i <= j && !(flags && flags[j])) {
      if (Rprev) {
        double sr = 0, si = 0;
        for (int q = i; q <= j; ++q) {
          const zc a = A[i][q], b = Ri[q][j];
          sr += a.x * b.x - a.y * b.y;
          si += a.x * b.y + a.y * b.x;
        }
        v = make_double2(sr, si);
      } else {
        v = A[i][j];
      }
    }
    Rout[i + ldo * j] = v;
  }
}

constexpr size_t WIDE_FACTOR_LDS = 2 * 64 * 65 * sizeof(zc);

void chol_factor_wide(tt_ctx* ctx, const zc* G, long ldg, int nb, double tau, bool absolute, const zc* Rprev,
                      zc* Rout, long ldo, const int* flags, zc* Rinv, int* bad) {
  if (nb < 1 || nb > 64) fail(TT_EINVAL, "chol_factor_wide: panel width must be 1..64");
  static bool attr_set = false;
  if (!attr_set) {
    TTF_HIP(hipFuncSetAttribute((const void*)chol_factor_wide_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)WIDE_FACTOR_LDS));
    attr_set = true;
  }
  KTimer kt(ctx, "chol_factor", (4.0 / 3.0) * 8.0 * nb * (double)nb * nb, 32.0 * nb * (double)nb, true);
  TTF_LAUNCH(kt, chol_factor_wide_kernel, dim3(1), dim3(1024), WIDE_FACTOR_LDS, ctx->stream, G, ldg, nb, tau,
             absolute ? 1 : 0, Rprev, Rout, ldo, flags, Rinv, bad);
  TTF_HIP(hipGetLastError());
}

// Z <- Z Rinv for the m x nb panel Z (ld ldz, nb <= 64), Rinv upper nb x nb
// (ld nb, zero below the diagonal): 64 rows per workgroup, the rows and
// Rinv staged in LDS; thread (a, b) forms the 4 x 4 outputs of rows
// a + 16 u and columns b + 16 v (consecutive lanes read consecutive rows,
// and the Rinv entries a wavefront reads are four distinct words)
__global__ __launch_bounds__(256) void panel_trmm_wide_kernel(zc* __restrict__ Z, long ldz, int m, int nb,
                                                              const zc* __restrict__ Rinv) {
  extern __shared__ double2 wide_lds[];
  zc (*tile)[65] = reinterpret_cast<zc (*)[65]>(wide_lds);            // tile[c][r]
  zc (*Ri)[65] = reinterpret_cast<zc (*)[65]>(wide_lds + 64 * 65);   // Ri[q][c]
  const long row0 = (long)blockIdx.x * 64;
  const int t = threadIdx.x;
  const int rows = (m - row0 < 64) ? (int)(m - row0) : 64;
  for (int e = t; e < 64 * nb; e += 256) {
    const int r = e & 63, c = e >> 6;
    tile[c][r] = (r < rows) ? Z[row0 + r + ldz * c] : make_double2(0.0, 0.0);
  }
  for (int e = t; e < nb * nb; e += 256) {
    const int q = e % nb, c = e / nb;
    Ri[q][c] = Rinv[e];
  }
  __syncthreads();
  const int a = t & 15, b = t >> 4;
  double ar[4][4], ai[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) ar[u][v] = ai[u][v] = 0.0;
  for (int q = 0; q < nb; ++q) {
    zc x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = tile[q][a + 16 * u];
#pragma unroll
    for (int v = 0; v < 4; ++v) y[v] = (b + 16 * v < nb) ? Ri[q][b + 16 * v] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ar[u][v] += x[u].x * y[v].x - x[u].y * y[v].y;
        ai[u][v] += x[u].x * y[v].y + x[u].y * y[v].x;
      }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = a + 16 * u;
    if (r >= rows) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = b + 16 * v;
      if (c < nb) Z[row0 + r + ldz * c] = make_double2(ar[u][v], ai[u][v]);
    }
  }
}

void panel_trmm_wide(tt_ctx* ctx, zc* Z, long ldz, int m, int nb, const zc* Rinv) {
  if (nb < 1 || nb > 64) fail(TT_EINVAL, "panel_trmm_wide: panel width must be 1..64");
  if (m <= 0) return;
  static bool attr_set = false;
  if (!attr_set) {
    TTF_HIP(hipFuncSetAttribute((const void*)panel_trmm_wide_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)WIDE_FACTOR_LDS));
    attr_set = true;
  }
  KTimer kt(ctx, "panel_trmm", 4.0 * (double)m * nb * nb, 32.0 * (double)m * nb, true);
  TTF_LAUNCH(kt, panel_trmm_wide_kernel, dim3((m + 63) / 64), dim3(256), WIDE_FACTOR_LDS, ctx->stream, Z, ldz, m, nb,
             Rinv);
  TTF_HIP(hipGetLastError());
}

__global__ void fill_zero_kernel(zc* x, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    x[e] = make_double2(0.0, 0.0);
}

void fill_zero(tt_ctx* ctx, zc* x, long n) {
  if (n <= 0) return;
  const int blocks = (int)std::min<long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, ctx->stream, x, n);
  TTF_HIP(hipGetLastError());
}

}  // namespace ttf
