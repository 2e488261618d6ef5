// Householder QR of tall blocks, one workgroup per block, explicit Q.
//
// This is the leaf factorisation of the tall-skinny QR (TSQR) used by every
// orthogonalisation of the TT sweeps: the QR of V(C) and the LQ of H(C)
// (App. A.1, Alg. 1 and Alg. 2), tree-reduced as in the paper's TSQR
// (App. A.3, Fig. tsqr-tree) but inside one GPU: leaves are row blocks
// factored by separate workgroups, their stacked R factors are factored
// again, and Q is assembled top-down with batched matrix-core GEMMs.
// Householder reflections keep Q orthonormal to working precision whatever
// the rank of the input, which matters here because MPO products and sums
// of TTs are routinely exactly rank-deficient.
//
// Per block (b x k, b >= k, in place): for j = 0..k-1 a reflector
// H_j = I - tau_j v_j v_j^H annihilates column j below the diagonal
// (v_j(0) = 1, beta real) and H_j^H is applied to the trailing columns;
// then R is copied out and Q = H_0 ... H_{k-1} [I; 0] is formed backwards
// in place of the block.
#include "common.hpp"
#include "dpp.hpp"
#include "rng.hpp"

namespace ttf {

constexpr int HH_THREADS = 1024;
constexpr int HH_KMAX = 512;
constexpr int HH_BMAX = 2048;
constexpr int HH_GROUPS = HH_THREADS / 16;

// Householder reflector for column j of the block (rows j..b-1), computed by
// one 16-lane group: v(j) = 1, the entries below the diagonal are scaled in
// place and copied to vb, A(j,j) becomes beta, tau goes to *tau_out.
__device__ inline void hh_reflector(zc* A, long ldq, int b, int j, int l16, zc* vb, zc* tau_out) {
  double xs = 0;
  for (int r = j + 1 + l16; r < b; r += 16) {
    const zc a = A[r + ldq * j];
    xs += a.x * a.x + a.y * a.y;
  }
  xs = row16_sum(xs);
  const zc al = A[j + ldq * j];
  zc tj, sc;
  double be;
  if (xs == 0.0 && al.y == 0.0) {
    tj = make_double2(0.0, 0.0);
    be = al.x;
    sc = make_double2(0.0, 0.0);
  } else {
    const double nrm = sqrt(al.x * al.x + al.y * al.y + xs);
    be = (al.x >= 0.0) ? -nrm : nrm;
    tj = make_double2((be - al.x) / be, -al.y / be);
    const double dr = al.x - be, di = al.y;
    const double den = dr * dr + di * di;
    sc = make_double2(dr / den, -di / den);  // 1 / (alpha - beta)
  }
  for (int r = j + 1 + l16; r < b; r += 16) {
    const zc a = A[r + ldq * j];
    const zc vr = make_double2(a.x * sc.x - a.y * sc.y, a.x * sc.y + a.y * sc.x);
    A[r + ldq * j] = vr;
    vb[r] = vr;
  }
  if (l16 == 0) {
    vb[j] = make_double2(1.0, 0.0);
    A[j + ldq * j] = make_double2(be, 0.0);
    *tau_out = tj;
  }
}

// A(j:b, c) -= s * v(j:b), s = t * (v^H A(j:b, c)); one 16-lane group.
__device__ inline void hh_apply_column(zc* A, long ldq, int b, int j, int c, int l16, const zc* v, zc t) {
  constexpr int RPL = 8;
  double dr = 0, di = 0;
  for (int r0 = j; r0 < b; r0 += 16 * RPL) {
    zc a[RPL], w[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = r0 + l16 + 16 * s;
      a[s] = (r < b) ? A[r + ldq * c] : make_double2(0.0, 0.0);
      w[s] = (r < b) ? v[r] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      dr += w[s].x * a[s].x + w[s].y * a[s].y;  // conj(v) a
      di += w[s].x * a[s].y - w[s].y * a[s].x;
    }
  }
  dr = row16_sum(dr);
  di = row16_sum(di);
  const double sr = t.x * dr - t.y * di, si = t.x * di + t.y * dr;
  for (int r0 = j; r0 < b; r0 += 16 * RPL) {
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = r0 + l16 + 16 * s;
      if (r < b) {
        const zc w = v[r];
        zc a = A[r + ldq * c];
        a.x -= w.x * sr - w.y * si;
        a.y -= w.x * si + w.y * sr;
        A[r + ldq * c] = a;
      }
    }
  }
}

// Leaf i holds rows [i*bl, i*bl + rows) of the m-row matrix, rows = bl for
// every leaf but the last, which takes the remainder (arranged by the host
// so that k <= rows <= HH_BMAX).  1024 threads = 64 groups of 16 lanes; each
// group updates one column at a time with 16-lane DPP reductions, and the
// group that updates column j+1 forms the next reflector right away
// (look-ahead), so each column step needs one barrier.
__global__ __launch_bounds__(HH_THREADS) void hh_leaf_kernel(zc* __restrict__ Qbase, long ldq, int bl, int nleaves,
                                                             int m, int k, zc* __restrict__ Rbase, long ldr,
                                                             long strideR) {
  __shared__ zc vbuf[2][HH_BMAX];
  __shared__ zc tau[HH_KMAX];
  const int leaf = blockIdx.x;
  zc* A = Qbase + (long)leaf * bl;
  const int b = (leaf == nleaves - 1) ? m - leaf * bl : bl;
  zc* R = Rbase + strideR * leaf;
  const int t = threadIdx.x, nt = blockDim.x, g = t >> 4, l16 = t & 15;

  // ---- factorisation
  if (g == 0) hh_reflector(A, ldq, b, 0, l16, vbuf[0], &tau[0]);
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    const zc* v = vbuf[j & 1];
    const zc tc = make_double2(tau[j].x, -tau[j].y);  // apply H_j^H
    const bool active = (tc.x != 0.0 || tc.y != 0.0);
    for (int c = j + 1 + g; c < k; c += HH_GROUPS) {
      if (active) hh_apply_column(A, ldq, b, j, c, l16, v, tc);
      if (c == j + 1) hh_reflector(A, ldq, b, j + 1, l16, vbuf[(j + 1) & 1], &tau[j + 1]);
    }
    __syncthreads();
  }
  // ---- R (upper triangle)
  for (long e = t; e < (long)k * k; e += nt) {
    const int p = (int)(e % k), c = (int)(e / k);
    R[p + ldr * c] = (p <= c) ? A[p + ldq * c] : make_double2(0.0, 0.0);
  }
  // ---- Q = H_0 ... H_{k-1} [I; 0], backwards and in place; the reflector
  // of the next (lower) column is prefetched into the other buffer
  for (int r = k + t; r < b; r += nt) vbuf[(k - 1) & 1][r] = A[r + ldq * (k - 1)];
  if (t == 0) vbuf[(k - 1) & 1][k - 1] = make_double2(1.0, 0.0);
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const zc* v = vbuf[j & 1];
    const zc tj = tau[j];
    if (j > 0) {
      zc* vn = vbuf[(j - 1) & 1];
      for (int r = j + t; r < b; r += nt) vn[r] = A[r + ldq * (j - 1)];
      if (t == 0) vn[j - 1] = make_double2(1.0, 0.0);
    }
    if (tj.x != 0.0 || tj.y != 0.0)
      for (int c = j + 1 + g; c < k; c += HH_GROUPS) hh_apply_column(A, ldq, b, j, c, l16, v, tj);
    for (int r = t; r < b; r += nt) {
      zc q;
      if (r < j)
        q = make_double2(0.0, 0.0);
      else if (r == j)
        q = make_double2(1.0 - tj.x, -tj.y);
      else {
        const zc vr = v[r];
        q = make_double2(-(tj.x * vr.x - tj.y * vr.y), -(tj.x * vr.y + tj.y * vr.x));
      }
      A[r + ldq * j] = q;
    }
    __syncthreads();
  }
}

void hh_leaves(tt_ctx* ctx, zc* Q, long ldq, int bl, int nleaves, int m, int k, zc* R, long ldr, long strideR) {
  if (k > HH_KMAX) fail(TT_EINVAL, "Householder QR: rank above the supported maximum of 512");
  const int last = m - (nleaves - 1) * bl;
  if (bl < k || last < k || last > HH_BMAX || bl > HH_BMAX) fail(TT_EINVAL, "Householder QR: bad leaf shape");
  // factor (4 b k^2 - 4/3 k^3 complex) and forming Q (same), real flops
  const double flops = 8.0 * (8.0 * (double)m * k * k - 8.0 / 3.0 * (double)k * k * k * nleaves);
  KTimer kt(ctx, "hhqr", flops, 32.0 * (double)m * k);
  hipLaunchKernelGGL(hh_leaf_kernel, dim3(nleaves), dim3(HH_THREADS), 0, ctx->stream, Q, ldq, bl, nleaves, m, k, R,
                     ldr, strideR);
  TTF_HIP(hipGetLastError());
}

int hh_max_rows() { return HH_BMAX; }

// ----------------------------------------------- LDS panel Householder QR
// Blocks of at most 256 rows x 32 columns held in LDS for the whole
// factorisation (Householder factor, R copy-out, explicit Q), one workgroup
// per block.  Used for the panels of the block Gram-Schmidt QR below and for
// the R-stack merges of its TSQR tree (eight 32 x 32 factors per block).
constexpr int PT_ROWS = 256;
constexpr int PT_COLS = 32;

__device__ inline void pt_reflector(zc (*A)[PT_ROWS + 1], int b, int j, int l16, zc* tau_out) {
  double xs = 0;
  for (int r = j + 1 + l16; r < b; r += 16) {
    const zc a = A[j][r];
    xs += a.x * a.x + a.y * a.y;
  }
  xs = row16_sum(xs);
  const zc al = A[j][j];
  zc tj, sc;
  double be;
  if (xs == 0.0 && al.y == 0.0) {
    tj = make_double2(0.0, 0.0);
    be = al.x;
    sc = make_double2(0.0, 0.0);
  } else {
    const double nrm = sqrt(al.x * al.x + al.y * al.y + xs);
    be = (al.x >= 0.0) ? -nrm : nrm;
    tj = make_double2((be - al.x) / be, -al.y / be);
    const double dr = al.x - be, di = al.y;
    const double den = dr * dr + di * di;
    sc = make_double2(dr / den, -di / den);
  }
  for (int r = j + 1 + l16; r < b; r += 16) {
    const zc a = A[j][r];
    A[j][r] = make_double2(a.x * sc.x - a.y * sc.y, a.x * sc.y + a.y * sc.x);
  }
  if (l16 == 0) {
    A[j][j] = make_double2(be, 0.0);
    *tau_out = tj;
  }
}

// column c (rows j..b-1) <- (I - t v v^H) column c, v = [1; A[j][j+1..b-1]]
// when vsrc == nullptr, else v from vsrc (with vsrc[j] = 1)
__device__ inline void pt_apply(zc (*A)[PT_ROWS + 1], int b, int j, int c, int l16, const zc* vsrc, zc t) {
  double dr = 0, di = 0;
  for (int r = j + l16; r < b; r += 16) {
    const zc w = vsrc ? vsrc[r] : (r == j ? make_double2(1.0, 0.0) : A[j][r]);
    const zc a = A[c][r];
    dr += w.x * a.x + w.y * a.y;
    di += w.x * a.y - w.y * a.x;
  }
  dr = row16_sum(dr);
  di = row16_sum(di);
  const double sr = t.x * dr - t.y * di, si = t.x * di + t.y * dr;
  for (int r = j + l16; r < b; r += 16) {
    const zc w = vsrc ? vsrc[r] : (r == j ? make_double2(1.0, 0.0) : A[j][r]);
    zc a = A[c][r];
    a.x -= w.x * sr - w.y * si;
    a.y -= w.x * si + w.y * sr;
    A[c][r] = a;
  }
}

// Householder QR of one row block per workgroup, entirely in LDS.  Leaf i
// owns rows [i m / P, (i+1) m / P) of the m x k matrix at Qbase (ld ldq),
// k <= 32 and every leaf 32..256 rows; it leaves the explicit Q factor in
// place and writes R_i (k x k upper) at Rbase + i strideR (ld ldr).
__global__ __launch_bounds__(1024) void pt_leaf_kernel(zc* __restrict__ Qbase, long ldq, int nleaves, int m, int k,
                                                       zc* __restrict__ Rbase, long ldr, long strideR) {
  __shared__ zc A[PT_COLS][PT_ROWS + 1];
  __shared__ zc vb[2][PT_ROWS];
  __shared__ zc tau[PT_COLS];
  const int leaf = blockIdx.x;
  const long r0 = (long)leaf * m / nleaves, r1 = (long)(leaf + 1) * m / nleaves;
  zc* G = Qbase + r0;
  const int b = (int)(r1 - r0);
  zc* R = Rbase + strideR * leaf;
  const int t = threadIdx.x, g = t >> 4, l16 = t & 15;
  for (int e = t; e < b * k; e += 1024) {
    const int r = e % b, c = e / b;
    A[c][r] = G[r + ldq * c];
  }
  __syncthreads();
  // factor: the group that updates column j+1 forms reflector j+1 next
  if (g == 0) pt_reflector(A, b, 0, l16, &tau[0]);
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    const zc tc = make_double2(tau[j].x, -tau[j].y);
    const int c = j + 1 + g;
    if (c < k) {
      if (tc.x != 0.0 || tc.y != 0.0) pt_apply(A, b, j, c, l16, nullptr, tc);
      if (c == j + 1) pt_reflector(A, b, j + 1, l16, &tau[j + 1]);
    }
    __syncthreads();
  }
  for (int e = t; e < k * k; e += 1024) {
    const int p = e % k, c = e / k;
    R[p + ldr * c] = (p <= c) ? A[c][p] : make_double2(0.0, 0.0);
  }
  // Q backwards; v_j staged in vb[j & 1], v_{j-1} prefetched meanwhile
  for (int r = k + t; r < b; r += 1024) vb[(k - 1) & 1][r] = A[k - 1][r];
  if (t == 0) vb[(k - 1) & 1][k - 1] = make_double2(1.0, 0.0);
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const zc* v = vb[j & 1];
    const zc tj = tau[j];
    if (j > 0) {
      for (int r = j + t; r < b; r += 1024) vb[(j - 1) & 1][r] = A[j - 1][r];
      if (t == 0) vb[(j - 1) & 1][j - 1] = make_double2(1.0, 0.0);
    }
    const int c = j + 1 + g;
    if (c < k && (tj.x != 0.0 || tj.y != 0.0)) pt_apply(A, b, j, c, l16, v, tj);
    if (g == k - j - 1) {
      // the first idle group (k <= 32 < 64 groups) rewrites column j
      for (int r = l16; r < b; r += 16) {
        zc q;
        if (r < j)
          q = make_double2(0.0, 0.0);
        else if (r == j)
          q = make_double2(1.0 - tj.x, -tj.y);
        else {
          const zc vr = v[r];
          q = make_double2(-(tj.x * vr.x - tj.y * vr.y), -(tj.x * vr.y + tj.y * vr.x));
        }
        A[j][r] = q;
      }
    }
    __syncthreads();
  }
  for (int e = t; e < b * k; e += 1024) {
    const int r = e % b, c = e / b;
    G[r + ldq * c] = A[c][r];
  }
}

void pt_leaves(tt_ctx* ctx, zc* Q, long ldq, int nleaves, int m, int k, zc* R, long ldr, long strideR) {
  // leaf sizes are floor(m / P) or ceil(m / P)
  if (k < 1 || k > PT_COLS || nleaves < 1 || m / nleaves < k || (m + nleaves - 1) / nleaves > PT_ROWS)
    fail(TT_EINVAL, "panel QR: bad block shape");
  const double flops = 8.0 * (8.0 * (double)m * k * k - 8.0 / 3.0 * (double)k * k * k * nleaves);
  KTimer kt(ctx, "hhqr", flops, 32.0 * (double)m * k);
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
  KTimer kt(ctx, "hhqr", 8.0 * (double)m * k * k, 48.0 * (double)m * k);
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
// flag[c] = 1 when the residual of panel column c after projection is below
// 1e-13 of the column's norm (residual^2 from the Gram G, projected part from
// the coefficients W, p0 rows, leading dimension ldw).
__global__ void bcgs_flag_kernel(const zc* __restrict__ G, int nb, const zc* __restrict__ W, long ldw, int p0,
                                 int* __restrict__ flags) {
  const int c = threadIdx.x;
  if (c >= nb) return;
  const double res2 = G[c + (long)nb * c].x;
  double w2 = 0;
  for (int i = 0; i < p0; ++i) {
    const zc w = W[i + ldw * c];
    w2 += w.x * w.x + w.y * w.y;
  }
  const double tot = res2 + w2;
  flags[c] = (!(res2 > 1e-26 * tot) || !(res2 > 0.0)) ? 1 : 0;
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

void bcgs_flag(tt_ctx* ctx, const zc* G, int nb, const zc* W, long ldw, int p0, int* flags) {
  hipLaunchKernelGGL(bcgs_flag_kernel, dim3(1), dim3(64), 0, ctx->stream, G, nb, W, ldw, p0, flags);
  TTF_HIP(hipGetLastError());
}

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
