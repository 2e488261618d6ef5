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

namespace ttf {

constexpr int HH_THREADS = 512;
constexpr int HH_KMAX = 512;
constexpr int HH_BMAX = 4096;

__device__ inline double hh_wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Leaf i holds rows [i*bl, i*bl + rows) of the m-row matrix, rows = bl for
// every leaf but the last, which takes the remainder (bl <= rows < bl + k,
// arranged by the host so that rows <= HH_BMAX).
__global__ __launch_bounds__(HH_THREADS) void hh_leaf_kernel(zc* __restrict__ Qbase, long ldq, int bl, int nleaves,
                                                             int m, int k, zc* __restrict__ Rbase, long ldr,
                                                             long strideR) {
  __shared__ zc v[HH_BMAX];
  __shared__ zc tau[HH_KMAX];
  const int leaf = blockIdx.x;
  zc* A = Qbase + (long)leaf * bl;
  const int b = (leaf == nleaves - 1) ? m - leaf * bl : bl;
  zc* R = Rbase + strideR * leaf;
  const int t = threadIdx.x, nt = blockDim.x, wave = t >> 6, lane = t & 63, nw = nt >> 6;

  // ---- factorisation
  for (int j = 0; j < k; ++j) {
    if (wave == 0) {
      double xs = 0;
      for (int r = j + 1 + lane; r < b; r += 64) {
        const zc a = A[r + ldq * j];
        xs += a.x * a.x + a.y * a.y;
      }
      xs = hh_wave_sum(xs);
      const zc al = A[j + ldq * j];
      zc tj;
      double be;
      zc sc;
      if (xs == 0.0 && al.y == 0.0) {
        tj = make_double2(0.0, 0.0);
        be = al.x;
        sc = make_double2(0.0, 0.0);
      } else {
        const double nrm = sqrt(al.x * al.x + al.y * al.y + xs);
        be = (al.x >= 0.0) ? -nrm : nrm;
        tj = make_double2((be - al.x) / be, -al.y / be);
        // sc = 1 / (alpha - beta)
        const double dr = al.x - be, di = al.y;
        const double den = dr * dr + di * di;
        sc = make_double2(dr / den, -di / den);
      }
      for (int r = j + 1 + lane; r < b; r += 64) {
        const zc a = A[r + ldq * j];
        const zc vr = make_double2(a.x * sc.x - a.y * sc.y, a.x * sc.y + a.y * sc.x);
        A[r + ldq * j] = vr;
        v[r] = vr;
      }
      if (lane == 0) {
        v[j] = make_double2(1.0, 0.0);
        A[j + ldq * j] = make_double2(be, 0.0);
        tau[j] = tj;
      }
    }
    __syncthreads();
    const zc tc = make_double2(tau[j].x, -tau[j].y);  // conj(tau): apply H_j^H
    if (tc.x != 0.0 || tc.y != 0.0) {
      for (int c = j + 1 + wave; c < k; c += nw) {
        double dr = 0, di = 0;
        for (int r = j + lane; r < b; r += 64) {
          const zc vr = v[r], a = A[r + ldq * c];
          dr += vr.x * a.x + vr.y * a.y;  // conj(v) a
          di += vr.x * a.y - vr.y * a.x;
        }
        dr = hh_wave_sum(dr);
        di = hh_wave_sum(di);
        // s = conj(tau) * dot
        const double sr = tc.x * dr - tc.y * di, si = tc.x * di + tc.y * dr;
        for (int r = j + lane; r < b; r += 64) {
          const zc vr = v[r];
          zc a = A[r + ldq * c];
          a.x -= vr.x * sr - vr.y * si;
          a.y -= vr.x * si + vr.y * sr;
          A[r + ldq * c] = a;
        }
      }
    }
    __syncthreads();
  }
  // ---- R (upper triangle)
  for (long e = t; e < (long)k * k; e += nt) {
    const int p = (int)(e % k), c = (int)(e / k);
    R[p + ldr * c] = (p <= c) ? A[p + ldq * c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  // ---- Q = H_0 ... H_{k-1} [I; 0], backwards and in place
  for (int j = k - 1; j >= 0; --j) {
    for (int r = j + 1 + t; r < b; r += nt) v[r] = A[r + ldq * j];
    if (t == 0) v[j] = make_double2(1.0, 0.0);
    __syncthreads();
    const zc tj = tau[j];
    if (tj.x != 0.0 || tj.y != 0.0) {
      for (int c = j + 1 + wave; c < k; c += nw) {
        double dr = 0, di = 0;
        for (int r = j + lane; r < b; r += 64) {
          const zc vr = v[r], a = A[r + ldq * c];
          dr += vr.x * a.x + vr.y * a.y;
          di += vr.x * a.y - vr.y * a.x;
        }
        dr = hh_wave_sum(dr);
        di = hh_wave_sum(di);
        const double sr = tj.x * dr - tj.y * di, si = tj.x * di + tj.y * dr;
        for (int r = j + lane; r < b; r += 64) {
          const zc vr = v[r];
          zc a = A[r + ldq * c];
          a.x -= vr.x * sr - vr.y * si;
          a.y -= vr.x * si + vr.y * sr;
          A[r + ldq * c] = a;
        }
      }
    }
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

}  // namespace ttf
