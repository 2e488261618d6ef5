// Complex double GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4f64).
//
// C[M x N] = alpha * op(A) * op(B) + beta * C, column major, op in
// {N, T, C(conjugate transpose)}, strided batches.  Every contraction of the
// TT arithmetic (orthogonalisation factors pushed into neighbour cores,
// Gram matrices, sketch contractions, Q * U products) is one of these.
//
// Workgroup tile 64 x 64, K step 16, 256 threads = 4 wavefronts of 64 lanes;
// each wavefront owns a 32 x 32 sub-tile = 2 x 2 MFMA tiles of 16 x 16.
// A complex product is four real MFMAs: Re += Ar Br - Ai Bi,
// Im += Ar Bi + Ai Br (the imaginary part of A is negated once in LDS for
// the subtraction).  Operand tiles are staged through LDS as separate real
// and imaginary planes so every MFMA operand is one 8-byte LDS read per lane.
// Large K with a small output grid is split over workgroups (split-K) into a
// workspace and reduced deterministically by a second kernel.
#include <string>

#include "common.hpp"

namespace ttf {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, PAD = 1;

struct GemmParams {
  int M, N, K, opA, opB, kchunk;
  const zc* A;
  long lda, sA;
  const zc* B;
  long ldb, sB;
  zc* C;
  long ldc, sC;
  zc alpha, beta;
  int batch;
  zc* ws;  // split-K partials: [split][batch][N][M] (column major M x N)
};

__device__ inline zc load_a(const GemmParams& p, const zc* A, int m, int k) {
  if (m >= p.M || k >= p.K) return make_double2(0.0, 0.0);
  if (p.opA == OPN) return A[m + p.lda * (long)k];
  zc v = A[k + p.lda * (long)m];
  if (p.opA == OPC) v.y = -v.y;
  return v;
}

__device__ inline zc load_b(const GemmParams& p, const zc* B, int k, int n) {
  if (k >= p.K || n >= p.N) return make_double2(0.0, 0.0);
  if (p.opB == OPN) return B[k + p.ldb * (long)n];
  zc v = B[n + p.ldb * (long)k];
  if (p.opB == OPC) v.y = -v.y;
  return v;
}

__global__ __launch_bounds__(256) void zgemm_kernel(GemmParams p) {
  __shared__ double Ar[BK][BM + PAD], Ai[BK][BM + PAD];  // Ai holds -Im(A)
  __shared__ double Br[BK][BN + PAD], Bi[BK][BN + PAD];
  __shared__ double Ap[BK][BM + PAD];                    // +Im(A)

  const int nsplit = gridDim.z / p.batch;
  const int bz = blockIdx.z % p.batch;
  const int split = blockIdx.z / p.batch;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int kbeg = split * p.kchunk;
  const int kend = min(p.K, kbeg + p.kchunk);
  const zc* A = p.A + p.sA * (long)bz;
  const zc* B = p.B + p.sB * (long)bz;

  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;

  dbl4 accR[2][2], accI[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = dbl4{0, 0, 0, 0};
      accI[i][j] = dbl4{0, 0, 0, 0};
    }

  zc ra[4], rb[4];
  auto gload = [&](int k0) {
    for (int r = 0; r < 4; ++r) {
      if (p.opA == OPN)
        ra[r] = load_a(p, A, m0 + (t & 63), k0 + (t >> 6) + 4 * r);
      else
        ra[r] = load_a(p, A, m0 + (t >> 4) + 16 * r, k0 + (t & 15));
      if (p.opB == OPN)
        rb[r] = load_b(p, B, k0 + (t & 15), n0 + (t >> 4) + 16 * r);
      else
        rb[r] = load_b(p, B, k0 + (t >> 6) + 4 * r, n0 + (t & 63));
    }
  };
  auto sstore = [&]() {
    for (int r = 0; r < 4; ++r) {
      int mm, kk;
      if (p.opA == OPN) {
        mm = t & 63;
        kk = (t >> 6) + 4 * r;
      } else {
        mm = (t >> 4) + 16 * r;
        kk = t & 15;
      }
      Ar[kk][mm] = ra[r].x;
      Ai[kk][mm] = -ra[r].y;
      Ap[kk][mm] = ra[r].y;
      int nn;
      if (p.opB == OPN) {
        kk = t & 15;
        nn = (t >> 4) + 16 * r;
      } else {
        kk = (t >> 6) + 4 * r;
        nn = t & 63;
      }
      Br[kk][nn] = rb[r].x;
      Bi[kk][nn] = rb[r].y;
    }
  };

  if (kbeg < kend) {
    gload(kbeg);
    sstore();
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) gload(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double ar[2], an[2], ap[2], br[2], bi[2];
      for (int i = 0; i < 2; ++i) {
        ar[i] = Ar[ks + lk][wm + 16 * i + lr];
        an[i] = Ai[ks + lk][wm + 16 * i + lr];
        ap[i] = Ap[ks + lk][wm + 16 * i + lr];
      }
      for (int j = 0; j < 2; ++j) {
        br[j] = Br[ks + lk][wn + 16 * j + lr];
        bi[j] = Bi[ks + lk][wn + 16 * j + lr];
      }
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], accR[i][j], 0, 0, 0);
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(an[i], bi[j], accR[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], accI[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[i], br[j], accI[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
    if (more) {
      sstore();
      __syncthreads();
    }
  }

  // v_mfma_f64_16x16x4f64 result layout: register v of lane l holds
  // D[4 v + l/16][l % 16] of each 16 x 16 tile
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + 16 * i + 4 * v + lk;
        const int n = n0 + wn + 16 * j + lr;
        if (m >= p.M || n >= p.N) continue;
        const double re = accR[i][j][v], im = accI[i][j][v];
        if (nsplit > 1) {
          zc* w = p.ws + ((long)split * p.batch + bz) * (long)p.M * p.N;
          w[m + (long)p.M * n] = make_double2(re, im);
        } else {
          zc* C = p.C + p.sC * (long)bz;
          zc out = make_double2(p.alpha.x * re - p.alpha.y * im, p.alpha.x * im + p.alpha.y * re);
          const long off = m + p.ldc * (long)n;
          if (p.beta.x != 0.0 || p.beta.y != 0.0) {
            const zc c = C[off];
            out.x += p.beta.x * c.x - p.beta.y * c.y;
            out.y += p.beta.x * c.y + p.beta.y * c.x;
          }
          C[off] = out;
        }
      }
}

__global__ void splitk_reduce(GemmParams p, int nsplit) {
  const long total = (long)p.M * p.N * p.batch;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int bz = (int)(e / ((long)p.M * p.N));
    const long mn = e - (long)bz * p.M * p.N;
    const int n = (int)(mn / p.M), m = (int)(mn - (long)n * p.M);
    double re = 0, im = 0;
    for (int s = 0; s < nsplit; ++s) {
      const zc v = p.ws[((long)s * p.batch + bz) * (long)p.M * p.N + mn];
      re += v.x;
      im += v.y;
    }
    zc* C = p.C + p.sC * (long)bz;
    zc out = make_double2(p.alpha.x * re - p.alpha.y * im, p.alpha.x * im + p.alpha.y * re);
    const long off = m + p.ldc * (long)n;
    if (p.beta.x != 0.0 || p.beta.y != 0.0) {
      const zc c = C[off];
      out.x += p.beta.x * c.x - p.beta.y * c.y;
      out.y += p.beta.x * c.y + p.beta.y * c.x;
    }
    C[off] = out;
  }
}

void zgemm(tt_ctx* ctx, int opA, int opB, int M, int N, int K, zc alpha, const zc* A, long lda,
           long strideA, const zc* B, long ldb, long strideB, zc beta, zc* C, long ldc, long strideC,
           int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) {
    // C = beta C: reuse the kernel with an empty K range (kernel writes alpha*0 + beta*C)
    K = 0;
  }
  GemmParams p;
  p.M = M; p.N = N; p.K = K; p.opA = opA; p.opB = opB;
  p.A = A; p.lda = lda; p.sA = strideA;
  p.B = B; p.ldb = ldb; p.sB = strideB;
  p.C = C; p.ldc = ldc; p.sC = strideC;
  p.alpha = alpha; p.beta = beta; p.batch = batch; p.ws = nullptr;
  const int gx = (M + BM - 1) / BM, gy = (N + BN - 1) / BN;
  const long tiles = (long)gx * gy * batch;
  // split K when the output grid alone cannot occupy the chip
  int nsplit = 1;
  const int kblocks = (K + BK - 1) / BK;
  if (tiles < 512 && kblocks >= 8) {
    nsplit = (int)std::min<long>((1024 + tiles - 1) / tiles, kblocks / 4);
    nsplit = std::max(1, std::min(nsplit, 64));
  }
  int kchunk = ((kblocks + nsplit - 1) / nsplit) * BK;
  if (K == 0) kchunk = 0;
  nsplit = (K == 0) ? 1 : (K + kchunk - 1) / kchunk;
  p.kchunk = kchunk;
  const double flops = 8.0 * M * N * (double)K * batch;
  const double bytes = 16.0 * ((double)M * K + (double)K * N + 2.0 * M * N) * batch;
  if (nsplit > 1) {
    p.ws = (zc*)ctx->get_ws("gemm_splitk", sizeof(zc) * (size_t)nsplit * batch * M * N);
  }
  if ((long)batch * nsplit > 65535) fail(TT_EINVAL, "zgemm: batch * split too large for the grid");
  {
    // with shape profiling on, the launch is also recorded under its shape
    std::string shape;
    if (ctx->profile_shapes) {
      const char ops[3] = {'N', 'T', 'C'};
      shape = std::string("zgemm:") + ops[opA] + ops[opB] + ":" + std::to_string(M) + "x" + std::to_string(N) + "x" +
              std::to_string(K) + "x" + std::to_string(batch);
    }
    KTimer kt2(ctx->profile_shapes ? ctx : nullptr, shape.c_str(), flops, bytes);
    KTimer kt(ctx, "zgemm", flops, bytes);
    hipLaunchKernelGGL(zgemm_kernel, dim3(gx, gy, batch * nsplit), dim3(256), 0, ctx->stream, p);
    if (nsplit > 1) {
      const long total = (long)M * N * batch;
      const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
      hipLaunchKernelGGL(splitk_reduce, dim3(blocks), dim3(256), 0, ctx->stream, p, nsplit);
    }
  }
  TTF_HIP(hipGetLastError());
}

}  // namespace ttf
