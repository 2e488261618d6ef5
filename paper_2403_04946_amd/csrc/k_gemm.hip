// Complex double GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4f64).
//
// C[M x N] = alpha * op(A) * op(B) + beta * C, column major, op in
// {N, T, C(conjugate transpose)}, strided batches.  Every contraction of the
// TT arithmetic (orthogonalisation factors pushed into neighbour cores,
// Gram matrices, sketch contractions, Q * U products) is one of these.
//
// Workgroup tiles 64 x 64, 128 x 32, 64 x 32, 32 x 32 or 32 x 64 (chosen by
// the output shape), K step 16, 256 threads = 4 wavefronts of 64 lanes in a
// 2 x 2 arrangement; operand ops are template parameters.
// A complex product is four real MFMAs: Re += Ar Br - Ai Bi,
// Im += Ar Bi + Ai Br (the imaginary part of A is negated once in LDS for
// the subtraction).  Operand tiles are staged through LDS as separate real
// and imaginary planes so every MFMA operand is one 8-byte LDS read per lane.
// Large K with a small output grid is split over workgroups (split-K) into a
// workspace and reduced deterministically by a second kernel.
//
// The FP32 form (TT_PREC_FP32) is the same kernel with the operands rounded
// to float in the LDS staging and v_mfma_f32_16x16x4f32 products; each K
// step of 16 is accumulated in float and then added into double
// accumulators, so the error per entry stays near 2^-24 times the sum of
// |a||b| of one K step, whatever K is.
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "common.hpp"

namespace ttf {

// ------------------------------------------------------ tuned choices
namespace {
using GemmKey = std::tuple<int, int, int, int, int, int, int>;
std::map<GemmKey, GemmChoice>& gemm_table() {
  static std::map<GemmKey, GemmChoice> t;
  return t;
}
std::mutex& gemm_table_mutex() {
  static std::mutex m;
  return m;
}
std::atomic<int> gemm_table_size{0};
thread_local const GemmChoice* gemm_forced = nullptr;
}  // namespace

void gemm_force(const GemmChoice* c) { gemm_forced = c; }

bool gemm_choice(int fmt, int opA, int opB, int M, int N, int K, int batch, GemmChoice* out) {
  if (gemm_forced) {
    *out = *gemm_forced;
    return true;
  }
  if (gemm_table_size.load(std::memory_order_relaxed) == 0) return false;
  std::lock_guard<std::mutex> lock(gemm_table_mutex());
  auto it = gemm_table().find(GemmKey{fmt, opA, opB, M, N, K, batch});
  if (it == gemm_table().end()) return false;
  *out = it->second;
  return true;
}

void gemm_table_put(const int* e) {
  std::lock_guard<std::mutex> lock(gemm_table_mutex());
  GemmChoice c;
  c.a = e[7];
  c.b = e[8];
  c.nsplit = e[9];
  gemm_table()[GemmKey{e[0], e[1], e[2], e[3], e[4], e[5], e[6]}] = c;
  gemm_table_size.store((int)gemm_table().size());
}

int gemm_table_count() {
  std::lock_guard<std::mutex> lock(gemm_table_mutex());
  return (int)gemm_table().size();
}

bool gemm_table_entry(int index, int* e) {
  std::lock_guard<std::mutex> lock(gemm_table_mutex());
  if (index < 0 || index >= (int)gemm_table().size()) return false;
  auto it = gemm_table().begin();
  std::advance(it, index);
  const GemmKey& k = it->first;
  e[0] = std::get<0>(k); e[1] = std::get<1>(k); e[2] = std::get<2>(k); e[3] = std::get<3>(k);
  e[4] = std::get<4>(k); e[5] = std::get<5>(k); e[6] = std::get<6>(k);
  e[7] = it->second.a; e[8] = it->second.b; e[9] = it->second.nsplit;
  return true;
}

void gemm_table_clear() {
  std::lock_guard<std::mutex> lock(gemm_table_mutex());
  gemm_table().clear();
  gemm_table_size.store(0);
}

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int BK = 16, PAD = 1;

struct GemmParams {
  int M, N, K, kchunk;
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

template <int OP>
__device__ inline zc load_op(const zc* X, long ld, int r, int c, int R, int Ccount) {
  // element (r, c) of op(X), R x Ccount, zero outside
  if (r >= R || c >= Ccount) return make_double2(0.0, 0.0);
  if (OP == OPN) return X[r + ld * (long)c];
  zc v = X[c + ld * (long)r];
  if (OP == OPC) v.y = -v.y;
  return v;
}

// Workgroup tile BM x BN, 256 threads = 2 x 2 wavefronts, each owning a
// (BM/2) x (BN/2) block of (BM/32) x (BN/32) MFMA tiles of 16 x 16.
// blockIdx.x runs over N tiles (fastest), so consecutive workgroups share
// the A tile through L2.
template <int OPA, int OPB, int BM, int BN, typename RT = double>
__global__ __launch_bounds__(256) void zgemm_kernel(GemmParams p) {
  constexpr bool F32 = sizeof(RT) == 4;
  constexpr int TI = BM / 32, TJ = BN / 32;
  constexpr int RA = BM * BK / 256, RB = BN * BK / 256;  // elements per thread
  __shared__ RT Ar[BK][BM + PAD], Ai[BK][BM + PAD];  // Ai holds -Im(A)
  __shared__ RT Ap[BK][BM + PAD];                    // +Im(A)
  __shared__ RT Br[BK][BN + PAD], Bi[BK][BN + PAD];

  const int nsplit = gridDim.z / p.batch;
  const int bz = blockIdx.z % p.batch;
  const int split = blockIdx.z / p.batch;
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * BM;
  const int kbeg = split * p.kchunk;
  const int kend = min(p.K, kbeg + p.kchunk);
  const zc* A = p.A + p.sA * (long)bz;
  const zc* B = p.B + p.sB * (long)bz;

  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);
  const int lr = lane & 15, lk = lane >> 4;

  dbl4 accR[TI][TJ], accI[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      accR[i][j] = dbl4{0, 0, 0, 0};
      accI[i][j] = dbl4{0, 0, 0, 0};
    }

  // thread -> (row, k) of the A tile and (k, col) of the B tile, following
  // the memory order of each operand so that global loads coalesce
  auto a_idx = [&](int r, int& mm, int& kk) {
    if (OPA == OPN) {
      mm = t % BM;
      kk = t / BM + (256 / BM) * r;
    } else {
      kk = t % BK;
      mm = t / BK + (256 / BK) * r;
    }
  };
  auto b_idx = [&](int r, int& kk, int& nn) {
    if (OPB == OPN) {
      kk = t % BK;
      nn = t / BK + (256 / BK) * r;
    } else {
      nn = t % BN;
      kk = t / BN + (256 / BN) * r;
    }
  };
  zc ra[RA], rb[RB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      int mm, kk;
      a_idx(r, mm, kk);
      ra[r] = load_op<OPA>(A, p.lda, m0 + mm, k0 + kk, p.M, kend);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int kk, nn;
      b_idx(r, kk, nn);
      rb[r] = load_op<OPB>(B, p.ldb, k0 + kk, n0 + nn, kend, p.N);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      int mm, kk;
      a_idx(r, mm, kk);
      Ar[kk][mm] = (RT)ra[r].x;
      Ai[kk][mm] = -(RT)ra[r].y;
      Ap[kk][mm] = (RT)ra[r].y;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int kk, nn;
      b_idx(r, kk, nn);
      Br[kk][nn] = (RT)rb[r].x;
      Bi[kk][nn] = (RT)rb[r].y;
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
    if constexpr (F32) {
      // one K step in float, then into the double accumulators
      flt4 fR[TI][TJ], fI[TI][TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          fR[i][j] = flt4{0, 0, 0, 0};
          fI[i][j] = flt4{0, 0, 0, 0};
        }
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
        float ar[TI], an[TI], ap[TI], br[TJ], bi[TJ];
#pragma unroll
        for (int i = 0; i < TI; ++i) {
          ar[i] = Ar[ks + lk][wm + 16 * i + lr];
          an[i] = Ai[ks + lk][wm + 16 * i + lr];
          ap[i] = Ap[ks + lk][wm + 16 * i + lr];
        }
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          br[j] = Br[ks + lk][wn + 16 * j + lr];
          bi[j] = Bi[ks + lk][wn + 16 * j + lr];
        }
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) {
            fR[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], br[j], fR[i][j], 0, 0, 0);
            fR[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(an[i], bi[j], fR[i][j], 0, 0, 0);
            fI[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bi[j], fI[i][j], 0, 0, 0);
            fI[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ap[i], br[j], fI[i][j], 0, 0, 0);
          }
      }
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            accR[i][j][v] += (double)fR[i][j][v];
            accI[i][j][v] += (double)fI[i][j][v];
          }
    } else {
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
        double ar[TI], an[TI], ap[TI], br[TJ], bi[TJ];
#pragma unroll
        for (int i = 0; i < TI; ++i) {
          ar[i] = Ar[ks + lk][wm + 16 * i + lr];
          an[i] = Ai[ks + lk][wm + 16 * i + lr];
          ap[i] = Ap[ks + lk][wm + 16 * i + lr];
        }
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          br[j] = Br[ks + lk][wn + 16 * j + lr];
          bi[j] = Bi[ks + lk][wn + 16 * j + lr];
        }
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) {
            accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], accR[i][j], 0, 0, 0);
            accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(an[i], bi[j], accR[i][j], 0, 0, 0);
            accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], accI[i][j], 0, 0, 0);
            accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[i], br[j], accI[i][j], 0, 0, 0);
          }
      }
    }
    __syncthreads();
    if (more) {
      sstore();
      __syncthreads();
    }
  }

  // result layout: register v of lane l holds D[4 v + l/16][l % 16] of
  // each 16 x 16 tile for v_mfma_f64_16x16x4f64, D[4 (l/16) + v][l % 16]
  // for v_mfma_f32_16x16x4f32
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + 16 * i + (F32 ? 4 * lk + v : 4 * v + lk);
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

// C = alpha sum_s ws[s] + beta C.  SK_LANES consecutive lanes share one
// element: lane u adds splits u, u + SK_LANES, ... (four independent sums),
// then the lanes' sums are combined by a fixed butterfly, so the result does
// not depend on timing; many lanes per element keep enough loads in flight
// for the small outputs (a few thousand elements, up to 128 splits) of the
// skinny projections.
constexpr int SK_LANES = 8;
__global__ __launch_bounds__(256) void splitk_reduce(GemmParams p, int nsplit) {
  const long total = (long)p.M * p.N * p.batch;
  const int u = threadIdx.x % SK_LANES;
  const long per_block = 256 / SK_LANES;
  const long stride = (long)p.batch * p.M * p.N;
  for (long e0 = blockIdx.x * per_block; e0 < total; e0 += (long)gridDim.x * per_block) {
    const long e = e0 + threadIdx.x / SK_LANES;
    const bool live = e < total;
    double pr[4] = {0, 0, 0, 0}, pi[4] = {0, 0, 0, 0};
    if (live) {
      const zc* src = p.ws + e;
      int s = u, q = 0;
      for (; s + 3 * SK_LANES < nsplit; s += 4 * SK_LANES) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const zc v = src[stride * (s + w * SK_LANES)];
          pr[w] += v.x;
          pi[w] += v.y;
        }
      }
      for (; s < nsplit; s += SK_LANES, ++q) {
        const zc v = src[stride * s];
        pr[q] += v.x;
        pi[q] += v.y;
      }
    }
    double re = (pr[0] + pr[1]) + (pr[2] + pr[3]);
    double im = (pi[0] + pi[1]) + (pi[2] + pi[3]);
#pragma unroll
    for (int off = 1; off < SK_LANES; off <<= 1) {
      re += __shfl_xor(re, off, 64);
      im += __shfl_xor(im, off, 64);
    }
    if (!live || u != 0) continue;
    const int bz = (int)(e / ((long)p.M * p.N));
    const long mn = e - (long)bz * p.M * p.N;
    const int n = (int)(mn / p.M), m = (int)(mn - (long)n * p.M);
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

void splitk_finish(tt_ctx* ctx, int M, int N, int batch, int nsplit, zc* ws, zc alpha, zc beta, zc* C, long ldc,
                   long strideC) {
  GemmParams p;
  p.M = M; p.N = N; p.K = 0; p.kchunk = 0;
  p.A = nullptr; p.lda = 0; p.sA = 0;
  p.B = nullptr; p.ldb = 0; p.sB = 0;
  p.C = C; p.ldc = ldc; p.sC = strideC;
  p.alpha = alpha; p.beta = beta; p.batch = batch; p.ws = ws;
  const long total = (long)M * N * batch;
  const int blocks = (int)std::min<long>((total + 256 / SK_LANES - 1) / (256 / SK_LANES), 8192);
  KTimer kt(ctx, "zgemm_reduce", 0.0, 16.0 * (double)total * (nsplit + 1 + (beta.x != 0.0 || beta.y != 0.0)));
  hipLaunchKernelGGL(splitk_reduce, dim3(blocks), dim3(256), 0, ctx->stream, p, nsplit);
}

template <int BM, int BN, typename RT = double>
void launch_tile(KTimer& kt, int opA, int opB, dim3 grid, hipStream_t st, const GemmParams& p) {
#define TTF_GEMM_CASE(OA, OB)                                                        \
  if (opA == OA && opB == OB) {                                                      \
    TTF_LAUNCH(kt, (zgemm_kernel<OA, OB, BM, BN, RT>), grid, dim3(256), 0, st, p); \
    return;                                                                          \
  }
  TTF_GEMM_CASE(OPN, OPN)
  TTF_GEMM_CASE(OPN, OPT)
  TTF_GEMM_CASE(OPN, OPC)
  TTF_GEMM_CASE(OPT, OPN)
  TTF_GEMM_CASE(OPT, OPT)
  TTF_GEMM_CASE(OPT, OPC)
  TTF_GEMM_CASE(OPC, OPN)
  TTF_GEMM_CASE(OPC, OPT)
  TTF_GEMM_CASE(OPC, OPC)
#undef TTF_GEMM_CASE
  fail(TT_EINVAL, "zgemm: bad op");
}

void zgemm_prec(int fmt, tt_ctx* ctx, int opA, int opB, int M, int N, int K, zc alpha, const zc* A,
                long lda, long strideA, const zc* B, long ldb, long strideB, zc beta, zc* C, long ldc,
                long strideC, int batch) {
  if (fmt == TT_PREC_BF16X3 || fmt == TT_PREC_FP16X3) {
    zgemm_split(fmt, ctx, opA, opB, M, N, K, alpha, A, lda, strideA, B, ldb, strideB, beta, C, ldc, strideC, batch);
    return;
  }
  if (fmt != TT_PREC_FP64 && fmt != TT_PREC_FP32) fail(TT_EINVAL, "zgemm: unknown precision");
  const bool f32 = fmt == TT_PREC_FP32;
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) {
    // C = beta C: reuse the kernel with an empty K range (kernel writes alpha*0 + beta*C)
    K = 0;
  }
  GemmParams p;
  p.M = M; p.N = N; p.K = K;
  p.A = A; p.lda = lda; p.sA = strideA;
  p.B = B; p.ldb = ldb; p.sB = strideB;
  p.C = C; p.ldc = ldc; p.sC = strideC;
  p.alpha = alpha; p.beta = beta; p.batch = batch; p.ws = nullptr;
  // tile shape: narrow outputs take 32-wide tiles, tall ones 128 rows
  int bm = 64, bn = 64;
  if (N <= 32) {
    bn = 32;
    bm = (M <= 32) ? 32 : (M >= 4096 ? 128 : 64);
  } else if (M <= 32) {
    bm = 32;
    bn = 64;
  }
  int gx = (N + bn - 1) / bn, gy = (M + bm - 1) / bm;
  const long tiles = (long)gx * gy * batch;
  // split K when the output grid alone cannot occupy the chip (fewer tiles
  // than compute units) and the output is small enough for the partial sums
  // to be cheap to reduce (at most 256K elements: the tall panel updates of
  // the QR factorisations run unsplit), up to about two workgroups per
  // compute unit, keeping at least two K steps per split
  int nsplit = 1;
  const int kb = BK;
  const int kblocks = (K + kb - 1) / kb;
  if (tiles < 256 && (long)M * N * batch <= (1L << 18) && kblocks >= 4) {
    nsplit = (int)std::min<long>((512 + tiles - 1) / tiles, kblocks / 2);
    nsplit = std::max(1, std::min(nsplit, 128));
  }
  {
    // a tuned launch shape for this GEMM replaces the rule above
    GemmChoice c;
    if (gemm_choice(fmt, opA, opB, M, N, K, batch, &c)) {
      const bool ok = (c.a == 64 && (c.b == 64 || c.b == 32)) || (c.a == 128 && c.b == 32) ||
                      (c.a == 32 && (c.b == 32 || c.b == 64));
      if (!ok || c.nsplit < 1 || c.nsplit > 128) fail(TT_EINVAL, "zgemm: bad tuned launch shape");
      bm = c.a;
      bn = c.b;
      gx = (N + bn - 1) / bn;
      gy = (M + bm - 1) / bm;
      nsplit = std::max(1, std::min(c.nsplit, std::max(1, kblocks)));
    }
  }
  nsplit = (int)std::max<size_t>(1, std::min<size_t>(nsplit, SPLITK_WS_ELEMS / std::max<size_t>(1, (size_t)M * N * batch)));
  int kchunk = ((kblocks + nsplit - 1) / nsplit) * kb;
  if (K == 0) kchunk = 0;
  nsplit = (K == 0) ? 1 : (K + kchunk - 1) / kchunk;
  p.kchunk = kchunk;
  const double flops = 8.0 * M * N * (double)K * batch;
  // algorithmic bytes of the product: operands read once, C written once
  // (and read once when beta != 0); split-K partials are the reduce's
  const double bytes = 16.0 * ((double)M * K + (double)K * N + (1.0 + (beta.x != 0.0 || beta.y != 0.0)) * M * N) * batch;
  if (nsplit > 1) {
    p.ws = (zc*)ctx->get_ws("gemm_splitk", sizeof(zc) * (size_t)nsplit * batch * M * N);
  }
  if ((long)batch * nsplit > 65535 || gy > 65535) fail(TT_EINVAL, "zgemm: grid too large");
  {
    // with shape profiling on, the launch is also recorded under its shape
    std::string shape;
    if (ctx->profile_shapes) {
      const char ops[3] = {'N', 'T', 'C'};
      shape = std::string(f32 ? "zgemm_fp32:" : "zgemm:") + ops[opA] + ops[opB] + ":" + std::to_string(M) + "x" +
              std::to_string(N) + "x" +
              std::to_string(K) + "x" + std::to_string(batch);
    }
    KTimer kt2(ctx->profile_shapes ? ctx : nullptr, shape.c_str(), flops, bytes);
    {
      KTimer kt(ctx, f32 ? "zgemm_fp32" : "zgemm", flops, bytes, true);
      const dim3 grid(gx, gy, batch * nsplit);
      if (f32) {
        if (bm == 64 && bn == 64)
          launch_tile<64, 64, float>(kt, opA, opB, grid, ctx->stream, p);
        else if (bm == 128)
          launch_tile<128, 32, float>(kt, opA, opB, grid, ctx->stream, p);
        else if (bm == 64)
          launch_tile<64, 32, float>(kt, opA, opB, grid, ctx->stream, p);
        else if (bn == 32)
          launch_tile<32, 32, float>(kt, opA, opB, grid, ctx->stream, p);
        else
          launch_tile<32, 64, float>(kt, opA, opB, grid, ctx->stream, p);
      } else if (bm == 64 && bn == 64)
        launch_tile<64, 64>(kt, opA, opB, grid, ctx->stream, p);
      else if (bm == 128)
        launch_tile<128, 32>(kt, opA, opB, grid, ctx->stream, p);
      else if (bm == 64)
        launch_tile<64, 32>(kt, opA, opB, grid, ctx->stream, p);
      else if (bn == 32)
        launch_tile<32, 32>(kt, opA, opB, grid, ctx->stream, p);
      else
        launch_tile<32, 64>(kt, opA, opB, grid, ctx->stream, p);
    }
    if (nsplit > 1) splitk_finish(ctx, M, N, batch, nsplit, p.ws, alpha, beta, C, ldc, strideC);
  }
  TTF_HIP(hipGetLastError());
}

void zgemm(tt_ctx* ctx, int opA, int opB, int M, int N, int K, zc alpha, const zc* A, long lda, long strideA,
           const zc* B, long ldb, long strideB, zc beta, zc* C, long ldc, long strideC, int batch) {
  zgemm_prec(TT_PREC_FP64, ctx, opA, opB, M, N, K, alpha, A, lda, strideA, B, ldb, strideB, beta, C, ldc, strideC,
             batch);
}

}  // namespace ttf
