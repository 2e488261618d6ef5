// Complex GEMM in split 16-bit arithmetic on the CDNA4 matrix cores: the
// mixed-precision form of the sketch contractions.
//
// C = alpha op(A) op(B) + beta C with FP64 complex operands and result, as
// zgemm, in two steps:
//  1. split_planes: each operand, with its op applied, is rewritten once as
//     rows of K (rows = M for A, N for B), K cut into blocks of 32.  Every
//     (row, block) is scaled by the power of two 2^(14 - e), e the largest
//     binary exponent of its components (exact), and each real component x
//     becomes hi + lo in the 16-bit format: hi = round(x), lo = round(x - hi)
//     (through an FP32 intermediate).  Layout per (row, block): 4 planes of
//     32 halves (Re hi, Re lo, Im hi, Im lo), K contiguous, 256 bytes; the
//     exponent e is stored beside it (one int per (row, block)).
//     FP16 halves keep about 22 significant bits, BF16 halves about 17.
//  2. zgemm_planes: a 16-bit GEMM over the planes.  Each real product is
//     hi*hi + hi*lo + lo*hi (three v_mfma_f32_16x16x32 products, FP32
//     accumulation), twelve per complex product.  After every K block the
//     FP32 accumulators are added into FP64 ones with the scale
//     2^(e_A(row) + e_B(col) - 28) undone, so no FP32 sum runs over more
//     than 32 terms of K and no operand range limit applies.
// Workgroup tiles (32 TI) x (32 TJ), 256 threads = 2 x 2 wavefronts each
// owning TI x TJ MFMA tiles of 16 x 16; the K block of both operand tiles
// is staged through LDS (rows padded by 16 bytes against bank conflicts).
// 16x16x32 operand layout: lane l holds row (l % 16) and the 8 consecutive
// K values starting at 8 (l / 16), for A and B alike (any K assignment
// shared by both operands gives the same sum); result register v of lane l
// holds D[4 (l / 16) + v][l % 16].
#include <string>

#include "common.hpp"

namespace ttf {

constexpr int SP_K = 32;          // K block
constexpr int SP_ROW = 4 * SP_K;  // halves per (row, block): four planes
constexpr int SP_EXP = 14;        // scaled block maxima lie in [2^14, 2^15)
constexpr int SP_LROW = SP_ROW + 8;  // LDS row stride in halves (272 bytes)

typedef _Float16 hf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float fl4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned short bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}

template <int FMT>
__device__ inline void split16(float x, unsigned short& hi, unsigned short& lo) {
  if constexpr (FMT == TT_PREC_BF16X3) {
    hi = bf16_round(x);
    lo = bf16_round(x - __uint_as_float((unsigned)hi << 16));
  } else {
    const _Float16 h = (_Float16)x;
    hi = __builtin_bit_cast(unsigned short, h);
    lo = __builtin_bit_cast(unsigned short, (_Float16)(x - (float)h));
  }
}

// ------------------------------------------------------------ split_planes
// Element (r, k) of the operand is X[r * sr + k * sk] (conjugated with
// conj), with (sr, sk) = (ld, 1) when K is contiguous (KCONTIG) and (1, ld)
// otherwise.  Grid (ceil(R / 64), KB, batch); 256 threads, four per row,
// eight K values each.
template <int FMT, bool KCONTIG>
__global__ __launch_bounds__(256) void split_planes_kernel(const zc* __restrict__ X, long ld, long sX, int R, int K,
                                                           int KB, int conj, unsigned short* __restrict__ H,
                                                           int* __restrict__ E) {
  const int bz = blockIdx.z, kb = blockIdx.y, r0 = blockIdx.x * 64;
  const zc* Xb = X + sX * (long)bz;
  const int t = threadIdx.x, row = t >> 2, ks = (t & 3) * 8;
  const int r = r0 + row;
  const int kbase = kb * SP_K;
  // the 64 x SP_K tile goes through LDS, read so that consecutive lanes
  // take consecutive addresses: along K (32 lanes per row) when K is
  // contiguous, along the rows otherwise
  __shared__ zc T[SP_K][65];
  if constexpr (KCONTIG) {
    const int kk = t & (SP_K - 1), k = kbase + kk;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int rr = (t >> 5) + 8 * j;
      T[kk][rr] = (r0 + rr < R && k < K) ? Xb[k + ld * (long)(r0 + rr)] : make_double2(0.0, 0.0);
    }
  } else {
    const int rr = t & 63;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kk = (t >> 6) + 4 * j, k = kbase + kk;
      T[kk][rr] = (r0 + rr < R && k < K) ? Xb[(r0 + rr) + ld * (long)k] : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  zc v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = T[ks + j][row];
  double mx = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (conj) v[j].y = -v[j].y;
    mx = fmax(mx, fmax(fabs(v[j].x), fabs(v[j].y)));
  }
  // the four lanes of a row are adjacent in one wavefront
  mx = fmax(mx, __shfl_xor(mx, 1, 64));
  mx = fmax(mx, __shfl_xor(mx, 2, 64));
  const int e = mx > 0.0 ? min(max(ilogb(mx), -1100), 1100) : 0;
  const int s = SP_EXP - e;
  unsigned short p[4][8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    split16<FMT>((float)ldexp(v[j].x, s), p[0][j], p[1][j]);
    split16<FMT>((float)ldexp(v[j].y, s), p[2][j], p[3][j]);
  }
  if (r < R) {
    unsigned short* out = H + (((long)bz * R + r) * KB + kb) * SP_ROW + ks;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      u4 w;
      w.x = p[q][0] | ((unsigned)p[q][1] << 16);
      w.y = p[q][2] | ((unsigned)p[q][3] << 16);
      w.z = p[q][4] | ((unsigned)p[q][5] << 16);
      w.w = p[q][6] | ((unsigned)p[q][7] << 16);
      *reinterpret_cast<u4*>(out + q * SP_K) = w;
    }
    if ((t & 3) == 0) E[((long)bz * R + r) * KB + kb] = e;
  }
}

static void split_planes(int fmt, tt_ctx* ctx, const zc* X, long ld, long sX, int R, int K, int batch, bool kcontig,
                         bool conj, unsigned short* H, int* E) {
  const int KB = (K + SP_K - 1) / SP_K;
  if (R <= 0 || KB <= 0 || batch <= 0) return;
  if (KB > 65535 || batch > 65535) fail(TT_EINVAL, "split_planes: grid too large");
  const dim3 grid((R + 63) / 64, KB, batch);
  const double elems = (double)R * K * batch;
  KTimer kt(ctx, "split_planes", 0.0, elems * (16.0 + 8.0) + 4.0 * (double)R * KB * batch);
#define TTF_SPLIT_LAUNCH(F, KC) \
  hipLaunchKernelGGL((split_planes_kernel<F, KC>), grid, dim3(256), 0, ctx->stream, X, ld, sX, R, K, KB, conj ? 1 : 0, H, E)
  if (fmt == TT_PREC_BF16X3) {
    if (kcontig) TTF_SPLIT_LAUNCH(TT_PREC_BF16X3, true); else TTF_SPLIT_LAUNCH(TT_PREC_BF16X3, false);
  } else {
    if (kcontig) TTF_SPLIT_LAUNCH(TT_PREC_FP16X3, true); else TTF_SPLIT_LAUNCH(TT_PREC_FP16X3, false);
  }
#undef TTF_SPLIT_LAUNCH
  TTF_HIP(hipGetLastError());
}

// ------------------------------------------------------------ zgemm_planes
struct PlaneGemm {
  const unsigned short* A;
  const int* Ea;
  long rowsA;  // rows per batch of the A planes (0: one A for every batch)
  const unsigned short* B;
  const int* Eb;
  long rowsB;
  int M, N, KB, kbchunk, batch;
  zc alpha, beta;
  zc* C;
  long ldc, sC;
  zc* ws;  // split-K partials [split][batch][N][M]
};

template <int FMT>
__device__ inline fl4 mfma32(u4 a, u4 b, fl4 c) {
  if constexpr (FMT == TT_PREC_BF16X3)
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(hf8, a), __builtin_bit_cast(hf8, b), c, 0, 0, 0);
}

template <int FMT, int TI, int TJ>
__global__ __launch_bounds__(256, 2) void zgemm_planes_kernel(PlaneGemm p) {
  constexpr int BM = 32 * TI, BN = 32 * TJ;
  constexpr int QA = BM / 16, QB = BN / 16;  // 16-byte chunks per thread
  // the operand tiles; after the K loop the same memory stages the output
  __shared__ __align__(16) unsigned short AB[(BM + BN) * SP_LROW];
  unsigned short* const As = AB;
  unsigned short* const Bs = AB + BM * SP_LROW;
  __shared__ int ea_s[BM], eb_s[BN];

  const int nsplit = gridDim.z / p.batch;
  const int bz = blockIdx.z % p.batch;
  const int split = blockIdx.z / p.batch;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int kb0 = split * p.kbchunk;
  const int kb1 = min(p.KB, kb0 + p.kbchunk);
  const long rA = p.rowsA * bz, rB = p.rowsB * bz;  // first row of this batch

  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);
  const int lr = lane & 15, lq = lane >> 4;

  double dR[TI][TJ][4], dI[TI][TJ][4];
  fl4 fR[TI][TJ], fI[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      fR[i][j] = fl4{0, 0, 0, 0};
      fI[i][j] = fl4{0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 4; ++v) dR[i][j][v] = dI[i][j][v] = 0.0;
    }

  u4 ra[QA], rb[QB];
  int rexp = 0;
  auto gload = [&](int kb) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int c = t + 256 * q, row = c >> 4, part = c & 15;
      const int m = m0 + row;
      ra[q] = m < p.M ? *reinterpret_cast<const u4*>(p.A + ((rA + m) * p.KB + kb) * SP_ROW + part * 8)
                      : u4{0, 0, 0, 0};
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int c = t + 256 * q, row = c >> 4, part = c & 15;
      const int n = n0 + row;
      rb[q] = n < p.N ? *reinterpret_cast<const u4*>(p.B + ((rB + n) * p.KB + kb) * SP_ROW + part * 8)
                      : u4{0, 0, 0, 0};
    }
    if (t < BM)
      rexp = m0 + t < p.M ? p.Ea[(rA + m0 + t) * p.KB + kb] : 0;
    else if (t < BM + BN)
      rexp = n0 + t - BM < p.N ? p.Eb[(rB + n0 + t - BM) * p.KB + kb] : 0;
  };
  auto sstore = [&]() {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int c = t + 256 * q, row = c >> 4, part = c & 15;
      *reinterpret_cast<u4*>(&As[row * SP_LROW + part * 8]) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int c = t + 256 * q, row = c >> 4, part = c & 15;
      *reinterpret_cast<u4*>(&Bs[row * SP_LROW + part * 8]) = rb[q];
    }
    if (t < BM)
      ea_s[t] = rexp;
    else if (t < BM + BN)
      eb_s[t - BM] = rexp;
  };

  if (kb0 < kb1) {
    gload(kb0);
    sstore();
  }
  __syncthreads();
  const u4 sign = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  for (int kb = kb0; kb < kb1; ++kb) {
    const bool more = kb + 1 < kb1;
    if (more) gload(kb + 1);
    u4 b[TJ][6];
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const unsigned short* src = &Bs[(wn + 16 * j + lr) * SP_LROW + 8 * lq];
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) b[j][pl] = *reinterpret_cast<const u4*>(src + pl * SP_K);
      b[j][4] = b[j][2] ^ sign;  // -Im hi, -Im lo
      b[j][5] = b[j][3] ^ sign;
    }
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      u4 a[4];
      const unsigned short* src = &As[(wm + 16 * i + lr) * SP_LROW + 8 * lq];
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) a[pl] = *reinterpret_cast<const u4*>(src + pl * SP_K);
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        fl4 r = fR[i][j], m = fI[i][j];
        // Re += Re A Re B + Im A (-Im B);  Im += Re A Im B + Im A Re B
        r = mfma32<FMT>(a[0], b[j][0], r);
        r = mfma32<FMT>(a[0], b[j][1], r);
        r = mfma32<FMT>(a[1], b[j][0], r);
        r = mfma32<FMT>(a[2], b[j][4], r);
        r = mfma32<FMT>(a[2], b[j][5], r);
        r = mfma32<FMT>(a[3], b[j][4], r);
        m = mfma32<FMT>(a[0], b[j][2], m);
        m = mfma32<FMT>(a[0], b[j][3], m);
        m = mfma32<FMT>(a[1], b[j][2], m);
        m = mfma32<FMT>(a[2], b[j][0], m);
        m = mfma32<FMT>(a[2], b[j][1], m);
        m = mfma32<FMT>(a[3], b[j][0], m);
        fR[i][j] = r;
        fI[i][j] = m;
      }
    }
    // fold the block into FP64 with its scales undone
    int eb[TJ];
#pragma unroll
    for (int j = 0; j < TJ; ++j) eb[j] = eb_s[wn + 16 * j + lr] - 2 * SP_EXP;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ea = ea_s[wm + 16 * i + 4 * lq + v];
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          dR[i][j][v] += ldexp((double)fR[i][j][v], ea + eb[j]);
          dI[i][j][v] += ldexp((double)fI[i][j][v], ea + eb[j]);
        }
      }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        fR[i][j] = fl4{0, 0, 0, 0};
        fI[i][j] = fl4{0, 0, 0, 0};
      }
    __syncthreads();
    if (more) {
      sstore();
      __syncthreads();
    }
  }

  // Output through LDS, half the tile's columns at a time (the two wave
  // columns in turn): each wave leaves its values in a column-major tile
  // (BM + 1 rows per column: conflict-free), then consecutive lanes store
  // consecutive rows of a column.
  constexpr int HN = BN / 2, LDT = BM + 1;
  static_assert(HN * LDT * 16 <= (BM + BN) * SP_LROW * 2, "output staging exceeds the operand tiles");
  zc* const T = reinterpret_cast<zc*>(AB);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();
    if ((wave >> 1) == h) {
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            T[(16 * j + lr) * LDT + wm + 16 * i + 4 * lq + v] = make_double2(dR[i][j][v], dI[i][j][v]);
    }
    __syncthreads();
    for (int e = t; e < BM * HN; e += 256) {
      const int row = e % BM, col = e / BM;
      const int m = m0 + row, n = n0 + h * HN + col;
      if (m >= p.M || n >= p.N) continue;
      const zc d = T[col * LDT + row];
      if (nsplit > 1) {
        zc* w = p.ws + ((long)split * p.batch + bz) * (long)p.M * p.N;
        w[m + (long)p.M * n] = d;
      } else {
        zc* C = p.C + p.sC * (long)bz;
        zc out = make_double2(p.alpha.x * d.x - p.alpha.y * d.y, p.alpha.x * d.y + p.alpha.y * d.x);
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
}

template <int TI, int TJ>
static void launch_planes(KTimer& kt, int fmt, dim3 grid, hipStream_t st, const PlaneGemm& p) {
  if (fmt == TT_PREC_BF16X3)
    TTF_LAUNCH(kt, (zgemm_planes_kernel<TT_PREC_BF16X3, TI, TJ>), grid, dim3(256), 0, st, p);
  else
    TTF_LAUNCH(kt, (zgemm_planes_kernel<TT_PREC_FP16X3, TI, TJ>), grid, dim3(256), 0, st, p);
}

void zgemm_split(int fmt, tt_ctx* ctx, int opA, int opB, int M, int N, int K, zc alpha, const zc* A, long lda,
                 long strideA, const zc* B, long ldb, long strideB, zc beta, zc* C, long ldc, long strideC,
                 int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  const int KB = K > 0 ? (K + SP_K - 1) / SP_K : 0;
  const int batchA = strideA == 0 ? 1 : batch, batchB = strideB == 0 ? 1 : batch;
  unsigned short* Ha = nullptr;
  unsigned short* Hb = nullptr;
  int* Ea = nullptr;
  int* Eb = nullptr;
  if (KB > 0) {
    const size_t blocksA = (size_t)batchA * M * KB, blocksB = (size_t)batchB * N * KB;
    Ha = (unsigned short*)ctx->get_ws("mx_planes_A", blocksA * SP_ROW * 2);
    Hb = (unsigned short*)ctx->get_ws("mx_planes_B", blocksB * SP_ROW * 2);
    Ea = (int*)ctx->get_ws("mx_exp_A", blocksA * 4);
    Eb = (int*)ctx->get_ws("mx_exp_B", blocksB * 4);
    // op(A)(m, k) is A[m + lda k] (N) or A[k + lda m] (T, C): K contiguous
    // unless N; op(B)(k, n) is B[k + ldb n] (N) or B[n + ldb k] (T, C)
    split_planes(fmt, ctx, A, lda, strideA, M, K, batchA, opA != OPN, opA == OPC, Ha, Ea);
    split_planes(fmt, ctx, B, ldb, strideB, N, K, batchB, opB == OPN, opB == OPC, Hb, Eb);
  }
  PlaneGemm p;
  p.A = Ha; p.Ea = Ea; p.rowsA = strideA == 0 ? 0 : M;
  p.B = Hb; p.Eb = Eb; p.rowsB = strideB == 0 ? 0 : N;
  p.M = M; p.N = N; p.KB = KB; p.batch = batch;
  p.alpha = alpha; p.beta = beta; p.C = C; p.ldc = ldc; p.sC = strideC; p.ws = nullptr;
  // tile: 64 x 64, or 32 rows / columns for narrow outputs
  int ti = 2, tj = 2;
  if (M <= 32) ti = 1;
  if (N <= 32) tj = 1;
  GemmChoice tuned;
  const bool have_tuned = gemm_choice(fmt, opA, opB, M, N, K, batch, &tuned);
  if (have_tuned) {
    if (tuned.a < 1 || tuned.a > 2 || tuned.b < 1 || tuned.b > 2 || tuned.nsplit < 1 || tuned.nsplit > 128)
      fail(TT_EINVAL, "zgemm_split: bad tuned launch shape");
    ti = tuned.a;
    tj = tuned.b;
  }
  const int bm = 32 * ti, bn = 32 * tj;
  const int gx = (M + bm - 1) / bm, gy = (N + bn - 1) / bn;
  const long tiles = (long)gx * gy * batch;
  int nsplit = 1;
  if (tiles < 512 && KB >= 4) nsplit = (int)std::max<long>(1, std::min<long>({(512 + tiles - 1) / tiles, KB / 2, 128}));
  if (have_tuned) nsplit = std::max(1, std::min(tuned.nsplit, std::max(1, KB)));
  nsplit = (int)std::max<size_t>(1, std::min<size_t>(nsplit, SPLITK_WS_ELEMS / std::max<size_t>(1, (size_t)M * N * batch)));
  int kbchunk = KB > 0 ? (KB + nsplit - 1) / nsplit : 0;
  nsplit = KB > 0 ? (KB + kbchunk - 1) / kbchunk : 1;
  p.kbchunk = kbchunk;
  if (nsplit > 1) p.ws = (zc*)ctx->get_ws("gemm_splitk", sizeof(zc) * (size_t)nsplit * batch * M * N);
  if ((long)batch * nsplit > 65535 || gy > 65535) fail(TT_EINVAL, "zgemm_split: grid too large");
  const double flops = 8.0 * M * N * (double)K * batch;
  const double bytes = 8.0 * ((double)M * batchA + (double)N * batchB) * KB * SP_K +
                       16.0 * (1.0 + (beta.x != 0.0 || beta.y != 0.0)) * M * N * batch;
  {
    std::string shape;
    if (ctx->profile_shapes) {
      const char ops[3] = {'N', 'T', 'C'};
      shape = std::string(fmt == TT_PREC_BF16X3 ? "zgemm_bf16x3:" : "zgemm_fp16x3:") + ops[opA] + ops[opB] + ":" +
              std::to_string(M) + "x" + std::to_string(N) + "x" + std::to_string(K) + "x" + std::to_string(batch);
    }
    KTimer kt2(ctx->profile_shapes ? ctx : nullptr, shape.c_str(), flops, bytes);
    {
      // the class counts the 16-bit products it executes (three per real
      // product) against the 16-bit matrix-core peak
      KTimer kt(ctx, fmt == TT_PREC_BF16X3 ? "zgemm_bf16x3" : "zgemm_fp16x3", 3.0 * flops, bytes, true);
      const dim3 grid(gx, gy, batch * nsplit);
      if (ti == 2 && tj == 2)
        launch_planes<2, 2>(kt, fmt, grid, ctx->stream, p);
      else if (ti == 1 && tj == 2)
        launch_planes<1, 2>(kt, fmt, grid, ctx->stream, p);
      else if (ti == 2)
        launch_planes<2, 1>(kt, fmt, grid, ctx->stream, p);
      else
        launch_planes<1, 1>(kt, fmt, grid, ctx->stream, p);
    }
    if (nsplit > 1) splitk_finish(ctx, M, N, batch, nsplit, p.ws, alpha, beta, C, ldc, strideC);
  }
  TTF_HIP(hipGetLastError());
}

}  // namespace ttf
