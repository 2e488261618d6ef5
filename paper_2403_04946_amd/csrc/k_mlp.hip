// The learned form's rank predictor: a small fully connected network
// (n_in -> width -> width -> 1, ReLU hidden layers) kept in FP16 on the
// device, with FP32 accumulation, FP32 master weights and Adam updates.
// The three products of each layer (forward, weight gradient, input
// gradient) run on the matrix cores (v_mfma_f32_16x16x4f32): the FP16
// weights widen to FP32 exactly, and the activations and deltas stay FP32,
// which an FP16 product would round.  Every sum has a fixed order (no
// atomics), so forward, gradients and training are deterministic.
//
// Parameters, as one vector: W1 (width x n_in, row-major), b1, W2 (width x
// width), b2, W3 (1 x width), b3.  Samples are rows of a B x n_in FP32
// matrix.  Loss: L = (1 / 2B) sum_b (y_b - t_b)^2.
#include "common.hpp"

namespace ttf {

typedef float flt4 __attribute__((ext_vector_type(4)));

// Epilogues of mlp_mfma_gemm
enum { MLP_BIAS_RELU = 0, MLP_BIAS = 1, MLP_RELU_MASK = 2, MLP_WGRAD = 3 };

// C(m, n) = sum_k A(m, k) B(k, n) with strided operands, A(m, k) =
// A[m sam + k sak] and B(k, n) = B[k sbk + n sbn], so one kernel serves
// Y = X W^T (forward), dX = dY W (input gradient) and gW = dY^T X (weight
// gradient) without transposed copies.
//   MLP_BIAS_RELU, MLP_BIAS: C[m ldc + n] = (relu) (sum + bias[n])
//   MLP_RELU_MASK:           C[m ldc + n] = H[m ldc + n] > 0 ? sum : 0
//   MLP_WGRAD:               column N - 1 of B is taken as ones, so its
//                            column of C, gb[m] = sum_k A(m, k), is the
//                            bias gradient; the others go to C[m ldc + n]
struct MlpGemm {
  const void* A;
  long sam, sak;
  const void* B;
  long sbk, sbn;
  int M, N, K;
  float* C;
  long ldc;
  const _Float16* bias;
  const float* H;
  float* gb;
};

// One workgroup of four waves per 16 x 16 tile of C.  Lane l holds
// A(m0 + l % 16, k + l / 16) and B(k + l / 16, n0 + l % 16) for each step of
// four in k, and register v of its result C(m0 + 4 (l / 16) + v, n0 + l % 16).
// Wave w takes the steps k = 4 w, 4 w + 16, ...; the waves' sums are added
// in the order 0, 1, 2, 3.
template <typename TA, typename TB, int EPI>
__global__ __launch_bounds__(256) void mlp_mfma_gemm(MlpGemm p) {
  __shared__ flt4 part[3][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int ntn = (p.N + 15) / 16;
  const int m0 = (int)(blockIdx.x / ntn) * 16, n0 = (int)(blockIdx.x % ntn) * 16;
  const int m = m0 + lr, n = n0 + lr;
  const TA* A = (const TA*)p.A;
  const TB* B = (const TB*)p.B;
  const bool ones = EPI == MLP_WGRAD && n == p.N - 1;
  flt4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 4 * wave; k0 < p.K; k0 += 16) {
    const int k = k0 + lk;
    float a = 0.0f, b = 0.0f;
    if (m < p.M && k < p.K) a = (float)A[m * p.sam + k * p.sak];
    if (k < p.K && n < p.N) b = ones ? 1.0f : (float)B[k * p.sbk + n * p.sbn];
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  if (wave > 0) part[wave - 1][lane] = acc;
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int w = 0; w < 3; ++w) acc += part[w][lane];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int mm = m0 + 4 * lk + v;
    if (mm >= p.M || n >= p.N) continue;
    const float s = acc[v];
    const long off = mm * p.ldc + n;
    if (EPI == MLP_BIAS_RELU) {
      const float y = s + (float)p.bias[n];
      p.C[off] = y < 0.0f ? 0.0f : y;
    } else if (EPI == MLP_BIAS) {
      p.C[off] = s + (float)p.bias[n];
    } else if (EPI == MLP_RELU_MASK) {
      p.C[off] = p.H[off] > 0.0f ? s : 0.0f;
    } else if (n == p.N - 1) {
      p.gb[mm] = s;
    } else {
      p.C[off] = s;
    }
  }
}

template <typename TA, typename TB, int EPI>
static void mlp_gemm(tt_ctx* ctx, const MlpGemm& g) {
  const unsigned tiles = (unsigned)(((g.M + 15) / 16) * (long)((g.N + 15) / 16));
  hipLaunchKernelGGL((mlp_mfma_gemm<TA, TB, EPI>), dim3(tiles), dim3(256), 0, ctx->stream, g);
}

// Y (B x nout) = act(X W^T + bias): X (B x nin, FP32), W (nout x nin, FP16)
static void linear_fwd(tt_ctx* ctx, const _Float16* W, const _Float16* bias, const float* X, float* Y, int B,
                       int nin, int nout, bool relu) {
  MlpGemm g{X, nin, 1, W, 1, nin, B, nout, nin, Y, nout, bias, nullptr, nullptr};
  if (relu)
    mlp_gemm<float, _Float16, MLP_BIAS_RELU>(ctx, g);
  else
    mlp_gemm<float, _Float16, MLP_BIAS>(ctx, g);
}

// gW (nout x nin) = dY^T X and gb (nout) = dY^T 1: dY (B x nout), X (B x nin)
static void linear_bwd_w(tt_ctx* ctx, const float* dY, const float* X, float* gW, float* gb, int B, int nin,
                         int nout) {
  MlpGemm g{dY, 1, nout, X, nin, 1, nout, nin + 1, B, gW, nin, nullptr, nullptr, gb};
  mlp_gemm<float, float, MLP_WGRAD>(ctx, g);
}

// dX (B x nin) = (dY W) masked by H > 0: dY (B x nout), W (nout x nin, FP16),
// H (B x nin) the ReLU output of the layer's input
static void linear_bwd_x(tt_ctx* ctx, const _Float16* W, const float* dY, const float* H, float* dX, int B,
                         int nin, int nout) {
  MlpGemm g{dY, nout, 1, W, nin, 1, B, nin, nout, dX, nin, nullptr, H, nullptr};
  mlp_gemm<float, _Float16, MLP_RELU_MASK>(ctx, g);
}

// dY[b] = (Y[b] - T[b]) / B and the per-sample squared errors
__global__ void mlp_out_grad(const float* __restrict__ Y, const float* __restrict__ T, float* __restrict__ dY,
                             float* __restrict__ sq, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float r = Y[b] - T[b];
  dY[b] = r / (float)B;
  sq[b] = r * r;
}

// loss = (1 / 2B) sum sq, one workgroup, fixed order
__global__ __launch_bounds__(256) void mlp_loss(const float* __restrict__ sq, int B, float* __restrict__ out) {
  __shared__ float part[256];
  float s = 0.0f;
  for (int b = threadIdx.x; b < B; b += 256) s += sq[b];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = 0.5f * part[0] / (float)B;
}

// Adam on the FP32 master weights; the FP16 copy follows
__global__ void mlp_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                         float* __restrict__ v, _Float16* __restrict__ ph, int n, float lr, float b1, float b2,
                         float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.0f - b1) * gi;
  const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  const float pi = p[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[e] = pi;
  ph[e] = (_Float16)pi;
}

__global__ void mlp_to_half(const float* __restrict__ p, _Float16* __restrict__ ph, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) ph[e] = (_Float16)p[e];
}

__global__ void mlp_from_half(const _Float16* __restrict__ ph, float* __restrict__ p, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = (float)ph[e];
}

static dim3 blocks_for(long n) { return dim3((unsigned)((n + 255) / 256)); }

void mlp_forward(tt_ctx* ctx, const MlpDev& m, const float* X, int B, float* h1, float* h2, float* y) {
  const int w = m.width, ni = m.n_in;
  const _Float16* W1 = m.ph;
  const _Float16* b1 = W1 + (long)w * ni;
  const _Float16* W2 = b1 + w;
  const _Float16* b2 = W2 + (long)w * w;
  const _Float16* W3 = b2 + w;
  const _Float16* b3 = W3 + w;
  KTimer kt(ctx, "mlp_forward", 2.0 * B * ((double)w * ni + (double)w * w + w), 0.0);
  linear_fwd(ctx, W1, b1, X, h1, B, ni, w, true);
  linear_fwd(ctx, W2, b2, h1, h2, B, w, w, true);
  linear_fwd(ctx, W3, b3, h2, y, B, w, 1, false);
  TTF_HIP(hipGetLastError());
}

void mlp_gradients(tt_ctx* ctx, const MlpDev& m, const float* X, const float* T, int B, float* loss_dev) {
  const int w = m.width, ni = m.n_in;
  float* h1 = m.act;
  float* h2 = h1 + (long)m.bcap * w;
  float* y = h2 + (long)m.bcap * w;
  float* d3 = y + m.bcap;
  float* sq = d3 + m.bcap;
  float* d2 = sq + m.bcap;
  float* d1 = d2 + (long)m.bcap * w;
  mlp_forward(ctx, m, X, B, h1, h2, y);
  const _Float16* W2 = m.ph + (long)w * ni + w;
  const _Float16* W3 = W2 + (long)w * w + w;
  float* gW1 = m.g;
  float* gb1 = gW1 + (long)w * ni;
  float* gW2 = gb1 + w;
  float* gb2 = gW2 + (long)w * w;
  float* gW3 = gb2 + w;
  float* gb3 = gW3 + w;
  KTimer kt(ctx, "mlp_backward", 4.0 * B * ((double)w * ni + (double)w * w + w), 0.0);
  hipLaunchKernelGGL(mlp_out_grad, blocks_for(B), dim3(256), 0, ctx->stream, y, T, d3, sq, B);
  hipLaunchKernelGGL(mlp_loss, dim3(1), dim3(256), 0, ctx->stream, sq, B, loss_dev);
  // output layer
  linear_bwd_w(ctx, d3, h2, gW3, gb3, B, w, 1);
  linear_bwd_x(ctx, W3, d3, h2, d2, B, w, 1);
  // second hidden layer
  linear_bwd_w(ctx, d2, h1, gW2, gb2, B, w, w);
  linear_bwd_x(ctx, W2, d2, h1, d1, B, w, w);
  // first hidden layer
  linear_bwd_w(ctx, d1, X, gW1, gb1, B, ni, w);
  TTF_HIP(hipGetLastError());
}

void mlp_adam_step(tt_ctx* ctx, MlpDev& m, float lr) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  m.step += 1;
  const float c1 = 1.0f - powf(b1, (float)m.step), c2 = 1.0f - powf(b2, (float)m.step);
  hipLaunchKernelGGL(mlp_adam, blocks_for(m.nparams), dim3(256), 0, ctx->stream, m.p, m.g, m.m, m.v, m.ph, m.nparams,
                     lr, b1, b2, eps, c1, c2);
  TTF_HIP(hipGetLastError());
}

void mlp_refresh_half(tt_ctx* ctx, MlpDev& m) {
  hipLaunchKernelGGL(mlp_to_half, blocks_for(m.nparams), dim3(256), 0, ctx->stream, m.p, m.ph, m.nparams);
  TTF_HIP(hipGetLastError());
}

void mlp_half_values(tt_ctx* ctx, const MlpDev& m, float* out_dev) {
  hipLaunchKernelGGL(mlp_from_half, blocks_for(m.nparams), dim3(256), 0, ctx->stream, m.ph, out_dev, m.nparams);
  TTF_HIP(hipGetLastError());
}

}  // namespace ttf
