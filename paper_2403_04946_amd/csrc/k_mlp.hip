// The learned form's rank predictor: a small fully connected network
// (n_in -> width -> width -> 1, ReLU hidden layers) kept in FP16 on the
// device, with FP32 accumulation, FP32 master weights and Adam updates.
// Batches of a few thousand samples: one thread per output element, every
// sum in a fixed order (no atomics), so forward, gradients and training are
// deterministic.
//
// Parameters, as one vector: W1 (width x n_in, row-major), b1, W2 (width x
// width), b2, W3 (1 x width), b3.  Samples are rows of a B x n_in FP32
// matrix.  Loss: L = (1 / 2B) sum_b (y_b - t_b)^2.
#include "common.hpp"

namespace ttf {

// Y[b][o] = act(sum_i W[o][i] X[b][i] + bias[o]), W and bias in FP16
__global__ void mlp_linear_fwd(const _Float16* __restrict__ W, const _Float16* __restrict__ bias,
                               const float* __restrict__ X, float* __restrict__ Y, int B, int nin, int nout,
                               int relu) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)B * nout) return;
  const int b = (int)(e / nout), o = (int)(e % nout);
  const _Float16* w = W + (long)o * nin;
  const float* x = X + (long)b * nin;
  float s = (float)bias[o];
  for (int i = 0; i < nin; ++i) s = fmaf((float)w[i], x[i], s);
  Y[e] = (relu && s < 0.0f) ? 0.0f : s;
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

// gW[o][i] = sum_b dY[b][o] X[b][i];  gb[o] = sum_b dY[b][o]
__global__ void mlp_linear_bwd_w(const float* __restrict__ dY, const float* __restrict__ X, float* __restrict__ gW,
                                 float* __restrict__ gb, int B, int nin, int nout) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nw = (long)nout * nin;
  if (e < nw) {
    const int o = (int)(e / nin), i = (int)(e % nin);
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s = fmaf(dY[(long)b * nout + o], X[(long)b * nin + i], s);
    gW[e] = s;
  } else if (e < nw + nout) {
    const int o = (int)(e - nw);
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += dY[(long)b * nout + o];
    gb[o] = s;
  }
}

// dX[b][i] = (sum_o dY[b][o] W[o][i]) * [H[b][i] > 0]  (H: the ReLU output)
__global__ void mlp_linear_bwd_x(const _Float16* __restrict__ W, const float* __restrict__ dY,
                                 const float* __restrict__ H, float* __restrict__ dX, int B, int nin, int nout) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)B * nin) return;
  const int b = (int)(e / nin), i = (int)(e % nin);
  float s = 0.0f;
  for (int o = 0; o < nout; ++o) s = fmaf(dY[(long)b * nout + o], (float)W[(long)o * nin + i], s);
  dX[e] = H[e] > 0.0f ? s : 0.0f;
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
  hipLaunchKernelGGL(mlp_linear_fwd, blocks_for((long)B * w), dim3(256), 0, ctx->stream, W1, b1, X, h1, B, ni, w, 1);
  hipLaunchKernelGGL(mlp_linear_fwd, blocks_for((long)B * w), dim3(256), 0, ctx->stream, W2, b2, h1, h2, B, w, w, 1);
  hipLaunchKernelGGL(mlp_linear_fwd, blocks_for(B), dim3(256), 0, ctx->stream, W3, b3, h2, y, B, w, 1, 0);
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
  hipLaunchKernelGGL(mlp_linear_bwd_w, blocks_for((long)w + 1), dim3(256), 0, ctx->stream, d3, h2, gW3, gb3, B, w, 1);
  hipLaunchKernelGGL(mlp_linear_bwd_x, blocks_for((long)B * w), dim3(256), 0, ctx->stream, W3, d3, h2, d2, B, w, 1);
  // second hidden layer
  hipLaunchKernelGGL(mlp_linear_bwd_w, blocks_for((long)w * w + w), dim3(256), 0, ctx->stream, d2, h1, gW2, gb2, B, w,
                     w);
  hipLaunchKernelGGL(mlp_linear_bwd_x, blocks_for((long)B * w), dim3(256), 0, ctx->stream, W2, d2, h1, d1, B, w, w);
  // first hidden layer
  hipLaunchKernelGGL(mlp_linear_bwd_w, blocks_for((long)w * ni + w), dim3(256), 0, ctx->stream, d1, X, gW1, gb1, B,
                     ni, w);
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
