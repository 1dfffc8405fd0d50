// Learned rank: a 512 -> 128 -> 128 -> 1 MLP (FP32, ReLU hidden layers) on
// the pivot-magnitude profile of a sketch's LUPP, with hand-written forward,
// backward and Adam kernels.  Samples are processed 16 per workgroup with
// the sample tile in LDS; batch sums of the gradients are written per
// workgroup and added in a fixed order (deterministic).
#include "rpid_internal.hpp"

namespace rpid {

namespace {
constexpr int IN = RPID_MLP_IN, H = RPID_MLP_H;
constexpr int SB = 16;  // samples per workgroup
constexpr int64_t OFF_W1 = 0, OFF_B1 = (int64_t)H * IN, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
                  OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H, NPARAM = OFF_B3 + 1;
static_assert(NPARAM == RPID_MLP_NPARAM, "parameter layout");

__global__ __launch_bounds__(128) void mlp_forward_kernel(const float* W, const float* x,
                                                          int64_t B, float* y, float* act) {
  __shared__ float xs[SB][IN];
  __shared__ float h1[SB][H];
  __shared__ float red[SB][2];
  const int o = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * SB;
  const int ns = (int)min((int64_t)SB, B - s0);
  for (int e = o; e < SB * IN; e += H) {
    const int s = e / IN, i = e % IN;
    xs[s][i] = (s < ns) ? x[(s0 + s) * IN + i] : 0.0f;
  }
  __syncthreads();
  float acc[SB];
#pragma unroll
  for (int s = 0; s < SB; ++s) acc[s] = W[OFF_B1 + o];
  for (int i = 0; i < IN; ++i) {
    const float w = W[OFF_W1 + (int64_t)o * IN + i];
#pragma unroll
    for (int s = 0; s < SB; ++s) acc[s] = fmaf(w, xs[s][i], acc[s]);
  }
#pragma unroll
  for (int s = 0; s < SB; ++s) h1[s][o] = fmaxf(acc[s], 0.0f);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SB; ++s) acc[s] = W[OFF_B2 + o];
  for (int i = 0; i < H; ++i) {
    const float w = W[OFF_W2 + (int64_t)o * H + i];
#pragma unroll
    for (int s = 0; s < SB; ++s) acc[s] = fmaf(w, h1[s][i], acc[s]);
  }
  const float w3 = W[OFF_W3 + o];
  float part[SB];
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    const float h2 = fmaxf(acc[s], 0.0f);
    if (act && s < ns) {
      act[(s0 + s) * 2 * H + o] = h1[s][o];
      act[(s0 + s) * 2 * H + H + o] = h2;
    }
    part[s] = w3 * h2;
  }
  // sum over the 128 hidden units: two waves of 64
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    float v = part[s];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((o & 63) == 0) red[s][o >> 6] = v;
  }
  __syncthreads();
  if (o < ns) y[s0 + o] = W[OFF_B3] + (red[o][0] + red[o][1]);
}

// Per-workgroup gradient of sum_s dy[s] * y[s] w.r.t. W, into gpart[blockIdx.x].
__global__ __launch_bounds__(128) void mlp_backward_kernel(const float* W, const float* x,
                                                           const float* act, const float* dy,
                                                           int64_t B, float* gpart) {
  __shared__ float xs[SB][IN];
  __shared__ float h1[SB][H];
  __shared__ float dz2[SB][H];
  __shared__ float dz1[SB][H];
  __shared__ float dys[SB];
  const int t = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * SB;
  const int ns = (int)min((int64_t)SB, B - s0);
  float* g = gpart + (int64_t)blockIdx.x * NPARAM;
  for (int e = t; e < SB * IN; e += H) {
    const int s = e / IN, i = e % IN;
    xs[s][i] = (s < ns) ? x[(s0 + s) * IN + i] : 0.0f;
  }
  if (t < SB) dys[t] = (t < ns) ? dy[s0 + t] : 0.0f;
  __syncthreads();
  const float w3 = W[OFF_W3 + t];
  float dw3 = 0.0f, db2 = 0.0f;
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    const float a1 = (s < ns) ? act[(s0 + s) * 2 * H + t] : 0.0f;
    const float a2 = (s < ns) ? act[(s0 + s) * 2 * H + H + t] : 0.0f;
    h1[s][t] = a1;
    dw3 = fmaf(dys[s], a2, dw3);
    const float d2 = (a2 > 0.0f) ? dys[s] * w3 : 0.0f;
    dz2[s][t] = d2;
    db2 += d2;
  }
  g[OFF_W3 + t] = dw3;
  g[OFF_B2 + t] = db2;
  if (t == 0) {
    float db3 = 0.0f;
    for (int s = 0; s < SB; ++s) db3 += dys[s];
    g[OFF_B3] = db3;
  }
  __syncthreads();
  // dW2[t][i] = sum_s dz2[s][t] h1[s][i]
  for (int i = 0; i < H; ++i) {
    float a = 0.0f;
#pragma unroll
    for (int s = 0; s < SB; ++s) a = fmaf(dz2[s][t], h1[s][i], a);
    g[OFF_W2 + (int64_t)t * H + i] = a;
  }
  // dh1[s][t] = sum_o W2[o][t] dz2[s][o];  dz1 = dh1 * (h1 > 0)
  float acc[SB];
#pragma unroll
  for (int s = 0; s < SB; ++s) acc[s] = 0.0f;
  for (int o = 0; o < H; ++o) {
    const float w = W[OFF_W2 + (int64_t)o * H + t];
#pragma unroll
    for (int s = 0; s < SB; ++s) acc[s] = fmaf(w, dz2[s][o], acc[s]);
  }
  float db1 = 0.0f;
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    const float d1 = (h1[s][t] > 0.0f) ? acc[s] : 0.0f;
    dz1[s][t] = d1;
    db1 += d1;
  }
  g[OFF_B1 + t] = db1;
  __syncthreads();
  // dW1[o][i] = sum_s dz1[s][o] x[s][i]; thread t covers columns i = t + 128 c
  for (int o = 0; o < H; ++o) {
#pragma unroll
    for (int c = 0; c < IN / H; ++c) {
      const int i = t + H * c;
      float a = 0.0f;
#pragma unroll
      for (int s = 0; s < SB; ++s) a = fmaf(dz1[s][o], xs[s][i], a);
      g[OFF_W1 + (int64_t)o * IN + i] = a;
    }
  }
}

__global__ void grad_reduce_kernel(const float* gpart, int parts, float* dW) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < NPARAM;
       p += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int w = 0; w < parts; ++w) s += gpart[(int64_t)w * NPARAM + p];
    dW[p] = s;
  }
}

__global__ void adam_kernel(float* W, const float* g, float* m1, float* m2, float lr, float c1,
                            float c2) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < NPARAM;
       p += (int64_t)gridDim.x * blockDim.x) {
    const float gp = g[p];
    const float a = 0.9f * m1[p] + 0.1f * gp;
    const float b = 0.999f * m2[p] + 0.001f * gp * gp;
    m1[p] = a;
    m2[p] = b;
    W[p] -= lr * (a / c1) / (sqrtf(b / c2) + 1e-8f);
  }
}

// Pinball (quantile) loss on the network output: r = target - yhat,
// loss = mean(tau max(r, 0) + (1 - tau) max(-r, 0)); dy = d loss / d yhat.
// One workgroup; the mean is summed in FP64 in a fixed order.
__global__ __launch_bounds__(256) void pinball_kernel(const float* yhat, const float* target,
                                                      int64_t B, float tau, float* dy,
                                                      float* loss) {
  __shared__ double part[256];
  double acc = 0.0;
  const float inv = 1.0f / (float)B;
  for (int64_t b = threadIdx.x; b < B; b += 256) {
    const float r = target[b] - yhat[b];
    const float l = (r > 0.0f) ? tau * r : (tau - 1.0f) * r;
    dy[b] = ((r > 0.0f) ? -tau : (r < 0.0f ? 1.0f - tau : 0.0f)) * inv;
    acc += (double)l;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(part[0] / (double)B);
}

template <typename T>
__global__ void features_kernel(const T* d, int64_t L, int64_t k_eff, float* f) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < L;
       t += (int64_t)gridDim.x * blockDim.x) {
    float v = -20.0f;
    if (t < k_eff && k_eff > 0) {
      const double r = (double)d[t] / (double)d[0];
      if (r > 0.0) v = fmaxf((float)log10(r), -20.0f);
    }
    f[t] = v;
  }
}
}  // namespace

size_t mlp_backward_workspace(int64_t B) {
  return (size_t)((B + SB - 1) / SB) * NPARAM * sizeof(float) + 256;
}

int mlp_forward(rpid_ctx ctx, const float* W, const float* feats, int64_t B, float* yhat,
                float* act) {
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((B + SB - 1) / SB)), dim3(H), 0,
                     ctx->stream, W, feats, B, yhat, act);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int mlp_backward(rpid_ctx ctx, const float* W, const float* feats, const float* act,
                 const float* dy, int64_t B, float* dW, size_t ws_off) {
  const int parts = (int)((B + SB - 1) / SB);
  float* gpart = ws_ptr<float>(ctx, ws_off);
  RPID_CHECK(ws_check(ctx, ws_off + (size_t)parts * NPARAM * sizeof(float)));
  hipLaunchKernelGGL(mlp_backward_kernel, dim3(parts), dim3(H), 0, ctx->stream, W, feats, act, dy,
                     B, gpart);
  RPID_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(grad_reduce_kernel, dim3(324), dim3(256), 0, ctx->stream, gpart, parts, dW);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int mlp_adam(rpid_ctx ctx, float* W, const float* dW, float* m1, float* m2, float lr, int64_t t) {
  const float c1 = 1.0f - powf(0.9f, (float)t);
  const float c2 = 1.0f - powf(0.999f, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3(324), dim3(256), 0, ctx->stream, W, dW, m1, m2, lr, c1,
                     c2);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int mlp_pinball(rpid_ctx ctx, const float* yhat, const float* target, int64_t B, float tau,
                float* dy, float* loss) {
  hipLaunchKernelGGL(pinball_kernel, dim3(1), dim3(256), 0, ctx->stream, yhat, target, B, tau, dy,
                     loss);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int mlp_features(rpid_ctx ctx, const void* diagU, bool f64, int64_t L, int64_t k_eff,
                 float* feats) {
  const unsigned blocks = (unsigned)((L + 255) / 256);
  if (f64)
    hipLaunchKernelGGL(features_kernel<double>, dim3(blocks), dim3(256), 0, ctx->stream,
                       (const double*)diagU, L, k_eff, feats);
  else
    hipLaunchKernelGGL(features_kernel<float>, dim3(blocks), dim3(256), 0, ctx->stream,
                       (const float*)diagU, L, k_eff, feats);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

}  // namespace rpid
