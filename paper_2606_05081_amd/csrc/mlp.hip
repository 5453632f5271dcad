// Engine-switch network kernels (fp32): forward pass, weighted softmax
// cross-entropy with its gradient, Adam, and a device-driven training loop.
//
// The network maps 12 standardised level features to 3 engine logits:
// h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3, with the
// parameters packed as W1[64][12], b1[64], W2[64][64], b2[64], W3[3][64],
// b3[3]. The paper does not contain it: its Conclusion names a more robust,
// graph-adaptive switching criterion as future work, and this network is
// that criterion, trained on per-level engine timings the library measures.
//
// The gradient kernel is one workgroup: 128-sample chunks are staged in LDS
// and every thread owns fixed output entries of each layer product, so the
// summation order is fixed and the result is deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "blest.h"

namespace {

constexpr int IN = BLEST_MLP_IN, H = BLEST_MLP_HIDDEN, OUT = BLEST_MLP_OUT;
constexpr int OW1 = 0, OB1 = OW1 + H * IN, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + OUT * H;
constexpr int NP = OB3 + OUT;
static_assert(NP == BLEST_MLP_NPARAMS, "parameter layout");

constexpr int GB = 256;  // threads of the gradient kernel
constexpr int CH = 128;  // samples per staged chunk

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Sample index i of a minibatch: either i itself (sampled == 0) or a
// counter-based draw from [0, nsamples) for training step `step`.
__device__ __forceinline__ int sample_index(int i, int sampled, int nsamples, unsigned long long seed, int step,
                                            int batch) {
  if (!sampled) return i;
  const unsigned long long r =
      mix64(seed + (static_cast<unsigned long long>(step) * batch + i + 1) * 0x9E3779B97F4A7C15ULL);
  return static_cast<int>((static_cast<unsigned __int128>(r) * static_cast<unsigned>(nsamples)) >> 64);
}

__global__ void __launch_bounds__(256) k_forward(const float* __restrict__ p, const float* __restrict__ x, int batch,
                                                 float* __restrict__ logits) {
  __shared__ float w[NP];
  for (int i = threadIdx.x; i < NP; i += blockDim.x) w[i] = p[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= batch) return;
  float xi[IN];
#pragma unroll
  for (int k = 0; k < IN; ++k) xi[k] = x[s * IN + k];
  float h1[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float a = w[OB1 + j];
#pragma unroll
    for (int k = 0; k < IN; ++k) a = fmaf(w[OW1 + j * IN + k], xi[k], a);
    h1[j] = fmaxf(a, 0.0f);
  }
  float z0 = w[OB3 + 0], z1 = w[OB3 + 1], z2 = w[OB3 + 2];
  for (int j = 0; j < H; ++j) {
    float a = w[OB2 + j];
#pragma unroll
    for (int k = 0; k < H; ++k) a = fmaf(w[OW2 + j * H + k], h1[k], a);
    const float h2 = fmaxf(a, 0.0f);
    z0 = fmaf(w[OW3 + j], h2, z0);
    z1 = fmaf(w[OW3 + H + j], h2, z1);
    z2 = fmaf(w[OW3 + 2 * H + j], h2, z2);
  }
  logits[s * OUT + 0] = z0;
  logits[s * OUT + 1] = z1;
  logits[s * OUT + 2] = z2;
}

// Loss and gradient of one minibatch. Single workgroup of GB threads.
// Thread t owns: gW2 entries t + GB*r (r < 16), gW1 entries t + GB*r (r < 3),
// gb1/gb2 entry t (t < 64), gW3 entries t (t < 192), gb3 entry t (t < 3).
__global__ void __launch_bounds__(GB) k_loss_grad(const float* __restrict__ p, const float* __restrict__ xall,
                                                  const int32_t* __restrict__ yall, const float* __restrict__ wall,
                                                  int batch, int sampled, int nsamples, unsigned long long seed,
                                                  int step, float* __restrict__ loss_out, float* __restrict__ grad) {
  __shared__ float w[NP];
  __shared__ float X[CH * IN];
  __shared__ float H1[CH * H];
  __shared__ float D2[CH * H];  // h2, then dA2
  __shared__ float D1[CH * H];  // dA1
  __shared__ float DZ[CH * OUT];
  __shared__ float red[GB];
  __shared__ float s_wsum;
  const int t = threadIdx.x;
  for (int i = t; i < NP; i += GB) w[i] = p[i];
  // total weight of the batch
  float ws = 0.0f;
  for (int i = t; i < batch; i += GB) {
    const int si = sample_index(i, sampled, nsamples, seed, step, batch);
    ws += wall ? wall[si] : 1.0f;
  }
  red[t] = ws;
  __syncthreads();
  for (int d = GB / 2; d > 0; d >>= 1) {
    if (t < d) red[t] += red[t + d];
    __syncthreads();
  }
  if (t == 0) s_wsum = red[0];
  __syncthreads();
  const float inv_w = 1.0f / s_wsum;
  float gW2[16], gW1[3], gb1 = 0.0f, gb2 = 0.0f, gW3 = 0.0f, gb3 = 0.0f, loss = 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) gW2[r] = 0.0f;
#pragma unroll
  for (int r = 0; r < 3; ++r) gW1[r] = 0.0f;

  for (int c0 = 0; c0 < batch; c0 += CH) {
    const int cn = min(CH, batch - c0);
    for (int i = t; i < cn * IN; i += GB) {
      const int s = i / IN, k = i % IN;
      const int si = sample_index(c0 + s, sampled, nsamples, seed, step, batch);
      X[i] = xall[static_cast<long long>(si) * IN + k];
    }
    __syncthreads();
    // layer 1
    for (int i = t; i < cn * H; i += GB) {
      const int s = i / H, j = i % H;
      float a = w[OB1 + j];
#pragma unroll
      for (int k = 0; k < IN; ++k) a = fmaf(w[OW1 + j * IN + k], X[s * IN + k], a);
      H1[i] = fmaxf(a, 0.0f);
    }
    __syncthreads();
    // layer 2 (h2 into D2)
    for (int i = t; i < cn * H; i += GB) {
      const int s = i / H, j = i % H;
      float a = w[OB2 + j];
      for (int k = 0; k < H; ++k) a = fmaf(w[OW2 + j * H + k], H1[s * H + k], a);
      D2[i] = fmaxf(a, 0.0f);
    }
    __syncthreads();
    // logits, softmax cross-entropy, dZ
    if (t < cn) {
      const int s = t;
      const int si = sample_index(c0 + s, sampled, nsamples, seed, step, batch);
      float z[OUT];
#pragma unroll
      for (int o = 0; o < OUT; ++o) {
        float a = w[OB3 + o];
        for (int j = 0; j < H; ++j) a = fmaf(w[OW3 + o * H + j], D2[s * H + j], a);
        z[o] = a;
      }
      const float zm = fmaxf(z[0], fmaxf(z[1], z[2]));
      const float e0 = expf(z[0] - zm), e1 = expf(z[1] - zm), e2 = expf(z[2] - zm);
      const float se = e0 + e1 + e2;
      const int y = yall[si];
      const float ww = (wall ? wall[si] : 1.0f) * inv_w;
      loss += ww * (logf(se) + zm - z[y]);
      const float inv_se = 1.0f / se;
      DZ[s * OUT + 0] = ww * (e0 * inv_se - (y == 0 ? 1.0f : 0.0f));
      DZ[s * OUT + 1] = ww * (e1 * inv_se - (y == 1 ? 1.0f : 0.0f));
      DZ[s * OUT + 2] = ww * (e2 * inv_se - (y == 2 ? 1.0f : 0.0f));
    }
    __syncthreads();
    // gW3, gb3
    if (t < OUT * H) {
      const int o = t / H, j = t % H;
      float a = 0.0f;
      for (int s = 0; s < cn; ++s) a = fmaf(DZ[s * OUT + o], D2[s * H + j], a);
      gW3 += a;
    }
    if (t < OUT) {
      float a = 0.0f;
      for (int s = 0; s < cn; ++s) a += DZ[s * OUT + t];
      gb3 += a;
    }
    __syncthreads();
    // dA2 = (dZ W3) * [h2 > 0], in place of h2
    for (int i = t; i < cn * H; i += GB) {
      const int s = i / H, j = i % H;
      const float g = DZ[s * OUT + 0] * w[OW3 + j] + DZ[s * OUT + 1] * w[OW3 + H + j] + DZ[s * OUT + 2] * w[OW3 + 2 * H + j];
      D2[i] = D2[i] > 0.0f ? g : 0.0f;
    }
    __syncthreads();
    // gW2[j][k] = sum_s dA2[s][j] h1[s][k]; gb2
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = t + GB * r, j = e / H, k = e % H;
      float a = 0.0f;
      for (int s = 0; s < cn; ++s) a = fmaf(D2[s * H + j], H1[s * H + k], a);
      gW2[r] += a;
    }
    if (t < H) {
      float a = 0.0f;
      for (int s = 0; s < cn; ++s) a += D2[s * H + t];
      gb2 += a;
    }
    // dA1 = (dA2 W2) * [h1 > 0]
    for (int i = t; i < cn * H; i += GB) {
      const int s = i / H, k = i % H;
      float a = 0.0f;
      for (int j = 0; j < H; ++j) a = fmaf(D2[s * H + j], w[OW2 + j * H + k], a);
      D1[i] = H1[i] > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    // gW1[j][k] = sum_s dA1[s][j] x[s][k]; gb1
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int e = t + GB * r, j = e / IN, k = e % IN;
      float a = 0.0f;
      for (int s = 0; s < cn; ++s) a = fmaf(D1[s * H + j], X[s * IN + k], a);
      gW1[r] += a;
    }
    if (t < H) {
      float a = 0.0f;
      for (int s = 0; s < cn; ++s) a += D1[s * H + t];
      gb1 += a;
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) grad[OW2 + t + GB * r] = gW2[r];
#pragma unroll
  for (int r = 0; r < 3; ++r) grad[OW1 + t + GB * r] = gW1[r];
  if (t < H) {
    grad[OB1 + t] = gb1;
    grad[OB2 + t] = gb2;
  }
  if (t < OUT * H) grad[OW3 + t] = gW3;
  if (t < OUT) grad[OB3 + t] = gb3;
  // loss: fixed-order tree sum over threads
  red[t] = loss;
  __syncthreads();
  for (int d = GB / 2; d > 0; d >>= 1) {
    if (t < d) red[t] += red[t + d];
    __syncthreads();
  }
  if (t == 0 && loss_out) *loss_out = red[0];
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

namespace blest {

hipError_t mlp_forward_launch(const float* params, const float* x, int32_t batch, float* logits, hipStream_t st) {
  hipLaunchKernelGGL(k_forward, dim3((batch + 255) / 256), dim3(256), 0, st, params, x, batch, logits);
  return hipGetLastError();
}

hipError_t mlp_loss_grad_launch(const float* params, const float* x, const int32_t* y, const float* w, int32_t batch,
                                float* loss, float* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_grad, dim3(1), dim3(GB), 0, st, params, x, y, w, batch, 0, batch, 0ULL, 0, loss, grad);
  return hipGetLastError();
}

hipError_t mlp_adam_launch(float* params, const float* grad, float* m, float* v, int32_t n, int32_t t, float lr,
                           float beta1, float beta2, float eps, hipStream_t st) {
  const float c1 = 1.0f - powf(beta1, static_cast<float>(t)), c2 = 1.0f - powf(beta2, static_cast<float>(t));
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, params, grad, m, v, n, lr, beta1, beta2, eps,
                     c1, c2);
  return hipGetLastError();
}

// `steps` Adam steps on minibatches drawn on the device; grad is a caller-
// provided NP-float scratch vector.
hipError_t mlp_train_launch(float* params, float* m, float* v, const float* x, const int32_t* y, const float* w,
                            int32_t nsamples, int32_t batch, int32_t steps, float lr, uint64_t seed, float* loss_log,
                            float* grad, hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int s = 0; s < steps; ++s) {
    hipLaunchKernelGGL(k_loss_grad, dim3(1), dim3(GB), 0, st, params, x, y, w, batch, 1, nsamples, seed, s,
                       loss_log ? loss_log + s : nullptr, grad);
    const int t = s + 1;
    const float c1 = 1.0f - powf(b1, static_cast<float>(t)), c2 = 1.0f - powf(b2, static_cast<float>(t));
    hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, st, params, grad, m, v, NP, lr, b1, b2, eps, c1,
                       c2);
  }
  return hipGetLastError();
}

}  // namespace blest
