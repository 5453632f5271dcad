// In-kernel inference of the engine-switch network (12 -> 64 -> 64 -> 3,
// ReLU): weights staged in LDS, one wave computes the logits. Shared by the
// single-source and the multi-source persistent kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "blest_internal.h"
#include "device_common.h"

namespace blest {

// Switch network in LDS: W1T[12][64], b1[64], W2T[64][64], b2[64], W3[3][64],
// b3[3], mean[12], inv_std[12] (W1 and W2 transposed for conflict-free reads).
constexpr int kLdsW1T = 0, kLdsB1 = 768, kLdsW2T = 832, kLdsB2 = 4928, kLdsW3 = 4992, kLdsB3 = 5184,
              kLdsMean = 5187, kLdsInvStd = 5199, kLdsMaxRatio = 5211, kLdsMlpFloats = 5212;

static __device__ __forceinline__ void mlp_to_lds(const MlpDev* mlp, float* s) {
  const float* p = mlp->params;
  for (int i = threadIdx.x; i < 768; i += blockDim.x) {
    int j = i / 12, k = i % 12;  // W1[j][k]
    s[kLdsW1T + k * 64 + j] = p[i];
  }
  for (int i = threadIdx.x; i < 4096; i += blockDim.x) {
    int j = i / 64, k = i % 64;  // W2[j][k]
    s[kLdsW2T + k * 64 + j] = p[832 + i];
  }
  for (int i = threadIdx.x; i < 64; i += blockDim.x) {
    s[kLdsB1 + i] = p[768 + i];
    s[kLdsB2 + i] = p[4928 + i];
  }
  for (int i = threadIdx.x; i < 195; i += blockDim.x) s[kLdsW3 + i] = p[4992 + i];
  for (int i = threadIdx.x; i < 12; i += blockDim.x) {
    s[kLdsMean + i] = mlp->mean[i];
    s[kLdsInvStd + i] = mlp->inv_std[i];
  }
  if (threadIdx.x == 0) s[kLdsMaxRatio] = mlp->max_ratio;
}

// Forward pass by one full wave; returns the argmax engine, or -1 when a
// standardised input lies outside [-6, 6] or the softmax probability of the
// argmax is below the model's confidence floor (caller falls back to Eq. 3).
static __device__ int mlp_choose_wave(const float* s, const float (&feat)[kMaxSwitchFeatures]) {
  float z[kMaxSwitchFeatures];
  bool ood = false;
#pragma unroll
  for (int k = 0; k < kMaxSwitchFeatures; ++k) {
    z[k] = (feat[k] - s[kLdsMean + k]) * s[kLdsInvStd + k];
    ood |= !(fabsf(z[k]) <= 6.0f);
  }
  if (ood) return -1;
  const int j = lane_id();
  float h = s[kLdsB1 + j];
#pragma unroll
  for (int k = 0; k < kMaxSwitchFeatures; ++k) h = fmaf(s[kLdsW1T + k * 64 + j], z[k], h);
  h = fmaxf(h, 0.0f);
  float g = s[kLdsB2 + j];
#pragma unroll 8
  for (int k = 0; k < 64; ++k) {
    float hk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(h), k));
    g = fmaf(s[kLdsW2T + k * 64 + j], hk, g);
  }
  g = fmaxf(g, 0.0f);
  float l0 = wave_sum(s[kLdsW3 + j] * g) + s[kLdsB3 + 0];
  float l1 = wave_sum(s[kLdsW3 + 64 + j] * g) + s[kLdsB3 + 1];
  float l2 = wave_sum(s[kLdsW3 + 128 + j] * g) + s[kLdsB3 + 2];
  int best = 0;
  float bv = l0;
  if (l1 > bv) { best = 1; bv = l1; }
  if (l2 > bv) { best = 2; bv = l2; }
  const float ratio = expf(l0 - bv) + expf(l1 - bv) + expf(l2 - bv);  // = 1 / p(best)
  if (!(ratio <= s[kLdsMaxRatio])) return -1;
  return best;
}

}  // namespace blest
