// ktmi_mlp.hpp -- small network that predicts the starting point of the
// per-cell root solve (learned guess).  Not part of the paper's method: the
// paper only notes that the root solve needs a variable number of iterations
// per cell (App. A.3).  4 -> 32 -> 32 -> 1, tanh hidden layers:
//   f = (ln E / 5, M/E, (M/E)^2, ln(max(lo/E, 1e-30)) / 10),
//   lo = max(0, E - M^2/E) (the root solve's lower bracket end),
//   guess = lo + sigmoid(z) (E - lo), always inside the bracket [lo, E].
// Parameters, flat FP32: W1[32][4], b1[32], W2[32][32], b2[32], w3[32], b3.
// The 32x32 layer of the wave-level forward runs on the BF16 matrix cores
// (v_mfma_f32_32x32x8_bf16, FP32 accumulation); the per-lane forward is FP32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ktmi {

constexpr int kMlpH = 32;
constexpr int kMlpNParam = kMlpH * 4 + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;  // 1249
constexpr int kOW1 = 0, kOB1 = 128, kOW2 = 160, kOB2 = 160 + 1024, kOW3 = kOB2 + 32,
              kOB3 = kOW3 + 32;
// Device copy used by the step kernels: the FP32 parameters padded to kMlpPad
// floats, then W2 as BF16 (row-major 32 x 32).
constexpr int kMlpPad = 1252;
constexpr size_t kMlpDevBytes = kMlpPad * 4 + kMlpH * kMlpH * 2;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Round-to-nearest-even FP32 -> BF16 bit pattern (finite inputs).
__host__ __device__ inline uint32_t to_bf16(float x) {
  const uint32_t u = __builtin_bit_cast(uint32_t, x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// tanh from its exponential form, tanh x = 1 - 2 / (e^{2x} + 1), with the
// hardware base-2 exponential and reciprocal (about one ulp each; no division
// sequence): saturates to +-1 for large |x|, absolute error of a few FP32 ulps.
__device__ __forceinline__ float mlp_tanh(float x) {
  const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * x);  // e^{2x} = 2^{2x log2 e}
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// Features of (E, M^2); lo = lower end of the root bracket.
__device__ __forceinline__ void mlp_features(double E, double M2, float f[4], double& lo) {
  const double r = sqrt(M2) / E;
  lo = E - M2 / E;
  lo = lo < 0.0 ? 0.0 : lo;
  double q = lo / E;
  q = q < 1e-30 ? 1e-30 : q;
  f[0] = 0.2f * __logf((float)E);
  f[1] = (float)r;
  f[2] = (float)(r * r);
  f[3] = 0.1f * __logf((float)q);
}

__device__ __forceinline__ void mlp_layer1(const float* __restrict__ prm, const float f[4],
                                           float h1[kMlpH]) {
#pragma unroll
  for (int j = 0; j < kMlpH; ++j) {
    float a = prm[kOB1 + j];
#pragma unroll
    for (int k = 0; k < 4; ++k) a += prm[kOW1 + j * 4 + k] * f[k];
    h1[j] = mlp_tanh(a);
  }
}

// FP32 layers 2 and 3 of one sample (per lane); h2 receives the hidden outputs.
__device__ __forceinline__ float mlp_z_fp32(const float* __restrict__ prm, const float h1[kMlpH],
                                            float h2[kMlpH]) {
  float z = prm[kOB3];
#pragma unroll
  for (int i = 0; i < kMlpH; ++i) {
    float a = prm[kOB2 + i];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) a += prm[kOW2 + i * kMlpH + j] * h1[j];
    h2[i] = mlp_tanh(a);
    z += prm[kOW3 + i] * h2[i];
  }
  return z;
}

// Layers 2 and 3 of 64 samples, one per lane, on the matrix cores.  Every lane
// of the wave must be active.  Z2^T (32 x 64) = W2 (32 x 32) * H1^T as two
// 32-sample column blocks (samples of lanes 0-31 and 32-63) and four K slices
// of 8.  Operand layout of v_mfma_f32_32x32x8_bf16: lane l holds
// A[l % 32][4 (l / 32) + j] and B[4 (l / 32) + j][l % 32] (j = 0..3), and
// D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] in accumulator register r.  A lane
// needs half of its B slice from its own sample and half from the sample of
// lane l ^ 32, exchanged with one cross-half shuffle per 32-bit pair; no LDS.
// w2bf: W2 as BF16 (row-major).  h2 (optional) receives the lane's own hidden
// outputs.
__device__ __forceinline__ float mlp_z_mfma(const float* __restrict__ prm,
                                            const uint16_t* __restrict__ w2bf,
                                            const float h1[kMlpH], float* h2 = nullptr) {
  const int l = threadIdx.x & 63;
  const bool upper = l >= 32;
  const int row = l & 31;
  uint32_t hb[kMlpH / 2];
#pragma unroll
  for (int q = 0; q < kMlpH / 2; ++q) hb[q] = to_bf16(h1[2 * q]) | (to_bf16(h1[2 * q + 1]) << 16);
  f32x16 acc0 = {}, acc1 = {};
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    // k range of this lane: 8 ks + 4 (l / 32) + 0..3
    const u32x2 a = *reinterpret_cast<const u32x2*>(w2bf + row * kMlpH + 8 * ks + (upper ? 4 : 0));
    const uint32_t own0 = upper ? hb[4 * ks + 2] : hb[4 * ks];
    const uint32_t own1 = upper ? hb[4 * ks + 3] : hb[4 * ks + 1];
    const uint32_t snd0 = upper ? hb[4 * ks] : hb[4 * ks + 2];
    const uint32_t snd1 = upper ? hb[4 * ks + 1] : hb[4 * ks + 3];
    const uint32_t rcv0 = (uint32_t)__shfl_xor((int)snd0, 32, 64);
    const uint32_t rcv1 = (uint32_t)__shfl_xor((int)snd1, 32, 64);
    u32x2 b0, b1;
    b0.x = upper ? rcv0 : own0;
    b0.y = upper ? rcv1 : own1;
    b1.x = upper ? own0 : rcv0;
    b1.y = upper ? own1 : rcv1;
    acc0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(__builtin_bit_cast(bf16x4, a),
                                                    __builtin_bit_cast(bf16x4, b0), acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(__builtin_bit_cast(bf16x4, a),
                                                    __builtin_bit_cast(bf16x4, b1), acc1, 0, 0, 0);
  }
  // rows held here: i(r) = 8 (r / 4) + 4 (l / 32) + r % 4, of samples l % 32
  // (acc0) and 32 + l % 32 (acc1); the lane's own sample is in acc0 for the
  // lower half and in acc1 for the upper half.
  float keep = 0.0f, send = 0.0f;
  float mine[16], other[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 8 * (r >> 2) + (upper ? 4 : 0) + (r & 3);
    const float t0 = mlp_tanh(acc0[r] + prm[kOB2 + i]);
    const float t1 = mlp_tanh(acc1[r] + prm[kOB2 + i]);
    mine[r] = upper ? t1 : t0;
    other[r] = upper ? t0 : t1;
    keep += prm[kOW3 + i] * mine[r];
    send += prm[kOW3 + i] * other[r];
  }
  const float z = prm[kOB3] + keep + __shfl_xor(send, 32, 64);
  if (h2) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float got = __shfl_xor(other[r], 32, 64);  // partner's rows of this lane's sample
      const int lo_i = 8 * (r >> 2) + (r & 3);
      h2[lo_i] = upper ? got : mine[r];
      h2[lo_i + 4] = upper ? mine[r] : got;
    }
  }
  return z;
}

// guess = lo + sigmoid(z) (E - lo); the sigmoid in FP32 (hardware exponential
// and reciprocal), clamped to [0, 1] so the guess stays inside the bracket.
__device__ __forceinline__ double mlp_guess_from_z(float z, double E, double lo) {
  const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * z);  // e^{-z}
  const float s = fminf(fmaxf(__builtin_amdgcn_rcpf(1.0f + e), 0.0f), 1.0f);
  return lo + (double)s * (E - lo);
}

// Guess of one lane (FP32 forward; divergent lanes allowed).
__device__ __forceinline__ double mlp_guess_lane(const float* __restrict__ prm, double E,
                                                 double M2) {
  float f[4], h1[kMlpH], h2[kMlpH];
  double lo;
  mlp_features(E, M2, f, lo);
  mlp_layer1(prm, f, h1);
  return mlp_guess_from_z(mlp_z_fp32(prm, h1, h2), E, lo);
}

// Guess of every lane of the wave (matrix-core forward; all lanes active).
__device__ __forceinline__ double mlp_guess_wave(const float* __restrict__ prm,
                                                 const uint16_t* __restrict__ w2bf, double E,
                                                 double M2) {
  float f[4], h1[kMlpH];
  double lo;
  mlp_features(E, M2, f, lo);
  mlp_layer1(prm, f, h1);
  return mlp_guess_from_z(mlp_z_mfma(prm, w2bf, h1), E, lo);
}

}  // namespace ktmi
