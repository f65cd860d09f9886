// ktmi_mlp.hip -- forward, gradient and Adam kernels of the learned root-solve
// guess (network in ktmi_mlp.hpp) and their C ABI.  Training runs on the GPU:
// per-sample forward (FP32, or BF16 matrix cores for the 32x32 layer) and FP32
// backward; each workgroup sweeps a fixed set of 128-sample chunks and folds
// their gradients through LDS into per-thread accumulators, then one kernel
// folds the workgroups in a fixed order (bitwise reproducible), then Adam.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ktmi.h"
#include "ktmi_mlp.hpp"

namespace ktmi {

constexpr int kMlpBlock = 128;                 // samples per chunk (= threads per workgroup)
constexpr int kMlpGrid = 512;                  // workgroups of the gradient kernel (at most)
constexpr int kMlpSlots = kMlpNParam + 2;      // gradient sums, loss sum, sample count

__device__ __forceinline__ void load_w2bf(const float* __restrict__ prm, uint16_t* w2bf) {
  for (int k = threadIdx.x; k < kMlpH * kMlpH; k += blockDim.x)
    w2bf[k] = (uint16_t)to_bf16(prm[kOW2 + k]);
  __syncthreads();
}

__device__ __forceinline__ bool mlp_sample_ok(double E, double M, double emin) {
  return E >= emin && E < 1e300 && M >= 0.0 && M < 1e300;
}

// guess[i] for n samples (E, M); MODE 0 FP32, 1 BF16 matrix cores.  Samples
// with E < emin (or non-finite) get guess = E.
template <int MODE>
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ prm, int n,
                                                     const double* __restrict__ E,
                                                     const double* __restrict__ M, double emin,
                                                     double* __restrict__ guess) {
  __shared__ uint16_t w2bf[kMlpH * kMlpH];
  if (MODE == 1) load_w2bf(prm, w2bf);
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const double e = s < n ? E[s] : 1.0, m = s < n ? M[s] : 0.0;
  const bool ok = s < n && mlp_sample_ok(e, m, emin);
  const double ee = ok ? e : 1.0, mm = ok ? m : 0.0;
  double g;
  if (MODE == 1) {
    g = mlp_guess_wave(prm, w2bf, ee, mm * mm);
  } else {
    g = mlp_guess_lane(prm, ee, mm * mm);
  }
  if (s < n) guess[s] = ok ? g : e;
}

// Gradient sums of the loss ((guess - e)/E)^2 over the samples with E >= emin,
// plus the loss sum and the sample count, per workgroup: part[block][slot].
template <int MODE>
__global__ __launch_bounds__(kMlpBlock) void k_mlp_grad(const float* __restrict__ prm, int n,
                                                        const double* __restrict__ E,
                                                        const double* __restrict__ M,
                                                        const double* __restrict__ eps,
                                                        double emin, float* __restrict__ part) {
  __shared__ uint16_t w2bf[kMlpH * kMlpH];
  __shared__ float A[kMlpBlock][kMlpH + 1];  // +1 keeps column reads off one bank
  __shared__ float B[kMlpBlock][kMlpH + 1];
  __shared__ float Fv[kMlpBlock][4];
  __shared__ float Dz[kMlpBlock];
  if (MODE == 1) load_w2bf(prm, w2bf);
  const int tid = threadIdx.x;
  // accumulators: W2 entries tid + 128 k (k < 8), W1 entry tid, and for
  // tid < 32 the b1, b2, w3 entries tid; thread 0 also b3, loss, count
  float gW2[8], gW1 = 0.0f, gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f, gb3 = 0.0f;
  double loss = 0.0, cnt = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) gW2[k] = 0.0f;
  const int nchunk = (n + kMlpBlock - 1) / kMlpBlock;
  for (int ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int s = ch * kMlpBlock + tid;
    const double e = s < n ? E[s] : 1.0, m = s < n ? M[s] : 0.0;
    const bool ok = s < n && mlp_sample_ok(e, m, emin);
    const double ee = ok ? e : 1.0, mm = ok ? m : 0.0, target = ok ? eps[s] : 0.5;
    float f[4], h1[kMlpH], h2[kMlpH];
    double lo;
    mlp_features(ee, mm * mm, f, lo);
    mlp_layer1(prm, f, h1);
    const float z = MODE == 1 ? mlp_z_mfma(prm, w2bf, h1, h2) : mlp_z_fp32(prm, h1, h2);
    const double sg = 1.0 / (1.0 + exp(-(double)z));
    const double r = (ee - lo) / ee;
    const double t = ee > lo ? (target - lo) / (ee - lo) : 0.0;
    const double d = r * (sg - t);
    const float dz = ok ? (float)(2.0 * d * r * sg * (1.0 - sg)) : 0.0f;
    Dz[tid] = dz;
    {
      // per-chunk loss and count, folded by thread 0 in sample order below
      A[tid][kMlpH] = ok ? (float)(d * d) : 0.0f;
    }
    float d2[kMlpH];
#pragma unroll
    for (int i = 0; i < kMlpH; ++i) {
      d2[i] = dz * prm[kOW3 + i] * (1.0f - h2[i] * h2[i]);
      A[tid][i] = d2[i];
      B[tid][i] = h1[i];
    }
    B[tid][kMlpH] = ok ? 1.0f : 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) Fv[tid][k] = f[k];
    __syncthreads();
    // dW2[i][j] += sum_s d2_i h1_j ; db2, dw3 partial, db3, loss, count
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int q = tid + kMlpBlock * k, i = q / kMlpH, j = q % kMlpH;
      float acc = 0.0f;
      for (int r2 = 0; r2 < kMlpBlock; ++r2) acc += A[r2][i] * B[r2][j];
      gW2[k] += acc;
    }
    if (tid < kMlpH) {
      float acc = 0.0f;
      for (int r2 = 0; r2 < kMlpBlock; ++r2) acc += A[r2][tid];
      gb2 += acc;
    }
    if (tid == 0) {
      float a = 0.0f;
      double l2 = 0.0, c2 = 0.0;
      for (int r2 = 0; r2 < kMlpBlock; ++r2) {
        a += Dz[r2];
        l2 += A[r2][kMlpH];
        c2 += B[r2][kMlpH];
      }
      gb3 += a;
      loss += l2;
      cnt += c2;
    }
    __syncthreads();
    // d1 = (W2^T d2)(1 - h1^2); dW1 += sum_s d1 f^T, db1, dw3 += sum_s dz h2
#pragma unroll 4
    for (int j = 0; j < kMlpH; ++j) {
      float a = 0.0f;
#pragma unroll
      for (int i = 0; i < kMlpH; ++i) a += prm[kOW2 + i * kMlpH + j] * d2[i];
      A[tid][j] = a * (1.0f - h1[j] * h1[j]);
      B[tid][j] = dz * h2[j];
    }
    __syncthreads();
    {
      const int j = tid / 4, k = tid % 4;
      float acc = 0.0f;
      for (int r2 = 0; r2 < kMlpBlock; ++r2) acc += A[r2][j] * Fv[r2][k];
      gW1 += acc;
    }
    if (tid < kMlpH) {
      float a1 = 0.0f, a3 = 0.0f;
      for (int r2 = 0; r2 < kMlpBlock; ++r2) {
        a1 += A[r2][tid];
        a3 += B[r2][tid];
      }
      gb1 += a1;
      gw3 += a3;
    }
    __syncthreads();  // A, B, Fv, Dz are rewritten by the next chunk
  }
  float* out = part + (size_t)blockIdx.x * kMlpSlots;
#pragma unroll
  for (int k = 0; k < 8; ++k) out[kOW2 + tid + kMlpBlock * k] = gW2[k];
  out[kOW1 + tid] = gW1;
  if (tid < kMlpH) {
    out[kOB1 + tid] = gb1;
    out[kOB2 + tid] = gb2;
    out[kOW3 + tid] = gw3;
  }
  if (tid == 0) {
    out[kOB3] = gb3;
    out[kMlpNParam] = (float)loss;
    out[kMlpNParam + 1] = (float)cnt;
  }
}

// out[p] = (sum over workgroups of part[.][p]) / count, folded in workgroup
// order; out[kMlpNParam] = mean loss, out[kMlpNParam + 1] = count.
__global__ void k_mlp_fold(const float* __restrict__ part, int nblk, float* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpSlots) return;
  double acc = 0.0, cnt = 0.0;
  for (int b = 0; b < nblk; ++b) {
    acc += part[(size_t)b * kMlpSlots + p];
    cnt += part[(size_t)b * kMlpSlots + kMlpNParam + 1];
  }
  out[p] = p == kMlpNParam + 1 ? (float)cnt : (cnt > 0.0 ? (float)(acc / cnt) : 0.0f);
}

// Adam (Kingma & Ba): bias-corrected first and second moments, t from 1.
__global__ void k_mlp_adam(float* __restrict__ prm, const float* __restrict__ g,
                           float* __restrict__ m, float* __restrict__ v, float c1, float c2,
                           float lr, float b1, float b2, float epsilon) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpNParam) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.0f - b1) * gp;
  const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  prm[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + epsilon);
}

static int mlp_grid(int n) {
  const int nchunk = (int)(((long)n + kMlpBlock - 1) / kMlpBlock);
  return nchunk < kMlpGrid ? nchunk : kMlpGrid;
}

// Largest sample count: the gradient kernel indexes samples with 32-bit ints
// (chunk * kMlpBlock + thread), which stay below 2^31 up to this n.
constexpr int kMlpMaxSamples = 0x7fffffff - kMlpBlock;

// Scratch of ktmi_mlp_grad_noalloc: the partial sums of the gradient kernel's
// workgroups (at most kMlpGrid records of kMlpSlots floats, 2.56 MB).  One copy
// per GPU, held until the process ends.  Its name is a host-side stand-in in
// host code: kernels get the device address from hipGetSymbolAddress.
constexpr size_t kMlpScratchFloats = (size_t)kMlpGrid * kMlpSlots;
static __device__ __align__(256) float scratch[kMlpScratchFloats];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[kMaxDevices];  // device address of scratch on each GPU

// Device address of scratch on the current GPU, looked up once per device.
static int scratch_on_current_device(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return KTMI_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return KTMI_EHIP;
    g_scratch_ptr[dev] = (float*)p;
  }
  *out = g_scratch_ptr[dev];
  return KTMI_OK;
}

// Gradient kernel, then the fixed-order fold of its workgroups, into out.
static int launch_mlp_grad(const float* params, int n, const double* E, const double* M,
                           const double* eps, double emin, int mode, float* out, float* part,
                           hipStream_t s) {
  const int nblk = mlp_grid(n);
  if (mode == KTMI_MLP_BF16)
    hipLaunchKernelGGL(k_mlp_grad<1>, dim3(nblk), dim3(kMlpBlock), 0, s, params, n, E, M, eps,
                       emin, part);
  else
    hipLaunchKernelGGL(k_mlp_grad<0>, dim3(nblk), dim3(kMlpBlock), 0, s, params, n, E, M, eps,
                       emin, part);
  hipLaunchKernelGGL(k_mlp_fold, dim3((kMlpSlots + 255) / 256), dim3(256), 0, s, part, nblk, out);
  return hipGetLastError() == hipSuccess ? KTMI_OK : KTMI_EHIP;
}

}  // namespace ktmi

using namespace ktmi;

extern "C" {

int ktmi_mlp_nparam(void) { return kMlpNParam; }

int ktmi_mlp_forward(const float* params, int n, const double* E, const double* M, double emin,
                     double* guess, int mode, void* stream) {
  if (!params || n < 0 || (n && (!E || !M || !guess)) || (mode != KTMI_MLP_FP32 &&
                                                         mode != KTMI_MLP_BF16))
    return KTMI_EINVAL;
  if (n == 0) return KTMI_OK;
  const dim3 grid((n + 255) / 256), block(256);
  hipStream_t s = (hipStream_t)stream;
  if (mode == KTMI_MLP_BF16)
    hipLaunchKernelGGL(k_mlp_forward<1>, grid, block, 0, s, params, n, E, M, emin, guess);
  else
    hipLaunchKernelGGL(k_mlp_forward<0>, grid, block, 0, s, params, n, E, M, emin, guess);
  return hipGetLastError() == hipSuccess ? KTMI_OK : KTMI_EHIP;
}

size_t ktmi_mlp_grad_workspace_bytes(int n) {
  if (n < 1) return 0;
  return (size_t)mlp_grid(n) * kMlpSlots * sizeof(float);
}

int ktmi_mlp_grad(const float* params, int n, const double* E, const double* M, const double* eps,
                  double emin, int mode, float* out, void* ws, size_t bytes, void* stream) {
  if (!params || n < 1 || !E || !M || !eps || !out || !ws ||
      (mode != KTMI_MLP_FP32 && mode != KTMI_MLP_BF16))
    return KTMI_EINVAL;
  if (n > kMlpMaxSamples || bytes < ktmi_mlp_grad_workspace_bytes(n)) return KTMI_EINVAL;
  return launch_mlp_grad(params, n, E, M, eps, emin, mode, out, (float*)ws, (hipStream_t)stream);
}

int ktmi_mlp_grad_noalloc(const float* params, int n, const double* E, const double* M,
                          const double* eps, double emin, int mode, float* out, void* stream) {
  if (!params || n < 1 || n > kMlpMaxSamples || !E || !M || !eps || !out ||
      (mode != KTMI_MLP_FP32 && mode != KTMI_MLP_BF16))
    return KTMI_EINVAL;
  // every sample count fits: the kernel never runs more than kMlpGrid workgroups
  if ((size_t)mlp_grid(n) * kMlpSlots > kMlpScratchFloats) return KTMI_EINVAL;
  float* part = nullptr;
  const int rc = scratch_on_current_device(&part);
  if (rc != KTMI_OK) return rc;
  return launch_mlp_grad(params, n, E, M, eps, emin, mode, out, part, (hipStream_t)stream);
}

int ktmi_mlp_adam(float* params, const float* grad, float* m, float* v, int t, float lr, float b1,
                  float b2, float epsilon, void* stream) {
  if (!params || !grad || !m || !v || t < 1 || !(lr > 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) ||
      !(b2 >= 0.0f && b2 < 1.0f) || !(epsilon > 0.0f))
    return KTMI_EINVAL;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpNParam + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, params, grad, m, v, c1, c2, lr, b1, b2, epsilon);
  return hipGetLastError() == hipSuccess ? KTMI_OK : KTMI_EHIP;
}

}  // extern "C"
