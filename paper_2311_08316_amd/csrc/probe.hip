// Measured hardware ceilings for the roofline figures the benchmark reports
// next to the datasheet peaks: a streaming copy (HBM bandwidth) and loops of
// independent matrix-core instructions (FP64 and FP32 MFMA throughput). Not
// part of the factorization.
#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;  // independent accumulators per wave

// dst[i] = src[i] for i < n2 pairs of doubles, 16 bytes per lane per access.
__global__ void __launch_bounds__(kThreads)
copy_kernel(const double2* __restrict__ src, double2* __restrict__ dst, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n2; i += stride)
    dst[i] = src[i];
}

// iters rounds of kChains independent 16x16x4 FP64 MFMAs per wave; one value
// per wave is stored so the chains stay live.
__global__ void __launch_bounds__(kThreads) mfma_f64_kernel(double* out, int iters) {
  const int lane = threadIdx.x & 63;
  const double a = 1.0 + 1e-3 * lane;
  const double b = 1.0 - 1e-3 * lane;
  d4_t acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = d4_t{0.0, 0.0, 0.0, (double)c};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c)
      acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (lane == 0) out[blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6)] = s;
}

__global__ void __launch_bounds__(kThreads) mfma_f32_kernel(double* out, int iters) {
  const int lane = threadIdx.x & 63;
  const float a = 1.0f + 1e-3f * lane;
  const float b = 1.0f - 1e-3f * lane;
  f4_t acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = f4_t{0.f, 0.f, 0.f, (float)c};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c)
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (lane == 0) out[blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6)] = (double)s;
}

}  // namespace

extern "C" {

int cqrrpt_probe_copy(const double* src, double* dst, int64_t n, void* stream) {
  if (!src) return -1;
  if (!dst) return -2;
  if (n < 2 || (n & 1)) return -3;
  const int64_t n2 = n / 2;
  int64_t grid = (n2 + kThreads - 1) / kThreads;
  const int64_t cap = (int64_t)cqh::device_info().num_cu * 16;
  if (grid > cap) grid = cap;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)grid), dim3(kThreads), 0,
                     static_cast<hipStream_t>(stream), reinterpret_cast<const double2*>(src),
                     reinterpret_cast<double2*>(dst), n2);
  return hipGetLastError() == hipSuccess ? CQRRPT_OK : CQRRPT_EHIP;
}

int cqrrpt_probe_mfma(int fp64, int iters, double* out, int64_t out_len, int64_t* flops,
                      void* stream) {
  if (iters < 1) return -2;
  if (!out) return -3;
  if (!flops) return -5;
  const int blocks = cqh::device_info().num_cu * 8;
  const int64_t waves = (int64_t)blocks * (kThreads / 64);
  if (out_len < waves) return -4;
  // One 16x16x4 instruction: 16 * 16 * 4 multiply-adds.
  *flops = waves * (int64_t)iters * kChains * 2 * 16 * 16 * 4;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (fp64)
    hipLaunchKernelGGL(mfma_f64_kernel, dim3(blocks), dim3(kThreads), 0, s, out, iters);
  else
    hipLaunchKernelGGL(mfma_f32_kernel, dim3(blocks), dim3(kThreads), 0, s, out, iters);
  return hipGetLastError() == hipSuccess ? CQRRPT_OK : CQRRPT_EHIP;
}

}  // extern "C"
