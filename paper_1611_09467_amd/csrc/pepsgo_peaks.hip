// Throughput probes of the units the evaluation runs on (float64 vector
// FMA, float64 / float32 / bfloat16 matrix cores).  Each wave runs
// independent chains long enough that issue, not latency, bounds it; the
// caller times the launch on its stream.  Measurement helpers only: nothing
// of the method runs here.
#include <hip/hip_runtime.h>

#include "pepsgo.h"
#include "pepsgo_internal.h"

namespace pg {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kChains = 8;  // independent matrix-core accumulators per wave

__global__ void __launch_bounds__(kProbeThreads) k_probe_fma64(int iters, double seed, double* sink) {
  double a[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) a[q] = seed + q + threadIdx.x;
  const double b = 1.0 - 0x1p-40, c = 0x1p-41;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = fma(a[q], b, c);
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += a[q];
  if (s == 12345.678) sink[blockIdx.x] = s;  // keeps the chains live
}

typedef double p_d4 __attribute__((ext_vector_type(4)));
typedef float p_f4 __attribute__((ext_vector_type(4)));
typedef short p_s4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kProbeThreads) k_probe_mfma64(int iters, double seed, double* sink) {
  p_d4 acc[kChains];
#pragma unroll
  for (int q = 0; q < kChains; ++q) acc[q] = p_d4{0.0, 0.0, 0.0, 0.0};
  const double a = seed + threadIdx.x, b = 1.0 / (1.0 + threadIdx.x);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < kChains; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kChains; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  if (s == 12345.678) sink[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kProbeThreads) k_probe_mfma32(int iters, double seed, double* sink) {
  p_f4 acc[kChains];
#pragma unroll
  for (int q = 0; q < kChains; ++q) acc[q] = p_f4{0.f, 0.f, 0.f, 0.f};
  const float a = (float)seed + threadIdx.x, b = 1.0f / (1.0f + threadIdx.x);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < kChains; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[q], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < kChains; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  if (s == 12345.678f) sink[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kProbeThreads) k_probe_mfma_bf16(int iters, double seed, double* sink) {
  p_f4 acc[kChains];
#pragma unroll
  for (int q = 0; q < kChains; ++q) acc[q] = p_f4{0.f, 0.f, 0.f, 0.f};
  p_s4 a, b;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    a[j] = (short)(0x3f80 + ((threadIdx.x + j + (int)seed) & 7));
    b[j] = (short)(0x3f00 + ((threadIdx.x * 3 + j) & 7));
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < kChains; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[q], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < kChains; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  if (s == 12345.678f) sink[blockIdx.x] = s;
}

}  // namespace
}  // namespace pg

extern "C" {

int pepsgo_peak_probe(int kind, int blocks, int iters, double* sink, double* flops, void* stream) {
  using namespace pg;
  if (blocks < 1 || iters < 1 || !sink || !flops)
    return api_fail(PEPSGO_EINVAL, "pepsgo_peak_probe: blocks %d, iters %d, NULL buffer", blocks, iters);
  hipStream_t s = (hipStream_t)stream;
  const double waves = (double)blocks * (kProbeThreads / 64);
  switch (kind) {
    case PEPSGO_PROBE_FMA64:
      hipLaunchKernelGGL(k_probe_fma64, dim3(blocks), dim3(kProbeThreads), 0, s, iters, 1.0, sink);
      *flops = 2.0 * 8.0 * iters * (double)blocks * kProbeThreads;
      break;
    case PEPSGO_PROBE_MFMA64:
      hipLaunchKernelGGL(k_probe_mfma64, dim3(blocks), dim3(kProbeThreads), 0, s, iters, 1.0, sink);
      *flops = 2.0 * 16 * 16 * 4 * kChains * (double)iters * waves;
      break;
    case PEPSGO_PROBE_MFMA32:
      hipLaunchKernelGGL(k_probe_mfma32, dim3(blocks), dim3(kProbeThreads), 0, s, iters, 1.0, sink);
      *flops = 2.0 * 16 * 16 * 4 * kChains * (double)iters * waves;
      break;
    case PEPSGO_PROBE_MFMA_BF16:
      hipLaunchKernelGGL(k_probe_mfma_bf16, dim3(blocks), dim3(kProbeThreads), 0, s, iters, 1.0, sink);
      *flops = 2.0 * 16 * 16 * 16 * kChains * (double)iters * waves;
      break;
    default:
      return api_fail(PEPSGO_EINVAL, "pepsgo_peak_probe: unknown kind %d", kind);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return api_fail(PEPSGO_EDEVICE, "pepsgo_peak_probe: %s", hipGetErrorString(e));
  return PEPSGO_OK;
}

}  // extern "C"
