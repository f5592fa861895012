// peaks.hip -- achievable device rates, measured beside the published peaks
// that the rooflines divide by: FP32 fused multiply-add issue (unpacked, as
// this library is compiled), FP32 reciprocal issue, and a streaming device
// copy.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "engine.h"

namespace hmd {
namespace {

constexpr int PK_TPB = 256;
constexpr int PK_CHAINS = 8;  // independent dependency chains per thread

// PK_CHAINS independent chains of fused multiply-adds per thread, iters deep:
// 2 PK_CHAINS iters FLOP per thread.  The sum is stored so nothing is elided.
__global__ __launch_bounds__(PK_TPB) void k_peak_fma(float* __restrict__ out, int iters, float a, float b) {
  float x[PK_CHAINS];
#pragma unroll
  for (int k = 0; k < PK_CHAINS; ++k) x[k] = 1.0f + 1e-3f * float(k) + 1e-7f * float(threadIdx.x);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < PK_CHAINS; ++k) x[k] = fmaf(x[k], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < PK_CHAINS; ++k) s += x[k];
  out[size_t(blockIdx.x) * PK_TPB + threadIdx.x] = s;
}

// The same chains of reciprocals (x -> 1/x keeps every value near 1).
__global__ __launch_bounds__(PK_TPB) void k_peak_rcp(float* __restrict__ out, int iters) {
  float x[PK_CHAINS];
#pragma unroll
  for (int k = 0; k < PK_CHAINS; ++k) x[k] = 1.0f + 1e-3f * float(k) + 1e-7f * float(threadIdx.x);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < PK_CHAINS; ++k) x[k] = __builtin_amdgcn_rcpf(x[k]);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < PK_CHAINS; ++k) s += x[k];
  out[size_t(blockIdx.x) * PK_TPB + threadIdx.x] = s;
}

// Streaming copy of n float4, a workgroup per PK_TPB * 4 of them: each
// thread's four loads are in flight together, then the four stores.
__global__ __launch_bounds__(PK_TPB) void k_peak_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                      size_t n) {
  const size_t base = size_t(blockIdx.x) * PK_TPB * 4 + threadIdx.x;
  float4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const size_t i = base + size_t(k) * PK_TPB;
    if (i < n) v[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const size_t i = base + size_t(k) * PK_TPB;
    if (i < n) dst[i] = v[k];
  }
}

}  // namespace
}  // namespace hmd

using namespace hmd;

extern "C" int hmd_measure_peaks(hmd_ctx* ctx, double* out) {
  if (!ctx || !out) return HMD_EINVAL;
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  int cus = 0;
  HMD_HIP(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
  const int blocks = std::max(1, cus) * 8;  // eight 256-thread workgroups per compute unit
  const int iters = 4096;
  const size_t copy_n = size_t(1) << 26;  // 64 Mi float4 = 1 GiB each way
  float* d_out = nullptr;
  float4 *d_src = nullptr, *d_dst = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = HMD_OK;
  auto timed = [&](auto launch, float* ms) -> int {
    launch();  // warm-up
    HMD_HIP(ctx, hipEventRecord(e0, s));
    for (int r = 0; r < 5; ++r) launch();
    HMD_HIP(ctx, hipEventRecord(e1, s));
    HMD_HIP(ctx, hipEventSynchronize(e1));
    HMD_HIP(ctx, hipEventElapsedTime(ms, e0, e1));
    *ms /= 5.0f;
    return HMD_OK;
  };
  do {
    if (hipMalloc(&d_out, sizeof(float) * size_t(blocks) * PK_TPB) != hipSuccess ||
        hipMalloc(&d_src, sizeof(float4) * copy_n) != hipSuccess ||
        hipMalloc(&d_dst, sizeof(float4) * copy_n) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      ctx->err = "hmd_measure_peaks: allocation failed";
      rc = HMD_ENOMEM;
      break;
    }
    if (hipMemsetAsync(d_src, 0, sizeof(float4) * copy_n, s) != hipSuccess) {
      rc = HMD_EDEVICE;
      break;
    }
    const double threads = double(blocks) * PK_TPB;
    float ms_fma = 0.0f, ms_rcp = 0.0f, ms_copy = 0.0f;
    if ((rc = timed([&] { hipLaunchKernelGGL(k_peak_fma, dim3(blocks), dim3(PK_TPB), 0, s, d_out, iters,
                                             0.999999f, 1e-7f); },
                    &ms_fma)) != HMD_OK)
      break;
    if ((rc = timed([&] { hipLaunchKernelGGL(k_peak_rcp, dim3(blocks), dim3(PK_TPB), 0, s, d_out, iters); },
                    &ms_rcp)) != HMD_OK)
      break;
    const unsigned copy_blocks = unsigned((copy_n + PK_TPB * 4 - 1) / (PK_TPB * 4));
    if ((rc = timed([&] { hipLaunchKernelGGL(k_peak_copy, dim3(copy_blocks), dim3(PK_TPB), 0, s, d_src, d_dst,
                                             copy_n); },
                    &ms_copy)) != HMD_OK)
      break;
    if (hipGetLastError() != hipSuccess) {
      rc = HMD_EDEVICE;
      break;
    }
    const double ops = threads * double(iters) * PK_CHAINS;  // instructions of each chain kind
    out[0] = 2.0 * ops / (double(ms_fma) * 1e-3) / 1e12;    // FP32 FMA TFLOP/s
    out[1] = ops / (double(ms_rcp) * 1e-3) / 1e12;          // reciprocals, tera per second
    out[2] = double(ms_rcp) / double(ms_fma);                // issue cost of a reciprocal in FMAs
    out[3] = 2.0 * sizeof(float4) * double(copy_n) / (double(ms_copy) * 1e-3) / 1e9;  // copy GB/s (read + write)
  } while (false);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (void* p : {(void*)d_out, (void*)d_src, (void*)d_dst})
    if (p) (void)hipFree(p);
  return rc;
}
