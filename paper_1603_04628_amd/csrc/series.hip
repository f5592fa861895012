// series.hip -- mean and standard error of sampled time series on the device.
//
// The paper (Sec. 2.3, hyperparameters) takes the noise of an MD run as the
// standard deviation of its mean output computed from the raw
// time-instantaneous data.  The flux of a channel stays correlated for a
// viscous time ~h^2/nu (thousands of steps in wide channels), so the
// estimator must account for the correlation.  Default: the initial
// monotone sequence estimator of Geyer (Statistical Science 7 (1992) 473,
// Sec. 3.3) over the empirical autocovariances; alternative: the standard
// deviation of nb contiguous block means.
//
// Rows: S series of n samples each, row stride ld, every sample multiplied
// by `scale` (the MD series holds sums of B steps; scale = 1/B).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "engine.h"
#include "series.h"

namespace hmd {

namespace {

constexpr int SER_TPB = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  // 256 threads: four wavefronts
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

}  // namespace

// out[s*4 + 0] = mean, [2] = mean of the first n/2 samples, [3] = mean of
// the rest; [1] (the standard error) is left to the estimator kernels.
__global__ __launch_bounds__(SER_TPB) void k_series_moments(const double* __restrict__ x, int64_t ld, int64_t n,
                                                           double scale, double* __restrict__ out) {
  __shared__ double red[4];
  const int s = blockIdx.x;
  const double* row = x + int64_t(s) * ld;
  const int64_t half = n / 2;
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < half; i += SER_TPB) a += row[i] * scale;
  for (int64_t i = half + threadIdx.x; i < n; i += SER_TPB) b += row[i] * scale;
  a = block_sum(a, red);
  b = block_sum(b, red);
  if (threadIdx.x == 0) {
    out[4 * s + 0] = (a + b) / double(n);
    out[4 * s + 2] = a / double(half);
    out[4 * s + 3] = b / double(n - half);
  }
}

// gamma_t = (1/n) sum_{i < n-t} d_i d_{i+t}, d = scale x - mean, for the
// 256 lags t0 .. t0+255 of this workgroup (grid: lag tiles x rows).  Each
// lag sums its products in ascending i; out-of-range terms are exact zeros.
__global__ __launch_bounds__(SER_TPB) void k_series_acov(const double* __restrict__ x, int64_t ld, int64_t n,
                                                        double scale, const double* __restrict__ mom,
                                                        double* __restrict__ gam, int64_t gld) {
  __shared__ double a[SER_TPB], b[2 * SER_TPB];
  const int s = blockIdx.y;
  const double* row = x + int64_t(s) * ld;
  const int64_t t0 = int64_t(blockIdx.x) * SER_TPB;
  const int tid = threadIdx.x;
  const double mean = mom[4 * s];
  double acc = 0.0;
  for (int64_t i0 = 0; i0 < n - t0; i0 += SER_TPB) {
    const int64_t ia = i0 + tid, ib = i0 + t0 + tid;
    a[tid] = ia < n ? row[ia] * scale - mean : 0.0;
    b[tid] = ib < n ? row[ib] * scale - mean : 0.0;
    b[tid + SER_TPB] = ib + SER_TPB < n ? row[ib + SER_TPB] * scale - mean : 0.0;
    __syncthreads();
#pragma unroll 8
    for (int j = 0; j < SER_TPB; ++j) acc += a[j] * b[j + tid];
    __syncthreads();
  }
  const int64_t t = t0 + tid;
  if (t < n) gam[int64_t(s) * gld + t] = acc / double(n);
}

// Geyer's initial monotone sequence: Gamma_k = gamma_2k + gamma_2k+1 while
// positive, each replaced by the smallest so far; sigma^2 = -gamma_0 +
// 2 sum Gamma_k; SE = sqrt(sigma^2 / n).  An empty sequence, or a sigma^2
// that is not positive, falls back to the iid value gamma_0.  One thread per
// row; pairs are read 16 at a time ahead of the sequential scan.
__global__ __launch_bounds__(64) void k_series_geyer(const double* __restrict__ gam, int64_t gld, int64_t n,
                                                     int S, double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const double* g = gam + int64_t(s) * gld;
  constexpr int CH = 16;
  const int64_t kmax = n / 2;  // pairs (2k, 2k+1) with 2k+1 < n
  double total = 0.0, smallest = INFINITY;
  int64_t used = 0;
  bool stop = false;
  for (int64_t k0 = 0; k0 < kmax && !stop; k0 += CH) {
    double p[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int64_t k = k0 + c;
      p[c] = k < kmax ? g[2 * k] + g[2 * k + 1] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (!stop) {
        if (k0 + c < kmax && p[c] > 0.0) {
          smallest = fmin(smallest, p[c]);
          total += smallest;
          ++used;
        } else {
          stop = true;
        }
      }
    }
  }
  double var = used > 0 ? -g[0] + 2.0 * total : g[0];
  if (!(var > 0.0)) var = g[0];
  out[4 * s + 1] = sqrt(var / double(n));
}

// Block rule: nb contiguous blocks of floor(n / nb) samples (the remainder
// dropped from the front); mean and halves are those of the block means.
__global__ __launch_bounds__(SER_TPB) void k_series_blocks(const double* __restrict__ x, int64_t ld, int64_t n,
                                                          double scale, int nb, double* __restrict__ out) {
  __shared__ double bm[1024];
  const int s = blockIdx.x;
  const double* row = x + int64_t(s) * ld;
  const int64_t B = n / nb, r = n - int64_t(nb) * B;
  for (int j = threadIdx.x; j < nb; j += SER_TPB) {
    double acc = 0.0;
    for (int64_t k = 0; k < B; ++k) acc += row[r + int64_t(j) * B + k] * scale;
    bm[j] = acc / double(B);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mean = 0.0;
    for (int j = 0; j < nb; ++j) mean += bm[j];
    mean /= double(nb);
    double var = 0.0;
    for (int j = 0; j < nb; ++j) var += (bm[j] - mean) * (bm[j] - mean);
    var /= double(nb - 1);
    const int h1 = nb / 2;
    double m1 = 0.0, m2 = 0.0;
    for (int j = 0; j < h1; ++j) m1 += bm[j];
    for (int j = h1; j < nb; ++j) m2 += bm[j];
    out[4 * s + 0] = mean;
    out[4 * s + 1] = sqrt(var / double(nb));
    out[4 * s + 2] = m1 / double(h1);
    out[4 * s + 3] = m2 / double(nb - h1);
  }
}

int series_stats_check(int S, int64_t n, int64_t ld, int n_blocks, std::string& err) {
  if (S < 1 || S > 65535 || n < 2 || ld < n || n_blocks < 0 || n_blocks == 1 || n_blocks > kSeriesMaxBlocks ||
      (n_blocks >= 2 && n < n_blocks)) {
    err = "series statistics: need 1..65535 rows of n >= 2 samples (row stride >= n) and n_blocks 0 or "
          "2..1024 with n >= n_blocks";
    return HMD_EINVAL;
  }
  return HMD_OK;
}

void series_stats_enqueue(hipStream_t st, const double* d_x, int S, int64_t n, int64_t ld, double scale,
                          int n_blocks, double* d_gam, double* d_out) {
  hipLaunchKernelGGL(k_series_moments, dim3(S), dim3(SER_TPB), 0, st, d_x, ld, n, scale, d_out);
  if (n_blocks >= 2) {
    hipLaunchKernelGGL(k_series_blocks, dim3(S), dim3(SER_TPB), 0, st, d_x, ld, n, scale, n_blocks, d_out);
    return;
  }
  const unsigned lag_tiles = unsigned((n + SER_TPB - 1) / SER_TPB);
  hipLaunchKernelGGL(k_series_acov, dim3(lag_tiles, S), dim3(SER_TPB), 0, st, d_x, ld, n, scale, d_out, d_gam, n);
  hipLaunchKernelGGL(k_series_geyer, dim3((S + 63) / 64), dim3(64), 0, st, d_gam, n, n, S, d_out);
}

// ---------------------------------------------------------------------------
// Allocation-free form.  The autocovariance scratch lives in a fixed device
// array, one copy per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// symbol): its device address is looked up once per device at context
// creation and that address is what the kernels receive.
// ---------------------------------------------------------------------------
namespace {

static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

int series_noalloc_init(int device, std::string& err) {
  if (device < 0 || device >= kMaxDevices) {
    err = "series scratch: device index out of range";
    return HMD_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return HMD_OK;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) prev = device;
  hipError_t e = hipSetDevice(device);
  void* ptr = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  (void)hipSetDevice(prev);
  if (e != hipSuccess || !ptr) {
    err = std::string("series scratch: hipGetSymbolAddress: ") + hipGetErrorString(e);
    return HMD_EDEVICE;
  }
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return HMD_OK;
}

double* series_noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace hmd

extern "C" int md_series_stats_noalloc(hmd_ctx* ctx, const double* d_x, int S, int64_t n, int64_t ld, int n_blocks,
                                       double* d_out, void* stream) {
  if (!ctx || !d_x || !d_out) return HMD_EINVAL;
  HMD_TRY(hmd::series_stats_check(S, n, ld, n_blocks, ctx->err));
  const int64_t need = n_blocks == 0 ? int64_t(S) * n : 0;
  if (need > hmd::kNoAllocScratchDoubles) {
    ctx->err = "md_series_stats_noalloc: S * n = " + std::to_string(need) + " exceeds the fixed scratch of " +
               std::to_string(hmd::kNoAllocScratchDoubles) + " doubles";
    return HMD_EINVAL;
  }
  double* sc = hmd::series_noalloc_scratch(ctx->device);
  if (!sc) {
    ctx->err = "md_series_stats_noalloc: no scratch address for this device (context not set up)";
    return HMD_EDEVICE;
  }
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
  hmd::series_stats_enqueue(s, d_x, S, n, ld, 1.0, n_blocks, sc, d_out);
  HMD_HIP(ctx, hipGetLastError());
  return HMD_OK;
}
