// series.h -- device statistics of sampled series (see series.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace hmd {

constexpr int kSeriesMaxBlocks = 1024;  // block rule: at most this many blocks
// entries of a system's sampled flux series (one per step up to this many
// sampled steps; beyond, each entry sums B consecutive steps)
constexpr int64_t kSeriesCap = int64_t(1) << 16;

// Fixed device scratch of the allocation-free form: 2^21 doubles (16 MiB)
// per GPU, enough for the autocovariances of S series of n samples with
// S n <= 2^21.
constexpr int64_t kNoAllocScratchDoubles = int64_t(1) << 21;

// Look up (once per device) the device address of the fixed scratch array;
// called when a context is created on that device.
int series_noalloc_init(int device, std::string& err);

// HMD_OK, or HMD_EINVAL with a message for arguments the kernels cannot take.
int series_stats_check(int S, int64_t n, int64_t ld, int n_blocks, std::string& err);
// Queue the statistics of S rows (n samples, row stride ld, each sample times
// `scale`) on stream st: d_out[4 S] receives mean, standard error, first-half
// and second-half means per row.  n_blocks 0: Geyer's initial monotone
// sequence estimator, which needs d_gam[S n] doubles of scratch (the
// autocovariances); n_blocks >= 2: the block rule (d_gam unused).
void series_stats_enqueue(hipStream_t st, const double* d_x, int S, int64_t n, int64_t ld, double scale,
                          int n_blocks, double* d_gam, double* d_out);

}  // namespace hmd
