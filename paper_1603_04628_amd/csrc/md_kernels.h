// md_kernels.h -- kernel declarations of the NEMD step (see md_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "engine.h"

namespace hmd {

constexpr int BIN_LDS = 128;  // LDS profile bins per block

// Pointers to one copy of the FP64 SoA state.
struct StateRef {
  double *x, *y, *z, *vx, *vy, *vz;
};

template <int MODE>
__global__ void k_integrate(int ntot, const SimDev* sims, const uint16_t* atom_sim, StateRef st, const float4* f4,
                            uint32_t* key, uint32_t* count, uint32_t* rank, Acc acc, const int64_t* dstate,
                            StepConst K);
__global__ void k_scan(const SimDev* sims, uint32_t* count, uint32_t* cursor, uint32_t* start, uint32_t* ncount,
                       int64_t* dstate, int advance);
__global__ void k_scatter(int ntot, const uint32_t* key, const uint32_t* start, const uint32_t* rank, uint32_t* perm);
__global__ void k_reorder(int ntot, const SimDev* sims, const uint16_t* cell_sim, const uint32_t* key,
                          const uint32_t* start, const uint32_t* ncount, const uint32_t* perm, StateRef src,
                          StateRef dst, const int* tag_src, int* tag_dst, float4* pos4);
template <int MODE>
__global__ void k_force(int ntot, const SimDev* sims, const uint16_t* atom_sim, const float4* pos4,
                        const uint32_t* start, const uint32_t* ncount, const float4* wpos4, const uint32_t* wstart,
                        const uint32_t* wcount, float4* f4, StateRef st, Acc acc, int64_t* dstate, StepConst K);
__global__ void k_set_i64(int64_t* p, int64_t v);

}  // namespace hmd
