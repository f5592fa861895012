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

// Step index of a launch: steps completed before it = *base + k (base null:
// k alone).
struct StepRef {
  const int64_t* base;
  int64_t k;
};

template <int MODE, int PATH>
__global__ void k_integrate(int ntot, const SimDev* sims, const uint16_t* atom_sim, StateRef st, const float4* f4,
                            uint32_t* key, uint32_t* count, uint32_t* rank, int4* pfix, const int4* pbuild,
                            int* flag, Acc acc, const int64_t* dstate, StepRef R, StepConst K);
__global__ void k_keys(int ntot, const SimDev* sims, const uint16_t* atom_sim, StateRef st, uint32_t* key,
                       uint32_t* count, uint32_t* rank, const int* flag, StepRef R);
__global__ void k_scan(const SimDev* sims, uint32_t* count, uint32_t* start, uint32_t* ncount, const int* flag,
                       StepRef R);
__global__ void k_scatter(int ntot, const uint32_t* key, const uint32_t* start, const uint32_t* rank, uint32_t* perm,
                          const int* flag, StepRef R);
template <int PATH>
__global__ void k_reorder(int ntot, const SimDev* sims, const uint16_t* cell_sim, const uint32_t* key,
                          const uint32_t* start, const uint32_t* ncount, const uint32_t* perm, StateRef src,
                          StateRef dst, const int* tag_src, int* tag_dst, float4* pos4, int4* pfix, int4* pbuild,
                          uint32_t* slot_cell, const int* flag, StepRef R);
__global__ void k_build_list(int ntot, int ld, int cap, const SimDev* sims, const uint16_t* atom_sim,
                             const uint32_t* slot_cell, const int4* pfix, const uint32_t* start,
                             const uint32_t* ncount, const uint32_t* wstart, const uint32_t* wcount, uint32_t* list,
                             uint32_t* nlist, StateRef from, StateRef to, const int* tag_from, int* tag_to,
                             int* overflow, const int* flag, StepRef R, float rl2);
template <int MODE>
__global__ void k_force_cell(int ntot, const SimDev* sims, const uint16_t* atom_sim, const float4* pos4,
                             const uint32_t* start, const uint32_t* ncount, const float4* wpos4,
                             const uint32_t* wstart, const uint32_t* wcount, float4* f4, StateRef st, Acc acc,
                             int64_t* dstate, StepRef R, StepConst K);
template <int MODE, int ENERGY, int UNI, int WS, int PR>
__global__ void k_force_list(int ntot, int ld, const SimDev* sims, const uint16_t* atom_sim, const int4* pfix,
                             const uint32_t* list, const uint32_t* nlist, float4* f4, StateRef st, Acc acc,
                             int64_t* dstate, StepRef R, StepConst K);
constexpr int TILE_THREADS = 256;  // threads per tile workgroup
// LDS capacity of a tile in atoms (x, y, z fixed point: 36 KiB, so four
// workgroups share a compute unit's 160 KiB); a
// compile-time size lets every LDS read carry its array offset as an immediate
constexpr int TILE_STAGE = 3072;
// cells of a tile's neighbourhood listed in LDS by the list build
constexpr int TILE_CTAB = 768;
// 32-bit words of a tile's range table, kept in memory from one list build
// to the next
constexpr int TILE_REC = 49;
template <int UNI>
__global__ void k_build_tiles(int ntot, int ld, int cap, const int4* tiles, const SimDev* sims,
                              const uint32_t* slot_cell, const int4* pfix, const uint32_t* start,
                              const uint32_t* ncount, const uint32_t* wstart, const uint32_t* wcount,
                              uint32_t* list, uint32_t* nlist, uint32_t* tilerec, StateRef from, StateRef to,
                              const int* tag_from, int* tag_to, int* overflow, const int* flag, StepRef R,
                              float rl2, int global_out);
template <int MODE, int ENERGY, int UNI, int WS, int PR>
__global__ void k_force_tiles(int ntot, int ld, const uint32_t* tilerec, const SimDev* sims, const int4* pfix,
                              const uint32_t* list, const uint32_t* nlist, float4* f4, StateRef st, Acc acc,
                              int64_t* dstate, StepRef R, StepConst K);
__global__ void k_stamp(unsigned long long* slot, const int* flag, StepRef R);
__global__ void k_set_i64(int64_t* p, int64_t v);
__global__ void k_add_i64(int64_t* p, int64_t v);
__global__ void k_set_i32(int* p, int v);

}  // namespace hmd
