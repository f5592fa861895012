// md_kernels.hip -- gfx950 kernels of the NEMD step (paper, Appendix A):
//   integrate  finish the previous step (Berendsen factor, sampling of the
//              mass flow rate), first half-kick, drift, periodic wrap, cell
//              key and per-cell count                       (memory bound)
//   scan       per-system exclusive scan of cell counts     (latency bound)
//   scatter    counting-sort scatter of slot indices        (memory bound)
//   reorder    stable placement inside each cell, permutation of the FP64
//              state, FP32 cell-relative position copy      (memory bound)
//   force      FP32 Lennard-Jones forces over the 27 neighbouring cells
//              (fluid and frozen wall atoms), second half-kick, thermostat
//              and energy sums                              (VALU bound)
// All systems of a batch are flattened: one launch per kernel covers them.
#include <hip/hip_runtime.h>

#include "engine.h"
#include "md_kernels.h"

namespace hmd {

namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ int dcell(double x, double inv, int n) {
  const double t = floor(x * inv);
  if (!(t >= 0.0)) return 0;
  if (t >= double(n - 1)) return n - 1;
  return int(t);
}

__device__ __forceinline__ double wrap_periodic(double x, double L) {
  double y = x;
  if (y >= L) y = y - L;
  else if (y < 0.0) y = y + L;
  if (y >= L) y = 0.0;
  return y;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// True when every active lane of the wave holds the same system index.
__device__ __forceinline__ bool wave_uniform(int s) {
  const int s0 = __shfl(s, 0);
  return __all(s == s0 || s < 0) != 0 && s0 >= 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// integrate: MODE 0 cell keys only; 1 full step; 2 finish-only (Berendsen
// factor applied in registers for the final sample, nothing written back).
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_integrate(int ntot, const SimDev* __restrict__ sims,
                                                   const uint16_t* __restrict__ atom_sim,
                                                   StateRef st, const float4* __restrict__ f4,
                                                   uint32_t* __restrict__ key, uint32_t* __restrict__ count,
                                                   uint32_t* __restrict__ rank, Acc acc,
                                                   const int64_t* __restrict__ dstate, StepConst K) {
  __shared__ double lds_vx[BIN_LDS];
  __shared__ double lds_cnt[BIN_LDS];
  __shared__ int lds_bin_base;

  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < ntot;
  const int s = valid ? int(atom_sim[i]) : -1;
  const SimDev* D = valid ? &sims[s] : nullptr;

  double r[3] = {0, 0, 0}, v[3] = {0, 0, 0};
  if (valid) {
    r[0] = st.x[i]; r[1] = st.y[i]; r[2] = st.z[i];
    v[0] = st.vx[i]; v[1] = st.vy[i]; v[2] = st.vz[i];
  }

  if (MODE != 0) {
    const int64_t n = dstate[0];
    const int64_t n_equil = dstate[1];
    const int64_t sampled = dstate[2];
    const bool pending = dstate[3] != 0;
    // Berendsen (Appendix A) on the thermostatted component, from the sum
    // gathered after the previous step's second half-kick.
    if (valid && pending) {
      const double Tc = acc.vc2[n & 1][s] * D->inv_nf;
      const double lam = sqrt(1.0 + K.dt_tau * (K.T0 / Tc - 1.0));
      v[K.axis] *= lam;
    }
    // Sample the completed step n (mass flow rate per unit span, Sec. 2.1).
    const int64_t ns = n - n_equil - 1;
    if (n > n_equil && n > sampled && ns >= K.r) {
      const int64_t b = (ns - K.r) / K.B;
      if (b < K.nb) {
        double q[4] = {v[0], v[0] * v[0], v[1] * v[1], v[2] * v[2]};
        if (wave_uniform(s)) {
#pragma unroll
          for (int k = 0; k < 4; ++k) q[k] = wave_sum(valid ? q[k] : 0.0);
          const int sw = __shfl(s, 0);
          if ((threadIdx.x & (WAVE - 1)) == 0 && sw >= 0) {
            const SimDev& Dw = sims[sw];
            atomicAdd(&acc.blocks[int64_t(sw) * K.nb + b], q[0] * Dw.inv_area);
            atomicAdd(&acc.tsum[3 * sw + 0], q[1] * Dw.inv_nf);
            atomicAdd(&acc.tsum[3 * sw + 1], q[2] * Dw.inv_nf);
            atomicAdd(&acc.tsum[3 * sw + 2], q[3] * Dw.inv_nf);
          }
        } else if (valid) {
          atomicAdd(&acc.blocks[int64_t(s) * K.nb + b], q[0] * D->inv_area);
          atomicAdd(&acc.tsum[3 * s + 0], q[1] * D->inv_nf);
          atomicAdd(&acc.tsum[3 * s + 1], q[2] * D->inv_nf);
          atomicAdd(&acc.tsum[3 * s + 2], q[3] * D->inv_nf);
        }
        if (K.bins_on) {
          // Wall-normal profile: aggregate in LDS relative to the block's
          // first bin, spill to global atomics when out of range.
          int gb = -1;
          if (valid) {
            int bb = int(floor(r[1] * D->inv_bin));
            bb = bb < 0 ? 0 : (bb >= D->nbins ? D->nbins - 1 : bb);
            gb = D->bin0 + bb;
          }
          for (int k = threadIdx.x; k < BIN_LDS; k += blockDim.x) { lds_vx[k] = 0.0; lds_cnt[k] = 0.0; }
          if (threadIdx.x == 0) lds_bin_base = 0x7fffffff;
          __syncthreads();
          if (gb >= 0) atomicMin(&lds_bin_base, gb);
          __syncthreads();
          const int base = lds_bin_base;
          if (gb >= 0) {
            const int o = gb - base;
            if (o < BIN_LDS) {
              atomicAdd(&lds_vx[o], v[0]);
              atomicAdd(&lds_cnt[o], 1.0);
            } else {
              atomicAdd(&acc.binvx[gb], v[0]);
              atomicAdd(&acc.bincnt[gb], 1.0);
            }
          }
          __syncthreads();
          for (int k = threadIdx.x; k < BIN_LDS; k += blockDim.x)
            if (lds_cnt[k] != 0.0) {
              atomicAdd(&acc.binvx[base + k], lds_vx[k]);
              atomicAdd(&acc.bincnt[base + k], lds_cnt[k]);
            }
        }
      }
    }
    if (MODE == 2) return;
    if (valid && i == D->a0) {
      const int p = int((n + 1) & 1);
      acc.vc2[p][s] = 0.0;
      acc.pe[p][s] = 0.0;
      acc.ke[p][s] = 0.0;
    }
    // First half-kick with the force of the previous step, drift, wrap.
    const float4 f = valid ? f4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    if (valid) {
      v[0] += K.hdt * (double(f.x) + D->g);
      v[1] += K.hdt * double(f.y);
      v[2] += K.hdt * double(f.z);
      r[0] = wrap_periodic(r[0] + K.dt * v[0], D->Lx);
      r[1] = r[1] + K.dt * v[1];
      r[2] = wrap_periodic(r[2] + K.dt * v[2], D->Lz);
    }
    if (valid) {
      st.x[i] = r[0]; st.y[i] = r[1]; st.z[i] = r[2];
      st.vx[i] = v[0]; st.vy[i] = v[1]; st.vz[i] = v[2];
      const bool bad = !(r[1] > 0.0 && r[1] < D->h) || !(r[0] >= 0.0 && r[0] < D->Lx) ||
                       !(r[2] >= 0.0 && r[2] < D->Lz) || !isfinite(v[0]) || !isfinite(v[1]) || !isfinite(v[2]);
      if (bad) atomicOr(&acc.status[s], 1);
    }
  }
  uint32_t c = 0;
  if (valid) {
    const int cx = dcell(r[0], D->inv_x, D->nx);
    const int cy = dcell(r[1], D->inv_y, D->ny);
    const int cz = dcell(r[2], D->inv_z, D->nz);
    c = uint32_t(D->c0 + (cz * D->ny + cy) * D->nx + cx);
    key[i] = c;
  }
  // Arrival rank inside the cell: lanes of a wave with the same key take one
  // atomic together (sorted neighbours share keys, so a wave has few keys).
  const int lane = threadIdx.x & (WAVE - 1);
  const unsigned long long lt = (1ull << lane) - 1ull;
  bool todo = valid;
  uint32_t rk = 0;
  while (__any(todo)) {
    const unsigned long long pm = __ballot(todo);
    const int leader = __ffsll(pm) - 1;
    const uint32_t ck = __shfl(c, leader);
    const bool mine = todo && c == ck;
    const unsigned long long m = __ballot(mine);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&count[ck], uint32_t(__popcll(m)));
    base = __shfl(base, leader);
    if (mine) {
      rk = base + uint32_t(__popcll(m & lt));
      todo = false;
    }
  }
  if (valid) rank[i] = rk;
}

// ---------------------------------------------------------------------------
// scan: one block per system; exclusive scan of the per-cell counts into
// global slot offsets; counters are cleared for the next step.  Block 0
// advances the device step counter when `advance` is set.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_scan(const SimDev* __restrict__ sims, uint32_t* __restrict__ count,
                                               uint32_t* __restrict__ cursor, uint32_t* __restrict__ start,
                                               uint32_t* __restrict__ ncount, int64_t* __restrict__ dstate,
                                               int advance) {
  __shared__ uint32_t wave_tot[1024 / WAVE];
  __shared__ uint32_t carry;
  const SimDev& D = sims[blockIdx.x];
  const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
  if (threadIdx.x == 0) carry = uint32_t(D.a0);
  __syncthreads();
  for (int base = 0; base < D.ncell; base += blockDim.x) {
    const int c = base + threadIdx.x;
    const uint32_t n = c < D.ncell ? count[D.c0 + c] : 0u;
    uint32_t incl = n;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const uint32_t t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    if (lane == WAVE - 1) wave_tot[wid] = incl;
    __syncthreads();
    if (wid == 0) {
      uint32_t w = lane < int(blockDim.x / WAVE) ? wave_tot[lane] : 0u;
      uint32_t wi = w;
#pragma unroll
      for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t t = __shfl_up(wi, o);
        if (lane >= o) wi += t;
      }
      if (lane < int(blockDim.x / WAVE)) wave_tot[lane] = wi - w;
    }
    __syncthreads();
    const uint32_t excl = carry + wave_tot[wid] + incl - n;
    if (c < D.ncell) {
      start[D.c0 + c] = excl;
      ncount[D.c0 + c] = n;
      count[D.c0 + c] = 0u;
      cursor[D.c0 + c] = 0u;
    }
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) carry = excl + n;
    __syncthreads();
  }
  if (advance && blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t n = dstate[0];
    if (n > dstate[1] && n > dstate[2]) dstate[2] = n;
    dstate[0] = n + 1;
  }
}

// scatter: counting-sort placement of every slot index into its cell's range
// at its arrival rank (the order inside a cell is fixed by the reorder kernel).
__global__ __launch_bounds__(256) void k_scatter(int ntot, const uint32_t* __restrict__ key,
                                                 const uint32_t* __restrict__ start,
                                                 const uint32_t* __restrict__ rank, uint32_t* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  perm[start[key[i]] + rank[i]] = uint32_t(i);
}

// reorder: inside each cell, the atom from old slot p goes to position
// (number of cell members with a smaller old slot) -- a stable counting sort
// of the previous order by cell.  Copies the FP64 state and the id, and
// writes the FP32 position relative to the cell's lower corner.
__global__ __launch_bounds__(256) void k_reorder(int ntot, const SimDev* __restrict__ sims,
                                                 const uint16_t* __restrict__ cell_sim,
                                                 const uint32_t* __restrict__ key,
                                                 const uint32_t* __restrict__ start,
                                                 const uint32_t* __restrict__ ncount,
                                                 const uint32_t* __restrict__ perm, StateRef src, StateRef dst,
                                                 const int* __restrict__ tag_src, int* __restrict__ tag_dst,
                                                 float4* __restrict__ pos4) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ntot) return;
  const uint32_t p = perm[j];
  const uint32_t c = key[p];
  const uint32_t st = start[c], n = ncount[c];
  uint32_t rank = 0;
  for (uint32_t m = 0; m < n; ++m) rank += perm[st + m] < p ? 1u : 0u;
  const uint32_t d = st + rank;
  const double x = src.x[p], y = src.y[p], z = src.z[p];
  dst.x[d] = x; dst.y[d] = y; dst.z[d] = z;
  dst.vx[d] = src.vx[p]; dst.vy[d] = src.vy[p]; dst.vz[d] = src.vz[p];
  tag_dst[d] = tag_src[p];
  const SimDev& D = sims[cell_sim[c]];
  const int lc = int(c) - D.c0;
  const int cx = lc % D.nx, cy = (lc / D.nx) % D.ny, cz = lc / (D.nx * D.ny);
  pos4[d] = make_float4(float(x - double(cx) * D.wx), float(y - double(cy) * D.wy),
                        float(z - double(cz) * D.wz), __int_as_float(lc));
}

// Second half-kick (MODE 1) and the per-system sums that the next step's
// Berendsen factor and the energy trace need.
template <int MODE>
__device__ __forceinline__ void finish_force(int i, bool valid, int s, const SimDev* __restrict__ sims, float fx,
                                             float fy, float fz, float pe, StateRef st, Acc acc,
                                             int64_t* __restrict__ dstate, const StepConst& K) {
  const int p = int(dstate[0] & 1);
  double vc2 = 0.0, ke = 0.0, pes = valid ? double(pe) : 0.0;
  if (MODE == 1 && valid) {
    const SimDev& D = sims[s];
    double v[3] = {st.vx[i] + K.hdt * (double(fx) + D.g), st.vy[i] + K.hdt * double(fy),
                   st.vz[i] + K.hdt * double(fz)};
    st.vx[i] = v[0]; st.vy[i] = v[1]; st.vz[i] = v[2];
    vc2 = v[K.axis] * v[K.axis];
    ke = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  }
  if (MODE == 1 || K.energy_on) {
    if (wave_uniform(s)) {
      vc2 = wave_sum(vc2);
      if (K.energy_on) { ke = wave_sum(ke); pes = wave_sum(pes); }
      const int sw = __shfl(s, 0);
      if ((threadIdx.x & (WAVE - 1)) == 0) {
        if (MODE == 1) atomicAdd(&acc.vc2[p][sw], vc2);
        if (K.energy_on) { atomicAdd(&acc.ke[p][sw], ke); atomicAdd(&acc.pe[p][sw], pes); }
      }
    } else if (valid) {
      if (MODE == 1) atomicAdd(&acc.vc2[p][s], vc2);
      if (K.energy_on) { atomicAdd(&acc.ke[p][s], ke); atomicAdd(&acc.pe[p][s], pes); }
    }
  }
  if (MODE == 1 && blockIdx.x == 0 && threadIdx.x == 0) dstate[3] = K.thermo_on;
}

// ---------------------------------------------------------------------------
// force (one thread per slot): shifted LJ (Eq. LJ) over the 27 neighbouring
// cells, fluid-fluid and wall-fluid, FP32.  Cell-relative coordinates keep
// the FP32 separations accurate; the image shift of a neighbouring cell is
// its offset times the cell width.  MODE 1 adds the second half-kick and the
// thermostat / energy sums.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_force(int ntot, const SimDev* __restrict__ sims,
                                               const uint16_t* __restrict__ atom_sim,
                                               const float4* __restrict__ pos4, const uint32_t* __restrict__ start,
                                               const uint32_t* __restrict__ ncount,
                                               const float4* __restrict__ wpos4, const uint32_t* __restrict__ wstart,
                                               const uint32_t* __restrict__ wcount, float4* __restrict__ f4,
                                               StateRef st, Acc acc, int64_t* __restrict__ dstate, StepConst K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < ntot;
  const int s = valid ? int(atom_sim[i]) : -1;
  float fx = 0.f, fy = 0.f, fz = 0.f, pe = 0.f;
  uint32_t nff = 0, nwf = 0;  // in-cutoff pairs (energy passes only)
  if (valid) {
    const SimDev& D = sims[s];
    const float4 me = pos4[i];
    const int lc = __float_as_int(me.w);
    const int cx = lc % D.nx, cy = (lc / D.nx) % D.ny, cz = lc / (D.nx * D.ny);
    for (int oz = -1; oz <= 1; ++oz) {
      int jz = cz + oz;
      jz += jz < 0 ? D.nz : (jz >= D.nz ? -D.nz : 0);
      const float az = me.z - float(oz) * D.fwz;
      for (int oy = -1; oy <= 1; ++oy) {
        const int jy = cy + oy;
        const float ay = me.y - float(oy) * D.fwy;
        const bool wall = jy < 0 || jy >= D.ny;
        for (int ox = -1; ox <= 1; ++ox) {
          int jx = cx + ox;
          jx += jx < 0 ? D.nx : (jx >= D.nx ? -D.nx : 0);
          const float ax = me.x - float(ox) * D.fwx;
          if (!wall) {
            const uint32_t gc = uint32_t(D.c0 + (jz * D.ny + jy) * D.nx + jx);
            const uint32_t b = start[gc], e = b + ncount[gc];
            for (uint32_t j = b; j < e; ++j) {
              const float4 o = pos4[j];
              const float dx = ax - o.x, dy = ay - o.y, dz = az - o.z;
              const float r2 = dx * dx + dy * dy + dz * dz;
              if (r2 < K.rc2 && j != uint32_t(i)) {
                const float ri2 = 1.0f / r2;
                const float ri6 = ri2 * ri2 * ri2;
                const float fr = 24.0f * ri6 * (2.0f * ri6 - 1.0f) * ri2;
                fx += fr * dx; fy += fr * dy; fz += fr * dz;
                if (K.energy_on) {
                  pe += 0.5f * (4.0f * ri6 * (ri6 - 1.0f) - K.ush_ff);
                  ++nff;
                }
              }
            }
          } else {
            const int slab = jy < 0 ? 0 : 1;
            const uint32_t wc = uint32_t(D.wc0 + (slab * D.nz + jz) * D.nx + jx);
            const uint32_t b = wstart[wc], e = b + wcount[wc];
            for (uint32_t j = b; j < e; ++j) {
              const float4 o = wpos4[j];
              const float dx = ax - o.x, dy = ay - o.y, dz = az - o.z;
              const float r2 = dx * dx + dy * dy + dz * dz;
              if (r2 < K.rc2) {
                const float ri2 = 1.0f / r2;
                const float s2 = K.sig2_wf * ri2;
                const float s6 = s2 * s2 * s2;
                const float fr = 24.0f * K.eps_wf * s6 * (2.0f * s6 - 1.0f) * ri2;
                fx += fr * dx; fy += fr * dy; fz += fr * dz;
                if (K.energy_on) {
                  pe += 4.0f * K.eps_wf * s6 * (s6 - 1.0f) - K.ush_wf;
                  ++nwf;
                }
              }
            }
          }
        }
      }
    }
    f4[i] = make_float4(fx, fy, fz, pe);
  }
  if (K.energy_on) {
    const unsigned long long a = wave_sum((unsigned long long)nff), w = wave_sum((unsigned long long)nwf);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
      atomicAdd(&acc.pairs[0], a);
      atomicAdd(&acc.pairs[1], w);
    }
  }
  finish_force<MODE>(i, valid, s, sims, fx, fy, fz, pe, st, acc, dstate, K);
}

template __global__ void k_integrate<0>(int, const SimDev*, const uint16_t*, StateRef, const float4*, uint32_t*,
                                        uint32_t*, uint32_t*, Acc, const int64_t*, StepConst);
template __global__ void k_integrate<1>(int, const SimDev*, const uint16_t*, StateRef, const float4*, uint32_t*,
                                        uint32_t*, uint32_t*, Acc, const int64_t*, StepConst);
template __global__ void k_integrate<2>(int, const SimDev*, const uint16_t*, StateRef, const float4*, uint32_t*,
                                        uint32_t*, uint32_t*, Acc, const int64_t*, StepConst);
template __global__ void k_force<0>(int, const SimDev*, const uint16_t*, const float4*, const uint32_t*,
                                    const uint32_t*, const float4*, const uint32_t*, const uint32_t*, float4*,
                                    StateRef, Acc, int64_t*, StepConst);
template __global__ void k_force<1>(int, const SimDev*, const uint16_t*, const float4*, const uint32_t*,
                                    const uint32_t*, const float4*, const uint32_t*, const uint32_t*, float4*,
                                    StateRef, Acc, int64_t*, StepConst);

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

}  // namespace hmd
