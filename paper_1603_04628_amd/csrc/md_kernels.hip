// md_kernels.hip -- gfx950 kernels of the NEMD step (paper, Appendix A:
// shifted LJ fluid between frozen walls, velocity Verlet, Berendsen on one
// velocity component, periodic in x and z; body force of Eq. momentumEq).
//
// Two force paths share the integrator and the counting sort:
//   cell path   every step: keys -> scan -> scatter -> reorder (stable
//               counting sort of the FP64 state by cell), then FP32 forces
//               over the 27 neighbouring cells from cell-relative positions;
//   pair path   fixed-point positions (32-bit per axis, so a periodic
//               minimum image is plain integer wrap-around); a Verlet pair
//               list with cut-off rc + skin is rebuilt from the same counting
//               sort only on steps where some atom has moved skin/2 since the
//               last build -- the rebuild kernels read a device flag and
//               return at once otherwise, so one captured graph serves every
//               step.
// Every kernel covers all systems of a batch (flattened slots and cells).
// Step n (1-based) is identified as base + k with base read from device
// memory (graph replays) or zero (direct launches).
#include <hip/hip_runtime.h>
#include <type_traits>

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

__device__ __forceinline__ uint32_t fix_axis(double v, double scale) {
  double t = v * scale;
  t = t < 0.0 ? 0.0 : (t > 4294967295.0 ? 4294967295.0 : t);
  return uint32_t(t);
}

// Fixed-point position: x, z over the periodic extents, y over the wall span.
__device__ __forceinline__ int4 to_fixed(double x, double y, double z, const SimDev& D) {
  return make_int4(int(fix_axis(x, D.fix_x)), int(fix_axis(y - D.y_lo, D.fix_y)), int(fix_axis(z, D.fix_z)), 0);
}

// Separation a - b in FP32 from fixed-point positions (wrap-around of the
// 32-bit difference is the periodic minimum image in x and z).
__device__ __forceinline__ float3 fixed_sep(const int4& a, const int4& b, const SimDev& D) {
  return make_float3(float(int(uint32_t(a.x) - uint32_t(b.x))) * D.unit_x,
                     float(int(uint32_t(a.y) - uint32_t(b.y))) * D.unit_y,
                     float(int(uint32_t(a.z) - uint32_t(b.z))) * D.unit_z);
}

__device__ __forceinline__ int64_t step_n(const StepRef& R) { return (R.base ? *R.base : 0) + R.k; }

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
// Renumber them so every XCD walks one contiguous range of slots: spatially
// sorted neighbours then share that XCD's L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int q = nb / NXCD, rem = nb % NXCD;
  const int x = b % NXCD, r = b / NXCD;
  return x < rem ? x * (q + 1) + r : rem * (q + 1) + (x - rem) * q + r;
}

__device__ __forceinline__ bool rebuild_needed(const int* flag, const StepRef& R) {
  return flag == nullptr || flag[(step_n(R) + 1) & 1] != 0;
}

// Arrival rank of each lane's key inside its cell: lanes of a wave with the
// same key take one atomic together (sorted neighbours share keys).
__device__ __forceinline__ void rank_in_cell(bool valid, uint32_t c, uint32_t* __restrict__ count,
                                             uint32_t* __restrict__ rank, int i) {
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

// Arrival rank of each slot in its cell, a block at a time (blockDim <= 256,
// all threads call it): the block counts its own atoms per cell in an LDS
// table, then takes one global atomic per distinct cell -- all in parallel,
// where the wavefront version takes one per cell in turn.
__device__ __forceinline__ void rank_in_cell_block(bool valid, uint32_t c, uint32_t* __restrict__ count,
                                                   uint32_t* __restrict__ rank, int i) {
  constexpr uint32_t H = 256, EMPTY = 0xffffffffu;
  __shared__ uint32_t hkey[H], hcnt[H], hbase[H];
  const uint32_t tid = threadIdx.x;
  for (uint32_t k = tid; k < H; k += blockDim.x) { hkey[k] = EMPTY; hcnt[k] = 0u; }
  __syncthreads();
  uint32_t h = c & (H - 1u), local = 0;
  if (valid) {  // open addressing: at most blockDim distinct keys in H slots
    for (;;) {
      const uint32_t old = atomicCAS(&hkey[h], EMPTY, c);
      if (old == EMPTY || old == c) break;
      h = (h + 1u) & (H - 1u);
    }
    local = atomicAdd(&hcnt[h], 1u);
  }
  __syncthreads();
  for (uint32_t k = tid; k < H; k += blockDim.x)
    if (hkey[k] != EMPTY) hbase[k] = atomicAdd(&count[hkey[k]], hcnt[k]);
  __syncthreads();
  if (valid) rank[i] = hbase[h] + local;
}

}  // namespace

// ---------------------------------------------------------------------------
// integrate.  MODE 0: no time step (cell path: keys and counts; pair path:
// fixed-point positions).  MODE 1: finish the previous step (Berendsen factor
// from the sum after its second half-kick), first half-kick with the stored
// force, drift, periodic wrap; the cell path then keys the slot, the pair
// path writes its fixed-point position and checks the displacement since the
// last list build.
// ---------------------------------------------------------------------------
template <int MODE, int PATH>
__global__ __launch_bounds__(256) void k_integrate(int ntot, const SimDev* __restrict__ sims,
                                                   const uint16_t* __restrict__ atom_sim, StateRef st,
                                                   const float4* __restrict__ f4, uint32_t* __restrict__ key,
                                                   uint32_t* __restrict__ count, uint32_t* __restrict__ rank,
                                                   int4* __restrict__ pfix, const int4* __restrict__ pbuild,
                                                   int* __restrict__ flag, Acc acc, const int64_t* __restrict__ dstate,
                                                   StepRef R, StepConst K) {
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  const bool valid = i < ntot;
  // The step of one atom for system s.  A wavefront whose atoms all belong
  // to one system (all but the few that straddle two) runs it with s in a
  // scalar register, so the system's constants come from scalar loads, not
  // one vector load per constant.
  auto body = [&](const int s) {
    const SimDev& D = sims[s];
    double r[3] = {0, 0, 0}, v[3] = {0, 0, 0};
    if (valid) {
      r[0] = st.x[i]; r[1] = st.y[i]; r[2] = st.z[i];
      v[0] = st.vx[i]; v[1] = st.vy[i]; v[2] = st.vz[i];
    }
    if (MODE == 1) {
      const int64_t n = step_n(R);  // steps completed before this one
      if (valid && dstate[3] != 0) {
        const double Tc = ((n & 1) ? acc.vc2[1] : acc.vc2[0])[s] * D.inv_nf;
        const double lam = sqrt(1.0 + K.dt_tau * (K.T0 / Tc - 1.0));
        v[0] *= K.axis == 0 ? lam : 1.0;
        v[1] *= K.axis == 1 ? lam : 1.0;
        v[2] *= K.axis == 2 ? lam : 1.0;
      }
      if (valid && i == D.a0) {
        const int p = int((n + 1) & 1);
        (p ? acc.vc2[1] : acc.vc2[0])[s] = 0.0;
        (p ? acc.pe[1] : acc.pe[0])[s] = 0.0;
        (p ? acc.ke[1] : acc.ke[0])[s] = 0.0;
      }
      if (PATH == 1 && i == 0 && flag) flag[n & 1] = 0;
      if (valid) {
        const float4 f = f4[i];
        v[0] += K.hdt * (double(f.x) + D.g);
        v[1] += K.hdt * double(f.y);
        v[2] += K.hdt * double(f.z);
        r[0] = wrap_periodic(r[0] + K.dt * v[0], D.Lx);
        r[1] = r[1] + K.dt * v[1];
        r[2] = wrap_periodic(r[2] + K.dt * v[2], D.Lz);
        st.x[i] = r[0]; st.y[i] = r[1]; st.z[i] = r[2];
        st.vx[i] = v[0]; st.vy[i] = v[1]; st.vz[i] = v[2];
        const bool bad = !(r[1] > 0.0 && r[1] < D.h) || !(r[0] >= 0.0 && r[0] < D.Lx) ||
                         !(r[2] >= 0.0 && r[2] < D.Lz) || !isfinite(v[0]) || !isfinite(v[1]) || !isfinite(v[2]);
        if (bad) atomicOr(&acc.status[s], 1);
      }
      if (PATH == 1) {
        if (valid) {
          const int4 p = to_fixed(r[0], r[1], r[2], D);
          pfix[i] = p;
          const float3 dd = fixed_sep(p, pbuild[i], D);
          if (dd.x * dd.x + dd.y * dd.y + dd.z * dd.z > K.half_skin2) flag[(n + 1) & 1] = 1;
        }
        return;
      }
    }
    if (PATH == 1) {
      if (valid) pfix[i] = to_fixed(r[0], r[1], r[2], D);
      return;
    }
    uint32_t c = 0;
    if (valid) {
      const int cx = dcell(r[0], D.inv_x, D.nx);
      const int cy = dcell(r[1], D.inv_y, D.ny);
      const int cz = dcell(r[2], D.inv_z, D.nz);
      c = uint32_t(D.c0) + D.rank[(cz * D.ny + cy) * D.nx + cx];
      key[i] = c;
    }
    rank_in_cell(valid, c, count, rank, i);
  };
  const int sl = valid ? int(atom_sim[i]) : 0;
  if (wave_uniform(valid ? sl : -1)) body(__builtin_amdgcn_readfirstlane(sl));
  else body(sl);
}

// Pair path: cell keys of the current positions on rebuild steps.
__global__ __launch_bounds__(256) void k_keys(int ntot, const SimDev* __restrict__ sims,
                                              const uint16_t* __restrict__ atom_sim, StateRef st,
                                              uint32_t* __restrict__ key, uint32_t* __restrict__ count,
                                              uint32_t* __restrict__ rank, const int* __restrict__ flag, StepRef R) {
  if (!rebuild_needed(flag, R)) return;
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  const bool valid = i < ntot;
  uint32_t c = 0;
  auto cell_of = [&](const int s) {
    const SimDev& D = sims[s];
    const int cx = dcell(st.x[i], D.inv_x, D.nx);
    const int cy = dcell(st.y[i], D.inv_y, D.ny);
    const int cz = dcell(st.z[i], D.inv_z, D.nz);
    return uint32_t(D.c0) + D.rank[(cz * D.ny + cy) * D.nx + cx];
  };
  const int sl = valid ? int(atom_sim[i]) : 0;
  if (wave_uniform(valid ? sl : -1)) {  // one system: its constants through scalar loads
    const int su = __builtin_amdgcn_readfirstlane(sl);
    if (valid) c = cell_of(su);
  } else if (valid) {
    c = cell_of(sl);
  }
  if (valid) key[i] = c;
  rank_in_cell_block(valid, c, count, rank, i);
}

// scan: one block per system; exclusive scan of the per-cell counts into
// global slot offsets; counters are cleared for the next sort.
__global__ __launch_bounds__(1024) void k_scan(const SimDev* __restrict__ sims, uint32_t* __restrict__ count,
                                               uint32_t* __restrict__ start, uint32_t* __restrict__ ncount,
                                               const int* __restrict__ flag, StepRef R) {
  if (!rebuild_needed(flag, R)) return;
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
      const uint32_t w = lane < int(blockDim.x / WAVE) ? wave_tot[lane] : 0u;
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
    }
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) carry = excl + n;
    __syncthreads();
  }
}

// scatter: counting-sort placement of every slot index into its cell's range
// at its arrival rank (the order inside a cell is fixed by the reorder kernel).
__global__ __launch_bounds__(256) void k_scatter(int ntot, const uint32_t* __restrict__ key,
                                                 const uint32_t* __restrict__ start,
                                                 const uint32_t* __restrict__ rank, uint32_t* __restrict__ perm,
                                                 const int* __restrict__ flag, StepRef R) {
  if (!rebuild_needed(flag, R)) return;
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  perm[start[key[i]] + rank[i]] = uint32_t(i);
}

// reorder: inside each cell, the atom from old slot p goes to position
// (number of cell members with a smaller old slot) -- a stable counting sort
// of the previous order by cell.  Copies the FP64 state and the id.  The cell
// path writes FP32 cell-relative positions; the pair path writes fixed-point
// positions (also the reference for the displacement test) and the cell of
// every new slot.
template <int PATH>
__global__ __launch_bounds__(256) void k_reorder(int ntot, const SimDev* __restrict__ sims,
                                                 const uint16_t* __restrict__ cell_sim,
                                                 const uint32_t* __restrict__ key, const uint32_t* __restrict__ start,
                                                 const uint32_t* __restrict__ ncount,
                                                 const uint32_t* __restrict__ perm, StateRef src, StateRef dst,
                                                 const int* __restrict__ tag_src, int* __restrict__ tag_dst,
                                                 float4* __restrict__ pos4, int4* __restrict__ pfix,
                                                 int4* __restrict__ pbuild, uint32_t* __restrict__ slot_cell,
                                                 const int* __restrict__ flag, StepRef R) {
  if (!rebuild_needed(flag, R)) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ntot) return;
  const uint32_t p = perm[j];
  const uint32_t c = key[p];
  const uint32_t st = start[c], n = ncount[c];
  // eight of the cell's entries in flight at a time (one at a time, each
  // waited for, made this loop the kernel's cost)
  uint32_t rank = 0, m = 0;
  for (; m + 8 <= n; m += 8) {
    uint32_t e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) e[u] = perm[st + m + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) rank += e[u] < p ? 1u : 0u;
  }
  for (; m < n; ++m) rank += perm[st + m] < p ? 1u : 0u;
  const uint32_t d = st + rank;
  const double x = src.x[p], y = src.y[p], z = src.z[p];
  dst.x[d] = x; dst.y[d] = y; dst.z[d] = z;
  dst.vx[d] = src.vx[p]; dst.vy[d] = src.vy[p]; dst.vz[d] = src.vz[p];
  tag_dst[d] = tag_src[p];
  const SimDev& D = sims[cell_sim[c]];
  const int lc = int(D.lin[int(c) - D.c0]);  // row-major id of the cell
  if (PATH == 0) {
    const int cx = lc % D.nx, cy = (lc / D.nx) % D.ny, cz = lc / (D.nx * D.ny);
    pos4[d] = make_float4(float(x - double(cx) * D.wx), float(y - double(cy) * D.wy),
                          float(z - double(cz) * D.wz), __int_as_float(lc));
  } else {
    const int4 q = to_fixed(x, y, z, D);
    pfix[d] = q;
    pbuild[d] = q;
    slot_cell[d] = c;
  }
}

// Pair path: Verlet list of every slot (fluid and wall atoms within rc + skin
// in the 27 neighbouring cells), stored transposed (entry k of slot i at
// k * ld + i); also moves the reordered FP64 state back to the primary copy.
__global__ __launch_bounds__(256) void k_build_list(int ntot, int ld, int cap, const SimDev* __restrict__ sims,
                                                    const uint16_t* __restrict__ atom_sim,
                                                    const uint32_t* __restrict__ slot_cell,
                                                    const int4* __restrict__ pfix, const uint32_t* __restrict__ start,
                                                    const uint32_t* __restrict__ ncount,
                                                    const uint32_t* __restrict__ wstart,
                                                    const uint32_t* __restrict__ wcount, uint32_t* __restrict__ list,
                                                    uint32_t* __restrict__ nlist, StateRef from, StateRef to,
                                                    const int* __restrict__ tag_from, int* __restrict__ tag_to,
                                                    int* __restrict__ overflow, const int* __restrict__ flag,
                                                    StepRef R, float rl2) {
  if (!rebuild_needed(flag, R)) return;
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  to.x[i] = from.x[i]; to.y[i] = from.y[i]; to.z[i] = from.z[i];
  to.vx[i] = from.vx[i]; to.vy[i] = from.vy[i]; to.vz[i] = from.vz[i];
  tag_to[i] = tag_from[i];
  const SimDev& D = sims[atom_sim[i]];
  const int4 me = pfix[i];
  const int lc = int(D.lin[int(slot_cell[i]) - D.c0]);
  const int cx = lc % D.nx, cy = (lc / D.nx) % D.ny, cz = lc / (D.nx * D.ny);
  if (i == 0) atomicAdd(&overflow[1], 1);  // builds so far
  // The 27 neighbouring cells are visited in ascending order of their first
  // entry in the position array (fluid slots, then wall atoms from ntot), so
  // every list comes out sorted by index: neighbouring slots then walk the
  // position array in step, which keeps the force kernel's gathers on shared
  // cache lines.  Key: first entry << 8 | entry count (the host guarantees
  // fewer than 2^24 entries; a cell of more than 255 atoms is reported as an
  // overflow).
  uint32_t key[32];
  bool big = false;
#pragma unroll
  for (int oz = -1; oz <= 1; ++oz) {
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy) {
#pragma unroll
      for (int ox = -1; ox <= 1; ++ox) {
        int jz = cz + oz;
        jz += jz < 0 ? D.nz : (jz >= D.nz ? -D.nz : 0);
        int jx = cx + ox;
        jx += jx < 0 ? D.nx : (jx >= D.nx ? -D.nx : 0);
        const int jy = cy + oy;
        uint32_t b, n;
        if (jy >= 0 && jy < D.ny) {
          const uint32_t gc = uint32_t(D.c0) + D.rank[(jz * D.ny + jy) * D.nx + jx];
          b = start[gc];
          n = ncount[gc];
        } else {
          const uint32_t wc = uint32_t(D.wc0 + ((jy < 0 ? 0 : 1) * D.nz + jz) * D.nx + jx);
          b = uint32_t(ntot) + wstart[wc];
          n = wcount[wc];
        }
        big |= n > 255u;
        key[(oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)] = (b << 8) | (n > 255u ? 255u : n);
      }
    }
  }
#pragma unroll
  for (int k = 27; k < 32; ++k) key[k] = 0xffffffffu;
  // bitonic sort of the 32 keys in registers (all indices compile-time)
#pragma unroll
  for (int size = 2; size <= 32; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
      for (int a = 0; a < 32; ++a) {
        const int c = a ^ stride;
        if (c > a) {
          const uint32_t lo = min(key[a], key[c]), hi = max(key[a], key[c]);
          const bool up = (a & size) == 0;
          key[a] = up ? lo : hi;
          key[c] = up ? hi : lo;
        }
      }
    }
  }
  if (big) atomicMax(&overflow[0], 1 << 30);
  // entries go out four at a time: group g of slot i is the 16 bytes at
  // (g * ld + i) * 4, so a wave's k-th groups form one contiguous run
  uint4* list4 = reinterpret_cast<uint4*>(list);
  uint4 buf = make_uint4(0u, 0u, 0u, 0u);
  uint32_t cnt = 0;
#pragma unroll 1
  for (int k = 0; k < 27; ++k) {
    // take the smallest remaining key and shift the rest down (register
    // moves; a run-time index into key[] would put it in private memory)
    const uint32_t kk = key[0];
#pragma unroll
    for (int t = 0; t < 26; ++t) key[t] = key[t + 1];
    const uint32_t b = kk >> 8, e = b + (kk & 255u);
    for (uint32_t q = b; q < e; ++q) {
      const float3 d = fixed_sep(me, pfix[q], D);
      const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
      if (r2 < rl2 && q != uint32_t(i)) {
        const uint32_t t = cnt & 3u;
        buf.x = t == 0 ? q : buf.x;
        buf.y = t == 1 ? q : buf.y;
        buf.z = t == 2 ? q : buf.z;
        buf.w = t == 3 ? q : buf.w;
        if (t == 3 && cnt < uint32_t(cap)) list4[size_t(cnt >> 2) * ld + i] = buf;
        ++cnt;
      }
    }
  }
  if ((cnt & 3u) != 0 && cnt < uint32_t(cap)) list4[size_t(cnt >> 2) * ld + i] = buf;
  if (cnt > uint32_t(cap)) {
    atomicMax(&overflow[0], int(cnt));
    cnt = cap;
  }
  nlist[i] = cnt;
}

// Second half-kick, sums for the next Berendsen factor and the energy trace,
// and the sample of the completed step (flux, temperatures, wall-normal
// profile).  Temperatures are stored with the Berendsen factor of this step
// applied: lambda^2 T_c = T_c + a (T0 - T_c), a = dt / tau.
// Whether step R + 1 is a sampled step (flux, temperatures, profile).
__device__ __forceinline__ bool sampled_step(int64_t nstep, const StepConst& K) {
  const int64_t ns = nstep - K.n_equil - 1;
  return nstep > K.n_equil && ns >= K.r && (ns - K.r) / K.B < K.nb;
}

// One atom's contribution to a tile's profile bin as a single 64-bit word, so
// that one integer LDS atomic adds both the streamwise velocity and the count
// (two FP32 LDS atomics per atom cost ~15 us per sampled step on the batch):
// count in the top 24 bits, v_x + TBIN_OFFSET in units of TBIN_UNIT below
// (40 bits hold 512 atoms of |v_x| < TBIN_OFFSET; the unit is 2.4e-7).
constexpr int TBIN_CNT_SHIFT = 40;
constexpr double TBIN_OFFSET = 16.0;
constexpr double TBIN_UNIT = 1.0 / 4194304.0;  // 2^-22
__device__ __forceinline__ unsigned long long tbin_word(double vx) {
  const double c = vx < -TBIN_OFFSET + 1e-3 ? -TBIN_OFFSET + 1e-3 : (vx > TBIN_OFFSET - 1e-3 ? TBIN_OFFSET - 1e-3 : vx);
  return (1ull << TBIN_CNT_SHIFT) + (unsigned long long)((c + TBIN_OFFSET) * (1.0 / TBIN_UNIT) + 0.5);
}

// vpre, ypre: the atom's velocity and its height in bin widths, when the
// caller has them already.
// TB = 1: the caller owns per-system profile bins in LDS (tbin, indexed from
// the system's first bin, packed as in tbin_word), cleared before and flushed
// after all of its atoms, and all of its lanes belong to one system; TB = 0:
// the bins are gathered here per call.
// Per-thread sums of a tile, reduced once per tile by the caller: thermostat
// component, kinetic and potential energy, then the flux and the three
// temperature components of a sampled step.
struct TileSums {
  double v[8];
};

template <int MODE, int TB = 0>
__device__ __forceinline__ void finish_force(int i, bool valid, int s, const SimDev* __restrict__ sims, float fx,
                                             float fy, float fz, float pe, StateRef st, Acc acc,
                                             int64_t* __restrict__ dstate, int64_t nstep, const StepConst& K,
                                             double* lds_vx, double* lds_cnt, int* lds_base,
                                             unsigned long long* tbin = nullptr,
                                             const double3* vpre = nullptr, TileSums* ts = nullptr,
                                             const double* ypre = nullptr, int tb_sampled = 0, float pw = 0.0f) {
  const int p = int(nstep & 1);
  double vc2 = 0.0, ke = 0.0, pes = valid ? double(pe) : 0.0;
  // scalars, not an array indexed by the run-time axis (that would live in
  // private memory)
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  if (MODE == 1 && valid) {
    const SimDev& D = sims[s];
    v0 = (vpre ? vpre->x : st.vx[i]) + K.hdt * (double(fx) + D.g);
    v1 = (vpre ? vpre->y : st.vy[i]) + K.hdt * double(fy);
    v2 = (vpre ? vpre->z : st.vz[i]) + K.hdt * double(fz);
    st.vx[i] = v0; st.vy[i] = v1; st.vz[i] = v2;
    const double vc = K.axis == 0 ? v0 : (K.axis == 1 ? v1 : v2);
    vc2 = vc * vc;
    ke = v0 * v0 + v1 * v1 + v2 * v2;
  }
  if (MODE == 1 || K.energy_on) {
    // parity-selected accumulators picked by value (indexing the by-value
    // pointer arrays with p would copy them to private memory)
    double* const acc_vc2 = p ? acc.vc2[1] : acc.vc2[0];
    double* const acc_ke = p ? acc.ke[1] : acc.ke[0];
    double* const acc_pe = p ? acc.pe[1] : acc.pe[0];
    if (TB) {  // the caller reduces over the tile
      ts->v[0] += vc2;
      if (K.energy_on) { ts->v[1] += ke; ts->v[2] += pes; }
    } else if (wave_uniform(valid ? s : -1)) {
      vc2 = wave_sum(vc2);
      if (K.energy_on) { ke = wave_sum(ke); pes = wave_sum(pes); }
      const int sw = TB ? s : __shfl(s, 0);  // tiles: s is uniform already
      if ((threadIdx.x & (WAVE - 1)) == 0) {
        if (MODE == 1) atomicAdd(&acc_vc2[sw], vc2);
        if (K.energy_on) { atomicAdd(&acc_ke[sw], ke); atomicAdd(&acc_pe[sw], pes); }
      }
    } else if (valid) {
      if (MODE == 1) atomicAdd(&acc_vc2[s], vc2);
      if (K.energy_on) { atomicAdd(&acc_ke[s], ke); atomicAdd(&acc_pe[s], pes); }
    }
  }
  if (MODE != 1) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) dstate[3] = K.thermo_on;
  // sample of step nstep (mass flow rate per unit span, Sec. 2.1)
  // tiles: the caller decides once per launch whether the step is sampled
  // (the block index needs a 64-bit division)
  int64_t b = 0;
  if (TB) {
    if (!tb_sampled) return;
  } else {
    const int64_t ns = nstep - K.n_equil - 1;
    if (nstep <= K.n_equil || ns < K.r) return;
    b = (ns - K.r) / K.B;
    if (b >= K.nb) return;
  }
  const double a = K.thermo_on ? K.dt_tau : 0.0;
  double q0 = v0, q1 = v0 * v0, q2 = v1 * v1, q3 = v2 * v2;
  if (K.axis == 0) q1 = (1.0 - a) * q1 + a * K.T0;
  else if (K.axis == 1) q2 = (1.0 - a) * q2 + a * K.T0;
  else q3 = (1.0 - a) * q3 + a * K.T0;
  // the wall normal pressure of the step (with pressure on): the atom's
  // share of (F_lo,y - F_hi,y) / 2, per unit area when added
  double q4 = valid ? 0.5 * double(pw) : 0.0;
  if (!valid) q0 = q1 = q2 = q3 = 0.0;
  if (TB) {
    ts->v[3] += q0; ts->v[4] += q1; ts->v[5] += q2; ts->v[6] += q3; ts->v[7] += q4;
  } else if (wave_uniform(valid ? s : -1)) {
    q0 = wave_sum(q0); q1 = wave_sum(q1); q2 = wave_sum(q2); q3 = wave_sum(q3);
    if (K.press_on) q4 = wave_sum(q4);
    const int sw = TB ? s : __shfl(s, 0);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
      const SimDev& Dw = sims[sw];
      atomicAdd(&acc.blocks[int64_t(sw) * K.nb + b], q0 * Dw.inv_area);
      atomicAdd(&acc.tsum[3 * sw + 0], q1 * Dw.inv_nf);
      atomicAdd(&acc.tsum[3 * sw + 1], q2 * Dw.inv_nf);
      atomicAdd(&acc.tsum[3 * sw + 2], q3 * Dw.inv_nf);
      if (K.press_on) atomicAdd(&acc.pblocks[int64_t(sw) * K.nb + b], q4 * Dw.inv_area);
    }
  } else if (valid) {
    const SimDev& D = sims[s];
    atomicAdd(&acc.blocks[int64_t(s) * K.nb + b], q0 * D.inv_area);
    atomicAdd(&acc.tsum[3 * s + 0], q1 * D.inv_nf);
    atomicAdd(&acc.tsum[3 * s + 1], q2 * D.inv_nf);
    atomicAdd(&acc.tsum[3 * s + 2], q3 * D.inv_nf);
    if (K.press_on) atomicAdd(&acc.pblocks[int64_t(s) * K.nb + b], q4 * D.inv_area);
  }
  if (!K.bins_on) return;
  // wall-normal profile: aggregate in LDS relative to the block's lowest bin
  int gb = -1;
  if (valid) {
    const SimDev& D = sims[s];
    int bb = int(floor(ypre ? *ypre : st.y[i] * D.inv_bin));
    bb = bb < 0 ? 0 : (bb >= D.nbins ? D.nbins - 1 : bb);
    gb = D.bin0 + bb;
    if (TB) {
      if (bb < BIN_LDS) {
        atomicAdd(&tbin[bb], tbin_word(v0));
      } else {
        atomicAdd(&acc.binvx[gb], v0);
        atomicAdd(&acc.bincnt[gb], 1.0);
      }
    }
  }
  if (TB) return;
  for (int k = threadIdx.x; k < BIN_LDS; k += blockDim.x) { lds_vx[k] = 0.0; lds_cnt[k] = 0.0; }
  if (threadIdx.x == 0) *lds_base = 0x7fffffff;
  __syncthreads();
  if (gb >= 0) atomicMin(lds_base, gb);
  __syncthreads();
  const int base = *lds_base;
  if (gb >= 0) {
    const int o = gb - base;
    if (o < BIN_LDS) {
      atomicAdd(&lds_vx[o], v0);
      atomicAdd(&lds_cnt[o], 1.0);
    } else {
      atomicAdd(&acc.binvx[gb], v0);
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

// ---------------------------------------------------------------------------
// Cell-path force (one thread per slot): shifted LJ (Eq. LJ) over the 27
// neighbouring cells, fluid-fluid and wall-fluid, FP32.  Cell-relative
// coordinates keep the separations accurate; the image shift of a
// neighbouring cell is its offset times the cell width.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_force_cell(int ntot, const SimDev* __restrict__ sims,
                                                    const uint16_t* __restrict__ atom_sim,
                                                    const float4* __restrict__ pos4,
                                                    const uint32_t* __restrict__ start,
                                                    const uint32_t* __restrict__ ncount,
                                                    const float4* __restrict__ wpos4,
                                                    const uint32_t* __restrict__ wstart,
                                                    const uint32_t* __restrict__ wcount, float4* __restrict__ f4,
                                                    StateRef st, Acc acc, int64_t* __restrict__ dstate, StepRef R,
                                                    StepConst K) {
  __shared__ double lds_vx[BIN_LDS];
  __shared__ double lds_cnt[BIN_LDS];
  __shared__ int lds_base;
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  const bool valid = i < ntot;
  const int s = valid ? int(atom_sim[i]) : 0;
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
            const uint32_t gc = uint32_t(D.c0) + D.rank[(jz * D.ny + jy) * D.nx + jx];
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
  finish_force<MODE>(i, valid, s, sims, fx, fy, fz, pe, st, acc, dstate, step_n(R) + 1, K, lds_vx, lds_cnt,
                     &lds_base);
}

// Shifted LJ (Eq. LJ) for one list entry from a fixed-point separation,
// accumulated into f (and pe, pair counts with ENERGY); entries past the
// cut-off add zero through a select.  WS: sigma_wf = eps_wf = 1.  UNI: one
// fixed-point unit u on every axis, so the separation stays in units -- r^2 compares with rc^2 / u^2,
// sigma^2 / r^2 takes 1 / u^2, and f carries a factor u removed once per
// atom by the caller (multiply by inv_u).
struct PairConst {
  float rc2, s2_ff, s2_wf, eps24_wf, eps4_wf, ush_ff, ush_wf;
};

template <int UNI>
__device__ __forceinline__ PairConst pair_const(const StepConst& K, const SimDev& D) {
  PairConst c;
  c.rc2 = UNI ? K.rc2 * D.inv_u2 : K.rc2;
  c.s2_ff = UNI ? D.inv_u2 : 1.0f;
  c.s2_wf = UNI ? K.sig2_wf * D.inv_u2 : K.sig2_wf;
  c.eps24_wf = 24.0f * K.eps_wf;
  c.eps4_wf = 4.0f * K.eps_wf;
  c.ush_ff = K.ush_ff;
  c.ush_wf = K.ush_wf;
  return c;
}

// PR: also the wall normal pressure term, f_r |dy| over wall pairs (every
// lower-wall atom lies below every fluid atom and every upper-wall atom above,
// so |dy| carries each wall's sign: the sum over wall pairs is
// F_lo,y - F_hi,y, the normal forces of the two walls on the fluid).
template <int ENERGY, int UNI, int WS, int PR = 0>
__device__ __forceinline__ void lj_term(int dx, int dy, int dz, bool wall_atom, const PairConst& c,
                                        const SimDev& D, float& fx, float& fy, float& fz, float& pe,
                                        uint32_t& nff, uint32_t& nwf, float& pw) {
  // WS: wall-fluid parameters equal the fluid's, so forces need no wall test
  const bool wall = (WS && !ENERGY) ? false : wall_atom;
  const float ax = UNI ? float(dx) : float(dx) * D.unit_x;
  const float ay = UNI ? float(dy) : float(dy) * D.unit_y;
  const float az = UNI ? float(dz) : float(dz) * D.unit_z;
  const float r2 = ax * ax + ay * ay + az * az;
  const bool in = r2 < c.rc2;
  const float ri2 = __builtin_amdgcn_rcpf(r2);  // 1 ulp
  const float s2 = (wall ? c.s2_wf : c.s2_ff) * ri2;
  const float s6 = s2 * s2 * s2;
  // 24 eps s6 (2 s6 - 1) / r^2 as s6 (48 eps s6 - 24 eps) / r^2: one fused step fewer
  const float eps24 = wall ? c.eps24_wf : 24.0f;
  const float eps48 = wall ? 2.0f * c.eps24_wf : 48.0f;
  const float fr = in ? s6 * (eps48 * s6 - eps24) * ri2 : 0.0f;
  fx += fr * ax; fy += fr * ay; fz += fr * az;
  if (PR) pw += (wall_atom ? fr : 0.0f) * fabsf(ay);
  if (ENERGY) {
    const float u = wall ? c.eps4_wf * s6 * (s6 - 1.0f) - c.ush_wf : 0.5f * (4.0f * s6 * (s6 - 1.0f) - c.ush_ff);
    pe += in ? u : 0.0f;
    nwf += (in && wall) ? 1u : 0u;
    nff += (in && !wall) ? 1u : 0u;
  }
}

// ---------------------------------------------------------------------------
// Pair-path force (one thread per slot): the same shifted LJ sum over the
// slot's Verlet list (entries >= ntot are wall atoms), FP32 from fixed-point
// separations.
// ---------------------------------------------------------------------------
template <int MODE, int ENERGY, int UNI, int WS, int PR>
__global__ __launch_bounds__(256) void k_force_list(int ntot, int ld, const SimDev* __restrict__ sims,
                                                    const uint16_t* __restrict__ atom_sim,
                                                    const int4* __restrict__ pfix, const uint32_t* __restrict__ list,
                                                    const uint32_t* __restrict__ nlist, float4* __restrict__ f4,
                                                    StateRef st, Acc acc, int64_t* __restrict__ dstate, StepRef R,
                                                    StepConst K) {
  __shared__ double lds_vx[BIN_LDS];
  __shared__ double lds_cnt[BIN_LDS];
  __shared__ int lds_base;
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  const bool valid = i < ntot;
  const int s = valid ? int(atom_sim[i]) : 0;
  float fx = 0.f, fy = 0.f, fz = 0.f, pe = 0.f, pw = 0.f;
  uint32_t nff = 0, nwf = 0;
  if (valid) {
    const SimDev& D = sims[s];
    const int4 me = pfix[i];
    const uint32_t n = nlist[i];
    const uint4* grp = reinterpret_cast<const uint4*>(list) + i;  // group g at grp[g * ld]
    const PairConst pc = pair_const<UNI>(K, D);
    auto pair = [&](uint32_t j, const int4& o) {
      lj_term<ENERGY, UNI, WS, PR>(int(uint32_t(me.x) - uint32_t(o.x)), int(uint32_t(me.y) - uint32_t(o.y)),
                                   int(uint32_t(me.z) - uint32_t(o.z)), j >= uint32_t(ntot), pc, D, fx, fy, fz,
                                   pe, nff, nwf, pw);
    };
    // One coalesced 16-byte load brings four entries.  The next group's load
    // is issued before this group's arithmetic so that its latency overlaps
    // the four position gathers and the pair terms.
    const uint32_t full = n >> 2, rest = n & 3u, ngrp = (n + 3u) >> 2;
    uint4 jj = ngrp ? grp[0] : make_uint4(0u, 0u, 0u, 0u);
    for (uint32_t g = 0; g < full; ++g) {
      const int4 o0 = pfix[jj.x], o1 = pfix[jj.y], o2 = pfix[jj.z], o3 = pfix[jj.w];
      const uint32_t gn = g + 1 < ngrp ? g + 1 : g;
      const uint4 jn = grp[size_t(gn) * ld];
      pair(jj.x, o0);
      pair(jj.y, o1);
      pair(jj.z, o2);
      pair(jj.w, o3);
      jj = jn;
    }
    if (rest) {  // jj holds the partial last group
      pair(jj.x, pfix[jj.x]);
      if (rest > 1) pair(jj.y, pfix[jj.y]);
      if (rest > 2) pair(jj.z, pfix[jj.z]);
    }
    if (UNI) { fx *= D.inv_u; fy *= D.inv_u; fz *= D.inv_u; pw *= D.inv_u; }
    f4[i] = make_float4(fx, fy, fz, pe);
  }
  if (ENERGY) {
    const unsigned long long a = wave_sum((unsigned long long)nff), w = wave_sum((unsigned long long)nwf);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
      atomicAdd(&acc.pairs[0], a);
      atomicAdd(&acc.pairs[1], w);
    }
  }
  finish_force<MODE>(i, valid, s, sims, fx, fy, fz, pe, st, acc, dstate, step_n(R) + 1, K, lds_vx, lds_cnt,
                     &lds_base, nullptr, nullptr, nullptr, nullptr, 0, PR ? pw : 0.0f);
}

// ---------------------------------------------------------------------------
// Tiled pair path.  Cells are numbered slab by slab ((z nx + x) ny + y), so a
// tile -- ncol whole columns of one z slab -- owns one contiguous slot range,
// and everything its atoms can reach lies in three slabs (z - 1, z, z + 1)
// over columns x0 - 1 .. x0 + ncol: per slab one contiguous range of fluid
// slots and one of wall atoms per wall (two of each where the columns wrap
// around x).  A workgroup copies those ranges into LDS (fluid ranges first,
// then walls) and its lists hold 16-bit LDS indices, so the force loop reads
// neighbour positions from LDS instead of gathering them from memory.  A
// tile whose ranges exceed the LDS capacity keeps 32-bit position indices
// and gathers from memory instead.
// ---------------------------------------------------------------------------
constexpr int TILE_TPB = 256;
constexpr int TILE_RUNS = 18;  // kind (fluid, lower wall, upper wall) x 3 slabs x 2 pieces


struct TileStage {
  uint32_t gb[TILE_RUNS];       // first entry of each range in the position array
  uint32_t off[TILE_RUNS + 1];  // LDS offset of each range (prefix sums)
  int pa[2], pb[2], npieces;    // column pieces of the x range
  int s, z, x0, ncol;
  uint32_t home0, home1;        // home slots
  uint32_t mode;                // 0: lists of LDS indices; 1: of position indices (LDS too small)
};
static_assert(sizeof(TileStage) == TILE_REC * sizeof(uint32_t), "tile record layout");

// Column pieces of x0 - 1 .. x0 + ncol with periodic wrap (one piece covers
// the whole row when the range would meet itself).
__device__ __forceinline__ void tile_pieces(int x0, int ncol, int nx, int* pa, int* pb, int* np) {
  if (ncol + 2 >= nx) {
    pa[0] = 0; pb[0] = nx - 1; *np = 1;
    return;
  }
  const int xa = x0 - 1, xb = x0 + ncol;
  if (xa < 0) {
    pa[0] = xa + nx; pb[0] = nx - 1; pa[1] = 0; pb[1] = xb; *np = 2;
  } else if (xb >= nx) {
    pa[0] = xa; pb[0] = nx - 1; pa[1] = 0; pb[1] = xb - nx; *np = 2;
  } else {
    pa[0] = xa; pb[0] = xb; *np = 1;
  }
}

// Fills the range table of tile t (all threads; ends with a barrier).
__device__ __forceinline__ void tile_ranges(const int4& tile, int ntot, const SimDev* __restrict__ sims,
                                            const uint32_t* __restrict__ start,
                                            const uint32_t* __restrict__ ncount,
                                            const uint32_t* __restrict__ wstart,
                                            const uint32_t* __restrict__ wcount, TileStage& T) {
  __shared__ uint32_t len[TILE_RUNS];
  const int tid = threadIdx.x;
  const SimDev& D = sims[tile.x];
  if (tid == 0) {
    T.s = tile.x; T.z = tile.y; T.x0 = tile.z; T.ncol = tile.w;
    tile_pieces(tile.z, tile.w, D.nx, T.pa, T.pb, &T.npieces);
    const uint32_t c_first = uint32_t(D.c0 + (tile.y * D.nx + tile.z) * D.ny);
    const uint32_t c_last = c_first + uint32_t(tile.w * D.ny) - 1u;
    T.home0 = start[c_first];
    T.home1 = start[c_last] + ncount[c_last];
  }
  __syncthreads();
  if (tid < TILE_RUNS) {
    const int kind = tid / 6, dz = (tid / 2) % 3 - 1, piece = tid & 1;
    uint32_t gb = 0, n = 0;
    if (piece < T.npieces) {
      int zz = T.z + dz;
      zz += zz < 0 ? D.nz : (zz >= D.nz ? -D.nz : 0);
      const int a = T.pa[piece], b = T.pb[piece];
      if (kind == 0) {
        const uint32_t c1 = uint32_t(D.c0 + (zz * D.nx + a) * D.ny);
        const uint32_t c2 = uint32_t(D.c0 + (zz * D.nx + b) * D.ny + D.ny - 1);
        gb = start[c1];
        n = start[c2] + ncount[c2] - gb;
      } else {
        const uint32_t w1 = uint32_t(D.wc0 + ((kind - 1) * D.nz + zz) * D.nx + a);
        const uint32_t w2 = uint32_t(D.wc0 + ((kind - 1) * D.nz + zz) * D.nx + b);
        gb = uint32_t(ntot) + wstart[w1];
        n = wstart[w2] + wcount[w2] - wstart[w1];
      }
    }
    T.gb[tid] = gb;
    len[tid] = n;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int r = 0; r < TILE_RUNS; ++r) {
      T.off[r] = acc;
      acc += len[r];
    }
    T.off[TILE_RUNS] = acc;
  }
  __syncthreads();
}

// Copies the tile's ranges into LDS in one flat pass over every staged
// entry, each thread with eight loads in flight (range by range, each short
// range would cost a whole memory latency of its own); put(e, p) stores
// entry e.  The range of entry e is the r with off[r] <= e < off[r + 1] (an
// empty range shares its start with the next; the last such r is taken).  A
// wavefront handles 64 consecutive entries at a time, so a ballot over the
// lanes that hold the range starts counts the starts at or before its first
// entry, and only the few starts inside those 64 are compared lane by lane.
// All threads of the block call it (the ballots need whole wavefronts).
template <class Put>
__device__ __forceinline__ void tile_stage_core(const TileStage& T, const int4* __restrict__ pfix, Put put) {
  constexpr int U = 8;
  const uint32_t total = T.off[TILE_RUNS];
  const uint32_t lane = threadIdx.x & (WAVE - 1);
  const uint32_t start_q = (lane >= 1 && lane < uint32_t(TILE_RUNS)) ? T.off[lane] : 0xffffffffu;
  // source of the last entry, read in place of entries past the end so that
  // every load is issued unconditionally and in bounds
  const int r_last = __popcll(__ballot(start_q < total));
  const uint32_t last_src = total ? T.gb[r_last] + (total - 1u - T.off[r_last]) : 0u;
  for (uint32_t w0 = threadIdx.x - lane; w0 < total; w0 += U * blockDim.x) {  // uniform per wavefront
    uint32_t src[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t ew = w0 + u * blockDim.x, e = ew + lane;
      int r = __popcll(__ballot(start_q <= ew));
      unsigned long long m = __ballot(start_q > ew && start_q < ew + WAVE);
      while (m) {
        const int q = __builtin_ctzll(m);
        m &= m - 1ull;
        r += e >= uint32_t(__builtin_amdgcn_readlane(int(start_q), q)) ? 1 : 0;
      }
      src[u] = T.gb[r] + (e - T.off[r]);
    }
    // the loads go out together
    int4 p[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t e = w0 + u * blockDim.x + lane;
      p[u] = pfix[e < total ? src[u] : last_src];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t e = w0 + u * blockDim.x + lane;
      if (e < total) put(e, p[u]);
    }
  }
  __syncthreads();
}

// Fixed-point copy (structure of arrays; the caller checks the capacity).
__device__ __forceinline__ void tile_stage(const TileStage& T, const int4* __restrict__ pfix, int* lx, int* ly,
                                           int* lz) {
  tile_stage_core(T, pfix, [&](uint32_t e, const int4& q) {
    lx[e] = q.x; ly[e] = q.y; lz[e] = q.z;
  });
}

// The same copy as FP32 offsets from a tile origin o (fixed-point units
// scaled by sc per axis), for the list build's screening: |offset| stays
// below half an extent, so the 32-bit difference is the unwrapped offset,
// and its FP32 rounding (2^-24 relative) is far below the screening margin.
__device__ __forceinline__ void tile_stage_rel(const TileStage& T, const int4* __restrict__ pfix, int* lx, int* ly,
                                               int* lz, const int4& o, const float3& sc) {
  tile_stage_core(T, pfix, [&](uint32_t e, const int4& q) {
    lx[e] = __float_as_int(float(int(uint32_t(q.x) - uint32_t(o.x))) * sc.x);
    ly[e] = __float_as_int(float(int(uint32_t(q.y) - uint32_t(o.y))) * sc.y);
    lz[e] = __float_as_int(float(int(uint32_t(q.z) - uint32_t(o.z))) * sc.z);
  });
}

// Range table of a tile as the last list build left it (the cell ranges only
// change when the cells are rebuilt, and every rebuild runs the list build).
__device__ __forceinline__ void tile_load(const uint32_t* __restrict__ rec, TileStage& T) {
  if (threadIdx.x < TILE_REC) reinterpret_cast<uint32_t*>(&T)[threadIdx.x] = rec[threadIdx.x];
  __syncthreads();
}

// Verlet lists of a tile's atoms (rebuild steps only).  Also completes the
// reorder (state copy back) for the tile's slots.  global_out writes 32-bit
// position indices (the layout of k_build_list) for every tile.
template <int UNI>
__global__ __launch_bounds__(TILE_TPB) void k_build_tiles(
    int ntot, int ld, int cap, const int4* __restrict__ tiles, const SimDev* __restrict__ sims,
    const uint32_t* __restrict__ slot_cell, const int4* __restrict__ pfix, const uint32_t* __restrict__ start,
    const uint32_t* __restrict__ ncount, const uint32_t* __restrict__ wstart, const uint32_t* __restrict__ wcount,
    uint32_t* __restrict__ list, uint32_t* __restrict__ nlist, uint32_t* __restrict__ tilerec, StateRef from,
    StateRef to, const int* __restrict__ tag_from,
    int* __restrict__ tag_to, int* __restrict__ overflow, const int* __restrict__ flag, StepRef R, float rl2,
    int global_out) {
  if (!rebuild_needed(flag, R)) return;
  __shared__ int lx[TILE_STAGE + 4], ly[TILE_STAGE + 4], lz[TILE_STAGE + 4];
  __shared__ TileStage T;
  // LDS index of each neighbourhood cell's first atom (<< 8) and its count,
  // by (slab, column offset, y + 1): the candidate loop then reads no cell
  // tables from memory
  __shared__ uint32_t ctab[TILE_CTAB];
  __shared__ int tab_ok;
  const int t = xcd_block();
  tile_ranges(tiles[t], ntot, sims, start, ncount, wstart, wcount, T);
  const uint32_t total = T.off[TILE_RUNS];
  // one LDS slot beyond the staged atoms holds the padding entry's position
  const bool local = !global_out && total < uint32_t(TILE_STAGE);
  if (threadIdx.x < TILE_REC)  // range table and mode, for the force kernels until the next rebuild
    tilerec[size_t(t) * TILE_REC + threadIdx.x] =
        threadIdx.x == TILE_REC - 1 ? (local ? 0u : 1u) : reinterpret_cast<const uint32_t*>(&T)[threadIdx.x];
  if (t == 0 && threadIdx.x == 0) atomicAdd(&overflow[1], 1);  // builds so far
  const SimDev& D = sims[__builtin_amdgcn_readfirstlane(T.s)];  // one system per tile: scalar loads
  const bool whole = T.npieces == 1 && T.pa[0] == 0 && T.pb[0] == D.nx - 1;
  const int ncolx = whole ? D.nx : T.ncol + 2, nyt = D.ny + 2;
  bool use_tab = local && 3 * ncolx * nyt <= TILE_CTAB;
  // Screening in FP32 offsets from the centre of the tile's neighbourhood
  // (no integer conversion per candidate) where that neighbourhood spans
  // less than an extent in x and z, so that no offset wraps.  Margin: offsets
  // stay below 2^31 units, so each is within 2^7 units of exact and r^2 within
  // ~1e-6 relative of exact; screening at (1 + 1e-5) r_l^2 keeps every pair
  // inside r_l (the surplus pairs beyond r_l add nothing to the forces).
  const bool flt = use_tab && !whole && D.nz >= 4;
  int4 org = make_int4(0, 0, 0, 0);
  float3 sc = make_float3(1.0f, 1.0f, 1.0f);
  if (flt) {
    const double xc = (double(T.x0 - 1) + 0.5 * double(T.ncol + 2)) * D.wx, zc = (double(T.z) + 0.5) * D.wz;
    org = make_int4(int(fix_axis(xc, D.fix_x)), int(0x80000000u), int(fix_axis(zc, D.fix_z)), 0);
    if (!UNI) sc = make_float3(D.unit_x, D.unit_y, D.unit_z);
    tile_stage_rel(T, pfix, lx, ly, lz, org, sc);
  } else if (local) {
    tile_stage(T, pfix, lx, ly, lz);
  }
  if (use_tab) {
    if (threadIdx.x == 0) tab_ok = 1;
    __syncthreads();
    for (int e = threadIdx.x; e < 3 * ncolx * nyt; e += blockDim.x) {
      const int si = e / (ncolx * nyt), xi = (e / nyt) % ncolx, jy = e % nyt - 1;
      int jz = T.z + si - 1;
      jz += jz < 0 ? D.nz : (jz >= D.nz ? -D.nz : 0);
      int jx = whole ? xi : T.x0 - 1 + xi;
      jx += jx < 0 ? D.nx : (jx >= D.nx ? -D.nx : 0);
      const int piece = (T.npieces == 1 || (jx >= T.pa[0] && jx <= T.pb[0])) ? 0 : 1;
      const int kind = jy < 0 ? 1 : (jy >= D.ny ? 2 : 0);
      uint32_t cb, cn;
      if (kind == 0) {
        const uint32_t gc = uint32_t(D.c0 + (jz * D.nx + jx) * D.ny + jy);
        cb = start[gc];
        cn = ncount[gc];
      } else {
        const uint32_t wc = uint32_t(D.wc0 + ((kind - 1) * D.nz + jz) * D.nx + jx);
        cb = uint32_t(ntot) + wstart[wc];
        cn = wcount[wc];
      }
      const int run = kind * 6 + si * 2 + piece;
      if (cn > 255u) tab_ok = 0;
      ctab[e] = ((T.off[run] + (cb - T.gb[run])) << 8) | (cn > 255u ? 255u : cn);
    }
    __syncthreads();
    use_tab = tab_ok != 0;
    if (flt && !use_tab) tile_stage(T, pfix, lx, ly, lz);  // the cell-by-cell loop reads fixed point
  }
  const bool rel = flt && use_tab;
  const bool copy = from.x != to.x;  // a rebuild outside the step sequence copies nothing
  for (uint32_t i = T.home0 + threadIdx.x; i < T.home1; i += blockDim.x) {
    if (copy) {
      to.x[i] = from.x[i]; to.y[i] = from.y[i]; to.z[i] = from.z[i];
      to.vx[i] = from.vx[i]; to.vy[i] = from.vy[i]; to.vz[i] = from.vz[i];
      tag_to[i] = tag_from[i];
    }
    const int4 me = pfix[i];
    // squared separation (in fixed-point units squared with UNI)
    const float rl2u = UNI ? rl2 * D.inv_u2 : rl2;
    const float rl2r = rl2u * 1.00001f;
    const float mx = float(int(uint32_t(me.x) - uint32_t(org.x))) * sc.x;
    const float my = float(int(uint32_t(me.y) - uint32_t(org.y))) * sc.y;
    const float mz = float(int(uint32_t(me.z) - uint32_t(org.z))) * sc.z;
    auto sep2r = [&](int ox, int oy, int oz) {
      const float ax = mx - __int_as_float(ox), ay = my - __int_as_float(oy), az = mz - __int_as_float(oz);
      return ax * ax + ay * ay + az * az;
    };
    auto sep2 = [&](int ox, int oy, int oz) {
      const float ax = float(int(uint32_t(me.x) - uint32_t(ox))) * (UNI ? 1.0f : D.unit_x);
      const float ay = float(int(uint32_t(me.y) - uint32_t(oy))) * (UNI ? 1.0f : D.unit_y);
      const float az = float(int(uint32_t(me.z) - uint32_t(oz))) * (UNI ? 1.0f : D.unit_z);
      return ax * ax + ay * ay + az * az;
    };
    const int r0 = int(slot_cell[i]) - D.c0;  // (z nx + x) ny + y
    const int cy = r0 % D.ny, cx = (r0 / D.ny) % D.nx, cz = r0 / (D.ny * D.nx);
    uint32_t cnt = 0;
    // entry c of slot i: 16-bit at ((c / 8) ld + i) 8 + c % 8 (LDS index),
    // 32-bit at ((c / 4) ld + i) 4 + c % 4 (position index).  16-bit entries
    // gather in a register group (g0..g3, shifted down one entry per hit, the
    // newest on top) that goes out as one 16-byte store when it holds eight:
    // the lanes of a wave then write whole, adjacent groups instead of one
    // scattered 16-bit store per hit.  Byte offsets are 32-bit (the list is
    // below 4 GiB); the group index is clamped to cap / 8, a spill group in
    // the half of the capacity that 16-bit entries leave unused (an
    // overflowing list is reported below and never used).
    char* const list_b = reinterpret_cast<char*>(list);
    uint32_t g0 = 0, g1 = 0, g2 = 0, g3 = 0;
    auto push16 = [&](uint32_t k) {
      g0 = __builtin_amdgcn_alignbit(g1, g0, 16);
      g1 = __builtin_amdgcn_alignbit(g2, g1, 16);
      g2 = __builtin_amdgcn_alignbit(g3, g2, 16);
      g3 = __builtin_amdgcn_alignbit(k, g3, 16);
    };
    auto store_group = [&](uint32_t g) {
      g = min(g, uint32_t(cap) >> 3);
      *reinterpret_cast<uint4*>(list_b + ((__umul24(g, uint32_t(ld)) + i) << 4)) = make_uint4(g0, g1, g2, g3);
    };
    auto put16 = [&](bool hit, uint32_t k) {
      if (hit) {
        push16(k);
        ++cnt;
        if ((cnt & 7u) == 0u) store_group((cnt - 1u) >> 3);
      }
    };
    auto put32 = [&](bool hit, uint32_t q) {
      if (hit && cnt < uint32_t(cap)) list[(size_t(cnt >> 2) * ld + i) * 4 + (cnt & 3u)] = q;
      cnt += hit ? 1u : 0u;
    };
    // candidates k in [a, b) of the LDS arrays, four LDS reads in flight;
    // only the atom's own cell (SELF) holds the atom itself
    auto screen = [&](auto self_cell, uint32_t a, uint32_t b, uint32_t myk) {
      constexpr bool SELF = decltype(self_cell)::value;
      uint32_t k = a;
      if (rel) {
        // whole blocks of four, the last one masked (its reads past b stay
        // inside the arrays, which hold four spare slots): no remainder loop
        for (; k < b; k += 4) {
          float r2[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) r2[u] = sep2r(lx[k + u], ly[k + u], lz[k + u]);
#pragma unroll
          for (int u = 0; u < 4; ++u) put16(r2[u] < rl2r && k + u < b && (!SELF || k + u != myk), k + u);
        }
      } else {
        for (; k + 4 <= b; k += 4) {
          float r2[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) r2[u] = sep2(lx[k + u], ly[k + u], lz[k + u]);
#pragma unroll
          for (int u = 0; u < 4; ++u) put16(r2[u] < rl2u && (!SELF || k + u != myk), k + u);
        }
        for (; k < b; ++k) put16(sep2(lx[k], ly[k], lz[k]) < rl2u && (!SELF || k != myk), k);
      }
    };
    if (use_tab) {
      // own LDS index, for the self test
      const int xs = whole ? cx : cx - T.x0 + 1;
      const uint32_t myk = (ctab[(ncolx + xs) * nyt + cy + 1] >> 8) + (i - start[slot_cell[i]]);
      // cell by cell: the lanes of a wave sit in neighbouring cells, so their
      // k-th neighbour cells (a wall column for the first and last fluid
      // cells) are screened side by side
      for (int dz = 0; dz < 3; ++dz)
        for (int dx = -1; dx <= 1; ++dx) {
          int jx = cx + dx;
          if (whole) jx += jx < 0 ? D.nx : (jx >= D.nx ? -D.nx : 0);
          else jx -= T.x0 - 1;
          const uint32_t* row = ctab + (dz * ncolx + jx) * nyt + cy;  // y offsets -1, 0, 1 -> row[0..2]
          for (int dy = 0; dy < 3; ++dy) {
            const uint32_t w = row[dy];
            if (dz == 1 && dx == 0 && dy == 1)
              screen(std::true_type{}, w >> 8, (w >> 8) + (w & 255u), myk);
            else
              screen(std::false_type{}, w >> 8, (w >> 8) + (w & 255u), myk);
          }
        }
    } else
    for (int dz = -1; dz <= 1; ++dz) {
      int jz = cz + dz;
      jz += jz < 0 ? D.nz : (jz >= D.nz ? -D.nz : 0);
      for (int dx = -1; dx <= 1; ++dx) {
        int jx = cx + dx;
        jx += jx < 0 ? D.nx : (jx >= D.nx ? -D.nx : 0);
        const int piece = (T.npieces == 1 || (jx >= T.pa[0] && jx <= T.pb[0])) ? 0 : 1;
        for (int dy = -1; dy <= 1; ++dy) {
          const int jy = cy + dy;
          const int kind = jy < 0 ? 1 : (jy >= D.ny ? 2 : 0);
          uint32_t cb, cn;
          if (kind == 0) {
            const uint32_t gc = uint32_t(D.c0 + (jz * D.nx + jx) * D.ny + jy);
            cb = start[gc];
            cn = ncount[gc];
          } else {
            const uint32_t wc = uint32_t(D.wc0 + ((kind - 1) * D.nz + jz) * D.nx + jx);
            cb = uint32_t(ntot) + wstart[wc];
            cn = wcount[wc];
          }
          const int run = kind * 6 + (dz + 1) * 2 + piece;
          const uint32_t base = T.off[run] + (cb - T.gb[run]);
          const uint32_t self = i - cb;  // candidate index of the atom itself (if in this cell)
          if (local) {
            // four candidates per pass: their LDS reads are in flight together
            uint32_t m = 0;
            for (; m + 4 <= cn; m += 4) {
              float r2[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const uint32_t k = base + m + u;
                r2[u] = sep2(lx[k], ly[k], lz[k]);
              }
#pragma unroll
              for (int u = 0; u < 4; ++u) put16(r2[u] < rl2u && m + u != self, base + m + u);
            }
            for (; m < cn; ++m) {
              const uint32_t k = base + m;
              put16(sep2(lx[k], ly[k], lz[k]) < rl2u && m != self, k);
            }
          } else {
            for (uint32_t m = 0; m < cn; ++m) {
              const int4 o = pfix[cb + m];
              put32(sep2(o.x, o.y, o.z) < rl2u && m != self, cb + m);
            }
          }
        }
      }
    }
    // LDS lists are padded to whole groups of eight with the slot after the
    // staged atoms, which the force kernels place half a box away in z (more
    // than r_c from every atom of the slab): the force loop then needs no
    // partial last group
    if (local && D.nz >= 4) {
      while (cnt & 7u) put16(true, total);
    } else if (local && (cnt & 7u)) {  // the partial last group, moved down to entry 0
      for (uint32_t e = cnt & 7u; e < 8u; ++e) push16(0u);
      store_group(cnt >> 3);
    }
    if (cnt > uint32_t(cap)) {
      atomicMax(&overflow[0], int(cnt));
      cnt = cap;
    }
    nlist[i] = cnt;
  }
}

// Forces of a tile's atoms from their lists, neighbour positions read from
// LDS (or gathered, for a tile built with 32-bit indices), then the second
// half-kick and the sample of the step.
template <int MODE, int ENERGY, int UNI, int WS, int PR>
__global__ __launch_bounds__(TILE_TPB) void k_force_tiles(
    int ntot, int ld, const uint32_t* __restrict__ tilerec, const SimDev* __restrict__ sims,
    const int4* __restrict__ pfix, const uint32_t* __restrict__ list,
    const uint32_t* __restrict__ nlist, float4* __restrict__ f4, StateRef st, Acc acc,
    int64_t* __restrict__ dstate, StepRef R, StepConst K) {
  __shared__ int lx[TILE_STAGE], ly[TILE_STAGE], lz[TILE_STAGE];
  __shared__ TileStage T;
  __shared__ unsigned long long tbin[BIN_LDS];
  const int t = xcd_block();
  const int64_t nstep = step_n(R) + 1;  // the step this launch completes
  const bool sampled = MODE == 1 && sampled_step(nstep, K);
  const bool bins = sampled && K.bins_on;
  if (bins)
    for (int k = threadIdx.x; k < BIN_LDS; k += blockDim.x) tbin[k] = 0ull;
  tile_load(tilerec + size_t(t) * TILE_REC, T);  // ends with a barrier
  const bool local = T.mode == 0;
  const int s = __builtin_amdgcn_readfirstlane(T.s);  // one system per tile
  const SimDev& D = sims[s];
  const double bin_c1 = D.inv_bin / D.fix_y, bin_c0 = D.y_lo * D.inv_bin;  // fixed-point y -> bins
  const uint32_t n_home = T.home1 - T.home0;
  // a pass's own positions, velocities, list lengths and first list groups
  // are requested one step ahead: the first pass's during the staging, the
  // next pass's during this one's arithmetic
  int4 me_nx = make_int4(0, 0, 0, 0);
  uint32_t n_nx = 0;
  uint4 g_nx = make_uint4(0u, 0u, 0u, 0u);
  double3 v_nx = make_double3(0.0, 0.0, 0.0);
  auto fetch = [&](uint32_t base) {
    const uint32_t i = T.home0 + base + threadIdx.x;
    if (base + threadIdx.x < n_home) {
      me_nx = pfix[i];
      n_nx = nlist[i];
      g_nx = reinterpret_cast<const uint4*>(list)[i];
      if (MODE == 1) v_nx = make_double3(st.vx[i], st.vy[i], st.vz[i]);
    }
  };
  fetch(0);
  if (local) {
    if (threadIdx.x == 0) {  // the padding slot: half a box from the slab's centre in z
      const uint32_t pad = T.off[TILE_RUNS];
      lx[pad] = 0;
      ly[pad] = 0;
      lz[pad] = int(fix_axis((double(T.z) + 0.5) * D.wz, D.fix_z) + 0x80000000u);
    }
    tile_stage(T, pfix, lx, ly, lz);
  }
  const uint32_t first_wall = local ? T.off[6] : uint32_t(ntot);  // walls come after the fluid ranges
  TileSums sums;
#pragma unroll
  for (int q = 0; q < 8; ++q) sums.v[q] = 0.0;
  for (uint32_t base = 0; base < n_home; base += blockDim.x) {
    const uint32_t i = T.home0 + base + threadIdx.x;
    const bool valid = base + threadIdx.x < n_home;
    const int4 me = me_nx;
    const uint32_t n = n_nx;
    const uint4 g0 = g_nx;
    const double3 v = v_nx;
    if (base + blockDim.x < n_home) fetch(base + blockDim.x);
    float fx = 0.f, fy = 0.f, fz = 0.f, pe = 0.f, pw = 0.f;
    uint32_t nff = 0, nwf = 0;
    if (valid) {
      const uint4* grp = reinterpret_cast<const uint4*>(list) + i;
      const PairConst pc = pair_const<UNI>(K, D);
      auto pair = [&](uint32_t j, int ox, int oy, int oz) {
        lj_term<ENERGY, UNI, WS, PR>(int(uint32_t(me.x) - uint32_t(ox)), int(uint32_t(me.y) - uint32_t(oy)),
                                     int(uint32_t(me.z) - uint32_t(oz)), j >= first_wall, pc, D, fx, fy, fz, pe,
                                     nff, nwf, pw);
      };
      if (local) {
        // eight 16-bit LDS indices per 16-byte group; the next group is
        // requested before this one's arithmetic
        const uint32_t full = n >> 3, rest = n & 7u, ngrp = (n + 7u) >> 3;
        uint4 jj = g0;
        auto two = [&](uint32_t w) {
          const uint32_t k0 = w & 0xffffu, k1 = w >> 16;
          pair(k0, lx[k0], ly[k0], lz[k0]);
          pair(k1, lx[k1], ly[k1], lz[k1]);
        };
        // group g of slot i at byte (g ld + i) 16: a 32-bit offset from the
        // list base (the list is below 4 GiB), no 64-bit address arithmetic
        const char* const list_b = reinterpret_cast<const char*>(list);
        for (uint32_t g = 0; g < full; ++g) {
          const uint32_t gn = g + 1 < ngrp ? g + 1 : g;
          const uint4 jn = *reinterpret_cast<const uint4*>(list_b + ((__umul24(gn, uint32_t(ld)) + i) << 4));
          two(jj.x); two(jj.y); two(jj.z); two(jj.w);
          jj = jn;
        }
        if (rest) {  // jj holds the partial last group
          const uint32_t w[4] = {jj.x, jj.y, jj.z, jj.w};
#pragma unroll
          for (int e = 0; e < 7; ++e)
            if (uint32_t(e) < rest) {
              const uint32_t k = (w[e >> 1] >> ((e & 1) * 16)) & 0xffffu;
              pair(k, lx[k], ly[k], lz[k]);
            }
        }
      } else {
        const uint32_t full = n >> 2, rest = n & 3u;
        for (uint32_t g = 0; g < full; ++g) {
          const uint4 jj = grp[size_t(g) * ld];
          const int4 o0 = pfix[jj.x], o1 = pfix[jj.y], o2 = pfix[jj.z], o3 = pfix[jj.w];
          pair(jj.x, o0.x, o0.y, o0.z);
          pair(jj.y, o1.x, o1.y, o1.z);
          pair(jj.z, o2.x, o2.y, o2.z);
          pair(jj.w, o3.x, o3.y, o3.z);
        }
        if (rest) {
          const uint4 jj = grp[size_t(full) * ld];
          const int4 o0 = pfix[jj.x];
          pair(jj.x, o0.x, o0.y, o0.z);
          if (rest > 1) { const int4 o1 = pfix[jj.y]; pair(jj.y, o1.x, o1.y, o1.z); }
          if (rest > 2) { const int4 o2 = pfix[jj.z]; pair(jj.z, o2.x, o2.y, o2.z); }
        }
      }
      if (UNI) { fx *= D.inv_u; fy *= D.inv_u; fz *= D.inv_u; pw *= D.inv_u; }
      f4[i] = make_float4(fx, fy, fz, pe);
    }
    if (ENERGY) {
      const unsigned long long a = wave_sum((unsigned long long)nff), w = wave_sum((unsigned long long)nwf);
      if ((threadIdx.x & (WAVE - 1)) == 0) {
        atomicAdd(&acc.pairs[0], a);
        atomicAdd(&acc.pairs[1], w);
      }
    }
    // wall-normal position in bin widths, from the fixed-point copy (within
    // one fixed-point unit of the FP64 one; no memory read)
    const double yb = double(uint32_t(me.y)) * bin_c1 + bin_c0;
    finish_force<MODE, 1>(int(i), valid, s, sims, fx, fy, fz, pe, st, acc, dstate, nstep, K, nullptr, nullptr,
                          nullptr, tbin, &v, &sums, &yb, sampled ? 1 : 0, PR ? pw : 0.0f);
  }
  // one atomic per sum and tile (per wave and pass they queue on a few
  // addresses per system)
  if (MODE == 1 || K.energy_on) {
    __shared__ double red[TILE_TPB / WAVE][8];
    const int64_t ns = nstep - K.n_equil - 1;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    // sums: 0 vc2, 1 ke, 2 pe, 3 q', 4-6 T components, 7 wall pressure
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bool need = q == 0 ? MODE == 1 : (q < 3 ? K.energy_on != 0 : (q < 7 ? sampled : PR && sampled));
      if (need) {
        const double w = wave_sum(sums.v[q]);
        if (lane == 0) red[wave][q] = w;
      }
    }
    __syncthreads();
    if (threadIdx.x < 8) {
      const int q = threadIdx.x;
      const bool need = q == 0 ? MODE == 1 : (q < 3 ? K.energy_on != 0 : (q < 7 ? sampled : PR && sampled));
      if (need) {
        double tot = 0.0;
        for (int w = 0; w < int(blockDim.x / WAVE); ++w) tot += red[w][q];
        const int p = int(nstep & 1);
        double* dst;
        if (q == 0) dst = (p ? acc.vc2[1] : acc.vc2[0]) + s;
        else if (q == 1) dst = (p ? acc.ke[1] : acc.ke[0]) + s;
        else if (q == 2) dst = (p ? acc.pe[1] : acc.pe[0]) + s;
        else if (q == 3) { dst = acc.blocks + int64_t(s) * K.nb + (ns - K.r) / K.B; tot *= D.inv_area; }
        else if (q == 7) { dst = acc.pblocks + int64_t(s) * K.nb + (ns - K.r) / K.B; tot *= D.inv_area; }
        else { dst = acc.tsum + 3 * s + (q - 4); tot *= D.inv_nf; }
        atomicAdd(dst, tot);
      }
    }
  }
  if (bins) {  // one flush of the tile's profile bins
    __syncthreads();
    const int nb = min(D.nbins, BIN_LDS);
    for (int k = threadIdx.x; k < nb; k += blockDim.x)
      if (tbin[k] != 0ull) {  // the tile's own FP64 accumulators: a plain add, no atomics
        double* const tb = acc.tbins + (size_t(t) * BIN_LDS + k) * 2;
        const double n = double(tbin[k] >> TBIN_CNT_SHIFT);
        tb[0] += double(tbin[k] & ((1ull << TBIN_CNT_SHIFT) - 1ull)) * TBIN_UNIT - TBIN_OFFSET * n;
        tb[1] += n;
      }
  }
}

// One timestamp of the device's constant-rate wall clock (timed graph
// replays bracket each kernel of a step with these).
// Device wall clock for per-kernel timing inside graphs; bit 63 carries
// whether the step being stamped rebuilds its pair lists (flag non-null).
__global__ void k_stamp(unsigned long long* slot, const int* flag, StepRef R) {
  if (threadIdx.x == 0)
    *slot = (unsigned long long)wall_clock64() | ((flag && rebuild_needed(flag, R)) ? (1ull << 63) : 0ull);
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }
__global__ void k_add_i64(int64_t* p, int64_t v) { *p += v; }
__global__ void k_set_i32(int* p, int v) { *p = v; }

#define HMD_INST_INTEGRATE(M, P)                                                                                  \
  template __global__ void k_integrate<M, P>(int, const SimDev*, const uint16_t*, StateRef, const float4*,         \
                                             uint32_t*, uint32_t*, uint32_t*, int4*, const int4*, int*, Acc,       \
                                             const int64_t*, StepRef, StepConst);
HMD_INST_INTEGRATE(0, 0)
HMD_INST_INTEGRATE(1, 0)
HMD_INST_INTEGRATE(0, 1)
HMD_INST_INTEGRATE(1, 1)
template __global__ void k_reorder<0>(int, const SimDev*, const uint16_t*, const uint32_t*, const uint32_t*,
                                      const uint32_t*, const uint32_t*, StateRef, StateRef, const int*, int*,
                                      float4*, int4*, int4*, uint32_t*, const int*, StepRef);
template __global__ void k_reorder<1>(int, const SimDev*, const uint16_t*, const uint32_t*, const uint32_t*,
                                      const uint32_t*, const uint32_t*, StateRef, StateRef, const int*, int*,
                                      float4*, int4*, int4*, uint32_t*, const int*, StepRef);
template __global__ void k_force_cell<0>(int, const SimDev*, const uint16_t*, const float4*, const uint32_t*,
                                         const uint32_t*, const float4*, const uint32_t*, const uint32_t*, float4*,
                                         StateRef, Acc, int64_t*, StepRef, StepConst);
template __global__ void k_force_cell<1>(int, const SimDev*, const uint16_t*, const float4*, const uint32_t*,
                                         const uint32_t*, const float4*, const uint32_t*, const uint32_t*, float4*,
                                         StateRef, Acc, int64_t*, StepRef, StepConst);
template __global__ void k_build_tiles<0>(int, int, int, const int4*, const SimDev*, const uint32_t*,
                                          const int4*, const uint32_t*, const uint32_t*, const uint32_t*,
                                          const uint32_t*, uint32_t*, uint32_t*, uint32_t*, StateRef, StateRef,
                                          const int*, int*, int*, const int*, StepRef, float, int);
template __global__ void k_build_tiles<1>(int, int, int, const int4*, const SimDev*, const uint32_t*,
                                          const int4*, const uint32_t*, const uint32_t*, const uint32_t*,
                                          const uint32_t*, uint32_t*, uint32_t*, uint32_t*, StateRef, StateRef,
                                          const int*, int*, int*, const int*, StepRef, float, int);

#define HMD_FORCE_TILES(M, E, U, W, PR)                                                                \
  template __global__ void k_force_tiles<M, E, U, W, PR>(int, int, const uint32_t*, const SimDev*,            \
                                                         const int4*, const uint32_t*,                         \
                                                         const uint32_t*, float4*, StateRef, Acc, int64_t*,    \
                                                         StepRef, StepConst);
#define HMD_FORCE_LIST(M, E, U, W, PR)                                                                 \
  template __global__ void k_force_list<M, E, U, W, PR>(int, int, const SimDev*, const uint16_t*, const int4*, \
                                                        const uint32_t*, const uint32_t*, float4*, StateRef, Acc, \
                                                        int64_t*, StepRef, StepConst);
#define HMD_FORCE_BOTH(M, E, U, W) HMD_FORCE_TILES(M, E, U, W, 0) HMD_FORCE_LIST(M, E, U, W, 0)
HMD_FORCE_BOTH(0, 0, 0, 0) HMD_FORCE_BOTH(0, 0, 0, 1) HMD_FORCE_BOTH(0, 0, 1, 0) HMD_FORCE_BOTH(0, 0, 1, 1)
HMD_FORCE_BOTH(0, 1, 0, 0) HMD_FORCE_BOTH(0, 1, 0, 1) HMD_FORCE_BOTH(0, 1, 1, 0) HMD_FORCE_BOTH(0, 1, 1, 1)
HMD_FORCE_BOTH(1, 0, 0, 0) HMD_FORCE_BOTH(1, 0, 0, 1) HMD_FORCE_BOTH(1, 0, 1, 0) HMD_FORCE_BOTH(1, 0, 1, 1)
HMD_FORCE_BOTH(1, 1, 0, 0) HMD_FORCE_BOTH(1, 1, 0, 1) HMD_FORCE_BOTH(1, 1, 1, 0) HMD_FORCE_BOTH(1, 1, 1, 1)
// sampling steps with the wall pressure recorded
#define HMD_FORCE_PR(E, U, W) HMD_FORCE_TILES(1, E, U, W, 1) HMD_FORCE_LIST(1, E, U, W, 1)
HMD_FORCE_PR(0, 0, 0) HMD_FORCE_PR(0, 0, 1) HMD_FORCE_PR(0, 1, 0) HMD_FORCE_PR(0, 1, 1)
HMD_FORCE_PR(1, 0, 0) HMD_FORCE_PR(1, 0, 1) HMD_FORCE_PR(1, 1, 0) HMD_FORCE_PR(1, 1, 1)
#undef HMD_FORCE_PR
#undef HMD_FORCE_BOTH
#undef HMD_FORCE_TILES
#undef HMD_FORCE_LIST

}  // namespace hmd
