// md_engine.hip -- host runtime of the batched NEMD micro-solve: builds the
// flattened device layout of many channel systems, runs the step loop as
// direct launches or replays of a captured HIP graph, and reduces results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>

#include "engine.h"
#include "md_kernels.h"
#include "series.h"

namespace hmd {

namespace {

constexpr double kTwo32 = 4294967296.0;

inline int blocks_for(int64_t n, int tpb) { return int((n + tpb - 1) / tpb); }

StateRef state_ref(hmd_batch* b, int which) {
  double** s = b->d_state[which];
  return StateRef{s[0], s[1], s[2], s[3], s[4], s[5]};
}

StepConst step_const(const hmd_batch* b, bool thermostat, bool energy) {
  const hmd_md_params& P = b->P;
  StepConst K{};
  K.dt = P.dt;
  K.hdt = 0.5 * P.dt;
  K.dt_tau = P.dt / P.tau_T;
  K.T0 = P.T0;
  K.n_equil = P.n_equil;
  K.rc2 = float(P.rc * P.rc);
  K.eps_wf = float(P.eps_wf);
  K.sig2_wf = float(P.sigma_wf * P.sigma_wf);
  const double ir6 = 1.0 / std::pow(P.rc, 6.0);
  K.ush_ff = float(4.0 * (ir6 * ir6 - ir6));
  const double sw6 = std::pow(P.sigma_wf / P.rc, 6.0);
  K.ush_wf = float(4.0 * P.eps_wf * (sw6 * sw6 - sw6));
  K.half_skin2 = float(0.25 * b->skin * b->skin);
  K.axis = P.thermo_axis;
  K.nb = int(b->nser);
  K.B = b->ser_B;
  K.r = b->ser_r;
  K.thermo_on = thermostat ? 1 : 0;
  K.bins_on = 1;
  K.energy_on = energy ? 1 : 0;
  K.press_on = P.pressure ? 1 : 0;
  return K;
}

template <typename T>
int dalloc(hmd_ctx* ctx, T** p, int64_t n) {
  HMD_HIP(ctx, hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * size_t(std::max<int64_t>(n, 1))));
  return HMD_OK;
}

// 3-D Morton code: bits of x, y, z interleaved (x lowest).
uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t m = 0;
  for (int b = 0; b < 21; ++b) {
    m |= uint64_t((x >> b) & 1u) << (3 * b);
    m |= uint64_t((y >> b) & 1u) << (3 * b + 1);
    m |= uint64_t((z >> b) & 1u) << (3 * b + 2);
  }
  return m;
}

uint32_t fix_axis_host(double v, double scale) {
  double t = v * scale;
  t = t < 0.0 ? 0.0 : (t > 4294967295.0 ? 4294967295.0 : t);
  return uint32_t(t);
}

// Launches of one kind, optionally timed.  Direct launches: HIP events
// around each kernel (marks).  Captured graphs, where events cannot be timed:
// stamp kernels writing the device wall clock into b->d_stamps, one before a
// stamped step's first kernel and one after each of its kernels; spans
// records (kernel, stamp before, stamp after).
struct Launcher {
  hmd_batch* b;
  hipStream_t s;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>>* marks;  // null: untimed
  int next_ev = 0;
  std::vector<std::array<int, 3>>* spans = nullptr;  // non-null: stamp mode
  int next_stamp = 0, last_stamp = -1;
  const int* flag = nullptr;  // stamp mode: rebuild flags, recorded in each stamp's bit 63
  StepRef R{nullptr, 0};      // stamp mode: the step being stamped

  void stamp() {
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, b->d_stamps + next_stamp, flag, R);
    last_stamp = next_stamp++;
  }
  void begin(int k) {
    if (spans) {
      if (last_stamp < 0) stamp();
      spans->push_back({k, last_stamp, next_stamp});
      return;
    }
    if (!marks) return;
    hipEvent_t e0 = b->ev[next_ev++], e1 = b->ev[next_ev++];
    (void)hipEventRecord(e0, s);
    marks->push_back({k, {e0, e1}});
  }
  void end() {
    if (spans) {
      stamp();
      return;
    }
    if (!marks) return;
    (void)hipEventRecord(marks->back().second.second, s);
  }
};

// Pair-list build (after a reorder into `from`: the build copies the state
// back into `to`; from == to copies nothing).
void launch_build(hmd_batch* b, hipStream_t s, const int* flag, StepRef R, StateRef from, StateRef to,
                  const int* tag_from, int* tag_to, int global_out) {
  const int nt = int(b->ntot), tpb = b->tpb, nb = blocks_for(nt, tpb);
  const float rl2 = float((b->P.rc + b->skin) * (b->P.rc + b->skin));
  if (b->path == 2) {
    hipLaunchKernelGGL(b->uniform ? k_build_tiles<1> : k_build_tiles<0>, dim3(b->ntiles), dim3(TILE_THREADS), 0,
                       s, nt,
                       b->list_ld, b->list_cap, b->d_tiles, b->d_sims, b->d_slot_cell, b->d_pfix,
                       b->d_start, b->d_ncount, b->d_wstart, b->d_wcount, b->d_list, b->d_nlist,
                       b->d_tilerec, from, to, tag_from, tag_to, b->d_flag + 2, flag, R, rl2,
                       global_out || b->force_gather ? 1 : 0);
    return;
  }
  hipLaunchKernelGGL(k_build_list, dim3(nb), dim3(tpb), 0, s, nt, b->list_ld, b->list_cap, b->d_sims,
                     b->d_atom_sim, b->d_slot_cell, b->d_pfix, b->d_start, b->d_ncount, b->d_wstart, b->d_wcount,
                     b->d_list, b->d_nlist, from, to, tag_from, tag_to, b->d_flag + 2, flag, R, rl2);
}

// Counting sort of the current state by cell (flag null: unconditional).
void enqueue_sort(hmd_batch* b, Launcher& L, const StepConst& K, const int* flag, StepRef R) {
  hipStream_t s = L.s;
  const int nt = int(b->ntot), tpb = b->tpb, nb = blocks_for(nt, tpb);
  if (b->path == 0) {
    const int src = b->cur, dst = 1 - b->cur;
    if (!flag && R.base == nullptr && R.k < 0) {  // keys for a sort outside a time step
      hipLaunchKernelGGL((k_integrate<0, 0>), dim3(nb), dim3(tpb), 0, s, nt, b->d_sims, b->d_atom_sim,
                         state_ref(b, src), b->d_f4, b->d_key, b->d_count, b->d_rank, b->d_pfix, b->d_pbuild,
                         b->d_flag, b->acc, b->d_dstate, StepRef{nullptr, 0}, K);
    }
    L.begin(K_SCAN);
    hipLaunchKernelGGL(k_scan, dim3(b->S), dim3(1024), 0, s, b->d_sims, b->d_count, b->d_start, b->d_ncount,
                       nullptr, R);
    L.end();
    L.begin(K_SCATTER);
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(tpb), 0, s, nt, b->d_key, b->d_start, b->d_rank, b->d_perm,
                       nullptr, R);
    L.end();
    L.begin(K_REORDER);
    hipLaunchKernelGGL(k_reorder<0>, dim3(nb), dim3(tpb), 0, s, nt, b->d_sims, b->d_cell_sim, b->d_key,
                       b->d_start, b->d_ncount, b->d_perm, state_ref(b, src), state_ref(b, dst), b->d_tag[src],
                       b->d_tag[dst], b->d_pos4, b->d_pfix, b->d_pbuild, b->d_slot_cell, nullptr, R);
    L.end();
    b->cur = dst;
    return;
  }
  L.begin(K_KEYS);
  hipLaunchKernelGGL(k_keys, dim3(nb), dim3(tpb), 0, s, nt, b->d_sims, b->d_atom_sim, state_ref(b, 0), b->d_key,
                     b->d_count, b->d_rank, flag, R);
  L.end();
  L.begin(K_SCAN);
  hipLaunchKernelGGL(k_scan, dim3(b->S), dim3(1024), 0, s, b->d_sims, b->d_count, b->d_start, b->d_ncount, flag,
                     R);
  L.end();
  L.begin(K_SCATTER);
  hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(tpb), 0, s, nt, b->d_key, b->d_start, b->d_rank, b->d_perm, flag,
                     R);
  L.end();
  L.begin(K_REORDER);
  hipLaunchKernelGGL(k_reorder<1>, dim3(nb), dim3(tpb), 0, s, nt, b->d_sims, b->d_cell_sim, b->d_key, b->d_start,
                     b->d_ncount, b->d_perm, state_ref(b, 0), state_ref(b, 1), b->d_tag[0], b->d_tag[1],
                     b->d_pos4, b->d_pfix, b->d_pbuild, b->d_slot_cell, flag, R);
  L.end();
  L.begin(K_LIST);
  launch_build(b, s, flag, R, state_ref(b, 1), state_ref(b, 0), b->d_tag[1], b->d_tag[0], 0);
  L.end();
}

// Pair-path force kernels by variant index ((mode 2 + energy) 2 + uniform
// unit) 2 + wall parameters equal to the fluid's; sampling steps with the
// wall pressure recorded take the PR table, indexed (energy 2 + uniform) 2 +
// walls.
#define HMD_V(K, M, E, U, W) &K<M, E, U, W, 0>
#define HMD_VP(K, E, U, W) &K<1, E, U, W, 1>
#define HMD_VARIANTS_PR(K)                                                                                  \
  HMD_VP(K, 0, 0, 0), HMD_VP(K, 0, 0, 1), HMD_VP(K, 0, 1, 0), HMD_VP(K, 0, 1, 1), HMD_VP(K, 1, 0, 0),         \
      HMD_VP(K, 1, 0, 1), HMD_VP(K, 1, 1, 0), HMD_VP(K, 1, 1, 1)
#define HMD_VARIANTS(K)                                                                                   \
  HMD_V(K, 0, 0, 0, 0), HMD_V(K, 0, 0, 0, 1), HMD_V(K, 0, 0, 1, 0), HMD_V(K, 0, 0, 1, 1),               \
      HMD_V(K, 0, 1, 0, 0), HMD_V(K, 0, 1, 0, 1), HMD_V(K, 0, 1, 1, 0), HMD_V(K, 0, 1, 1, 1),           \
      HMD_V(K, 1, 0, 0, 0), HMD_V(K, 1, 0, 0, 1), HMD_V(K, 1, 0, 1, 0), HMD_V(K, 1, 0, 1, 1),           \
      HMD_V(K, 1, 1, 0, 0), HMD_V(K, 1, 1, 0, 1), HMD_V(K, 1, 1, 1, 0), HMD_V(K, 1, 1, 1, 1)
decltype(&k_force_tiles<0, 0, 0, 0, 0>) force_tiles_variant(int v, bool pr) {
  static const decltype(&k_force_tiles<0, 0, 0, 0, 0>) tab[16] = {HMD_VARIANTS(k_force_tiles)};
  static const decltype(&k_force_tiles<0, 0, 0, 0, 0>) tab_pr[8] = {HMD_VARIANTS_PR(k_force_tiles)};
  return pr ? tab_pr[v & 7] : tab[v];
}
decltype(&k_force_list<0, 0, 0, 0, 0>) force_list_variant(int v, bool pr) {
  static const decltype(&k_force_list<0, 0, 0, 0, 0>) tab[16] = {HMD_VARIANTS(k_force_list)};
  static const decltype(&k_force_list<0, 0, 0, 0, 0>) tab_pr[8] = {HMD_VARIANTS_PR(k_force_list)};
  return pr ? tab_pr[v & 7] : tab[v];
}
#undef HMD_VARIANTS
#undef HMD_VARIANTS_PR
#undef HMD_V
#undef HMD_VP

void enqueue_force(hmd_batch* b, hipStream_t s, int mode, const StepConst& K, StepRef R) {
  const int nt = int(b->ntot), tpb = b->tpb, nb = blocks_for(nt, tpb);
  const int src = b->cur;
  if (b->path == 0) {
    if (mode == 0)
      hipLaunchKernelGGL(k_force_cell<0>, dim3(nb), dim3(tpb), 0, s, nt, b->d_sims, b->d_atom_sim, b->d_pos4,
                         b->d_start, b->d_ncount, b->d_wpos4, b->d_wstart, b->d_wcount, b->d_f4, state_ref(b, src),
                         b->acc, b->d_dstate, R, K);
    else
      hipLaunchKernelGGL(k_force_cell<1>, dim3(nb), dim3(tpb), 0, s, nt, b->d_sims, b->d_atom_sim, b->d_pos4,
                         b->d_start, b->d_ncount, b->d_wpos4, b->d_wstart, b->d_wcount, b->d_f4, state_ref(b, src),
                         b->acc, b->d_dstate, R, K);
  } else {
    const int v = ((mode * 2 + (K.energy_on ? 1 : 0)) * 2 + (b->uniform ? 1 : 0)) * 2 + (b->walls_same ? 1 : 0);
    const bool pr = mode == 1 && K.press_on;
    if (b->path == 2) {
      hipLaunchKernelGGL(force_tiles_variant(v, pr), dim3(b->ntiles), dim3(TILE_THREADS), 0, s, nt, b->list_ld,
                         b->d_tilerec, b->d_sims, b->d_pfix, b->d_list,
                         b->d_nlist, b->d_f4, state_ref(b, 0), b->acc, b->d_dstate, R, K);
    } else {
      hipLaunchKernelGGL(force_list_variant(v, pr), dim3(nb), dim3(tpb), 0, s, nt, b->list_ld, b->d_sims,
                         b->d_atom_sim, b->d_pfix, b->d_list, b->d_nlist, b->d_f4, state_ref(b, 0), b->acc,
                         b->d_dstate, R, K);
    }
  }
}

// One velocity-Verlet step over the whole batch.
void enqueue_step(hmd_batch* b, Launcher& L, const StepConst& K, StepRef R) {
  hipStream_t s = L.s;
  const int nt = int(b->ntot), tpb = b->tpb, nb = blocks_for(nt, tpb);
  L.begin(K_INTEGRATE);
  if (b->path == 0)
    hipLaunchKernelGGL((k_integrate<1, 0>), dim3(nb), dim3(tpb), 0, s, nt, b->d_sims, b->d_atom_sim,
                       state_ref(b, b->cur), b->d_f4, b->d_key, b->d_count, b->d_rank, b->d_pfix, b->d_pbuild,
                       b->d_flag, b->acc, b->d_dstate, R, K);
  else
    hipLaunchKernelGGL((k_integrate<1, 1>), dim3(nb), dim3(tpb), 0, s, nt, b->d_sims, b->d_atom_sim,
                       state_ref(b, 0), b->d_f4, b->d_key, b->d_count, b->d_rank, b->d_pfix, b->d_pbuild, b->d_flag,
                       b->acc, b->d_dstate, R, K);
  L.end();
  enqueue_sort(b, L, K, b->path == 0 ? nullptr : b->d_flag, R);
  L.begin(K_FORCE);
  enqueue_force(b, s, 1, K, R);
  L.end();
}

// Unconditional sort of the current positions (creation, new state).
void sort_now(hmd_batch* b, const StepConst& K) {
  Launcher L{b, b->ctx->stream, nullptr, 0};
  enqueue_sort(b, L, K, nullptr, StepRef{nullptr, -1});
}

// Forces for the current positions; potential energy and pair counts go to
// acc.pe[(done + 1) & 1] and acc.pairs (cleared first).
int forces_now(hmd_batch* b, bool energy) {
  hmd_ctx* ctx = b->ctx;
  hipStream_t s = ctx->stream;
  StepConst K = step_const(b, b->thermo_on, energy);
  const int p = int((b->done + 1) & 1);
  HMD_HIP(ctx, hipMemsetAsync(b->acc.pe[p], 0, sizeof(double) * b->S, s));
  HMD_HIP(ctx, hipMemsetAsync(b->acc.ke[p], 0, sizeof(double) * b->S, s));
  HMD_HIP(ctx, hipMemsetAsync(b->acc.pairs, 0, 2 * sizeof(unsigned long long), s));
  enqueue_force(b, s, 0, K, StepRef{nullptr, b->done});
  HMD_HIP(ctx, hipGetLastError());
  return HMD_OK;
}

void release_graphs(hmd_batch* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& kv : b->graph_defs) (void)hipGraphDestroy(kv.second);
  b->graphs.clear();
  b->graph_defs.clear();
  b->graph_spans.clear();
  b->graph_nstamps.clear();
}

int ensure_events(hmd_batch* b, size_t n) {
  while (b->ev.size() < n) {
    hipEvent_t e;
    HMD_HIP(b->ctx, hipEventCreate(&e));
    b->ev.push_back(e);
  }
  return HMD_OK;
}

int harvest(hmd_batch* b, std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>>& marks) {
  if (marks.empty()) return HMD_OK;
  HMD_HIP(b->ctx, hipEventSynchronize(marks.back().second.second));
  for (auto& m : marks) {
    float ms = 0.f;
    HMD_HIP(b->ctx, hipEventElapsedTime(&ms, m.second.first, m.second.second));
    b->kern_ms[m.first] += ms;
    b->kern_n[m.first] += 1;
  }
  marks.clear();
  return HMD_OK;
}

// Executable graph of `chunk` steps; its step indices are read from
// d_dstate[0], which its last node advances by `chunk`.  With timing on, the
// kernels of up to kStampedSteps evenly spaced steps (the last one among
// them) are bracketed by stamp kernels, and one more stamp after the last
// measures the gap of an empty interval.
int get_graph(hmd_batch* b, int chunk, const StepConst& K, hipGraphExec_t* out) {
  const int key = chunk * 4 + (K.thermo_on ? 1 : 0) + (b->timing ? 2 : 0);
  auto it = b->graphs.find(key);
  if (it != b->graphs.end()) {
    *out = it->second;
    return HMD_OK;
  }
  hmd_ctx* ctx = b->ctx;
  hipStream_t s = ctx->stream;
  const int cur0 = b->cur;
  auto& spans = b->graph_spans[key];
  spans.clear();
  const int every = std::max(1, chunk / kStampedSteps);
  Launcher L{b, s, nullptr, 0};
  HMD_HIP(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < chunk; ++k) {
    const bool stamped = b->timing && (chunk - 1 - k) % every == 0 && (chunk - 1 - k) / every < kStampedSteps;
    L.spans = stamped ? &spans : nullptr;
    L.last_stamp = -1;
    L.flag = b->path == 0 ? nullptr : b->d_flag;
    L.R = StepRef{b->d_dstate, k};
    enqueue_step(b, L, K, StepRef{b->d_dstate, k});
  }
  if (b->timing) {  // calibration: an empty interval after the last stamp
    L.spans = &spans;
    L.stamp();
  }
  hipLaunchKernelGGL(k_add_i64, dim3(1), dim3(1), 0, s, b->d_dstate, int64_t(chunk));
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  b->cur = cur0;  // capture did not execute anything
  if (e != hipSuccess) {
    ctx->err = std::string("graph capture: ") + hipGetErrorString(e);
    return HMD_EDEVICE;
  }
  if (b->timing) b->graph_nstamps[key] = L.next_stamp;
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    ctx->err = std::string("graph instantiate: ") + hipGetErrorString(e);
    return HMD_EDEVICE;
  }
  b->graph_defs[key] = g;
  b->graphs[key] = ex;
  *out = ex;
  return HMD_OK;
}

}  // namespace

// Tiles of the tiled path: per system and z slab, runs of whole columns
// sized so that a tile holds about one to two workgroups of atoms and its
// staged neighbourhood fits the LDS capacity.
int make_tiles(hmd_batch* b) {
  hmd_ctx* ctx = b->ctx;
  constexpr int kStageCap = TILE_STAGE;
  b->stage_cap = kStageCap;
  std::vector<int4> tiles;
  b->tile_first.assign(b->S + 1, 0);
  for (int k = 0; k < b->S; ++k) {
    b->tile_first[k] = int(tiles.size());
    const SimDev& D = b->sims[k];
    const HostSystem& H = b->host[k];
    const double per_col = double(D.nf) / double(D.nx * D.nz);
    const double wall_col = double(H.nw) / double(2 * D.nx * D.nz);
    // columns per tile: the most home atoms per unit of cost, cost being
    // the lanes of whole 256-lane passes plus tile_alpha per staged atom
    // (a wider tile stages less halo per home atom); 2% hysteresis keeps
    // the narrower of two near-equal choices
    int best = 1;
    double best_use = -1.0;
    for (int nc = 1; nc <= D.nx; ++nc) {
      const double atoms = nc * per_col;
      const double staged = 3.0 * std::min(nc + 2, D.nx) * (per_col + 2.0 * wall_col);
      if (staged > 0.9 * kStageCap && nc > 1) break;
      const double passes = std::ceil(atoms / TILE_THREADS);
      const double use = atoms / (passes * TILE_THREADS + b->tile_alpha * staged);
      if (use > best_use + 0.02 * (b->tile_alpha > 0.0 ? best_use : 1.0)) {
        best_use = use;
        best = nc;
      }
    }
    const int ntx = (D.nx + best - 1) / best;
    for (int z = 0; z < D.nz; ++z)
      for (int t = 0; t < ntx; ++t) {  // columns split as evenly as possible
        const int x0 = int(int64_t(t) * D.nx / ntx), x1 = int(int64_t(t + 1) * D.nx / ntx);
        tiles.push_back(make_int4(k, z, x0, x1 - x0));
      }
  }
  b->ntiles = int(tiles.size());
  b->tile_first[b->S] = b->ntiles;
  HMD_TRY(dalloc(ctx, &b->d_tbins, int64_t(b->ntiles) * BIN_LDS * 2));
  HMD_HIP(ctx, hipMemsetAsync(b->d_tbins, 0, sizeof(double) * size_t(b->ntiles) * BIN_LDS * 2, ctx->stream));
  HMD_TRY(dalloc(ctx, &b->d_tiles, b->ntiles));
  HMD_TRY(dalloc(ctx, &b->d_tilerec, int64_t(b->ntiles) * TILE_REC));
  HMD_HIP(ctx, hipMemcpyAsync(b->d_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice,
                              ctx->stream));
  HMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return HMD_OK;
}

int batch_create(hmd_ctx* ctx, const hmd_md_job* jobs, int n, hmd_batch** out) {
  if (!ctx || !out || !jobs || n < 1 || n > 65535) {
    if (ctx) ctx->err = "md batch: need 1..65535 jobs";
    return HMD_EINVAL;
  }
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  auto* b = new hmd_batch();
  b->ctx = ctx;
  b->P = ctx->params;
  b->S = n;
  b->n_sample = jobs[0].n_sample;
  const int64_t min_sample = std::max(2, b->P.n_blocks);
  for (int k = 0; k < n; ++k)
    if (jobs[k].n_sample != b->n_sample || jobs[k].n_sample < 0 ||
        (jobs[k].n_sample > 0 && jobs[k].n_sample < min_sample)) {
      ctx->err = "md batch: every job needs the same n_sample (0, or at least max(2, n_blocks))";
      delete b;
      return HMD_EINVAL;
    }
  if (b->n_sample > 0) {  // one series entry per sampled step up to the cap, then groups of B steps
    const int64_t B = (b->n_sample + kSeriesCap - 1) / kSeriesCap;
    b->ser_B = int(B);
    b->nser = b->n_sample / B;
    b->ser_r = int(b->n_sample - b->nser * B);
  }
  {
    const Config c = choose_config(ctx, jobs, n);
    b->path = c.path;
    b->skin = c.skin;
    b->tpb = c.tpb;
    b->tile_alpha = c.tile_alpha;
    b->cell_w = c.cell_w;
    b->chunk = c.chunk;
  }
  if (b->path == 3) {  // the tiled path with every tile on its gather fallback
    b->path = 2;
    b->force_gather = true;
  }
  const double wmin = std::max(b->path >= 1 ? b->P.rc + b->skin : b->P.rc, b->cell_w);
  b->host.resize(n);
  for (int k = 0; k < n; ++k) {
    hmd_md_params Pk = b->P;  // the job's own density, where it gives one
    if (jobs[k].rho > 0.0) Pk.rho = jobs[k].rho;
    int rc = build_system(Pk, jobs[k].h, jobs[k].g, jobs[k].seed, wmin, b->host[k], ctx->err);
    if (rc != HMD_OK) {
      delete b;
      return rc;
    }
  }
  // flattened layout
  b->sims.resize(n);
  int64_t a0 = 0, c0 = 0, wc0 = 0, bin0 = 0, w0 = 0;
  const double half = 0.5 * std::cbrt(4.0 / b->P.rho_wall);
  for (int k = 0; k < n; ++k) {
    const HostSystem& H = b->host[k];
    SimDev& D = b->sims[k];
    std::memset(&D, 0, sizeof(D));
    D.Lx = H.Lx; D.Lz = H.Lz; D.h = H.h;
    D.inv_x = H.inv_x; D.inv_y = H.inv_y; D.inv_z = H.inv_z;
    D.wx = H.wx; D.wy = H.wy; D.wz = H.wz;
    D.g = H.g;
    D.inv_area = 1.0 / (H.Lx * H.Lz);
    D.inv_bin = 1.0 / b->P.bin_dy;
    D.inv_nf = 1.0 / double(H.nf);
    const double margin = double(b->P.wall_layers) * half + 1.0;  // beyond the outermost wall layer
    D.y_lo = -margin;
    D.fix_x = kTwo32 / H.Lx;
    D.fix_z = kTwo32 / H.Lz;
    // y takes the x unit when the wall span fits in 2^32 of them (then, with
    // Lx = Lz, one unit serves every axis)
    const double span_y = H.h + 2.0 * margin;
    D.fix_y = span_y < H.Lx ? D.fix_x : kTwo32 / span_y;
    D.unit_x = float(H.Lx / kTwo32);
    D.unit_y = float(1.0 / D.fix_y);
    D.unit_z = float(H.Lz / kTwo32);
    D.inv_u = float(D.fix_x);
    D.inv_u2 = float(D.fix_x * D.fix_x);
    D.fwx = float(H.wx); D.fwy = float(H.wy); D.fwz = float(H.wz);
    D.nx = H.nx; D.ny = H.ny; D.nz = H.nz;
    D.a0 = int(a0); D.nf = int(H.nf);
    D.c0 = int(c0); D.ncell = H.nx * H.ny * H.nz;
    D.wc0 = int(wc0);
    D.w0 = int(w0);
    D.nbins = H.nbins; D.bin0 = int(bin0);
    a0 += H.nf;
    c0 += D.ncell;
    wc0 += 2 * int64_t(H.nx) * H.nz;
    bin0 += H.nbins;
    w0 += H.nw;
  }
  if (a0 + w0 >= (int64_t(1) << 31) || c0 >= (int64_t(1) << 31)) {
    ctx->err = "md batch: too many atoms or cells for one batch";
    delete b;
    return HMD_EINVAL;
  }
  b->ntot = a0; b->ncell = c0; b->nwcell = wc0; b->nbins = bin0; b->nwall = w0;
  b->walls_same = b->P.eps_wf == 1.0 && b->P.sigma_wf == 1.0;
  b->uniform = true;
  for (const SimDev& D : b->sims)
    b->uniform = b->uniform && D.fix_x == D.fix_y && D.fix_x == D.fix_z;
  // the pair-list build packs a position index into 24 bits
  if (b->path == 1 && b->ntot + b->nwall >= (int64_t(1) << 24)) b->path = 0;
  if (b->path == 2 && b->P.wall_layers < 1) b->path = 1;
  if (b->P.pressure && b->path == 0) {
    ctx->err = "md batch: the wall pressure needs a pair path (force_path 1 or 2)";
    delete b;
    return HMD_EINVAL;
  }
  // pair-list capacity: neighbours within rc + skin at twice the fluid density
  // plus a wall half-space, rounded up to a multiple of 32
  const double rl = b->P.rc + b->skin;
  double rho_max = b->P.rho;
  for (int k = 0; k < n; ++k) rho_max = std::max(rho_max, jobs[k].rho);
  const double est = 2.0 * std::max(rho_max, 0.8) * 4.18879 * rl * rl * rl +
                     2.0 * b->P.rho_wall * 2.0944 * rl * rl * rl;
  b->list_cap = b->path >= 1 ? int(32 * std::ceil(est / 32.0)) : 0;
  b->list_ld = int(64 * ((b->ntot + 63) / 64));

  int rc = HMD_OK;
  auto fail = [&](int code) {
    batch_free(b);
    return code;
  };
  if ((rc = dalloc(ctx, &b->d_sims, n)) || (rc = dalloc(ctx, &b->d_atom_sim, b->ntot)) ||
      (rc = dalloc(ctx, &b->d_cell_sim, b->ncell)) || (rc = dalloc(ctx, &b->d_f4, b->ntot)) ||
      (rc = dalloc(ctx, &b->d_key, b->ntot)) || (rc = dalloc(ctx, &b->d_count, b->ncell)) ||
      (rc = dalloc(ctx, &b->d_rank, b->ntot)) || (rc = dalloc(ctx, &b->d_start, b->ncell)) ||
      (rc = dalloc(ctx, &b->d_ncount, b->ncell)) || (rc = dalloc(ctx, &b->d_perm, b->ntot)) ||
      (rc = dalloc(ctx, &b->d_wpos4, b->nwall)) || (rc = dalloc(ctx, &b->d_wstart, b->nwcell)) ||
      (rc = dalloc(ctx, &b->d_wcount, b->nwcell)) || (rc = dalloc(ctx, &b->d_dstate, 4)) ||
      (rc = dalloc(ctx, &b->d_tag[0], b->ntot)) || (rc = dalloc(ctx, &b->d_tag[1], b->ntot)) ||
      (rc = dalloc(ctx, &b->d_flag, 4)) ||
      (rc = dalloc(ctx, &b->d_stamps, kMaxStamps)))
    return fail(rc);
  if (b->path == 0) {
    if ((rc = dalloc(ctx, &b->d_pos4, b->ntot))) return fail(rc);
  } else {
    if ((rc = dalloc(ctx, &b->d_pfix, b->ntot + b->nwall)) || (rc = dalloc(ctx, &b->d_pbuild, b->ntot)) ||
        (rc = dalloc(ctx, &b->d_slot_cell, b->ntot)) || (rc = dalloc(ctx, &b->d_nlist, b->ntot)) ||
        (rc = dalloc(ctx, &b->d_list, int64_t(b->list_cap) * b->list_ld)))
      return fail(rc);
  }
  for (int w = 0; w < 2; ++w)
    for (int a = 0; a < 6; ++a)
      if ((rc = dalloc(ctx, &b->d_state[w][a], b->ntot))) return fail(rc);
  // cell numbering of every system (rank tables, then inverses): Morton
  // order, or slab order (z, x, y) for the tiled path
  if ((rc = dalloc(ctx, &b->d_cellmap, 2 * b->ncell))) return fail(rc);
  b->cell_rank.assign(b->ncell, 0);
  std::vector<uint32_t> cell_lin(b->ncell);
  for (int k = 0; k < n; ++k) {
    SimDev& D = b->sims[k];
    std::vector<std::pair<uint64_t, uint32_t>> order(D.ncell);
    for (int lid = 0; lid < D.ncell; ++lid) {
      const uint32_t cx = lid % D.nx, cy = (lid / D.nx) % D.ny, cz = lid / (D.nx * D.ny);
      const uint64_t key = b->path == 2 ? (uint64_t(cz) * D.nx + cx) * D.ny + cy : morton3(cx, cy, cz);
      order[lid] = {key, uint32_t(lid)};
    }
    std::sort(order.begin(), order.end());
    for (int r = 0; r < D.ncell; ++r) {
      b->cell_rank[D.c0 + order[r].second] = uint32_t(r);
      cell_lin[D.c0 + r] = order[r].second;
    }
    D.rank = b->d_cellmap + D.c0;
    D.lin = b->d_cellmap + b->ncell + D.c0;
  }
  if (b->path == 2 && (rc = make_tiles(b))) return fail(rc);
  HMD_HIP(ctx, hipMemcpyAsync(b->d_cellmap, b->cell_rank.data(), 4 * b->ncell, hipMemcpyHostToDevice, ctx->stream));
  HMD_HIP(ctx, hipMemcpyAsync(b->d_cellmap + b->ncell, cell_lin.data(), 4 * b->ncell, hipMemcpyHostToDevice,
                              ctx->stream));
  const int64_t nacc = 6 * int64_t(n) + 2 * int64_t(n) * b->nser + 3 * int64_t(n) + 2 * b->nbins;
  if ((rc = dalloc(ctx, &b->d_accbuf, nacc)) || (rc = dalloc(ctx, &b->d_status, n)) ||
      (rc = dalloc(ctx, &b->acc.pairs, 2)) || (rc = dalloc(ctx, &b->d_sout, 4 * int64_t(n))))
    return fail(rc);
  if (b->n_sample > 0 && b->P.n_blocks == 0 && (rc = dalloc(ctx, &b->d_gam, int64_t(n) * b->nser)))
    return fail(rc);
  double* q = b->d_accbuf;
  for (int p = 0; p < 2; ++p) { b->acc.vc2[p] = q; q += n; }
  for (int p = 0; p < 2; ++p) { b->acc.pe[p] = q; q += n; }
  for (int p = 0; p < 2; ++p) { b->acc.ke[p] = q; q += n; }
  b->acc.blocks = q; q += int64_t(n) * b->nser;
  b->acc.pblocks = q; q += int64_t(n) * b->nser;
  b->acc.tsum = q; q += 3 * int64_t(n);
  b->acc.binvx = q; q += b->nbins;
  b->acc.bincnt = q;
  b->acc.tbins = b->d_tbins;
  b->acc.status = b->d_status;

  hipStream_t s = ctx->stream;
  // host staging
  std::vector<double> hs[6];
  for (auto& v : hs) v.resize(b->ntot);
  std::vector<int> tag(b->ntot);
  std::vector<uint16_t> atom_sim(b->ntot), cell_sim(b->ncell);
  std::vector<float4> wpos(std::max<int64_t>(b->nwall, 1));
  std::vector<int4> wfix(std::max<int64_t>(b->nwall, 1));
  std::vector<uint32_t> wstart(b->nwcell), wcount(b->nwcell, 0);
  b->wall_id.assign(std::max<int64_t>(b->nwall, 1), 0);
  for (int k = 0; k < n; ++k) {
    HostSystem& H = b->host[k];
    const SimDev& D = b->sims[k];
    for (int64_t i = 0; i < H.nf; ++i) {
      const int64_t g = D.a0 + i;
      for (int a = 0; a < 3; ++a) {
        hs[a][g] = H.x[3 * i + a];
        hs[3 + a][g] = H.v[3 * i + a];
      }
      tag[g] = int(i);
      atom_sim[g] = uint16_t(k);
    }
    for (int c = 0; c < D.ncell; ++c) cell_sim[D.c0 + c] = uint16_t(k);
    // wall columns: slab 0 below the channel, 1 above; ascending wall id
    const int ncol = 2 * D.nx * D.nz;
    std::vector<int> wkey(H.nw);
    for (int64_t w = 0; w < H.nw; ++w) {
      const int cx = cell_coord(H.xw[3 * w], H.inv_x, H.nx);
      const int cz = cell_coord(H.xw[3 * w + 2], H.inv_z, H.nz);
      const int slab = H.xw[3 * w + 1] <= 0.0 ? 0 : 1;
      wkey[w] = (slab * H.nz + cz) * H.nx + cx;
      wcount[D.wc0 + wkey[w]]++;
    }
    uint32_t acc0 = uint32_t(D.w0);
    for (int c = 0; c < ncol; ++c) {
      wstart[D.wc0 + c] = acc0;
      acc0 += wcount[D.wc0 + c];
    }
    std::vector<uint32_t> fill(ncol, 0);
    for (int64_t w = 0; w < H.nw; ++w) {
      const int c = wkey[w];
      const uint32_t slot = wstart[D.wc0 + c] + fill[c]++;
      b->wall_id[slot] = int(w);
      const int cx = c % H.nx, cz = (c / H.nx) % H.nz, slab = c / (H.nx * H.nz);
      const double oy = slab == 0 ? -H.wy : double(H.ny) * H.wy;
      const double* p = &H.xw[3 * w];
      wpos[slot] = make_float4(float(p[0] - double(cx) * H.wx), float(p[1] - oy), float(p[2] - double(cz) * H.wz),
                               0.0f);
      wfix[slot] = make_int4(int(fix_axis_host(p[0], D.fix_x)), int(fix_axis_host(p[1] - D.y_lo, D.fix_y)),
                             int(fix_axis_host(p[2], D.fix_z)), 0);
    }
    // the big host arrays are no longer needed
    H.x.clear(); H.x.shrink_to_fit();
    H.v.clear(); H.v.shrink_to_fit();
    H.xw.clear(); H.xw.shrink_to_fit();
  }
  const int64_t dstate[4] = {0, b->P.n_equil, 0, 0};
  auto up = [&](void* d, const void* h, size_t bytes) -> int {
    HMD_HIP(ctx, hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
    return HMD_OK;
  };
  if ((rc = up(b->d_sims, b->sims.data(), sizeof(SimDev) * n)) ||
      (rc = up(b->d_atom_sim, atom_sim.data(), 2 * b->ntot)) ||
      (rc = up(b->d_cell_sim, cell_sim.data(), 2 * b->ncell)) || (rc = up(b->d_tag[0], tag.data(), 4 * b->ntot)) ||
      (rc = up(b->d_wpos4, wpos.data(), sizeof(float4) * b->nwall)) ||
      (rc = up(b->d_wstart, wstart.data(), 4 * b->nwcell)) ||
      (rc = up(b->d_wcount, wcount.data(), 4 * b->nwcell)) || (rc = up(b->d_dstate, dstate, sizeof(dstate))))
    return fail(rc);
  if (b->path >= 1 && (rc = up(b->d_pfix + b->ntot, wfix.data(), sizeof(int4) * b->nwall))) return fail(rc);
  for (int a = 0; a < 6; ++a)
    if ((rc = up(b->d_state[0][a], hs[a].data(), 8 * b->ntot))) return fail(rc);
  HMD_HIP(ctx, hipMemsetAsync(b->d_accbuf, 0, sizeof(double) * nacc, s));
  HMD_HIP(ctx, hipMemsetAsync(b->d_status, 0, sizeof(int) * n, s));
  HMD_HIP(ctx, hipMemsetAsync(b->d_count, 0, 4 * b->ncell, s));
  HMD_HIP(ctx, hipMemsetAsync(b->d_flag, 0, 4 * sizeof(int), s));
  b->cur = 0;
  StepConst K = step_const(b, true, true);
  sort_now(b, K);
  if ((rc = forces_now(b, true))) return fail(rc);
  HMD_HIP(ctx, hipStreamSynchronize(s));
  HMD_HIP(ctx, hipGetLastError());
  *out = b;
  return HMD_OK;
}

void batch_free(hmd_batch* b) {
  if (!b) return;
  release_graphs(b);
  for (auto e : b->ev) (void)hipEventDestroy(e);
  void* ptrs[] = {b->d_sims, b->d_atom_sim, b->d_cell_sim, b->d_f4, b->d_pos4, b->d_pfix, b->d_pbuild,
                  b->d_slot_cell, b->d_list, b->d_nlist, b->d_flag, b->d_key, b->d_count, b->d_rank, b->d_start,
                  b->d_ncount, b->d_perm, b->d_wpos4, b->d_wstart, b->d_wcount, b->d_dstate, b->d_tag[0],
                  b->d_tag[1], b->d_accbuf, b->d_status, b->acc.pairs, b->d_cellmap, b->d_tiles,
                  b->d_tilerec, b->d_tbins, b->d_gam, b->d_sout, b->d_stamps};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int w = 0; w < 2; ++w)
    for (int a = 0; a < 6; ++a)
      if (b->d_state[w][a]) (void)hipFree(b->d_state[w][a]);
  delete b;
}

int batch_run(hmd_batch* b, int64_t steps, int graph_chunk, bool thermostat, double* energy_trace) {
  hmd_ctx* ctx = b->ctx;
  if (steps < 0 || graph_chunk < 0 || (graph_chunk & 1)) {
    ctx->err = "md run: steps >= 0 and an even graph chunk";
    return HMD_EINVAL;
  }
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  b->thermo_on = thermostat;
  const bool energy = energy_trace != nullptr;
  const StepConst K = step_const(b, thermostat, energy);
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  const int per_sync = 32;
  if (b->timing) HMD_TRY(ensure_events(b, size_t(2 * K_COUNT) * per_sync + 2));
  Launcher L{b, s, b->timing ? &marks : nullptr, 2};

  auto direct_step = [&](int64_t k) -> int {
    enqueue_step(b, L, K, StepRef{nullptr, b->done});
    if (energy) {
      HMD_HIP(ctx, hipStreamSynchronize(s));
      const int p = int((b->done + 1) & 1);
      double pe = 0, ke = 0, vc2 = 0;
      HMD_HIP(ctx, hipMemcpy(&pe, b->acc.pe[p], sizeof(double), hipMemcpyDeviceToHost));
      HMD_HIP(ctx, hipMemcpy(&ke, b->acc.ke[p], sizeof(double), hipMemcpyDeviceToHost));
      HMD_HIP(ctx, hipMemcpy(&vc2, b->acc.vc2[p], sizeof(double), hipMemcpyDeviceToHost));
      const double nf = double(b->sims[0].nf);
      double lam2 = 1.0;
      if (thermostat) lam2 = 1.0 + K.dt_tau * (K.T0 / (vc2 / nf) - 1.0);
      energy_trace[k] = (0.5 * (ke + (lam2 - 1.0) * vc2) + pe) / nf;
    }
    b->done += 1;
    if (b->timing && int(marks.size()) >= per_sync * (K_COUNT - 1)) {
      HMD_TRY(harvest(b, marks));
      L.next_ev = 2;
    }
    return HMD_OK;
  };

  int64_t k = 0;
  if (graph_chunk > 0 && !energy && steps >= graph_chunk) {
    if (b->cur != 0) HMD_TRY(direct_step(k++));
    if (b->timing) {
      HMD_TRY(harvest(b, marks));
      L.next_ev = 2;
    }
    // timing mode: one replay in kStampEvery is the stamped graph (timed
    // by events, then its stamps read back); the others replay the plain
    // graph with no host synchronisation, as outside timing mode
    hipGraphExec_t ex = nullptr, ex_plain = nullptr;
    HMD_TRY(get_graph(b, graph_chunk, K, &ex));
    if (b->timing) {
      b->timing = false;
      const int rc = get_graph(b, graph_chunk, K, &ex_plain);
      b->timing = true;
      HMD_TRY(rc);
    }
    const int gkey = graph_chunk * 4 + (K.thermo_on ? 1 : 0) + (b->timing ? 2 : 0);
    if (b->timing && b->clock_khz <= 0.0) {
      int khz = 0;
      HMD_HIP(ctx, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device));
      if (khz <= 0) {
        ctx->err = "md run: the device reports no wall-clock rate for timed graph replays";
        return HMD_EDEVICE;
      }
      b->clock_khz = double(khz);
    }
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, b->d_dstate, b->done);
    for (int64_t rep = 0; steps - k >= graph_chunk; ++rep) {
      if (b->timing && rep % kStampEvery == 0) {
        hipEvent_t e0 = b->ev[0], e1 = b->ev[1];
        HMD_HIP(ctx, hipEventRecord(e0, s));
        HMD_HIP(ctx, hipGraphLaunch(ex, s));
        HMD_HIP(ctx, hipEventRecord(e1, s));
        HMD_HIP(ctx, hipEventSynchronize(e1));
        float ms = 0.f;
        HMD_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
        b->graph_ms += ms;
        b->graph_steps += graph_chunk;
        // the stamped steps of the replay: each kernel's time is the span
        // between its stamps less the gap of the empty interval at the end
        // the list build's time is also kept apart for steps that rebuild
        // and steps that do not (bit 63 of its opening stamp)
        const auto& spans = b->graph_spans[gkey];
        const int ns = b->graph_nstamps[gkey];
        unsigned long long st[kMaxStamps];
        HMD_HIP(ctx, hipMemcpy(st, b->d_stamps, sizeof(unsigned long long) * size_t(ns), hipMemcpyDeviceToHost));
        constexpr unsigned long long kClock = ~(1ull << 63);
        const double gap = double((st[ns - 1] & kClock) - (st[ns - 2] & kClock));
        for (const auto& sp : spans) {
          const double ticks = std::max(0.0, double((st[sp[2]] & kClock) - (st[sp[1]] & kClock)) - gap);
          b->kern_ms[sp[0]] += ticks / b->clock_khz;
          b->kern_n[sp[0]] += 1;
          if (sp[0] == K_LIST) {
            const int r = (st[sp[1]] >> 63) ? 1 : 0;
            b->list_ms[r] += ticks / b->clock_khz;
            b->list_n[r] += 1;
          }
        }
      } else {
        HMD_HIP(ctx, hipGraphLaunch(b->timing ? ex_plain : ex, s));
      }
      k += graph_chunk;
      b->done += graph_chunk;
    }
  }
  while (k < steps) HMD_TRY(direct_step(k++));
  if (b->timing) HMD_TRY(harvest(b, marks));
  b->pending = thermostat && b->done > 0;
  HMD_HIP(ctx, hipGetLastError());
  HMD_HIP(ctx, hipStreamSynchronize(s));
  return HMD_OK;
}

int batch_results(hmd_batch* b, hmd_md_result* out) {
  hmd_ctx* ctx = b->ctx;
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  HMD_TRY(forces_now(b, true));
  const int n = b->S;
  // the sampling window is complete once every one of its n_sample steps ran
  const bool complete = b->n_sample > 0 && b->done - b->P.n_equil >= b->n_sample;
  hipStream_t s = ctx->stream;
  std::vector<double> sout(4 * size_t(n)), pout(4 * size_t(n), 0.0), tsum(3 * size_t(n)), pe(n);
  if (complete && b->P.pressure) {  // the pressure series first: d_sout is reused
    series_stats_enqueue(s, b->acc.pblocks, n, b->nser, b->nser, 1.0 / double(b->ser_B), b->P.n_blocks,
                         b->d_gam, b->d_sout);
    HMD_HIP(ctx, hipMemcpyAsync(pout.data(), b->d_sout, 8 * pout.size(), hipMemcpyDeviceToHost, s));
  }
  if (complete)
    series_stats_enqueue(s, b->acc.blocks, n, b->nser, b->nser, 1.0 / double(b->ser_B), b->P.n_blocks, b->d_gam,
                         b->d_sout);
  std::vector<int> status(n);
  int flags[4] = {0, 0, 0, 0};
  if (complete)
    HMD_HIP(ctx, hipMemcpyAsync(sout.data(), b->d_sout, 8 * sout.size(), hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipMemcpyAsync(tsum.data(), b->acc.tsum, 8 * tsum.size(), hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipMemcpyAsync(pe.data(), b->acc.pe[(b->done + 1) & 1], 8 * size_t(n), hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipMemcpyAsync(status.data(), b->d_status, 4 * size_t(n), hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipMemcpyAsync(flags, b->d_flag, sizeof(flags), hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipStreamSynchronize(s));
  HMD_HIP(ctx, hipGetLastError());
  for (int k = 0; k < n; ++k) {
    hmd_md_result& R = out[k];
    std::memset(&R, 0, sizeof(R));
    const SimDev& D = b->sims[k];
    R.n_fluid = D.nf;
    R.pe = pe[k] * D.inv_nf;
    // an overflowing pair list drops interactions: every result is suspect
    int st = (status[k] & 1) || flags[2] > 0 ? HMD_EUNSTABLE : HMD_OK;
    if (complete) {
      const double* so = &sout[4 * size_t(k)];
      R.flux = so[0];
      R.flux_se = so[1];
      R.jflux = so[0] / D.h;
      if (b->P.pressure) {
        R.p = pout[4 * size_t(k)];
        R.p_se = pout[4 * size_t(k) + 1];
      }
      // temperatures are summed over every sampled step
      for (int a = 0; a < 3; ++a) R.T[a] = tsum[3 * k + a] / double(b->n_sample);
      // non-convergence (critical shear, Sec. 3.2): the two halves of the
      // series differ by more than 8 SE, or the spanwise temperature runs away
      if (st == HMD_OK && (std::fabs(so[3] - so[2]) > 8.0 * R.flux_se || R.T[2] > 1.5 * b->P.T0))
        st = HMD_ENOTCONV;
    } else if (st == HMD_OK) {
      st = HMD_EINVAL;  // sampling window not complete
    }
    R.status = st;
  }
  if (flags[2] > 0)
    ctx->err = flags[2] >= (1 << 30) ? std::string("pair list build: a cell holds more than 255 atoms")
                                     : "pair list overflow: " + std::to_string(flags[2]) + " > capacity";
  return HMD_OK;
}

// The sampled q' series of one system: nser entries (each the mean of ser_B
// consecutive sampled steps), as far as sampling has reached.
int batch_series(hmd_batch* b, int sim, double* q, int64_t* n, int which) {
  hmd_ctx* ctx = b->ctx;
  if (sim < 0 || sim >= b->S || b->n_sample <= 0 || which < 0 || which > 1 || (which == 1 && !b->P.pressure)) {
    ctx->err = "md series: need a valid system of a batch with n_sample > 0 (pressure series: pressure on)";
    return HMD_EINVAL;
  }
  if (n) *n = b->nser;
  if (!q) return HMD_OK;
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  const double* src = which ? b->acc.pblocks : b->acc.blocks;
  HMD_HIP(ctx, hipMemcpy(q, src + int64_t(sim) * b->nser, 8 * size_t(b->nser), hipMemcpyDeviceToHost));
  for (int64_t k = 0; k < b->nser; ++k) q[k] /= double(b->ser_B);
  return HMD_OK;
}

// ---------------------------------------------------------------------------
// state of every system at once, and single-system hooks (`sim` selects the
// system of the batch)
// ---------------------------------------------------------------------------
namespace {

int download_state(hmd_batch* b, std::vector<double> (&hs)[6], std::vector<int>& tag) {
  hmd_ctx* ctx = b->ctx;
  hipStream_t s = ctx->stream;
  for (int a = 0; a < 6; ++a) {
    hs[a].resize(b->ntot);
    HMD_HIP(ctx, hipMemcpyAsync(hs[a].data(), b->d_state[b->cur][a], 8 * b->ntot, hipMemcpyDeviceToHost, s));
  }
  tag.resize(b->ntot);
  HMD_HIP(ctx, hipMemcpyAsync(tag.data(), b->d_tag[b->cur], 4 * b->ntot, hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipStreamSynchronize(s));
  return HMD_OK;
}

}  // namespace

int batch_get_all_states(hmd_batch* b, std::vector<std::vector<double>>& x, std::vector<std::vector<double>>& v) {
  hmd_ctx* ctx = b->ctx;
  std::vector<double> hs[6];
  std::vector<int> tag;
  HMD_TRY(download_state(b, hs, tag));
  std::vector<double> vc2(b->S, 0.0);
  if (b->pending)  // the device holds velocities before the last Berendsen factor
    HMD_HIP(ctx, hipMemcpy(vc2.data(), b->acc.vc2[b->done & 1], 8 * size_t(b->S), hipMemcpyDeviceToHost));
  x.assign(b->S, {});
  v.assign(b->S, {});
  for (int k = 0; k < b->S; ++k) {
    const SimDev& D = b->sims[k];
    const double lam =
        b->pending ? std::sqrt(1.0 + (b->P.dt / b->P.tau_T) * (b->P.T0 / (vc2[k] * D.inv_nf) - 1.0)) : 1.0;
    x[k].resize(3 * size_t(D.nf));
    v[k].resize(3 * size_t(D.nf));
    for (int i = 0; i < D.nf; ++i) {
      const int64_t g = D.a0 + i;
      const int id = tag[g];
      for (int a = 0; a < 3; ++a) {
        x[k][3 * id + a] = hs[a][g];
        v[k][3 * id + a] = hs[3 + a][g] * (a == b->P.thermo_axis ? lam : 1.0);
      }
    }
  }
  return HMD_OK;
}

int batch_set_all_states(hmd_batch* b, const std::vector<std::vector<double>>& x,
                         const std::vector<std::vector<double>>& v) {
  hmd_ctx* ctx = b->ctx;
  if (int(x.size()) != b->S || int(v.size()) != b->S) return HMD_EINVAL;
  std::vector<double> hs[6];
  std::vector<int> tag;
  HMD_TRY(download_state(b, hs, tag));
  for (int k = 0; k < b->S; ++k) {
    const SimDev& D = b->sims[k];
    if (x[k].empty() && v[k].empty()) continue;  // this system keeps its state
    if (int64_t(x[k].size()) != 3 * int64_t(D.nf) || int64_t(v[k].size()) != 3 * int64_t(D.nf)) return HMD_EINVAL;
    for (int i = 0; i < D.nf; ++i) {
      const int64_t g = D.a0 + i;
      const int id = tag[g];
      for (int a = 0; a < 3; ++a) {
        hs[a][g] = x[k][3 * id + a];
        hs[3 + a][g] = v[k][3 * id + a];
      }
    }
  }
  hipStream_t s = ctx->stream;
  for (int a = 0; a < 6; ++a)
    HMD_HIP(ctx, hipMemcpyAsync(b->d_state[b->cur][a], hs[a].data(), 8 * b->ntot, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, b->d_dstate + 3, int64_t(0));
  b->pending = false;
  StepConst K = step_const(b, b->thermo_on, true);
  sort_now(b, K);
  HMD_TRY(forces_now(b, true));
  HMD_HIP(ctx, hipStreamSynchronize(s));
  return HMD_OK;
}

int batch_get_state(hmd_batch* b, int sim, double* x, double* v) {
  hmd_ctx* ctx = b->ctx;
  if (sim < 0 || sim >= b->S) return HMD_EINVAL;
  std::vector<double> hs[6];
  std::vector<int> tag;
  HMD_TRY(download_state(b, hs, tag));
  const SimDev& D = b->sims[sim];
  double lam = 1.0;
  if (b->pending) {  // the device holds velocities before the last Berendsen factor
    double vc2 = 0.0;
    HMD_HIP(ctx, hipMemcpy(&vc2, b->acc.vc2[b->done & 1] + sim, sizeof(double), hipMemcpyDeviceToHost));
    lam = std::sqrt(1.0 + (b->P.dt / b->P.tau_T) * (b->P.T0 / (vc2 * D.inv_nf) - 1.0));
  }
  for (int i = 0; i < D.nf; ++i) {
    const int64_t g = D.a0 + i;
    const int id = tag[g];
    for (int a = 0; a < 3; ++a) {
      if (x) x[3 * id + a] = hs[a][g];
      if (v) v[3 * id + a] = hs[3 + a][g] * (a == b->P.thermo_axis ? lam : 1.0);
    }
  }
  return HMD_OK;
}

int batch_set_state(hmd_batch* b, int sim, const double* x, const double* v) {
  hmd_ctx* ctx = b->ctx;
  if (sim < 0 || sim >= b->S || !x || !v) return HMD_EINVAL;
  std::vector<double> hs[6];
  std::vector<int> tag;
  HMD_TRY(download_state(b, hs, tag));
  const SimDev& D = b->sims[sim];
  for (int i = 0; i < D.nf; ++i) {
    const int64_t g = D.a0 + i;
    const int id = tag[g];
    for (int a = 0; a < 3; ++a) {
      hs[a][g] = x[3 * id + a];
      hs[3 + a][g] = v[3 * id + a];
    }
  }
  hipStream_t s = ctx->stream;
  for (int a = 0; a < 6; ++a)
    HMD_HIP(ctx, hipMemcpyAsync(b->d_state[b->cur][a], hs[a].data(), 8 * b->ntot, hipMemcpyHostToDevice, s));
  // the new velocities are final: no Berendsen factor is pending
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, b->d_dstate + 3, int64_t(0));
  b->pending = false;
  StepConst K = step_const(b, b->thermo_on, true);
  sort_now(b, K);
  HMD_TRY(forces_now(b, true));
  HMD_HIP(ctx, hipStreamSynchronize(s));
  return HMD_OK;
}

int batch_forces(hmd_batch* b, int sim, float* f, double* pe) {
  hmd_ctx* ctx = b->ctx;
  if (sim < 0 || sim >= b->S) return HMD_EINVAL;
  HMD_TRY(forces_now(b, true));
  std::vector<float4> f4(b->ntot);
  std::vector<int> tag(b->ntot);
  hipStream_t s = ctx->stream;
  HMD_HIP(ctx, hipMemcpyAsync(f4.data(), b->d_f4, sizeof(float4) * b->ntot, hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipMemcpyAsync(tag.data(), b->d_tag[b->cur], 4 * b->ntot, hipMemcpyDeviceToHost, s));
  double pes = 0.0;
  HMD_HIP(ctx, hipMemcpyAsync(&pes, b->acc.pe[(b->done + 1) & 1] + sim, 8, hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipStreamSynchronize(s));
  const SimDev& D = b->sims[sim];
  for (int i = 0; i < D.nf; ++i) {
    const int64_t g = D.a0 + i;
    const int id = tag[g];
    if (f) {
      f[3 * id + 0] = f4[g].x;
      f[3 * id + 1] = f4[g].y;
      f[3 * id + 2] = f4[g].z;
    }
  }
  if (pe) *pe = pes;
  return HMD_OK;
}

int batch_cells(hmd_batch* b, int sim, uint32_t* cell_of, uint32_t* counts, uint32_t* order) {
  hmd_ctx* ctx = b->ctx;
  if (sim < 0 || sim >= b->S) return HMD_EINVAL;
  const SimDev& D = b->sims[sim];
  std::vector<int> tag(b->ntot);
  std::vector<uint32_t> nc(D.ncell), cell(b->ntot);
  hipStream_t s = ctx->stream;
  if (b->path == 0) {
    std::vector<float4> p4(b->ntot);
    HMD_HIP(ctx, hipMemcpyAsync(p4.data(), b->d_pos4, sizeof(float4) * b->ntot, hipMemcpyDeviceToHost, s));
    HMD_HIP(ctx, hipStreamSynchronize(s));
    for (int64_t g = 0; g < b->ntot; ++g) {
      int lc;
      std::memcpy(&lc, &p4[g].w, 4);
      cell[g] = uint32_t(lc);
    }
  } else {
    // slots carry the Morton-ordered cell; report the row-major id
    std::vector<uint32_t> lin(D.ncell);
    for (int lid = 0; lid < D.ncell; ++lid) lin[b->cell_rank[D.c0 + lid]] = uint32_t(lid);
    HMD_HIP(ctx, hipMemcpyAsync(cell.data(), b->d_slot_cell, 4 * b->ntot, hipMemcpyDeviceToHost, s));
    HMD_HIP(ctx, hipStreamSynchronize(s));
    for (int64_t g = D.a0; g < D.a0 + D.nf; ++g) cell[g] = lin[cell[g] - uint32_t(D.c0)];
  }
  std::vector<uint32_t> st(D.ncell);
  HMD_HIP(ctx, hipMemcpyAsync(tag.data(), b->d_tag[b->cur], 4 * b->ntot, hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipMemcpyAsync(nc.data(), b->d_ncount + D.c0, 4 * size_t(D.ncell), hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipMemcpyAsync(st.data(), b->d_start + D.c0, 4 * size_t(D.ncell), hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipStreamSynchronize(s));
  if (cell_of)
    for (int i = 0; i < D.nf; ++i) cell_of[tag[D.a0 + i]] = cell[D.a0 + i];
  // counts and members are stored in Morton order of the cells; report them
  // in row-major cell order, members in the library's order inside a cell
  int64_t w = 0;
  for (int lid = 0; lid < D.ncell; ++lid) {
    const uint32_t key = b->cell_rank[D.c0 + lid];
    if (counts) counts[lid] = nc[key];
    for (uint32_t m = 0; m < nc[key]; ++m, ++w)
      if (order) order[w] = uint32_t(tag[st[key] + m]);
  }
  return HMD_OK;
}

int batch_neighbors(hmd_batch* b, int sim, uint32_t* counts, uint32_t* idx, int64_t cap, int64_t* total) {
  hmd_ctx* ctx = b->ctx;
  if (sim < 0 || sim >= b->S || b->path == 0) return HMD_EINVAL;
  const SimDev& D = b->sims[sim];
  std::vector<uint32_t> nl(b->ntot), list(size_t(b->list_cap) * b->list_ld);
  std::vector<int> tag(b->ntot);
  hipStream_t s = ctx->stream;
  // tiled lists hold LDS indices: rebuild them with position indices to read
  // them out, then rebuild them as they were
  if (b->path == 2)
    launch_build(b, s, nullptr, StepRef{nullptr, -1}, state_ref(b, 0), state_ref(b, 0), b->d_tag[0],
                 b->d_tag[0], 1);
  HMD_HIP(ctx, hipMemcpyAsync(nl.data(), b->d_nlist, 4 * b->ntot, hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipMemcpyAsync(list.data(), b->d_list, 4 * list.size(), hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipMemcpyAsync(tag.data(), b->d_tag[0], 4 * b->ntot, hipMemcpyDeviceToHost, s));
  if (b->path == 2)
    launch_build(b, s, nullptr, StepRef{nullptr, -1}, state_ref(b, 0), state_ref(b, 0), b->d_tag[0],
                 b->d_tag[0], 0);
  HMD_HIP(ctx, hipStreamSynchronize(s));
  // per atom id: neighbour ids (fluid ids, or N_f + wall index of the system)
  std::vector<std::vector<uint32_t>> per(D.nf);
  int64_t tot = 0;
  for (int i = 0; i < D.nf; ++i) {
    const int64_t g = D.a0 + i;
    auto& v = per[tag[g]];
    for (uint32_t k = 0; k < nl[g]; ++k) {
      const uint32_t j = list[(size_t(k >> 2) * b->list_ld + size_t(g)) * 4 + (k & 3u)];
      v.push_back(j < uint32_t(b->ntot) ? uint32_t(tag[j])
                                        : uint32_t(D.nf) + uint32_t(b->wall_id[j - uint32_t(b->ntot)]));
    }
    tot += int64_t(v.size());
  }
  int64_t w = 0;
  for (int id = 0; id < D.nf; ++id) {
    auto& v = per[id];
    std::sort(v.begin(), v.end());
    if (counts) counts[id] = uint32_t(v.size());
    for (uint32_t j : v) {
      if (idx && w < cap) idx[w] = j;
      ++w;
    }
  }
  if (total) *total = tot;
  return HMD_OK;
}

int batch_pairs(hmd_batch* b, int64_t* ff, int64_t* wf) {
  hmd_ctx* ctx = b->ctx;
  HMD_TRY(forces_now(b, true));
  unsigned long long h[2] = {0, 0};
  HMD_HIP(ctx, hipMemcpyAsync(h, b->acc.pairs, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  HMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (ff) *ff = int64_t(h[0]);
  if (wf) *wf = int64_t(h[1]);
  return HMD_OK;
}

int batch_list_builds(hmd_batch* b, int64_t* builds) {
  hmd_ctx* ctx = b->ctx;
  int flags[4] = {0, 0, 0, 0};
  HMD_HIP(ctx, hipMemcpyAsync(flags, b->d_flag, sizeof(flags), hipMemcpyDeviceToHost, ctx->stream));
  HMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (builds) *builds = b->path >= 1 ? int64_t(flags[3]) : 0;
  return HMD_OK;
}

int batch_profile(hmd_batch* b, int sim, double* mvx, double* cnt) {
  hmd_ctx* ctx = b->ctx;
  if (sim < 0 || sim >= b->S) return HMD_EINVAL;
  const SimDev& D = b->sims[sim];
  // per-system bins plus, on the tiled path, the system's per-tile bins
  std::vector<double> a(D.nbins), c(D.nbins);
  HMD_HIP(ctx, hipMemcpy(a.data(), b->acc.binvx + D.bin0, 8 * a.size(), hipMemcpyDeviceToHost));
  HMD_HIP(ctx, hipMemcpy(c.data(), b->acc.bincnt + D.bin0, 8 * c.size(), hipMemcpyDeviceToHost));
  if (b->d_tbins) {
    const int t0 = b->tile_first[sim], t1 = b->tile_first[sim + 1];
    std::vector<double> tb(size_t(t1 - t0) * BIN_LDS * 2);
    HMD_HIP(ctx, hipMemcpy(tb.data(), b->d_tbins + size_t(t0) * BIN_LDS * 2, 8 * tb.size(), hipMemcpyDeviceToHost));
    const int nb = std::min(D.nbins, BIN_LDS);
    for (int t = 0; t < t1 - t0; ++t)
      for (int k = 0; k < nb; ++k) {
        a[k] += tb[(size_t(t) * BIN_LDS + k) * 2];
        c[k] += tb[(size_t(t) * BIN_LDS + k) * 2 + 1];
      }
  }
  if (mvx) std::copy(a.begin(), a.end(), mvx);
  if (cnt) std::copy(c.begin(), c.end(), cnt);
  return HMD_OK;
}

}  // namespace hmd
