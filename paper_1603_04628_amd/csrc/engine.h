// engine.h -- internal types of libhmd (context, MD batch, device layout).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "hmd.h"
#include "md_setup.h"

struct hmd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hmd_md_params params{};
  std::string err;
  // tuned choices keyed by a workload signature (see tune.cpp)
  std::map<std::string, std::vector<double>> tuned;
  // device scratch of md_series_stats_dev (autocovariances), grown on demand
  double* d_series_scratch = nullptr;
  int64_t series_scratch_n = 0;
};

namespace hmd {

// Returns from the enclosing int-returning function on a HIP error.
#define HMD_HIP(ctx, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);                   \
      return e_ == hipErrorOutOfMemory ? HMD_ENOMEM : HMD_EDEVICE;                      \
    }                                                                                   \
  } while (0)

#define HMD_TRY(expr)              \
  do {                             \
    int rc_ = (expr);              \
    if (rc_ != HMD_OK) return rc_; \
  } while (0)

// Per-system constants read by every kernel (device copy, one per system).
struct SimDev {
  double Lx, Lz, h;
  double inv_x, inv_y, inv_z;  // n_a / L_a: cell rule floor(x * inv)
  double wx, wy, wz;           // cell widths
  double g;                    // body-force acceleration along +x
  double inv_area;             // 1 / (Lx Lz)
  double inv_bin;              // 1 / bin width
  double inv_nf;               // 1 / N_f
  double fix_x, fix_y, fix_z;  // fixed-point scales (2^32 per extent)
  double y_lo;                 // fixed-point origin in y
  float unit_x, unit_y, unit_z;  // length of one fixed-point unit
  float inv_u, inv_u2;         // 1 / unit_x and its square (same unit on every axis: uniform scale)
  float fwx, fwy, fwz;         // FP32 cell widths (neighbour-cell shifts)
  int nx, ny, nz;
  int a0, nf;                  // fluid slots [a0, a0 + nf)
  int c0, ncell;               // global fluid cells [c0, c0 + ncell)
  int wc0;                     // wall columns [wc0, wc0 + 2 nx nz)
  int w0;                      // wall atoms [w0, w0 + nw) of the wall arrays
  int nbins, bin0;             // profile bins [bin0, bin0 + nbins)
  // Cells are numbered in Morton (Z) order of their coordinates so that
  // consecutive slots form compact 3-D clusters: rank maps the row-major
  // cell id (cz ny + cy) nx + cx to its place in that order, lin inverts it.
  const uint32_t* rank;
  const uint32_t* lin;
};

// Step constants passed by value.
struct StepConst {
  double dt, hdt, dt_tau, T0;
  int64_t n_equil;
  float rc2, eps_wf, sig2_wf, ush_ff, ush_wf, half_skin2;
  int axis;        // thermostatted velocity component
  int nb, B, r;    // SE blocks, block length, samples dropped at the front
  int thermo_on;   // thermostat active in this run
  int bins_on;     // accumulate the wall-normal profile
  int energy_on;   // accumulate potential and kinetic energy
  int press_on;    // sampled steps also record the wall normal pressure
};

// Per-system FP64 accumulators (device).
struct Acc {
  double* vc2[2];   // sum v_c^2 after the second half-kick, by step parity
  double* pe[2];    // sum of per-atom potential energy, by step parity
  double* ke[2];    // sum |v|^2 after the second half-kick, by step parity
  double* blocks;   // [S * nb] the sampled q' series: entry k of a system holds the sum of
                    // B consecutive steps' q' (B = 1 unless n_sample exceeds the series cap)
  double* pblocks;  // [S * nb] the sampled wall-pressure series, laid out as blocks
  double* tsum;     // [S * 3] sums of T_a over sampled steps
  double* binvx;    // [bins] sum v_x
  double* bincnt;   // [bins] counts
  double* tbins;    // [tiles * BIN_LDS * 2] the tiled path's bins: (sum v_x, count) per tile and bin,
                    // each tile adding to its own (no atomics; summed per system when read)
  int* status;      // [S] bit 0: unstable
  unsigned long long* pairs;  // [2] in-cutoff fluid-fluid (ordered) and wall-fluid pairs
};

enum Kern { K_INTEGRATE = 0, K_SCAN, K_SCATTER, K_REORDER, K_FORCE, K_KEYS, K_LIST, K_COUNT };
constexpr int kStampedSteps = 10;  // steps per stamped graph replay whose kernels are stamped
constexpr int kStampEvery = 10;    // in timing mode, one replay in this many is the stamped graph
constexpr int kMaxStamps = 96;     // stamps of one timed replay (kernels + 1 per stamped step, + 1)

}  // namespace hmd

struct hmd_batch {
  hmd_ctx* ctx = nullptr;
  hmd_md_params P{};
  int S = 0;
  int64_t n_sample = 0;
  // sampled series per system: nser entries of ser_B steps each, the first
  // ser_r sampled steps left out (ser_B = 1 and ser_r = 0 up to the cap)
  int64_t nser = 1;
  int ser_B = 1 << 30, ser_r = 0;
  double* d_gam = nullptr;   // [S * nser] autocovariances (results)
  double* d_sout = nullptr;  // [S * 4] mean, SE, half means (results)
  int path = 1;           // 0 cell path, 1 pair path
  int tpb = 256;          // threads per block of the per-slot kernels
  double skin = 0.3;
  double tile_alpha = 0.0;  // tiled path: weight of staged atoms in the tile choice
  double cell_w = 0.0;      // cell width parameter in use
  int chunk = 100;          // graph chunk of whole-run calls
  int list_cap = 0, list_ld = 0;
  bool uniform = false;   // one fixed-point unit on all axes in every system
  bool walls_same = false;  // wall-fluid LJ parameters equal the fluid's
  bool force_gather = false;  // tiled path: every tile on the gather fallback
  std::vector<hmd::HostSystem> host;  // geometry (atom arrays released after upload)
  std::vector<int> wall_id;           // wall slot (column order) -> wall id within its system
  std::vector<uint32_t> cell_rank;    // per system, concatenated: row-major cell id -> Morton rank
  uint32_t* d_cellmap = nullptr;      // device copies: rank tables, then inverse tables
  std::vector<hmd::SimDev> sims;
  int64_t ntot = 0, ncell = 0, nwall = 0, nwcell = 0, nbins = 0;

  // device buffers
  hmd::SimDev* d_sims = nullptr;
  uint16_t* d_atom_sim = nullptr;   // slot -> system
  uint16_t* d_cell_sim = nullptr;   // global fluid cell -> system
  double* d_state[2][6] = {};       // x y z vx vy vz: current copy and reorder target
  int* d_tag[2] = {};               // atom id within its system
  float4* d_f4 = nullptr;           // force (w: potential energy) per slot
  float4* d_pos4 = nullptr;         // cell path: cell-relative FP32 position (w: local cell id bits)
  int4* d_pfix = nullptr;           // pair path: fixed-point positions, fluid slots then wall atoms
  int4* d_pbuild = nullptr;         // pair path: positions at the last list build
  uint32_t* d_slot_cell = nullptr;  // pair path: cell of each slot at the last build
  uint32_t* d_list = nullptr;       // pair path: list_cap x list_ld entries
  int4* d_tiles = nullptr;          // tiled path: (system, z slab, first column, columns) per workgroup
  uint32_t* d_tilerec = nullptr;    // tiled path: range table and list mode per tile, written by each list build
  double* d_tbins = nullptr;        // tiled path: profile bins per tile (Acc::tbins)
  std::vector<int> tile_first;      // tiled path: first tile of each system (S + 1 entries)
  int ntiles = 0, stage_cap = 0;    // tiles; LDS capacity in atoms
  uint32_t* d_nlist = nullptr;
  int* d_flag = nullptr;            // [2] rebuild flags by step parity, list overflow, builds so far
  uint32_t* d_key = nullptr;        // global cell of each slot
  uint32_t* d_count = nullptr;      // atomic counters per cell
  uint32_t* d_rank = nullptr;       // arrival rank of each slot inside its new cell
  uint32_t* d_start = nullptr;      // first slot of each cell
  uint32_t* d_ncount = nullptr;     // atoms per cell after the sort
  uint32_t* d_perm = nullptr;       // scatter target -> source slot
  float4* d_wpos4 = nullptr;        // wall atoms, column order, column-relative
  uint32_t* d_wstart = nullptr;
  uint32_t* d_wcount = nullptr;
  int64_t* d_dstate = nullptr;      // [0] steps done at a graph's start, [3] Berendsen factor pending
  hmd::Acc acc{};
  double* d_accbuf = nullptr;
  int* d_status = nullptr;

  int cur = 0;  // cell path: which state copy is current (pair path: always 0)
  int64_t done = 0;
  bool pending = false;
  bool thermo_on = true;

  std::map<int, hipGraphExec_t> graphs;  // key -> executable graph
  std::map<int, hipGraph_t> graph_defs;
  // timed graphs: (kernel, stamp before, stamp after) of the stamped steps
  std::map<int, std::vector<std::array<int, 3>>> graph_spans;
  std::map<int, int> graph_nstamps;
  unsigned long long* d_stamps = nullptr;  // [kMaxStamps] wall-clock stamps of a timed replay
  double clock_khz = 0.0;                  // device wall-clock rate

  bool timing = false;
  std::vector<hipEvent_t> ev;             // event pool for timing
  double kern_ms[hmd::K_COUNT] = {};
  int64_t kern_n[hmd::K_COUNT] = {};
  double list_ms[2] = {};   // stamped list-build time on steps without / with a rebuild
  int64_t list_n[2] = {};
  double graph_ms = 0.0;     // timed graph replays
  int64_t graph_steps = 0;
};

struct hmd_sys {
  hmd_batch* b = nullptr;
};

namespace hmd {
int batch_create(hmd_ctx* ctx, const hmd_md_job* jobs, int n, hmd_batch** out);
int batch_run(hmd_batch* b, int64_t steps, int graph_chunk, bool thermostat, double* energy_trace);
int batch_results(hmd_batch* b, hmd_md_result* out);
void batch_free(hmd_batch* b);
int batch_get_state(hmd_batch* b, int sim, double* x, double* v);
int batch_set_state(hmd_batch* b, int sim, const double* x, const double* v);
int batch_forces(hmd_batch* b, int sim, float* f, double* pe);
int batch_cells(hmd_batch* b, int sim, uint32_t* cell_of, uint32_t* counts, uint32_t* order);
int batch_profile(hmd_batch* b, int sim, double* mvx, double* cnt);
int batch_pairs(hmd_batch* b, int64_t* ff, int64_t* wf);
int batch_list_builds(hmd_batch* b, int64_t* builds);
int batch_series(hmd_batch* b, int sim, double* q, int64_t* n, int which);
int batch_neighbors(hmd_batch* b, int sim, uint32_t* counts, uint32_t* idx, int64_t cap, int64_t* total);
// Implementation choices of a batch.
struct Config {
  int path = 2;
  double skin = 0.3;
  int tpb = 256;
  double tile_alpha = 0.0;
  double cell_w = 0.0;
  int chunk = 100;
};
// Resolved implementation choices for a batch of these jobs on this context.
Config choose_config(hmd_ctx* ctx, const hmd_md_job* jobs, int n);
// Graph chunk of whole-run calls for these jobs.
int run_chunk(hmd_ctx* ctx, const hmd_md_job* jobs, int n);
// The state of every system at once (atom id order, one download), and its
// inverse (one upload; a system given empty vectors keeps its state).
int batch_get_all_states(hmd_batch* b, std::vector<std::vector<double>>& x, std::vector<std::vector<double>>& v);
int batch_set_all_states(hmd_batch* b, const std::vector<std::vector<double>>& x,
                         const std::vector<std::vector<double>>& v);
}  // namespace hmd
