// engine.h -- internal types of libhmd (context, MD batch, device layout).
#pragma once

#include <hip/hip_runtime.h>

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
  int force_variant = -1;  // -1: pick per batch; otherwise a fixed force kernel variant
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

// Per-system constants read by every kernel (device copy, one per system).
struct SimDev {
  double Lx, Lz, h;
  double inv_x, inv_y, inv_z;  // n_a / L_a: cell rule floor(x * inv)
  double wx, wy, wz;           // cell widths
  double g;                    // body-force acceleration along +x
  double inv_area;             // 1 / (Lx Lz)
  double inv_bin;              // 1 / bin width
  double inv_nf;               // 1 / N_f
  float fwx, fwy, fwz, fpad;   // FP32 cell widths (neighbour-cell shifts)
  int nx, ny, nz;
  int a0, nf;                  // fluid slots [a0, a0 + nf)
  int c0, ncell;               // global fluid cells [c0, c0 + ncell)
  int wc0;                     // wall columns [wc0, wc0 + 2 nx nz)
  int nbins, bin0;             // profile bins [bin0, bin0 + nbins)
  int pad;
};

// Step constants passed by value.
struct StepConst {
  double dt, hdt, dt_tau, T0;
  float rc2, eps_wf, sig2_wf, ush_ff, ush_wf;
  int axis;        // thermostatted velocity component
  int nb, B, r;    // SE blocks, block length, samples dropped at the front
  int thermo_on;   // thermostat active in this run
  int bins_on;     // accumulate the wall-normal profile
  int energy_on;   // accumulate potential and kinetic energy
};

// Per-system FP64 accumulators (device).
struct Acc {
  double* vc2[2];   // sum v_c^2 after the second half-kick, by step parity
  double* pe[2];    // sum of per-atom potential energy, by step parity
  double* ke[2];    // sum |v|^2 after the second half-kick, by step parity
  double* blocks;   // [S * nb] block sums of q'
  double* tsum;     // [S * 3] sums of T_a over sampled steps
  double* binvx;    // [bins] sum v_x
  double* bincnt;   // [bins] counts
  int* status;      // [S] bit 0: unstable
  unsigned long long* pairs;  // [2] in-cutoff fluid-fluid (ordered) and wall-fluid pairs
};

enum Kern { K_INTEGRATE = 0, K_SCAN, K_SCATTER, K_REORDER, K_FORCE, K_COUNT };

}  // namespace hmd

struct hmd_batch {
  hmd_ctx* ctx = nullptr;
  hmd_md_params P{};
  int S = 0;
  int64_t n_sample = 0;
  std::vector<hmd::HostSystem> host;  // geometry (atom arrays released after upload)
  std::vector<hmd::SimDev> sims;
  int64_t ntot = 0, ncell = 0, nwall = 0, nwcell = 0, nbins = 0;
  int force_variant = 0;

  // device buffers
  hmd::SimDev* d_sims = nullptr;
  uint16_t* d_atom_sim = nullptr;   // slot -> system
  uint16_t* d_cell_sim = nullptr;   // global fluid cell -> system
  double* d_state[2][6] = {};       // x y z vx vy vz, ping-pong
  int* d_tag[2] = {};               // atom id within its system
  float4* d_f4 = nullptr;           // force (w: potential energy) per slot
  float4* d_pos4 = nullptr;         // cell-relative FP32 position (w: local cell id bits)
  uint32_t* d_key = nullptr;        // global cell of each slot
  uint32_t* d_count = nullptr;      // atomic counters per cell
  uint32_t* d_cursor = nullptr;     // scatter cursors per cell
  uint32_t* d_start = nullptr;      // first slot of each cell
  uint32_t* d_ncount = nullptr;     // atoms per cell after the sort
  uint32_t* d_perm = nullptr;       // scatter target -> source slot
  uint32_t* d_rank = nullptr;       // arrival rank of each slot inside its new cell
  float4* d_wpos4 = nullptr;        // wall atoms, column order, column-relative
  uint32_t* d_wstart = nullptr;
  uint32_t* d_wcount = nullptr;
  int64_t* d_dstate = nullptr;      // done, n_equil, sampled_upto, lambda pending
  hmd::Acc acc{};
  double* d_accbuf = nullptr;
  int* d_status = nullptr;

  int cur = 0;  // which state buffer is current
  int64_t done = 0, sampled_upto = 0;
  bool pending = false;
  bool thermo_on = true;

  std::map<int, hipGraphExec_t> graphs;  // chunk length -> executable graph
  std::map<int, hipGraph_t> graph_defs;
  std::map<int, std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>>> graph_marks;

  bool timing = false;
  std::vector<hipEvent_t> ev;             // event pool for timing
  double kern_ms[hmd::K_COUNT] = {};
  int64_t kern_n[hmd::K_COUNT] = {};
  double graph_ms = 0.0;     // timed graph replays
  int64_t graph_steps = 0;
};

struct hmd_sys {
  hmd_batch* b = nullptr;
};

namespace hmd {
struct StepConst;
void launch_force(hmd_batch* b, hipStream_t s, int mode, const StepConst& K);
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
}  // namespace hmd
