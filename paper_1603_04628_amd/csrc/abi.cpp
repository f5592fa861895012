// abi.cpp -- extern "C" entry points of libhmd for the MD micro-solve (the
// declarations and their contracts are in include/hmd.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "engine.h"
#include "series.h"

namespace {

// Default graph chunk for whole-run calls: long enough to amortise launch
// gaps, short enough that a remainder runs quickly as direct launches.
constexpr int kDefaultChunk = 100;

template <typename F>
int guarded(hmd_ctx* ctx, F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed";
    return HMD_ENOMEM;
  } catch (...) {
    if (ctx) ctx->err = "internal error";
    return HMD_EDEVICE;
  }
}

}  // namespace

extern "C" {

void hmd_md_params_default(hmd_md_params* p) {
  if (!p) return;
  p->rho = 0.8; p->T0 = 1.0; p->rc = 2.5;
  p->eps_wf = 1.0; p->sigma_wf = 1.0; p->rho_wall = 1.0;
  p->wall_layers = 4; p->thermo_axis = 1;
  p->dt = 0.005; p->tau_T = 0.1;
  p->Lx_nom = 12.0; p->Lz_nom = 12.0; p->bin_dy = 0.25;
  p->n_equil = 0; p->n_blocks = 0; p->n_fluid = 0; p->delta = 1.0;
  p->force_path = -1; p->skin = 0.3; p->cell_w = 0.0;
  p->tile_alpha = 0.0; p->graph_chunk = 0;
  p->pressure = 0;
}

int hmd_create(const hmd_md_params* params, int device, void* hip_stream, hmd_ctx** out) {
  if (!out) return HMD_EINVAL;
  *out = nullptr;
  auto* ctx = new (std::nothrow) hmd_ctx();
  if (!ctx) return HMD_ENOMEM;
  if (params) ctx->params = *params;
  else hmd_md_params_default(&ctx->params);
  ctx->device = device;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    delete ctx;
    return HMD_EDEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return HMD_EDEVICE;
  }
  // the device address of the allocation-free entry point's fixed scratch,
  // looked up once per device
  if (hmd::series_noalloc_init(device, ctx->err) != HMD_OK) {
    delete ctx;
    return HMD_EDEVICE;
  }
  if (hip_stream) {
    ctx->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
      delete ctx;
      return HMD_EDEVICE;
    }
    ctx->own_stream = true;
  }
  *out = ctx;
  return HMD_OK;
}

void hmd_destroy(hmd_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->d_series_scratch) {  // md_series_stats_dev may have used another stream
    (void)hipDeviceSynchronize();
    (void)hipFree(ctx->d_series_scratch);
  }
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char* hmd_last_error(const hmd_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int hmd_get_params(const hmd_ctx* ctx, hmd_md_params* params) {
  if (!ctx || !params) return HMD_EINVAL;
  *params = ctx->params;
  return HMD_OK;
}

int hmd_set_params(hmd_ctx* ctx, const hmd_md_params* params) {
  if (!ctx || !params) return HMD_EINVAL;
  ctx->params = *params;
  return HMD_OK;
}

// ----------------------------------------------------------------- batches
int md_batch_create(hmd_ctx* ctx, const hmd_md_job* jobs, int n, hmd_batch** out) {
  if (!ctx || !jobs || !out) return HMD_EINVAL;
  return guarded(ctx, [&] { return hmd::batch_create(ctx, jobs, n, out); });
}

int md_batch_run(hmd_batch* b, int64_t steps, int graph_chunk) {
  if (!b) return HMD_EINVAL;
  return guarded(b->ctx, [&] { return hmd::batch_run(b, steps, graph_chunk, true, nullptr); });
}

int md_batch_results(hmd_batch* b, hmd_md_result* out) {
  if (!b || !out) return HMD_EINVAL;
  return guarded(b->ctx, [&] { return hmd::batch_results(b, out); });
}

int64_t md_batch_atoms(const hmd_batch* b) { return b ? b->ntot : 0; }

int md_batch_set_timing(hmd_batch* b, int on) {
  if (!b) return HMD_EINVAL;
  b->timing = on != 0;
  for (int k = 0; k < hmd::K_COUNT; ++k) {
    b->kern_ms[k] = 0.0;
    b->kern_n[k] = 0;
  }
  for (int r = 0; r < 2; ++r) {
    b->list_ms[r] = 0.0;
    b->list_n[r] = 0;
  }
  b->graph_ms = 0.0;
  b->graph_steps = 0;
  return HMD_OK;
}

int md_batch_kernel_ms(const hmd_batch* b, const char* kernel, double* ms, int64_t* launches) {
  if (!b || !kernel || !ms) return HMD_EINVAL;
  static const char* names[hmd::K_COUNT] = {"integrate", "scan", "scatter", "reorder", "force", "keys", "list"};
  if (std::strcmp(kernel, "graph_step") == 0) {
    *ms = b->graph_steps ? b->graph_ms / double(b->graph_steps) : 0.0;
    if (launches) *launches = b->graph_steps;
    return HMD_OK;
  }
  for (int r = 0; r < 2; ++r)
    if (std::strcmp(kernel, r ? "list_rebuild" : "list_idle") == 0) {
      *ms = b->list_n[r] ? b->list_ms[r] / double(b->list_n[r]) : 0.0;
      if (launches) *launches = b->list_n[r];
      return HMD_OK;
    }
  for (int k = 0; k < hmd::K_COUNT; ++k)
    if (std::strcmp(kernel, names[k]) == 0) {
      *ms = b->kern_n[k] ? b->kern_ms[k] / double(b->kern_n[k]) : 0.0;
      if (launches) *launches = b->kern_n[k];
      return HMD_OK;
    }
  return HMD_EINVAL;
}

int md_batch_pair_count(hmd_batch* b, int64_t* fluid_pairs, int64_t* wall_pairs) {
  if (!b) return HMD_EINVAL;
  return guarded(b->ctx, [&] { return hmd::batch_pairs(b, fluid_pairs, wall_pairs); });
}

int md_batch_get_state(hmd_batch* b, int sim, double* x, double* v, int64_t* n_fluid) {
  if (!b || sim < 0 || sim >= b->S) return HMD_EINVAL;
  if (n_fluid) *n_fluid = b->sims[sim].nf;
  if (!x && !v) return HMD_OK;
  return guarded(b->ctx, [&] { return hmd::batch_get_state(b, sim, x, v); });
}

int md_batch_forces(hmd_batch* b, int sim, float* f, double* pe) {
  if (!b || sim < 0 || sim >= b->S) return HMD_EINVAL;
  return guarded(b->ctx, [&] { return hmd::batch_forces(b, sim, f, pe); });
}

int md_batch_list_builds(hmd_batch* b, int64_t* builds) {
  if (!b) return HMD_EINVAL;
  return guarded(b->ctx, [&] { return hmd::batch_list_builds(b, builds); });
}

int md_batch_set_state(hmd_batch* b, int sim, const double* x, const double* v) {
  if (!b || sim < 0 || sim >= b->S || !x || !v) return HMD_EINVAL;
  return guarded(b->ctx, [&] { return hmd::batch_set_state(b, sim, x, v); });
}

int md_batch_set_states(hmd_batch* b, int m, const int* sims, const double* const* x, const double* const* v) {
  if (!b || m < 0 || (m > 0 && (!sims || !x || !v))) return HMD_EINVAL;
  return guarded(b->ctx, [&]() -> int {
    std::vector<std::vector<double>> xs(b->S), vs(b->S);
    for (int j = 0; j < m; ++j) {
      const int k = sims[j];
      if (k < 0 || k >= b->S || !x[j] || !v[j] || !xs[k].empty()) {
        b->ctx->err = "md_batch_set_states: bad or repeated system index, or a null array";
        return HMD_EINVAL;
      }
      const size_t n3 = 3 * size_t(b->sims[k].nf);
      xs[k].assign(x[j], x[j] + n3);
      vs[k].assign(v[j], v[j] + n3);
    }
    if (m == 0) return HMD_OK;
    return hmd::batch_set_all_states(b, xs, vs);
  });
}

int md_batch_get_states(hmd_batch* b, double* const* x, double* const* v) {
  if (!b || !x || !v) return HMD_EINVAL;
  return guarded(b->ctx, [&]() -> int {
    std::vector<std::vector<double>> xs, vs;
    HMD_TRY(hmd::batch_get_all_states(b, xs, vs));
    for (int k = 0; k < b->S; ++k) {
      if (x[k]) std::copy(xs[k].begin(), xs[k].end(), x[k]);
      if (v[k]) std::copy(vs[k].begin(), vs[k].end(), v[k]);
    }
    return HMD_OK;
  });
}

int md_batch_series(hmd_batch* b, int sim, double* q, int64_t* n) {
  if (!b) return HMD_EINVAL;
  return guarded(b->ctx, [&] { return hmd::batch_series(b, sim, q, n, 0); });
}

int md_batch_pressure_series(hmd_batch* b, int sim, double* p, int64_t* n) {
  if (!b) return HMD_EINVAL;
  return guarded(b->ctx, [&] { return hmd::batch_series(b, sim, p, n, 1); });
}

void md_batch_free(hmd_batch* b) { hmd::batch_free(b); }

int md_series_stats(hmd_ctx* ctx, const double* x, int S, int64_t n, int64_t ld, int n_blocks, double* out) {
  if (!ctx || !x || !out) return HMD_EINVAL;
  HMD_TRY(hmd::series_stats_check(S, n, ld, n_blocks, ctx->err));
  return guarded(ctx, [&]() -> int {
    HMD_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    double *dx = nullptr, *dg = nullptr, *dout = nullptr;
    auto release = [&] {
      if (dx) (void)hipFree(dx);
      if (dg) (void)hipFree(dg);
      if (dout) (void)hipFree(dout);
    };
    const size_t nx = size_t(S) * size_t(ld), ng = n_blocks == 0 ? size_t(S) * size_t(n) : 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&dx), 8 * nx);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&dg), 8 * ng);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&dout), 8 * 4 * size_t(S));
    if (e == hipSuccess) e = hipMemcpyAsync(dx, x, 8 * nx, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      hmd::series_stats_enqueue(s, dx, S, n, ld, 1.0, n_blocks, dg, dout);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, 8 * 4 * size_t(S), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    release();
    if (e != hipSuccess) {
      ctx->err = std::string("md_series_stats: ") + hipGetErrorString(e);
      return e == hipErrorOutOfMemory ? HMD_ENOMEM : HMD_EDEVICE;
    }
    return HMD_OK;
  });
}

int md_series_stats_dev(hmd_ctx* ctx, const double* d_x, int S, int64_t n, int64_t ld, int n_blocks, double* d_out,
                        void* stream) {
  if (!ctx || !d_x || !d_out) return HMD_EINVAL;
  HMD_TRY(hmd::series_stats_check(S, n, ld, n_blocks, ctx->err));
  return guarded(ctx, [&]() -> int {
    HMD_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
    const int64_t need = n_blocks == 0 ? int64_t(S) * n : 1;
    if (need > ctx->series_scratch_n) {  // grows; earlier work on the scratch must be done first
      HMD_HIP(ctx, hipDeviceSynchronize());
      if (ctx->d_series_scratch) HMD_HIP(ctx, hipFree(ctx->d_series_scratch));
      ctx->d_series_scratch = nullptr;
      ctx->series_scratch_n = 0;
      HMD_HIP(ctx, hipMalloc(reinterpret_cast<void**>(&ctx->d_series_scratch), 8 * size_t(need)));
      ctx->series_scratch_n = need;
    }
    hmd::series_stats_enqueue(s, d_x, S, n, ld, 1.0, n_blocks, ctx->d_series_scratch, d_out);
    HMD_HIP(ctx, hipGetLastError());
    return HMD_OK;
  });
}

int md_flux_batch(hmd_ctx* ctx, const hmd_md_job* jobs, int n, hmd_md_result* out) {
  if (!ctx || !jobs || !out || n < 1) {
    if (ctx) ctx->err = "md_flux_batch: null argument or n < 1";
    return HMD_EINVAL;
  }
  return guarded(ctx, [&]() -> int {
    // one batch per distinct sampling length
    std::map<int64_t, std::vector<int>> groups;
    for (int k = 0; k < n; ++k) {
      if (jobs[k].n_sample < std::max(2, ctx->params.n_blocks)) {
        ctx->err = "md_flux_batch: n_sample must be at least max(2, n_blocks)";
        return HMD_EINVAL;
      }
      groups[jobs[k].n_sample].push_back(k);
    }
    for (auto& kv : groups) {
      std::vector<hmd_md_job> sub;
      for (int k : kv.second) sub.push_back(jobs[k]);
      hmd_batch* b = nullptr;
      int rc = hmd::batch_create(ctx, sub.data(), int(sub.size()), &b);
      if (rc != HMD_OK) return rc;
      rc = hmd::batch_run(b, ctx->params.n_equil + kv.first, b->chunk, true, nullptr);
      std::vector<hmd_md_result> res(sub.size());
      if (rc == HMD_OK) rc = hmd::batch_results(b, res.data());
      hmd::batch_free(b);
      if (rc != HMD_OK) return rc;
      for (size_t j = 0; j < sub.size(); ++j) out[kv.second[j]] = res[j];
    }
    return HMD_OK;
  });
}

int md_flux_batch_dev(hmd_ctx* ctx, const hmd_md_job* jobs, int n, double* d_flux, double* d_se, int* d_status,
                      void* stream) {
  if (!ctx || !jobs || n < 1 || !d_flux || !d_se || !d_status) {
    if (ctx) ctx->err = "md_flux_batch_dev: null argument or n < 1";
    return HMD_EINVAL;
  }
  std::vector<hmd_md_result> res(n);
  int rc = md_flux_batch(ctx, jobs, n, res.data());
  if (rc != HMD_OK) return rc;
  std::vector<double> f(n), se(n);
  std::vector<int> st(n);
  for (int k = 0; k < n; ++k) {
    f[k] = res[k].flux;
    se[k] = res[k].flux_se;
    st[k] = res[k].status;
  }
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
  HMD_HIP(ctx, hipMemcpyAsync(d_flux, f.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  HMD_HIP(ctx, hipMemcpyAsync(d_se, se.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  HMD_HIP(ctx, hipMemcpyAsync(d_status, st.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
  HMD_HIP(ctx, hipStreamSynchronize(s));  // the host staging arrays end here
  return HMD_OK;
}

int md_flux(hmd_ctx* ctx, double h, double g, uint64_t seed, int64_t steps, double* flux, double* se) {
  if (!ctx) return HMD_EINVAL;
  hmd_md_job job{h, g, seed, steps};
  hmd_md_result r{};
  const int rc = md_flux_batch(ctx, &job, 1, &r);
  if (rc != HMD_OK) return rc;
  if (flux) *flux = r.flux;
  if (se) *se = r.flux_se;
  return r.status;
}

// ----------------------------------------------------------- single system
int md_sys_create(hmd_ctx* ctx, double h, double g, uint64_t seed, hmd_sys** out) {
  if (!ctx || !out) return HMD_EINVAL;
  return guarded(ctx, [&]() -> int {
    hmd_md_job job{h, g, seed, 0};
    hmd_batch* b = nullptr;
    const int rc = hmd::batch_create(ctx, &job, 1, &b);
    if (rc != HMD_OK) return rc;
    auto* s = new hmd_sys();
    s->b = b;
    *out = s;
    return HMD_OK;
  });
}

int md_sys_info(hmd_sys* s, int64_t* n_fluid, int64_t* n_wall, double box[3], int ncell[3]) {
  if (!s) return HMD_EINVAL;
  const hmd::HostSystem& H = s->b->host[0];
  if (n_fluid) *n_fluid = H.nf;
  if (n_wall) *n_wall = H.nw;
  if (box) { box[0] = H.Lx; box[1] = H.h; box[2] = H.Lz; }
  if (ncell) { ncell[0] = H.nx; ncell[1] = H.ny; ncell[2] = H.nz; }
  return HMD_OK;
}

int md_set_state(hmd_sys* s, const double* x, const double* v) {
  if (!s || !x || !v) return HMD_EINVAL;
  return guarded(s->b->ctx, [&] { return hmd::batch_set_state(s->b, 0, x, v); });
}

int md_get_state(hmd_sys* s, double* x, double* v, int64_t* n_fluid) {
  if (!s) return HMD_EINVAL;
  if (n_fluid) *n_fluid = s->b->host[0].nf;
  return guarded(s->b->ctx, [&] { return hmd::batch_get_state(s->b, 0, x, v); });
}

int md_compute_forces(hmd_sys* s, float* f, double* pe) {
  if (!s) return HMD_EINVAL;
  return guarded(s->b->ctx, [&] { return hmd::batch_forces(s->b, 0, f, pe); });
}

int md_cell_lists(hmd_sys* s, uint32_t* cell_of_atom, uint32_t* cell_count, uint32_t* order) {
  if (!s) return HMD_EINVAL;
  return guarded(s->b->ctx, [&] { return hmd::batch_cells(s->b, 0, cell_of_atom, cell_count, order); });
}

int md_run(hmd_sys* s, int64_t steps, int thermostat_on, double* energy_trace) {
  if (!s) return HMD_EINVAL;
  return guarded(s->b->ctx, [&] {
    return hmd::batch_run(s->b, steps, energy_trace ? 0 : kDefaultChunk, thermostat_on != 0, energy_trace);
  });
}

int md_sys_profile(hmd_sys* s, double* mvx, double* cnt) {
  if (!s) return HMD_EINVAL;
  return guarded(s->b->ctx, [&] { return hmd::batch_profile(s->b, 0, mvx, cnt); });
}

int md_neighbor_lists(hmd_sys* s, uint32_t* counts, uint32_t* idx, int64_t cap, int64_t* total) {
  if (!s) return HMD_EINVAL;
  return guarded(s->b->ctx, [&] { return hmd::batch_neighbors(s->b, 0, counts, idx, cap, total); });
}

int md_sys_config(hmd_sys* s, int* path, double* skin, int* tpb, int* list_cap) {
  if (!s) return HMD_EINVAL;
  return md_batch_config(s->b, path, skin, tpb, list_cap);
}

void md_sys_free(hmd_sys* s) {
  if (!s) return;
  hmd::batch_free(s->b);
  delete s;
}

}  // extern "C"
