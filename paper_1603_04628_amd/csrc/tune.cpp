// tune.cpp -- implementation choices of a batch (force path, pair-list skin,
// threads per block, tile size, cell width, graph chunk) and the autotuner
// that picks them by timing the actual jobs.  Results are cached in the
// context under a workload signature: the number of systems, the total fluid
// atoms (to a factor of 2), the periodic box and the mean channel height (to
// 1 sigma).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "engine.h"

namespace hmd {

namespace {

constexpr int kDefaultChunk = 100;

std::string signature(const hmd_ctx* ctx, const hmd_md_job* jobs, int n) {
  const hmd_md_params& P = ctx->params;
  double hsum = 0.0, atoms = 0.0;
  for (int k = 0; k < n; ++k) {
    hsum += jobs[k].h;
    atoms += P.rho * P.Lx_nom * P.Lz_nom * jobs[k].h;
  }
  char buf[160];
  std::snprintf(buf, sizeof(buf), "n%d_a%d_L%.1fx%.1f_h%.0f_rc%.2f", n, int(std::log2(atoms + 1.0)), P.Lx_nom,
                P.Lz_nom, hsum / n, P.rc);
  return buf;
}

// ctx->tuned layout: path, skin, tpb, tile_alpha, cell_w, chunk
std::vector<double> pack(const Config& c) {
  return {double(c.path), c.skin, double(c.tpb), c.tile_alpha, c.cell_w, double(c.chunk)};
}

}  // namespace

Config choose_config(hmd_ctx* ctx, const hmd_md_job* jobs, int n) {
  const hmd_md_params& P = ctx->params;
  Config c;
  c.path = 2;  // LDS-staged tiles unless tuned or asked otherwise
  c.skin = P.skin > 0.0 ? P.skin : 0.3;
  c.tpb = 256;
  c.tile_alpha = P.tile_alpha;
  c.cell_w = P.cell_w;
  c.chunk = P.graph_chunk > 0 ? P.graph_chunk : kDefaultChunk;
  if (P.force_path >= 0 && P.force_path <= 3) {
    c.path = P.force_path;
    return c;
  }
  auto it = ctx->tuned.find(signature(ctx, jobs, n));
  if (it != ctx->tuned.end() && it->second.size() >= 6) {
    const std::vector<double>& t = it->second;
    c.path = int(t[0]);
    c.skin = t[1];
    c.tpb = int(t[2]);
    c.tile_alpha = t[3];
    c.cell_w = t[4];
    c.chunk = int(t[5]);
  }
  return c;
}

int run_chunk(hmd_ctx* ctx, const hmd_md_job* jobs, int n) { return choose_config(ctx, jobs, n).chunk; }

}  // namespace hmd

using namespace hmd;

extern "C" {

int md_autotune(hmd_ctx* ctx, const hmd_md_job* jobs, int n, int probe_steps, double* table, int* n_rows) {
  if (!ctx || !jobs || n < 1 || probe_steps < 2) {
    if (ctx) ctx->err = "md_autotune: need jobs and probe_steps >= 2";
    return HMD_EINVAL;
  }
  const std::string sig = signature(ctx, jobs, n);
  const hmd_md_params saved = ctx->params;
  const int steps = (probe_steps + 1) & ~1;
  // probe without the sampling schedule: open-ended runs
  std::vector<hmd_md_job> probe(jobs, jobs + n);
  for (auto& j : probe) j.n_sample = 0;
  auto restore = [&](int rc) {
    ctx->params = saved;
    return rc;
  };

  // warm-up: the default configuration from the start lattice, then the
  // warmed state of every system is the start of each candidate
  std::vector<std::vector<double>> wx(n), wv(n);
  {
    ctx->params.force_path = -1;
    ctx->tuned.erase(sig);
    hmd_batch* b = nullptr;
    int rc = batch_create(ctx, probe.data(), n, &b);
    if (rc == HMD_OK) rc = batch_run(b, steps, std::min(kDefaultChunk, steps), true, nullptr);
    if (rc == HMD_OK) rc = batch_get_all_states(b, wx, wv);
    if (b) batch_free(b);
    if (rc != HMD_OK) return restore(rc);
  }

  int row = 0;
  const int max_rows = 64;
  // time one candidate: ms per step over `steps` graph-replayed steps
  auto time_cand = [&](const Config& c, double* ms) -> int {
    ctx->params.force_path = -1;
    ctx->tuned[sig] = pack(c);
    hmd_batch* b = nullptr;
    int rc = batch_create(ctx, probe.data(), n, &b);
    if (rc != HMD_OK) return rc;
    rc = batch_set_all_states(b, wx, wv);
    const int chunk = std::min(c.chunk, steps) & ~1;
    if (rc == HMD_OK) rc = batch_run(b, chunk, chunk, true, nullptr);  // capture the graph
    if (rc == HMD_OK) {
      HMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
      const auto t0 = std::chrono::steady_clock::now();
      rc = batch_run(b, steps, chunk, true, nullptr);
      *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / steps;
    }
    batch_free(b);
    if (rc == HMD_OK && table && row < max_rows) {
      double* t = table + 7 * row;
      t[0] = c.path; t[1] = c.skin; t[2] = c.tpb; t[3] = c.tile_alpha; t[4] = c.cell_w; t[5] = c.chunk;
      t[6] = *ms;
    }
    if (rc == HMD_OK) ++row;
    return rc;
  };

  Config best;
  best.path = 2;
  best.skin = 0.35;
  best.tpb = 256;
  best.tile_alpha = 0.0;
  best.cell_w = 0.0;
  best.chunk = kDefaultChunk;
  double best_ms = 1e300;
  auto axis = [&](std::vector<Config> cands) -> int {
    for (const Config& c : cands) {
      double ms = 1e300;
      const int rc = time_cand(c, &ms);
      if (rc != HMD_OK) return rc;
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    return HMD_OK;
  };
  auto vary = [&](auto set, const std::vector<double>& vals) {
    std::vector<Config> out;
    for (double v : vals) {
      Config c = best;
      set(c, v);
      out.push_back(c);
    }
    return out;
  };
  int rc = HMD_OK;
  // 1. force path and threads per block (the path's own default skin)
  {
    std::vector<Config> cands;
    for (int path : {2, 1, 0})
      for (int tpb : {256, 128}) {
        if (path == 2 && tpb == 128) continue;
        if (path == 0 && saved.pressure) continue;  // the wall pressure needs a pair path
        Config c = best;
        c.path = path;
        c.tpb = tpb;
        cands.push_back(c);
      }
    rc = axis(cands);
  }
  // 2. skin (pair paths only)
  if (rc == HMD_OK && best.path >= 1)
    rc = axis(vary([](Config& c, double v) { c.skin = v; }, {0.25, 0.30, 0.40, 0.45}));
  // 3. tile size (tiled path)
  if (rc == HMD_OK && best.path == 2)
    rc = axis(vary([](Config& c, double v) { c.tile_alpha = v; }, {0.25, 0.5, 1.0}));
  // 4. cell width beyond the minimum
  if (rc == HMD_OK) {
    const double wmin = saved.rc + (best.path >= 1 ? best.skin : 0.0);
    rc = axis(vary([](Config& c, double v) { c.cell_w = v; }, {1.1 * wmin, 1.25 * wmin}));
  }
  // 5. graph chunk of whole-run calls
  if (rc == HMD_OK)
    rc = axis(vary([](Config& c, double v) { c.chunk = int(v); }, {20.0, 50.0, 200.0}));
  if (rc != HMD_OK) {
    ctx->tuned.erase(sig);
    return restore(rc);
  }
  ctx->params = saved;
  ctx->tuned[sig] = pack(best);
  if (n_rows) *n_rows = row;
  return HMD_OK;
}

int md_batch_config(const hmd_batch* b, int* path, double* skin, int* tpb, int* list_cap) {
  if (!b) return HMD_EINVAL;
  if (path) *path = b->path;
  if (skin) *skin = b->skin;
  if (tpb) *tpb = b->tpb;
  if (list_cap) *list_cap = b->list_cap;
  return HMD_OK;
}

int md_batch_tuning(const hmd_batch* b, double out[8]) {
  if (!b || !out) return HMD_EINVAL;
  out[0] = b->path;
  out[1] = b->skin;
  out[2] = b->tpb;
  out[3] = b->tile_alpha;
  out[4] = b->sims.empty() ? 0.0 : b->sims[0].wx;
  out[5] = b->chunk;
  out[6] = b->ntiles;
  out[7] = b->list_cap;
  return HMD_OK;
}

}  // extern "C"
