// tune.cpp -- implementation choices for a batch (force path, pair-list
// skin, threads per block) and the autotuner that picks them by timing short
// probe runs of the actual jobs.  Results are cached in the context under a
// workload signature: the number of systems, the total fluid atoms (to a
// factor of 2), the periodic box and the mean channel height (to 1 sigma).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "engine.h"

namespace hmd {

namespace {

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

}  // namespace

void choose_path(hmd_ctx* ctx, const hmd_md_job* jobs, int n, int* path, double* skin, int* tpb) {
  const hmd_md_params& P = ctx->params;
  *path = 2;  // LDS-staged tiles unless tuned or asked otherwise
  *skin = P.skin > 0.0 ? P.skin : 0.3;
  *tpb = 256;
  if (P.force_path >= 0 && P.force_path <= 3) {
    *path = P.force_path;
    return;
  }
  auto it = ctx->tuned.find(signature(ctx, jobs, n));
  if (it != ctx->tuned.end() && it->second.size() >= 3) {
    *path = int(it->second[0]);
    *skin = it->second[1];
    *tpb = int(it->second[2]);
  }
}

}  // namespace hmd

using namespace hmd;

extern "C" {

int md_autotune(hmd_ctx* ctx, const hmd_md_job* jobs, int n, int probe_steps, double* table, int* n_rows) {
  if (!ctx || !jobs || n < 1 || probe_steps < 2) return HMD_EINVAL;
  const std::string sig = signature(ctx, jobs, n);
  struct Cand {
    int path;
    double skin;
    int tpb;
  };
  std::vector<Cand> cands = {{0, 0.0, 128}, {0, 0.0, 256}, {1, 0.2, 256}, {1, 0.3, 128}, {1, 0.3, 256},
                             {1, 0.4, 256}, {1, 0.5, 256}, {2, 0.3, 256}, {2, 0.4, 256}, {2, 0.5, 256}};
  const hmd_md_params saved = ctx->params;
  // probe without the sampling schedule: open-ended runs
  std::vector<hmd_md_job> probe(jobs, jobs + n);
  for (auto& j : probe) j.n_sample = 0;
  const int chunk = std::min(100, probe_steps) & ~1;
  double best = 1e300;
  Cand pick = cands[2];
  int row = 0;
  for (const Cand& c : cands) {
    ctx->params.force_path = -1;
    ctx->tuned[sig] = {double(c.path), c.skin > 0.0 ? c.skin : saved.skin, double(c.tpb)};
    hmd_batch* b = nullptr;
    int rc = batch_create(ctx, probe.data(), n, &b);
    if (rc != HMD_OK) {
      ctx->params = saved;
      ctx->tuned.erase(sig);
      return rc;
    }
    double ms = 1e300;
    rc = batch_run(b, std::max(2, probe_steps / 4) & ~1, chunk, true, nullptr);  // warm-up
    if (rc == HMD_OK) {
      const auto t0 = std::chrono::steady_clock::now();
      rc = batch_run(b, probe_steps, chunk, true, nullptr);
      ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / probe_steps;
    }
    batch_free(b);
    if (rc != HMD_OK) {
      ctx->params = saved;
      ctx->tuned.erase(sig);
      return rc;
    }
    if (table) {
      table[4 * row + 0] = c.path;
      table[4 * row + 1] = c.skin;
      table[4 * row + 2] = c.tpb;
      table[4 * row + 3] = ms;
    }
    ++row;
    if (ms < best) {
      best = ms;
      pick = c;
    }
  }
  ctx->params = saved;
  ctx->tuned[sig] = {double(pick.path), pick.skin > 0.0 ? pick.skin : saved.skin, double(pick.tpb)};
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

}  // extern "C"
