// pending.cpp -- entry points declared in hmd.h whose implementation is not
// in this build yet: each returns HMD_ENOSYS.
#include "hmd.h"

extern "C" {
void hmd_ens_cfg_default(hmd_ens_cfg* c) {
  if (!c) return;
  c->members = 5; c->hidden = 64; c->iters = 5000; c->lr = 1e-3; c->seed = 0;
}
int ens_fit(hmd_ctx*, const double*, const double*, int, const hmd_ens_cfg*, hmd_ens**) { return HMD_ENOSYS; }
int ens_predict(hmd_ens*, const double*, int, double*, double*) { return HMD_ENOSYS; }
int ens_loss(const hmd_ens*, double*) { return HMD_ENOSYS; }
int ens_grad_init(hmd_ctx*, const double*, const double*, int, const hmd_ens_cfg*, int, double*, double*, int*) {
  return HMD_ENOSYS;
}
void ens_free(hmd_ens*) {}
void hmd_hybrid_cfg_default(hmd_hybrid_cfg*) {}
int hybrid_create(hmd_ctx*, const hmd_hybrid_cfg*, hmd_gp*, hmd_ens*, hmd_hybrid**) { return HMD_ENOSYS; }
int hybrid_step(hmd_hybrid*, hmd_hybrid_stats*) { return HMD_ENOSYS; }
int hybrid_get(hmd_hybrid*, double*, double*, double*, uint8_t*) { return HMD_ENOSYS; }
void hybrid_free(hmd_hybrid*) {}
}
