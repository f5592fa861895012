// pending.cpp -- entry points declared in hmd.h whose implementation is not
// in this build yet: each returns HMD_ENOSYS.
#include "hmd.h"

extern "C" {
void hmd_hybrid_cfg_default(hmd_hybrid_cfg*) {}
int hybrid_create(hmd_ctx*, const hmd_hybrid_cfg*, hmd_gp*, hmd_ens*, hmd_hybrid**) { return HMD_ENOSYS; }
int hybrid_step(hmd_hybrid*, hmd_hybrid_stats*) { return HMD_ENOSYS; }
int hybrid_get(hmd_hybrid*, double*, double*, double*, uint8_t*) { return HMD_ENOSYS; }
void hybrid_free(hmd_hybrid*) {}
}
