// Planner stub (filled in below by the full planner).
#include "engine.h"

namespace fastmm {

int64_t default_leaf() { return 1024; }

int plan_choose(Library& L, int64_t M, int64_t N, int64_t K, int mode, fastmm_plan_t* out) {
  (void)L;
  (void)mode;
  out->depth = 16;
  out->leaf = default_leaf();
  out->tile = kTile128x128;
  out->workspace_bytes = 0;
  out->predicted_ms = -1.0;
  out->source = FASTMM_PLAN_DEFAULT;
  out->depth = effective_depth(M, N, K, 16, out->leaf);
  return kSuccess;
}

}  // namespace fastmm
