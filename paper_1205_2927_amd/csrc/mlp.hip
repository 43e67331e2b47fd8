// Cost-model network kernels (placeholder until the planner lands).
#include <hip/hip_runtime.h>

#include "engine.h"

using namespace fastmm;

extern "C" {
int fastmm_mlp_forward(int, const float*, const float*, float*) { set_error("not implemented"); return kNotSupported; }
int fastmm_mlp_backward(int, const float*, const float*, const float*, float*, float*) { set_error("not implemented"); return kNotSupported; }
int fastmm_mlp_adam(const float*, float*, float*, float*, int, float, float, float, float) { set_error("not implemented"); return kNotSupported; }
int fastmm_plan(int64_t M, int64_t N, int64_t K, int mode, fastmm_plan_t* out) {
  if (!out) return kInvalidValue;
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return plan_choose(L, M, N, K, mode, out);
}
int fastmm_set_plan_mode(int mode) { lib().plan_mode = mode; return kSuccess; }
int fastmm_planner_load(const char*, const char*) { return kNotSupported; }
int fastmm_planner_save(const char*, const char*) { return kNotSupported; }
int fastmm_planner_train(int, int, float, uint64_t, float*) { return kNotSupported; }
int64_t fastmm_planner_records(void) { return 0; }
}
