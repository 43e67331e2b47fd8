// Batched products: many independent C_i = A_i B_i in one level-wise
// schedule (one grouped launch per level and per leaf tile shape).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "engine.h"

namespace fastmm {
namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

void do_batched(Library& L, int count, const int64_t* M, const int64_t* N, const int64_t* K,
                const float* const* A, const int64_t* lda, const float* const* B,
                const int64_t* ldb, float* const* C, const int64_t* ldc, const int* depth,
                const int64_t* leaf) {
  if (count < 0) throw Error(kInvalidValue, "count < 0");
  if (count == 0) return;
  if (!M || !N || !K || !A || !lda || !B || !ldb || !C || !ldc)
    throw Error(kInvalidValue, "NULL array argument");
  for (int i = 0; i < count; ++i) {
    try {
      validate_gemm_args(M[i], N[i], K[i], A[i], lda[i], B[i], ldb[i], C[i], ldc[i],
                         depth ? depth[i] : 0);
    } catch (const Error& e) {
      throw Error(e.code, "problem " + std::to_string(i) + ": " + e.what());
    }
  }
  ensure_init(L);
  // Residency: every problem all-device or all-host, and the same for all.
  int on_dev = -1;
  for (int i = 0; i < count; ++i) {
    if (M[i] == 0 || N[i] == 0) continue;
    const int d = operands_on_device(M[i], N[i], K[i], A[i], B[i], C[i]) ? 1 : 0;
    if (on_dev >= 0 && d != on_dev)
      throw Error(kNotSupported, "batched problems must all be device or all be host");
    on_dev = d;
  }
  if (on_dev < 0) return;  // every problem empty

  std::vector<Problem> probs;
  std::vector<int> idx;
  size_t stage_bytes = 0, temp_bytes = 0;
  std::vector<size_t> a_off, b_off, c_off;
  for (int i = 0; i < count; ++i) {
    if (M[i] == 0 || N[i] == 0) continue;
    Problem p;
    p.M = M[i];
    p.N = N[i];
    p.K = K[i];
    int dep = depth ? depth[i] : -1;
    int64_t lf = leaf ? leaf[i] : default_leaf();
    int tile = kTile128x128;
    if (dep < 0) {
      fastmm_plan_t pl{};
      int rc = plan_choose(L, p.M, p.N, p.K, L.plan_mode, &pl);
      if (rc != kSuccess) throw Error(rc, "planner failed");
      dep = pl.depth;
      lf = pl.leaf;
      tile = pl.tile;
    }
    p.depth = p.K == 0 ? 0 : effective_depth(p.M, p.N, p.K, dep, lf);
    p.tile = tile;
    if (!on_dev) {
      a_off.push_back(stage_bytes);
      stage_bytes += align_up((size_t)p.M * p.K * 4, 256);
      b_off.push_back(stage_bytes);
      stage_bytes += align_up((size_t)p.K * p.N * 4, 256);
      c_off.push_back(stage_bytes);
      stage_bytes += align_up((size_t)p.M * p.N * 4, 256);
    }
    temp_bytes += align_up(problem_temp_bytes(p), 256);
    probs.push_back(p);
    idx.push_back(i);
  }
  // Size descriptors with placeholder pointers.
  Schedule s;
  {
    std::vector<Problem> q = probs;
    for (auto& x : q) {
      x.A = reinterpret_cast<const float*>(256);
      x.B = x.A;
      x.C = const_cast<float*>(x.A);
      x.lda = std::max<int64_t>(x.K, 1);
      x.ldb = std::max<int64_t>(x.N, 1);
      x.ldc = std::max<int64_t>(x.N, 1);
    }
    build_schedule(q, reinterpret_cast<char*>(256), s);
  }
  const size_t d_bytes = align_up(schedule_desc_bytes(s), 256) + 256;
  char* ws = ensure_arena(L, stage_bytes + temp_bytes + d_bytes);
  char* desc_host = ensure_pinned(L, d_bytes);
  hipStream_t sm = L.stream;
  for (size_t j = 0; j < probs.size(); ++j) {
    Problem& p = probs[j];
    const int i = idx[j];
    if (on_dev) {
      p.A = A[i];
      p.B = B[i];
      p.C = C[i];
      p.lda = lda[i];
      p.ldb = ldb[i];
      p.ldc = ldc[i];
    } else {
      float* dA = reinterpret_cast<float*>(ws + a_off[j]);
      float* dB = reinterpret_cast<float*>(ws + b_off[j]);
      p.A = dA;
      p.B = dB;
      p.C = reinterpret_cast<float*>(ws + c_off[j]);
      p.lda = std::max<int64_t>(p.K, 1);
      p.ldb = p.N;
      p.ldc = p.N;
      if (p.K > 0) {
        FASTMM_HIP(hipMemcpy2DAsync(dA, p.K * 4, A[i], lda[i] * 4, p.K * 4, p.M,
                                    hipMemcpyHostToDevice, sm));
        FASTMM_HIP(hipMemcpy2DAsync(dB, p.N * 4, B[i], ldb[i] * 4, p.N * 4, p.K,
                                    hipMemcpyHostToDevice, sm));
      }
    }
    if (p.K == 0) FASTMM_HIP(hipMemset2DAsync(p.C, p.ldc * 4, 0, p.N * 4, p.M, sm));
  }
  // Problems with K == 0 are done; the rest go through the schedule.
  std::vector<Problem> work;
  for (auto& p : probs)
    if (p.K > 0) work.push_back(p);
  int launches = 0;
  if (!work.empty()) {
    build_schedule(work, ws + stage_bytes, s);
    launches = enqueue_schedule(L, s, ws + stage_bytes + temp_bytes, desc_host);
  }
  if (!on_dev) {
    for (size_t j = 0; j < probs.size(); ++j) {
      const Problem& p = probs[j];
      const int i = idx[j];
      FASTMM_HIP(hipMemcpy2DAsync(C[i], ldc[i] * 4, p.C, p.N * 4, p.N * 4, p.M,
                                  hipMemcpyDeviceToHost, sm));
    }
  }
  FASTMM_HIP(hipStreamSynchronize(sm));
  fastmm_stats_t st{};
  st.h2d_ms = st.preadd_ms = st.leaf_ms = st.postadd_ms = st.d2h_ms = st.total_ms = -1.0;
  st.depth = s.max_depth;
  st.leaves = s.leaves;
  st.leaf_flops = s.leaf_flops;
  st.add_bytes = s.add_bytes;
  st.launches = launches;
  st.workspace_bytes = L.arena_bytes;
  L.stats = st;
}

}  // namespace
}  // namespace fastmm

using namespace fastmm;

extern "C" int fastmm_gemm_batched(int count, const int64_t* M, const int64_t* N,
                                   const int64_t* K, const float* const* A, const int64_t* lda,
                                   const float* const* B, const int64_t* ldb, float* const* C,
                                   const int64_t* ldc, const int* depth, const int64_t* leaf) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return run_guarded([&] { do_batched(L, count, M, N, K, A, lda, B, ldb, C, ldc, depth, leaf); });
}
