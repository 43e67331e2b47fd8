// Batched products: many independent C_i = A_i B_i of uneven extents, each
// with its own plan, in one level-wise schedule -- one grouped launch per
// recursion level and per leaf tile shape for the whole batch -- captured
// once into a HIP graph and replayed.
//
// What a replay needs to change between calls is only data: the operand
// pointers live in the descriptor arrays, which are copied to the device
// (outside the graph) before every replay.  The kernels' own arguments (the
// device addresses of those arrays, counts, grid sizes, vector-path flags)
// are the graph's key: a call whose launches would have exactly these
// arguments replays the graph, anything else captures a new one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "engine.h"

namespace fastmm {
namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct GraphCache {
  struct Entry {
    hipGraphExec_t exec;
    int launches;  // kernel launches the captured schedule holds
  };
  std::map<std::string, Entry> execs;
  int64_t captures = 0, replays = 0;
};

GraphCache& graphs() {
  static GraphCache G;
  return G;
}

// A call that repeats one of the last few -- the same problems (extents,
// operand pointers, leading dimensions, requested depths and leaves), the
// same planner mode, planner state and settings, the same workspace --
// replays the graph that call used without classifying, planning or
// building anything again.  Only the descriptor arrays are copied to the
// device again, since another call may have used that part of the
// workspace in between.
struct RecentCall {
  std::vector<int64_t> key;
  std::string graph;       // its GraphCache entry
  std::vector<char> desc;  // host image of its descriptor arrays
  char* desc_dev = nullptr;
  fastmm_stats_t stats{};
};

constexpr size_t kRecentCalls = 8;

std::vector<RecentCall>& recent_calls() {  // most recent last
  static std::vector<RecentCall> R;
  return R;
}

std::vector<int64_t> call_key(const Library& L, int count, const int64_t* M, const int64_t* N,
                              const int64_t* K, const float* const* A, const int64_t* lda,
                              const float* const* B, const int64_t* ldb, float* const* C,
                              const int64_t* ldc, const int* depth, const int64_t* leaf) {
  auto env = [](const char* n) {
    const char* e = std::getenv(n);
    return (int64_t)(e ? (unsigned char)e[0] : 0);
  };
  std::vector<int64_t> k;
  k.reserve(8 + (size_t)count * 11);
  k.push_back(count);
  k.push_back(L.plan_mode);
  k.push_back((int64_t)L.arena_generation);
  k.push_back(reinterpret_cast<int64_t>(L.stream));
  k.push_back((int64_t)planner_epoch());
  k.push_back(env("FASTMM_PERSISTENT"));
  k.push_back(env("FASTMM_GRAPH"));
  k.push_back(env("FASTMM_TREE_ADDS"));
  k.push_back(env("FASTMM_FUSED_PACK"));
  for (int i = 0; i < count; ++i) {
    k.push_back(M[i]);
    k.push_back(N[i]);
    k.push_back(K[i]);
    k.push_back(reinterpret_cast<int64_t>(A[i]));
    k.push_back(lda[i]);
    k.push_back(reinterpret_cast<int64_t>(B[i]));
    k.push_back(ldb[i]);
    k.push_back(reinterpret_cast<int64_t>(C[i]));
    k.push_back(ldc[i]);
    k.push_back(depth ? depth[i] : -1);
    k.push_back(leaf ? leaf[i] : -1);
  }
  return k;
}

// Kernel arguments of every launch the schedule issues, in order.
std::string signature(const Schedule& s) {
  std::ostringstream o;
  auto blocks_pre = [](const std::vector<PreAddNode>& v) {
    return v.empty() ? 0 : v.back().block_begin + (int)add_blocks_for(v.back().h_r, v.back().h_c);
  };
  auto blocks_post = [](const std::vector<PostAddNode>& v) {
    return v.empty() ? 0 : v.back().block_begin + (int)add_blocks_for(v.back().h_r, v.back().h_c);
  };
  for (int l = 0; l < s.max_depth; ++l)
    o << "a" << (const void*)s.d_preA[l] << ',' << s.preA[l].size() << ',' << blocks_pre(s.preA[l])
      << ',' << (int)s.vec_preA[l] << "b" << (const void*)s.d_preB[l] << ',' << s.preB[l].size()
      << ',' << blocks_pre(s.preB[l]) << ',' << (int)s.vec_preB[l] << ';';
  for (int t = 0; t < kNumTiles; ++t)
    o << "g" << t << (const void*)s.d_leaf[t] << ',' << s.leaf[t].size() << ','
      << s.leaf_tiles_total[t] << ',' << (int)s.vec_leaf[t] << ',' << s.xcd_chunk[t] << ','
      << (int)s.persistent << ';';
  for (int l = s.max_depth - 1; l >= 0; --l)
    o << "p" << (const void*)s.d_post[l] << ',' << s.post[l].size() << ',' << blocks_post(s.post[l])
      << ',' << (int)s.vec_post[l] << ';';
  for (const auto& t : s.trees)
    o << "t" << t.kind << ',' << t.level << ',' << t.levels << ',' << t.width << ',' << t.clip << ','
      << (const void*)t.d_nodes << ','
      << t.nodes.size() << ',' << t.blocks << ';';
  o << "f" << (int)s.fused_post << ';';
  for (int fmt = 0; fmt < 2; ++fmt)
    for (int side = 0; side < 2; ++side)
      o << "k" << fmt << side << (const void*)s.d_pack[fmt][side] << ',' << s.pack[fmt][side].size()
        << ',' << s.pack_units[fmt][side] << ';';
  return o.str();
}

// Launch the schedule through a (possibly new) graph on L.stream.
int launch_graphed(Library& L, Schedule& s, bool& replayed) {
  GraphCache& G = graphs();
  const std::string key = signature(s);
  auto it = G.execs.find(key);
  replayed = it != G.execs.end();
  if (!replayed) {
    hipGraph_t graph = nullptr;
    FASTMM_HIP(hipStreamBeginCapture(L.stream, hipStreamCaptureModeRelaxed));
    try {
      launch_schedule(L, s, nullptr, nullptr, false);
    } catch (...) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(L.stream, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      throw;
    }
    FASTMM_HIP(hipStreamEndCapture(L.stream, &graph));
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    FASTMM_HIP(e);
    if (G.execs.size() >= 32) {  // bound the cache
      (void)hipGraphExecDestroy(G.execs.begin()->second.exec);
      G.execs.erase(G.execs.begin());
    }
    it = G.execs.emplace(key, GraphCache::Entry{exec, s.launches}).first;
    ++G.captures;
  } else {
    ++G.replays;
  }
  FASTMM_HIP(hipGraphLaunch(it->second.exec, L.stream));
  return it->second.launches;
}

void do_batched(Library& L, int count, const int64_t* M, const int64_t* N, const int64_t* K,
                const float* const* A, const int64_t* lda, const float* const* B,
                const int64_t* ldb, float* const* C, const int64_t* ldc, const int* depth,
                const int64_t* leaf) {
  if (count < 0) throw Error(kInvalidValue, "count < 0");
  if (count == 0) return;
  if (!M || !N || !K || !A || !lda || !B || !ldb || !C || !ldc)
    throw Error(kInvalidValue, "NULL array argument");
  // An exact repeat replays its graph at once, unless the workspace
  // controls (a cap, NaN-poisoning) are set: those act on every call.
  const char* poison = std::getenv("FASTMM_POISON");
  const bool ws_controls = std::getenv("FASTMM_WORKSPACE_LIMIT") || (poison && poison[0] == '1');
  if (L.initialised && !ws_controls) {
    const std::vector<int64_t> key = call_key(L, count, M, N, K, A, lda, B, ldb, C, ldc, depth, leaf);
    std::vector<RecentCall>& R = recent_calls();
    GraphCache& G = graphs();
    auto hit = R.end();
    for (auto r = R.begin(); r != R.end(); ++r)
      if (r->key == key) hit = r;
    const auto it = hit != R.end() ? G.execs.find(hit->graph) : G.execs.end();
    if (it != G.execs.end()) {
      const RecentCall& F = *hit;
      char* host = ensure_pinned(L, F.desc.size());
      std::memcpy(host, F.desc.data(), F.desc.size());
      FASTMM_HIP(hipMemcpyAsync(F.desc_dev, host, F.desc.size(), hipMemcpyHostToDevice, L.stream));
      if (L.profiling) FASTMM_HIP(hipEventRecord(L.ev[5], L.stream));
      FASTMM_HIP(hipGraphLaunch(it->second.exec, L.stream));
      ++G.replays;
      if (L.profiling) FASTMM_HIP(hipEventRecord(L.ev[6], L.stream));
      FASTMM_HIP(hipStreamSynchronize(L.stream));
      fastmm_stats_t st = F.stats;
      st.graph_replayed = 1;
      st.total_ms = -1.0;
      if (L.profiling) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, L.ev[5], L.ev[6]) == hipSuccess) st.total_ms = ms;
        else (void)hipGetLastError();
      }
      L.stats = st;
      return;
    }
    if (hit != R.end()) R.erase(hit);  // its graph is gone
  }
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
  std::vector<Staging> stg;
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
      int rc = plan_choose_batched(L, p.M, p.N, p.K, L.plan_mode, &pl);
      if (rc != kSuccess) throw Error(rc, "planner failed");
      dep = pl.depth;
      lf = pl.leaf;
      tile = pl.tile;
    }
    p.depth = p.K == 0 ? 0 : effective_depth(p.M, p.N, p.K, dep, lf);
    p.tile = tile;
    // The same staging as a single call (so each result equals it bit for
    // bit): host operands, and device operands the 16-byte path cannot read.
    const Staging g = plan_staging(M[i], N[i], K[i], A[i], lda[i], B[i], ldb[i], on_dev == 1);
    p.K = g.K4;
    p.N = g.N4;
    p.c_cols = N[i];
    a_off.push_back(stage_bytes);
    stage_bytes += g.a_bytes;
    b_off.push_back(stage_bytes);
    stage_bytes += g.b_bytes;
    c_off.push_back(stage_bytes);
    if (!on_dev) stage_bytes += align_up((size_t)M[i] * N[i] * 4, 256);
    stg.push_back(g);
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
    const Staging& g = stg[j];
    float* dA = g.a ? reinterpret_cast<float*>(ws + a_off[j]) : const_cast<float*>(A[i]);
    float* dB = g.b ? reinterpret_cast<float*>(ws + b_off[j]) : const_cast<float*>(B[i]);
    p.A = dA;
    p.B = dB;
    p.lda = g.a ? std::max<int64_t>(g.K4, 1) : lda[i];
    p.ldb = g.b ? g.N4 : ldb[i];
    if (on_dev) {
      p.C = C[i];
      p.ldc = ldc[i];
    } else {
      p.C = reinterpret_cast<float*>(ws + c_off[j]);
      p.ldc = N[i];
    }
    stage_operands(g, M[i], N[i], K[i], A[i], lda[i], B[i], ldb[i], dA, dB, sm);
    if (p.K == 0) FASTMM_HIP(hipMemset2DAsync(p.C, p.ldc * 4, 0, N[i] * 4, p.M, sm));
  }
  // Problems with K == 0 are done; the rest go through the schedule.
  std::vector<Problem> work;
  for (auto& p : probs)
    if (p.K > 0) work.push_back(p);
  int launches = 0;
  bool replayed = false;
  if (L.profiling) FASTMM_HIP(hipEventRecord(L.ev[5], sm));
  if (!work.empty()) {
    build_schedule(work, ws + stage_bytes, s);
    // Leaves of every problem in one persistent launch per tile shape, its
    // workgroups taking tiles (longest reduction first) from a device
    // counter; FASTMM_PERSISTENT=0 launches one workgroup per tile instead.
    const char* pe = std::getenv("FASTMM_PERSISTENT");
    s.persistent = !(pe && pe[0] == '0');
    upload_schedule(L, s, ws + stage_bytes + temp_bytes, desc_host);
    const char* g = std::getenv("FASTMM_GRAPH");
    if (g && g[0] == '0')
      launches = launch_schedule(L, s, nullptr, nullptr, false);
    else
      launches = launch_graphed(L, s, replayed);
  }
  if (L.profiling) FASTMM_HIP(hipEventRecord(L.ev[6], sm));
  if (!on_dev) {
    for (size_t j = 0; j < probs.size(); ++j) {
      const Problem& p = probs[j];
      const int i = idx[j];
      FASTMM_HIP(hipMemcpy2DAsync(C[i], ldc[i] * 4, p.C, N[i] * 4, N[i] * 4, p.M,
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
  st.leaf_launches = 0;
  for (int t = 0; t < kNumTiles; ++t) st.leaf_launches += s.leaf_tiles_total[t] > 0 ? 1 : 0;
  if (L.profiling && !work.empty()) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, L.ev[5], L.ev[6]) == hipSuccess) st.total_ms = ms;
    else (void)hipGetLastError();
  }
  st.graph_replayed = replayed ? 1 : 0;
  L.stats = st;
  // Remember a graphed all-device call for an exact repeat, its key taken
  // now that the workspace is in place.
  // (Not when a problem has K == 0 or an operand was staged: those copies
  // and fills run outside the graph.)
  const char* ge = std::getenv("FASTMM_GRAPH");
  bool outside = false;
  for (const auto& p : probs) outside = outside || p.K == 0;
  for (const auto& g : stg) outside = outside || g.a || g.b;
  if (on_dev == 1 && !work.empty() && !outside && !(ge && ge[0] == '0')) {
    RecentCall F;
    F.key = call_key(L, count, M, N, K, A, lda, B, ldb, C, ldc, depth, leaf);
    F.graph = signature(s);
    const size_t n = schedule_desc_bytes(s);
    F.desc.assign(desc_host, desc_host + n);
    F.desc_dev = ws + stage_bytes + temp_bytes;
    F.stats = st;
    std::vector<RecentCall>& R = recent_calls();
    for (auto r = R.begin(); r != R.end(); ++r)
      if (r->key == F.key) {
        R.erase(r);
        break;
      }
    if (R.size() >= kRecentCalls) R.erase(R.begin());
    R.push_back(std::move(F));
  }
}

}  // namespace

void destroy_graphs() {
  for (auto& kv : graphs().execs) (void)hipGraphExecDestroy(kv.second.exec);
  graphs().execs.clear();
  recent_calls().clear();
}

int64_t graph_captures() { return graphs().captures; }
int64_t graph_replays() { return graphs().replays; }

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
