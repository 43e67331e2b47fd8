// Planner: chooses recursion depth and leaf tile per shape.
//
// The paper picks its leaf engine from the problem size with fixed
// thresholds found by experiment (Table 2 and the K0 / K1 operating points of
// Section 3.2) and stops the recursion at a fixed size (Section 3.1).  Three
// modes here:
//   DEFAULT     the fixed rule: split while the leaf stays >= 1280, tile
//               128x128 (the analogue of the paper's size thresholds and
//               recursion point, set from measured Winograd-vs-classic
//               crossovers on MI355X: with additions grouped over levels
//               the fastest depth leaves 1024..2432 in every dimension for
//               square n from 3072 to 22528, and 1280 is the cutoff that
//               is never more than 3% off the fastest depth there while
//               keeping n = 19456 at depth 3 (1216-wide leaves lose 6%)); a
//               launch that would have fewer than 512 tiles of 128x128
//               (under half the device's 1024 workgroup slots) takes 64x64
//               tiles instead (n = 1024: 0.081 against 0.129 ms, 1536:
//               0.150 / 0.165, 2560: 0.361 / 0.384; a tie at 2048);
//   EXHAUSTIVE  time every candidate (depth, tile) on the device with
//               device-resident operands, keep the fastest; every timing is
//               a record of the timing database;
//   MODEL       a learned cost model -- kModelNets networks 5 -> 64 -> 64 -> 1
//               (mlp.hip), each trained on the GPU on the whole timing
//               database from its own seeded initialisation and minibatch
//               order -- predicts every candidate's log2 run time as the
//               mean of the networks' predictions; the argmin over all
//               candidates (depth and tile) is taken, unless it is predicted
//               within kModelMargin of the fixed rule's choice, which then
//               stays.  With no trained model it falls back to EXHAUSTIVE.
//               Measured on held-out shapes (timings of 160 training shapes,
//               256 evaluation shapes, one MI355X): one network has mean
//               regret 1.5-2.7% against the fastest candidate depending on
//               its seed (worst single choice up to 52% slower); three have
//               1.4%, and the 1% margin brings that to 1.1% with no choice
//               worse than 17% (the fixed rule: 3.1%, worst 47%).
// Candidates: depth 0..4 with leaves of at least 128 in every dimension,
// times five leaf tiles (64x64 to 256x256).  Ties go to the smaller depth, then tile id.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "engine.h"

namespace fastmm {

// mlp.hip
size_t mlp_scratch_floats(int batch);
void mlp_forward(int batch, const float* p, const float* X, float* y, float* cache, hipStream_t s);
void mlp_backward(int batch, const float* p, const float* X, const float* t, float* grad,
                  float* loss, float* scratch, hipStream_t s);
void mlp_adam(const float* g, float* p, float* m, float* v, int step, float lr, float b1,
              float b2, float eps, hipStream_t s);
// engine.cpp
void gemm_impl(Library& L, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
               const float* B, int64_t ldb, float* C, int64_t ldc, int depth, int64_t leaf,
               int tile);

namespace {

constexpr int kNParams = FASTMM_MLP_PARAMS;
constexpr int kModelNets = FASTMM_MODEL_NETS;
constexpr int64_t kMinLeaf = 128;   // smallest leaf extent a candidate may reach
constexpr int kMaxDepth = 4;
constexpr int64_t kDefaultLeaf = 1280;
// Tiles the planner considers: one per macro-tile area (the area is the
// model's tile feature), the best-measured variant of each.
constexpr int kPlannerTiles[] = {kTile128x128, kTile128x64, kTile64x64, kTile256x128w8,
                                 kTile256x256w8};

struct Record {
  int64_t M, N, K;
  int depth, tile;
  double ms;
};

struct Planner {
  std::vector<Record> db;
  std::map<std::tuple<int64_t, int64_t, int64_t, int>, fastmm_plan_t> cache;
  // Exhaustive timings per shape: (depth, tile) -> ms.
  std::map<std::tuple<int64_t, int64_t, int64_t>, std::map<std::pair<int, int>, double>> table;
  bool trained = false;
  std::vector<float> params;  // host copy of the model: kModelNets x kNParams
  // MODEL's choices per shape (0: a single product, 1: a problem of a batch),
  // so that a repeated shape costs no inference on the device; cleared
  // whenever the model changes.
  std::map<std::tuple<int64_t, int64_t, int64_t, int>, fastmm_plan_t> model_cache;
  uint64_t epoch = 0;  // bumped whenever the timings or the model change
};

Planner& planner() {
  static Planner P;
  return P;
}

// SplitMix64 (Steele, Lea and Flood 2014): the planner's own seeded draws
// (weight initialisation, minibatch order).
uint64_t splitmix64(uint64_t& state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

double uniform01(uint64_t& s) { return (double)(splitmix64(s) >> 11) * 0x1p-53; }

// Features of a candidate, scaled to roughly [-1, 1].
void features(int64_t M, int64_t N, int64_t K, int depth, int tile, float* f) {
  const TileShape ts = tile_shape(tile);
  f[0] = (float)((std::log2((double)M) - 10.0) / 2.0);
  f[1] = (float)((std::log2((double)N) - 10.0) / 2.0);
  f[2] = (float)((std::log2((double)K) - 10.0) / 2.0);
  f[3] = (float)((depth - 2.0) / 2.0);
  f[4] = (float)(std::log2((double)ts.bm * ts.bn) - 14.0);
}

std::vector<std::pair<int, int>> candidates(int64_t M, int64_t N, int64_t K) {
  std::vector<std::pair<int, int>> c;
  const int64_t mn = std::min(std::min(M, N), K);
  for (int d = 0; d <= kMaxDepth; ++d) {
    if (d > 0 && (mn >> d) < kMinLeaf) break;
    for (int t : kPlannerTiles) c.push_back({d, t});
  }
  return c;
}

fastmm_plan_t make_plan(int depth, int tile, double ms, int source) {
  fastmm_plan_t p{};
  p.depth = depth;
  p.leaf = depth == 0 ? kDefaultLeaf : 1;  // depth is reachable: leaves >= kMinLeaf
  p.tile = tile;
  p.workspace_bytes = 0;
  p.predicted_ms = ms;
  p.source = source;
  return p;
}

__global__ void fill_uniform_kernel(float* x, int64_t n, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    x[i] = (float)((double)((int64_t)(z >> 40) - (1 << 23)) * 0x1p-23);
  }
}

// Time every candidate of (M, N, K) with device-resident operands.
fastmm_plan_t tune_exhaustive(Library& L, int64_t M, int64_t N, int64_t K) {
  Planner& P = planner();
  float *dA = nullptr, *dB = nullptr, *dC = nullptr;
  FASTMM_HIP(hipMalloc(&dA, (size_t)M * K * 4));
  FASTMM_HIP(hipMalloc(&dB, (size_t)K * N * 4));
  FASTMM_HIP(hipMalloc(&dC, (size_t)M * N * 4));
  auto release = [&] {
    (void)hipFree(dA);
    (void)hipFree(dB);
    (void)hipFree(dC);
  };
  fastmm_plan_t best{};
  double best_ms = 1e30;
  try {
    hipLaunchKernelGGL(fill_uniform_kernel, dim3(1024), dim3(256), 0, L.stream, dA, M * K, 0x5eedULL);
    hipLaunchKernelGGL(fill_uniform_kernel, dim3(1024), dim3(256), 0, L.stream, dB, K * N, 0xbeefULL);
    FASTMM_HIP(hipGetLastError());
    hipEvent_t e0 = L.tune_ev[0], e1 = L.tune_ev[1];
    for (auto [d, t] : candidates(M, N, K)) {
      const int64_t leaf = d == 0 ? kDefaultLeaf : 1;
      gemm_impl(L, M, N, K, dA, K, dB, N, dC, N, d, leaf, t);  // warm-up
      double ms = 1e30;
      for (int rep = 0; rep < 3; ++rep) {
        FASTMM_HIP(hipEventRecord(e0, L.stream));
        gemm_impl(L, M, N, K, dA, K, dB, N, dC, N, d, leaf, t);
        FASTMM_HIP(hipEventRecord(e1, L.stream));
        FASTMM_HIP(hipEventSynchronize(e1));
        float x = 0.f;
        FASTMM_HIP(hipEventElapsedTime(&x, e0, e1));
        ms = std::min(ms, (double)x);
      }
      P.db.push_back({M, N, K, d, t, ms});
      ++P.epoch;
      P.table[std::make_tuple(M, N, K)][{d, t}] = ms;
      if (ms < best_ms) {  // strict: earlier (smaller depth, tile) wins ties
        best_ms = ms;
        best = make_plan(d, t, ms, FASTMM_PLAN_EXHAUSTIVE);
      }
    }
  } catch (...) {
    release();
    throw;
  }
  release();
  return best;
}

// Device copies of the model parameters and a small inference buffer.
struct ModelDev {
  float* params = nullptr;  // kModelNets x kNParams
  float* buf = nullptr;     // features (64 x 5) and outputs (kModelNets x 64)
};

ModelDev& model_dev() {
  static ModelDev D;
  return D;
}

void upload_model(Library& L) {
  planner().model_cache.clear();
  ++planner().epoch;
  ModelDev& D = model_dev();
  if (!D.params) FASTMM_HIP(hipMalloc(&D.params, (size_t)kModelNets * kNParams * 4));
  if (!D.buf) FASTMM_HIP(hipMalloc(&D.buf, (size_t)64 * (5 + kModelNets) * 4));
  FASTMM_HIP(hipMemcpyAsync(D.params, planner().params.data(), (size_t)kModelNets * kNParams * 4,
                            hipMemcpyHostToDevice, L.stream));
  FASTMM_HIP(hipStreamSynchronize(L.stream));
}

// The fixed rule's tile for a depth-d product: 64x64 when the leaf launch
// would have fewer than 512 tiles of 128x128 (under half the device's
// workgroup slots), else 128x128.
int rule_tile(int64_t M, int64_t N, int d) {
  int64_t leaves = 1;
  for (int l = 0; l < d; ++l) leaves *= 7;
  const int64_t m = d ? leaf_extent(M, d) : M, n = d ? leaf_extent(N, d) : N;
  const int64_t tiles = leaves * ((m + 127) / 128) * ((n + 127) / 128);
  return tiles < 512 ? kTile64x64 : kTile128x128;
}

// The fixed rule: the deepest split whose leaves stay >= kDefaultLeaf, with
// rule_tile's tile.
std::pair<int, int> default_choice(int64_t M, int64_t N, int64_t K) {
  const int d = effective_depth(M, N, K, 16, kDefaultLeaf);
  return {d, rule_tile(M, N, d)};
}

// The model's choice stays with the fixed rule's unless another candidate is
// predicted at least this much faster (a tie-break inside the networks'
// spread: on held-out shapes it took the three networks' mean regret from
// 1.4% to 1.1%).
constexpr double kModelMargin = 1.01;
constexpr double kBatchMargin = 1.05;

// Mean predicted log2 time of the networks for each candidate.
std::vector<double> model_predict(Library& L, int64_t M, int64_t N, int64_t K,
                                  const std::vector<std::pair<int, int>>& cand) {
  ModelDev& D = model_dev();
  const int n = (int)cand.size();
  if (n > 64) throw Error(kDeviceError, "planner: too many candidates for the inference buffer");
  std::vector<float> X((size_t)n * 5), y((size_t)kModelNets * 64);
  for (int i = 0; i < n; ++i) features(M, N, K, cand[i].first, cand[i].second, &X[(size_t)i * 5]);
  float* dX = D.buf;
  float* dy = D.buf + 64 * 5;
  FASTMM_HIP(hipMemcpyAsync(dX, X.data(), X.size() * 4, hipMemcpyHostToDevice, L.stream));
  for (int j = 0; j < kModelNets; ++j)
    mlp_forward(n, D.params + (size_t)j * kNParams, dX, dy + (size_t)j * 64, nullptr, L.stream);
  FASTMM_HIP(hipMemcpyAsync(y.data(), dy, y.size() * 4, hipMemcpyDeviceToHost, L.stream));
  FASTMM_HIP(hipStreamSynchronize(L.stream));
  std::vector<double> pred(n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < kModelNets; ++j) pred[i] += (double)y[(size_t)j * 64 + i];
    pred[i] /= kModelNets;
  }
  return pred;
}

fastmm_plan_t plan_model(Library& L, int64_t M, int64_t N, int64_t K) {
  const auto cand = candidates(M, N, K);
  const int n = (int)cand.size();
  const std::vector<double> pred = model_predict(L, M, N, K, cand);
  const auto def = default_choice(M, N, K);
  int bi = 0, di = -1;
  for (int i = 0; i < n; ++i) {
    if (pred[i] < pred[bi]) bi = i;  // strict: earlier (smaller depth, tile) wins ties
    if (cand[i] == def) di = i;
  }
  if (di >= 0 && pred[di] <= pred[bi] + std::log2(kModelMargin)) bi = di;
  return make_plan(cand[bi].first, cand[bi].second, std::exp2(pred[bi]), FASTMM_PLAN_MODEL);
}

// 128x128 tiles of a depth-d product's leaf launch.
int64_t leaf_tiles_128(int64_t M, int64_t N, int d) {
  int64_t leaves = 1;
  for (int l = 0; l < d; ++l) leaves *= 7;
  const int64_t m = d ? leaf_extent(M, d) : M, n = d ? leaf_extent(N, d) : N;
  return leaves * ((m + 127) / 128) * ((n + 127) / 128);
}

}  // namespace

int64_t default_leaf() { return kDefaultLeaf; }

uint64_t planner_epoch() { return planner().epoch; }

// A problem of a batch: its leaves join one launch with every other
// problem's, which fills the device, so the tile is always 128x128 (the
// fixed rule's smaller tiles only help a product alone fill the device).  A
// single-product timing (EXHAUSTIVE) or prediction (MODEL) measures the
// batch's situation only where the product alone already fills the device
// with long leaves -- a leaf launch of at least 1024 tiles of 128x128, every
// leaf extent at least 1024 --: a deeper plan for a smaller product mostly
// buys occupancy that the batch already has, at the price of additions and
// short reductions (measured on the 256-problem batch: taking the fastest
// single-product depth wherever the product fills the device alone made
// the batch 6% slower under EXHAUSTIVE and 22% slower under MODEL than the
// fixed rule).  So the mode's choice is taken among those candidates,
// against the fixed rule's depth, which stays unless one of them is at
// least kBatchMargin faster alone (measured or, for MODEL, predicted): a
// product's own timing overstates what a Winograd level saves inside the
// batch, whose one persistent leaf launch keeps the device full anyway.
int plan_choose_batched(Library& L, int64_t M, int64_t N, int64_t K, int mode, fastmm_plan_t* out) {
  if (mode < FASTMM_PLAN_DEFAULT || mode > FASTMM_PLAN_EXHAUSTIVE)
    throw Error(kInvalidValue, "unknown planner mode");
  const int def = (M > 0 && N > 0 && K > 0) ? default_choice(M, N, K).first : 0;
  *out = make_plan(def, kTile128x128, -1.0, mode);
  out->leaf = kDefaultLeaf;
  if (mode == FASTMM_PLAN_DEFAULT || M <= 0 || N <= 0 || K <= 0) return kSuccess;
  ensure_init(L);
  Planner& P = planner();
  std::vector<std::pair<int, int>> cand;
  for (auto c : candidates(M, N, K))
    if (c.second == kTile128x128 &&
        (c.first == def ||
         (leaf_tiles_128(M, N, c.first) >= 1024 && std::min(std::min(M, N), K) >> c.first >= 1024)))
      cand.push_back(c);
  // The rule's own depth must be among them (beyond the candidates' depth
  // limit the rule stands).
  bool has_def = false;
  for (const auto& c : cand) has_def = has_def || c.first == def;
  if (cand.size() <= 1 || !has_def) return kSuccess;
  int best = -1;
  if (mode == FASTMM_PLAN_MODEL && P.trained) {
    const auto key = std::make_tuple(M, N, K, 1);
    const auto hit = P.model_cache.find(key);
    if (hit != P.model_cache.end()) {
      *out = hit->second;
      return kSuccess;
    }
    const std::vector<double> pred = model_predict(L, M, N, K, cand);
    int di = 0;
    for (int i = 0; i < (int)cand.size(); ++i) {
      if (best < 0 || pred[i] < pred[best]) best = i;
      if (cand[i].first == def) di = i;
    }
    if (pred[di] <= pred[best] + std::log2(kBatchMargin)) best = di;
  } else {
    fastmm_plan_t ex{};
    plan_choose(L, M, N, K, FASTMM_PLAN_EXHAUSTIVE, &ex);  // fills the timing table
    const auto& t = P.table[std::make_tuple(M, N, K)];
    int di = -1;
    for (int i = 0; i < (int)cand.size(); ++i) {
      auto f = t.find(cand[i]);
      if (f == t.end()) continue;
      if (cand[i].first == def) di = i;
      if (best < 0 || f->second < t.at(cand[best])) best = i;
    }
    if (di >= 0 && best >= 0 && t.at(cand[di]) <= t.at(cand[best]) * kBatchMargin) best = di;
  }
  if (best >= 0 && cand[best].first != def) {
    *out = make_plan(cand[best].first, kTile128x128, -1.0, mode);
  }
  if (mode == FASTMM_PLAN_MODEL && P.trained) P.model_cache[std::make_tuple(M, N, K, 1)] = *out;
  return kSuccess;
}

int plan_choose(Library& L, int64_t M, int64_t N, int64_t K, int mode, fastmm_plan_t* out) {
  if (mode < FASTMM_PLAN_DEFAULT || mode > FASTMM_PLAN_EXHAUSTIVE)
    throw Error(kInvalidValue, "unknown planner mode");
  if (M <= 0 || N <= 0 || K <= 0) {
    *out = make_plan(0, kTile128x128, -1.0, FASTMM_PLAN_DEFAULT);
    return kSuccess;
  }
  if (mode == FASTMM_PLAN_DEFAULT) {
    const auto def = default_choice(M, N, K);
    *out = make_plan(def.first, def.second, -1.0, FASTMM_PLAN_DEFAULT);
    out->leaf = kDefaultLeaf;
    return kSuccess;
  }
  ensure_init(L);
  Planner& P = planner();
  if (mode == FASTMM_PLAN_MODEL && P.trained) {
    const auto key = std::make_tuple(M, N, K, 0);
    auto it = P.model_cache.find(key);
    if (it == P.model_cache.end()) it = P.model_cache.emplace(key, plan_model(L, M, N, K)).first;
    *out = it->second;
    return kSuccess;
  }
  auto key = std::make_tuple(M, N, K, (int)FASTMM_PLAN_EXHAUSTIVE);
  auto it = P.cache.find(key);
  if (it == P.cache.end()) it = P.cache.emplace(key, tune_exhaustive(L, M, N, K)).first;
  *out = it->second;
  return kSuccess;
}

namespace {

void train_network(Library& L, const std::vector<float>& X, const std::vector<float>& t, int n,
                   int batch, int epochs, float lr, float tmean, uint64_t& s, std::vector<float>& p,
                   float& loss);

// Trains the kModelNets networks of the cost model on the whole timing
// database (targets: log2 of the measured milliseconds), network j from the
// seed + j stream.  *loss_out: the networks' mean full-data loss.
void train(Library& L, int epochs, int batch, float lr, uint64_t seed, float* loss_out) {
  Planner& P = planner();
  if (P.db.empty()) throw Error(kInvalidValue, "timing database is empty");
  if (epochs < 1 || batch < 1) throw Error(kInvalidValue, "epochs and batch must be positive");
  ensure_init(L);
  const int n = (int)P.db.size();
  batch = std::min(batch, n);
  std::vector<float> X((size_t)n * 5), t(n);
  double tmean = 0.0;
  for (int i = 0; i < n; ++i) {
    const Record& r = P.db[i];
    features(r.M, r.N, r.K, r.depth, r.tile, &X[(size_t)i * 5]);
    t[i] = (float)std::log2(std::max(r.ms, 1e-4));
    tmean += t[i];
  }
  tmean /= n;
  std::vector<float> all((size_t)kModelNets * kNParams);
  double loss_sum = 0.0;
  for (int net = 0; net < kModelNets; ++net) {
    // Network `net` draws its initialisation and minibatch order from its
    // own seeded stream.
    uint64_t s = seed + (uint64_t)net;
    std::vector<float> p(kNParams, 0.f);
    float loss = 0.f;
    train_network(L, X, t, n, batch, epochs, lr, (float)tmean, s, p, loss);
    std::copy(p.begin(), p.end(), all.begin() + (size_t)net * kNParams);
    loss_sum += loss;
  }
  if (loss_out) *loss_out = (float)(loss_sum / kModelNets);
  P.params = all;
  P.trained = true;
  upload_model(L);
}

// One network of the cost model: He-uniform initialisation from the seeded
// stream s (last bias: the mean target), then `epochs` passes of Adam over
// minibatches in an order shuffled from s; `loss` = full-data loss.
void train_network(Library& L, const std::vector<float>& X, const std::vector<float>& t, int n,
                   int batch, int epochs, float lr, float tmean, uint64_t& s, std::vector<float>& p,
                   float& loss) {
  auto init = [&](int off, int fan_in, int count) {
    const double a = std::sqrt(6.0 / fan_in);
    for (int i = 0; i < count; ++i) p[off + i] = (float)((2.0 * uniform01(s) - 1.0) * a);
  };
  init(0, 5, 5 * 64);
  init(5 * 64 + 64, 64, 64 * 64);
  init(5 * 64 + 64 + 64 * 64 + 64, 64, 64);
  p[kNParams - 1] = tmean;

  float *dp = nullptr, *dm = nullptr, *dv = nullptr, *dg = nullptr, *dX = nullptr, *dt = nullptr,
        *dscr = nullptr, *dloss = nullptr, *hbuf = nullptr;
  auto release = [&] {
    for (float* q : {dp, dm, dv, dg, dX, dt, dscr, dloss}) (void)hipFree(q);
    if (hbuf) (void)hipHostFree(hbuf);
  };
  try {
    FASTMM_HIP(hipMalloc(&dp, kNParams * 4));
    FASTMM_HIP(hipMalloc(&dm, kNParams * 4));
    FASTMM_HIP(hipMalloc(&dv, kNParams * 4));
    FASTMM_HIP(hipMalloc(&dg, kNParams * 4));
    FASTMM_HIP(hipMalloc(&dX, (size_t)n * 5 * 4));
    FASTMM_HIP(hipMalloc(&dt, (size_t)n * 4));
    FASTMM_HIP(hipMalloc(&dscr, mlp_scratch_floats(n) * 4));
    FASTMM_HIP(hipMalloc(&dloss, 4));
    FASTMM_HIP(hipHostMalloc((void**)&hbuf, (size_t)2 * batch * 6 * 4, hipHostMallocDefault));
    FASTMM_HIP(hipMemcpyAsync(dp, p.data(), kNParams * 4, hipMemcpyHostToDevice, L.stream));
    FASTMM_HIP(hipMemsetAsync(dm, 0, kNParams * 4, L.stream));
    FASTMM_HIP(hipMemsetAsync(dv, 0, kNParams * 4, L.stream));
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    int step = 0;
    for (int e = 0; e < epochs; ++e) {
      for (int i = n - 1; i > 0; --i) {  // Fisher-Yates with the seeded stream
        const int j = (int)(splitmix64(s) % (uint64_t)(i + 1));
        std::swap(order[i], order[j]);
      }
      for (int b0 = 0; b0 + batch <= n; b0 += batch) {
        // Alternate two pinned halves so a copy in flight is never rewritten.
        float* hx = hbuf + (size_t)(step & 1) * batch * 6;
        float* ht = hx + (size_t)batch * 5;
        FASTMM_HIP(hipStreamSynchronize(L.stream));
        for (int k = 0; k < batch; ++k) {
          std::memcpy(hx + (size_t)k * 5, &X[(size_t)order[b0 + k] * 5], 5 * 4);
          ht[k] = t[order[b0 + k]];
        }
        FASTMM_HIP(hipMemcpyAsync(dX, hx, (size_t)batch * 5 * 4, hipMemcpyHostToDevice, L.stream));
        FASTMM_HIP(hipMemcpyAsync(dt, ht, (size_t)batch * 4, hipMemcpyHostToDevice, L.stream));
        mlp_backward(batch, dp, dX, dt, dg, nullptr, dscr, L.stream);
        mlp_adam(dg, dp, dm, dv, ++step, lr, 0.9f, 0.999f, 1e-8f, L.stream);
      }
    }
    // Full-data loss of the trained model.
    FASTMM_HIP(hipMemcpyAsync(dX, X.data(), (size_t)n * 5 * 4, hipMemcpyHostToDevice, L.stream));
    FASTMM_HIP(hipMemcpyAsync(dt, t.data(), (size_t)n * 4, hipMemcpyHostToDevice, L.stream));
    mlp_backward(n, dp, dX, dt, dg, dloss, dscr, L.stream);
    FASTMM_HIP(hipMemcpyAsync(&loss, dloss, 4, hipMemcpyDeviceToHost, L.stream));
    FASTMM_HIP(hipMemcpyAsync(p.data(), dp, kNParams * 4, hipMemcpyDeviceToHost, L.stream));
    FASTMM_HIP(hipStreamSynchronize(L.stream));
  } catch (...) {
    release();
    throw;
  }
  release();
}

// Timing database: a flat JSON list of records.
void save_db(const char* path) {
  FILE* f = std::fopen(path, "w");
  if (!f) throw Error(kInvalidValue, std::string("cannot write ") + path);
  std::fprintf(f, "{\"device\": \"gfx950\", \"records\": [\n");
  const auto& db = planner().db;
  for (size_t i = 0; i < db.size(); ++i)
    std::fprintf(f, "  {\"M\": %lld, \"N\": %lld, \"K\": %lld, \"depth\": %d, \"tile\": %d, \"ms\": %.6f}%s\n",
                 (long long)db[i].M, (long long)db[i].N, (long long)db[i].K, db[i].depth,
                 db[i].tile, db[i].ms, i + 1 < db.size() ? "," : "");
  std::fprintf(f, "]}\n");
  std::fclose(f);
}

void load_db(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) throw Error(kInvalidValue, std::string("cannot read ") + path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  std::vector<Record> recs;
  size_t pos = 0;
  while ((pos = text.find("{\"M\":", pos)) != std::string::npos) {
    long long M, N, K;
    int d, t;
    double ms;
    if (std::sscanf(text.c_str() + pos,
                    "{\"M\": %lld, \"N\": %lld, \"K\": %lld, \"depth\": %d, \"tile\": %d, \"ms\": %lf}",
                    &M, &N, &K, &d, &t, &ms) != 6 ||
        M <= 0 || N <= 0 || K <= 0 || d < 0 || d > 16 || t < 0 || t >= kNumTiles || !(ms > 0))
      throw Error(kInvalidValue, std::string("malformed timing record in ") + path);
    recs.push_back({M, N, K, d, t, ms});
    pos += 5;
  }
  auto& db = planner().db;
  db.insert(db.end(), recs.begin(), recs.end());
}

}  // namespace

}  // namespace fastmm

using namespace fastmm;

extern "C" {

int fastmm_plan(int64_t M, int64_t N, int64_t K, int mode, fastmm_plan_t* out) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return run_guarded([&] {
    if (!out) throw Error(kInvalidValue, "out is NULL");
    if (M < 0 || N < 0 || K < 0) throw Error(kInvalidValue, "negative dimension");
    const int rc = plan_choose(L, M, N, K, mode, out);
    if (rc != kSuccess) throw Error(rc, "planner failed");
    // Temporaries of the level-wise schedule (K and N padded to 4 as staged
    // operands would be); staging copies of host or misaligned operands
    // come on top.
    out->workspace_bytes = 0;
    if (M > 0 && N > 0 && K > 0) {
      Problem q;
      q.M = M;
      q.N = (N + 3) / 4 * 4;
      q.K = (K + 3) / 4 * 4;
      q.depth = out->depth;
      q.tile = out->tile;
      out->workspace_bytes = problem_temp_bytes(q);
    }
  });
}

int fastmm_set_plan_mode(int mode) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return run_guarded([&] {
    if (mode < FASTMM_PLAN_DEFAULT || mode > FASTMM_PLAN_EXHAUSTIVE)
      throw Error(kInvalidValue, "unknown planner mode");
    L.plan_mode = mode;
  });
}

int fastmm_planner_load(const char* db_path, const char* model_path) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return run_guarded([&] {
    if (db_path) {
      load_db(db_path);
      ++planner().epoch;
    }
    if (model_path) {
      FILE* f = std::fopen(model_path, "rb");
      if (!f) throw Error(kInvalidValue, std::string("cannot read ") + model_path);
      std::vector<float> p((size_t)kModelNets * kNParams);
      const size_t got = std::fread(p.data(), 4, p.size(), f);
      const bool extra = std::fgetc(f) != EOF;
      std::fclose(f);
      if (got != p.size() || extra)
        throw Error(kInvalidValue, std::string("model file has the wrong size: ") + model_path);
      for (float x : p)
        if (!std::isfinite(x)) throw Error(kInvalidValue, "model file holds non-finite values");
      ensure_init(L);
      planner().params = p;
      planner().trained = true;
      upload_model(L);
    }
  });
}

int fastmm_planner_save(const char* db_path, const char* model_path) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return run_guarded([&] {
    if (db_path) save_db(db_path);
    if (model_path) {
      if (!planner().trained) throw Error(kInvalidValue, "no trained model to save");
      FILE* f = std::fopen(model_path, "wb");
      if (!f) throw Error(kInvalidValue, std::string("cannot write ") + model_path);
      std::fwrite(planner().params.data(), 4, planner().params.size(), f);
      std::fclose(f);
    }
  });
}

int fastmm_planner_train(int epochs, int batch, float lr, uint64_t seed, float* loss) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return run_guarded([&] { train(L, epochs, batch, lr, seed, loss); });
}

int64_t fastmm_planner_records(void) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return (int64_t)planner().db.size();
}

}  // extern "C"
