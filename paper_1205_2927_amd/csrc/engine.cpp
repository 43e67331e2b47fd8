// Recursion engine and the C ABI of the single-product path.
//
// The paper's recursion (Section 3.1) splits every operand into the four
// quadrants of equation (1) and recurses until the operands are small enough
// for a leaf (Table 2); its leaf call copies A and B to the device, runs the
// kernel, copies C back and returns (the three-step call of Section 3.3).
// Here the recursion is Winograd's 7-product form and it runs level by level
// (breadth first): every level is one pre-addition launch per operand, all
// 7^d leaves are one grouped MFMA launch, and every level is one
// post-addition launch, so a depth-d product costs 2d + d + 1 launches
// instead of thousands; levels that halve exactly share their additions'
// launches, up to three levels each (4 launches at depth 3).  Quadrants that
// are plain sub-blocks (A11, A12, A22, B11, B21, B22) are strided views,
// never copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "engine.h"

namespace fastmm {

namespace {
thread_local std::string t_last_error;

constexpr size_t kAlignFloats = 64;  // 256-byte alignment of every buffer

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// A strided operand view with a valid extent (outside: zero).
struct View {
  const float* p;
  int64_t ld;
  int64_t vrows, vcols;
};

// Quadrant (qr, qc) of a view whose quadrants are h_r x h_c (equation (1)).
View quadrant(const View& v, int qr, int qc, int64_t h_r, int64_t h_c) {
  View q;
  q.p = v.p + (int64_t)qr * h_r * v.ld + (int64_t)qc * h_c;
  q.ld = v.ld;
  q.vrows = std::min(std::max<int64_t>(v.vrows - qr * h_r, 0), h_r);
  q.vcols = std::min(std::max<int64_t>(v.vcols - qc * h_c, 0), h_c);
  return q;
}

}  // namespace

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// 16-byte accesses need every quadrant and output row start 16-byte aligned.
bool pre_vec_ok(const PreAddNode& n) {
  return aligned16(n.src) && aligned16(n.dst) && n.ld % 4 == 0 && n.h_c % 4 == 0 &&
         n.bot_off % 4 == 0 && n.out_stride % 4 == 0 && n.right_off % 4 == 0;
}

bool post_vec_ok(const PostAddNode& n) {
  return aligned16(n.P) && aligned16(n.dst) && n.ld % 4 == 0 && n.h_c % 4 == 0 &&
         n.bot_off % 4 == 0 && n.p_stride % 4 == 0 && n.right_off % 4 == 0;
}

void set_error(const std::string& msg) { t_last_error = msg; }

Library& lib() {
  static Library L;
  return L;
}

void ensure_init(Library& L) {
  if (L.initialised) return;
  FASTMM_HIP(hipGetDevice(&L.device));
  hipDeviceProp_t prop;
  FASTMM_HIP(hipGetDeviceProperties(&prop, L.device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    throw Error(kNotSupported, std::string("fastmm is built for gfx950; device is ") +
                                   prop.gcnArchName);
  // A blocking stream: it waits for work the caller queued on the legacy
  // default stream (e.g. the copies that produced A and B) and the default
  // stream waits for it.
  FASTMM_HIP(hipStreamCreate(&L.own_stream));
  if (!L.stream) L.stream = L.own_stream;
  for (auto& e : L.ev) FASTMM_HIP(hipEventCreate(&e));
  // The staged path's copy streams and second compute stream (default
  // priority, ordered against the library stream by events) run alongside
  // the library stream, so each needs a hardware queue of its own.  HIP
  // hands a new stream a queue that other streams already use once
  // GPU_MAX_HW_QUEUES queues exist (4 by default; the caller's default
  // stream usually holds one), and a compute stream that shared a queue with
  // the copy-in stream would wait for every copy queued before its work.
  // A stream created with a CU mask gets a queue of its own; the mask here
  // enables every CU.
  {
    std::vector<uint32_t> mask(((size_t)prop.multiProcessorCount + 31) / 32, 0u);
    for (int cu = 0; cu < prop.multiProcessorCount; ++cu) mask[cu / 32] |= 1u << (cu % 32);
    for (hipStream_t* sp : {&L.h2d_stream, &L.d2h_stream, &L.aux_stream})
      FASTMM_HIP(hipExtStreamCreateWithCUMask(sp, (uint32_t)mask.size(), mask.data()));
  }
  for (auto& e : L.sync_ev) FASTMM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (auto& e : L.leaf_ev) FASTMM_HIP(hipEventCreate(&e));
  for (auto& e : L.tune_ev) FASTMM_HIP(hipEventCreate(&e));
  // The persistent leaf launches' two counters: the head of the statically
  // allocated device workspace (noalloc.cpp), so that initialisation itself
  // allocates no device memory.
  L.leaf_queue = reinterpret_cast<int*>(bind_static_scratch(L.device));
  FASTMM_HIP(hipMemset(L.leaf_queue, 0, static_queue_bytes()));
  L.initialised = true;
}

char* ensure_arena(Library& L, size_t bytes) {
  bytes = std::max<size_t>(bytes, 1);
  // Debug/test controls, read on every call: a cap on the workspace, and
  // NaN-poisoning of the workspace so that a read of a temporary that was
  // never written shows up in the result.
  L.limit = 0;
  if (const char* s = std::getenv("FASTMM_WORKSPACE_LIMIT")) L.limit = std::strtoull(s, nullptr, 10);
  const char* poison = std::getenv("FASTMM_POISON");
  if (poison && poison[0] == '1' && L.arena && bytes <= L.arena_bytes)
    FASTMM_HIP(hipMemsetAsync(L.arena, 0xFF, L.arena_bytes, L.stream));
  if (L.limit && bytes > L.limit)
    throw Error(kOutOfMemory, "workspace of " + std::to_string(bytes) +
                                  " bytes exceeds FASTMM_WORKSPACE_LIMIT=" + std::to_string(L.limit));
  if (bytes <= L.arena_bytes) return L.arena;
  FASTMM_HIP(hipStreamSynchronize(L.stream));
  size_t free_b = 0, total_b = 0;
  FASTMM_HIP(hipMemGetInfo(&free_b, &total_b));
  if (bytes > free_b + L.arena_bytes)
    throw Error(kOutOfMemory, "workspace of " + std::to_string(bytes) + " bytes exceeds free device memory (" +
                                  std::to_string(free_b + L.arena_bytes) + ")");
  if (L.arena) {
    FASTMM_HIP(hipFree(L.arena));
    L.arena = nullptr;
    L.arena_bytes = 0;
  }
  // Grow geometrically to avoid reallocating on every slightly larger call,
  // but leave a margin of free memory to the rest of the process.
  const size_t margin = std::min<size_t>(free_b / 16, size_t(2) << 30);
  const size_t room = free_b + L.arena_bytes > margin ? free_b + L.arena_bytes - margin : 0;
  size_t want = std::max(bytes, std::min(bytes + bytes / 4, room));
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    want = bytes;
    FASTMM_HIP(hipMalloc(&p, want));
  }
  L.arena = static_cast<char*>(p);
  L.arena_bytes = want;
  ++L.arena_generation;
  if (poison && poison[0] == '1') FASTMM_HIP(hipMemsetAsync(L.arena, 0xFF, L.arena_bytes, L.stream));
  return L.arena;
}

char* ensure_pinned(Library& L, size_t bytes) {
  bytes = std::max<size_t>(bytes, 4096);
  if (bytes <= L.pinned_bytes) return L.pinned;
  FASTMM_HIP(hipStreamSynchronize(L.stream));
  if (L.pinned) FASTMM_HIP(hipHostFree(L.pinned));
  L.pinned = nullptr;
  L.pinned_bytes = 0;
  void* p = nullptr;
  FASTMM_HIP(hipHostMalloc(&p, bytes, hipHostMallocDefault));
  L.pinned = static_cast<char*>(p);
  L.pinned_bytes = bytes;
  return L.pinned;
}

int effective_depth(int64_t M, int64_t N, int64_t K, int depth, int64_t leaf) {
  int d = 0;
  int64_t m = M, k = K, n = N;
  while (splits(m, k, n, depth - d, leaf)) {
    m = split_half(m);
    k = split_half(k);
    n = split_half(n);
    ++d;
  }
  return d;
}

namespace {

std::vector<Dims> level_dims(const Problem& p) {
  std::vector<Dims> dims{{p.M, p.K, p.N}};
  for (int l = 0; l < p.depth; ++l) {
    const Dims& d = dims.back();
    const int left = p.depth - l;
    dims.push_back({split_at(d.m, left), split_at(d.k, left), split_at(d.n, left)});
  }
  return dims;
}

int64_t pow7(int l) {
  int64_t r = 1;
  for (int i = 0; i < l; ++i) r *= 7;
  return r;
}

}  // namespace

size_t b_tree_bytes(int64_t M, int64_t K, int64_t N, int depth) {
  Problem p;
  p.M = M;
  p.K = K;
  p.N = N;
  p.depth = depth;
  const auto dims = level_dims(p);
  size_t floats = 0;
  for (int l = 0; l < depth; ++l)
    floats += align_up((size_t)pow7(l) * 4 * dims[l + 1].k * dims[l + 1].n, kAlignFloats);
  return floats * sizeof(float);
}

size_t a_tree_bytes(int64_t M, int64_t K, int64_t N, int depth) {
  Problem p;
  p.M = M;
  p.K = K;
  p.N = N;
  p.depth = depth;
  const auto dims = level_dims(p);
  size_t floats = 0;
  for (int l = 0; l < depth; ++l)
    floats += align_up((size_t)pow7(l) * 4 * dims[l + 1].m * dims[l + 1].k, kAlignFloats);
  return floats * sizeof(float);
}

size_t problem_temp_bytes(const Problem& p) {
  const auto dims = level_dims(p);
  size_t floats = 0;
  for (int l = 0; l < p.depth; ++l) {
    const Dims& c = dims[l + 1];
    if (!p.a_tree) floats += align_up((size_t)pow7(l) * 4 * c.m * c.k, kAlignFloats);
    if (!p.b_tree) floats += align_up((size_t)pow7(l) * 4 * c.k * c.n, kAlignFloats);
  }
  for (int l = 1; l <= p.depth; ++l)
    floats += align_up((size_t)pow7(l) * dims[l].m * dims[l].n, kAlignFloats);
  // Split-precision leaves: both operands of every leaf packed as hi/lo
  // 16-bit tiles; for FP16 also one int exponent per row of A and per
  // column of B.
  const Dims& lf = dims[p.depth];
  if (p.tile == kTileBf16x3 || p.tile == kTileFp16x3)
    floats += align_up((size_t)pow7(p.depth) * (size_t)leaf_packed_bytes(lf.m, lf.n, lf.k) / 4,
                       kAlignFloats);
  if (p.tile == kTileFp16x3)
    floats += align_up((size_t)pow7(p.depth) * (size_t)leaf_scale_bytes(lf.m, lf.n, lf.k) / 4,
                       kAlignFloats);
  return floats * sizeof(float);
}

// Order in which the seven products of a node enter its result when the
// last level's post-additions are fused into the leaves: every quadrant's
// chain (C11 = P1 + P2; C12 = ((P1 + P6) + P5) + P3; C21 = ((P1 + P6) + P7)
// - P4; C22 = ((P1 + P6) + P7) + P5) then takes its operands in the
// post-addition kernel's order, so the result is bit for bit the same.
// Per product (P1..P7): quadrants entered (bit 0 C11, 1 C12, 2 C21, 3 C22),
// stored (first operand of the chain), subtracted.
constexpr int kFusedPostOrder[7] = {0, 5, 6, 4, 1, 2, 3};
constexpr int kFusedMask[7] = {0xF, 0x1, 0x2, 0x4, 0xA, 0xE, 0xC};
constexpr int kFusedFirst[7] = {0xF, 0, 0, 0, 0, 0, 0};
constexpr int kFusedSub[7] = {0, 0, 0, 0x4, 0, 0, 0};

void build_schedule(const std::vector<Problem>& probs, char* ws, Schedule& s) {
  s = Schedule();
  {
    const char* fp = std::getenv("FASTMM_FUSED_POST");
    s.fused_post = fp && fp[0] == '1' && probs.size() == 1 && probs[0].depth >= 1 &&
                   probs[0].tile == kTile128x128;
  }
  // Split-BF16 leaves take the last level's pre-additions and the pack pass
  // in one fused pass (FASTMM_FUSED_PACK=0: the two passes, for comparison).
  const char* fe = std::getenv("FASTMM_FUSED_PACK");
  const bool fuse_allowed = !(fe && fe[0] == '0');
  // Subtrees that split exactly take up to three levels of additions per
  // launch (FASTMM_TREE_ADDS=1: one level per launch; 2: at most two).
  const char* te = std::getenv("FASTMM_TREE_ADDS");
  const int tree_max = (te && te[0] >= '0' && te[0] <= '9') ? std::min(kMaxTreeLevels, std::atoi(te))
                                                            : kMaxTreeLevels;
  auto add_tree = [&](int kind, int level, int levels, int width, const TreeNode& tn) {
    for (auto& t : s.trees)
      if (t.kind == kind && t.level == level && t.levels == levels && t.width == width) {
        t.nodes.push_back(tn);
        return;
      }
    Schedule::TreeLaunch t;
    t.kind = kind;
    t.level = level;
    t.levels = levels;
    t.width = width;
    t.nodes.push_back(tn);
    s.trees.push_back(std::move(t));
  };
  int maxd = 0;
  for (const auto& p : probs) maxd = std::max(maxd, p.depth);
  s.max_depth = maxd;
  s.preA.resize(maxd);
  s.preB.resize(maxd);
  s.post.resize(maxd);
  float* base = reinterpret_cast<float*>(ws);
  size_t off = 0;  // floats
  auto carve = [&](size_t nfloats) {
    float* p = base + off;
    off += align_up(nfloats, kAlignFloats);
    return p;
  };

  for (const auto& p : probs) {
    const auto dims = level_dims(p);
    const int d = p.depth;
    std::vector<View> Av{{p.A, p.lda, p.ar(), p.ac()}}, Bv{{p.B, p.ldb, p.br(), p.bc()}};
    size_t t_off = 0;  // floats into p.b_tree
    size_t s_off = 0;  // floats into p.a_tree
    // Fused pre-addition and pack (split-BF16 leaves, depth >= 1, no shared
    // B tree): nodes of the last level whose quadrants allow 16-byte access.
    const bool fuse = fuse_allowed && (p.tile == kTileBf16x3 || p.tile == kTileFp16x3) && d >= 1 &&
                      !p.b_tree && !p.a_tree;
    const int fmt = p.tile == kTileFp16x3 ? 1 : 0;
    struct Fused {
      int64_t x;
      PreAddNode a, b;
    };
    std::vector<Fused> fused;
    // Level-wise nodes and bytes per level, and the S / T block bases; the
    // launches are chosen once every level is known.
    std::vector<std::vector<PreAddNode>> lvA(d), lvB(d);
    std::vector<float*> Sb(d), Tb(d);
    std::vector<double> byA(d, 0.0), byB(d, 0.0);
    // Pre-additions, level by level; the next level's operands are views
    // of this level's operands or of the new S / T blocks.
    for (int l = 0; l < d; ++l) {
      const Dims c = dims[l + 1];
      const int64_t nodes = pow7(l);
      float* S;
      if (p.a_tree) {
        S = p.a_tree + s_off;
        s_off += align_up((size_t)nodes * 4 * c.m * c.k, kAlignFloats);
      } else {
        S = carve((size_t)nodes * 4 * c.m * c.k);
      }
      float* T;
      if (p.b_tree) {
        T = p.b_tree + t_off;
        t_off += align_up((size_t)nodes * 4 * c.k * c.n, kAlignFloats);
      } else {
        T = carve((size_t)nodes * 4 * c.k * c.n);
      }
      std::vector<View> nA(7 * nodes), nB(7 * nodes);
      const int64_t sa = c.m * c.k, tb = c.k * c.n;
      for (int64_t x = 0; x < nodes; ++x) {
        const View& a = Av[x];
        const View& b = Bv[x];
        const PreAddNode na = preadd_node(a.p, a.ld, a.vrows, a.vcols, c.m, c.k, S + x * 4 * sa);
        const PreAddNode nb = preadd_node(b.p, b.ld, b.vrows, b.vcols, c.k, c.n, T + x * 4 * tb);
        if (fuse && l == d - 1 && pre_vec_ok(na) && pre_vec_ok(nb)) {
          fused.push_back({x, na, nb});
        } else {
          if (!p.a_tree_ready) lvA[l].push_back(na);
          if (!p.b_tree_ready) lvB[l].push_back(nb);
        }
        const View a11 = quadrant(a, 0, 0, c.m, c.k), a12 = quadrant(a, 0, 1, c.m, c.k),
                   a22 = quadrant(a, 1, 1, c.m, c.k);
        const View b11 = quadrant(b, 0, 0, c.k, c.n), b21 = quadrant(b, 1, 0, c.k, c.n),
                   b22 = quadrant(b, 1, 1, c.k, c.n);
        auto sv = [&](int i) { return View{S + (x * 4 + i) * sa, c.k, c.m, c.k}; };
        auto tv = [&](int i) { return View{T + (x * 4 + i) * tb, c.n, c.k, c.n}; };
        // P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4,
        // P5 = S1 T1,   P6 = S2 T2,   P7 = S3 T3
        const View ca[7] = {a11, a12, sv(3), a22, sv(0), sv(1), sv(2)};
        const View cb[7] = {b11, b21, b22, tv(3), tv(0), tv(1), tv(2)};
        for (int i = 0; i < 7; ++i) {
          nA[7 * x + i] = ca[i];
          nB[7 * x + i] = cb[i];
        }
      }
      Av.swap(nA);
      Bv.swap(nB);
      Sb[l] = S;
      Tb[l] = T;
      byA[l] = p.a_tree_ready ? 0.0 : (double)nodes * 32.0 * c.m * c.k;
      byB[l] = p.b_tree_ready ? 0.0 : (double)nodes * 32.0 * c.k * c.n;
    }
    // Group the levels from the bottom up: the deepest levels hold the most
    // nodes, so they gain most from sharing a pass.  g[l] = levels of the
    // launch whose top level is l (1: level-wise), 0 inside a group.  A
    // group needs every level below its top exactly twice the next (the
    // split rule gives that; the top node itself may be clipped).
    // side 0: A's extents (m, k); 1: B's (k, n); 2: the products' (m, n).
    auto exact = [&](int a, int b, int side) {
      for (int j = a + 1; j < b; ++j) {
        const Dims &x = dims[j], &y = dims[j + 1];
        const bool ok = side == 0   ? (x.m == 2 * y.m && x.k == 2 * y.k)
                        : side == 1 ? (x.k == 2 * y.k && x.n == 2 * y.n)
                                    : (x.m == 2 * y.m && x.n == 2 * y.n);
        if (!ok) return false;
      }
      return true;
    };
    auto group_levels = [&](int top, const std::function<bool(int, int)>& group_ok) {
      std::vector<int> g(d, 1);
      int hi = top;
      while (hi > 0) {
        int L = std::min(tree_max, hi);
        while (L > 1 && !group_ok(hi - L, L)) --L;
        L = std::max(L, 1);
        for (int j = hi - L; j < hi; ++j) g[j] = 0;
        g[hi - L] = L;
        hi -= L;
      }
      return g;
    };
    // Pre-addition groups stop above a level fused with the pack pass.
    const int pre_top = fuse ? d - 1 : d;
    auto pre_side = [&](int kind, std::vector<std::vector<PreAddNode>>& lv,
                        const std::vector<float*>& base, const std::vector<double>& by,
                        std::vector<std::vector<PreAddNode>>& out) {
      const std::vector<int> g = group_levels(pre_top, [&](int l, int L) {
        return (int64_t)lv[l].size() == pow7(l) && exact(l, l + L, kind);
      });
      for (int l = 0; l < d; ++l) {
        if (g[l] == 1) {
          out[l].insert(out[l].end(), lv[l].begin(), lv[l].end());
          s.add_bytes += by[l];
        } else if (g[l] > 1) {
          const int L = g[l];
          const Dims& cell = dims[l + L];
          const int64_t br = kind == 0 ? cell.m : cell.k, bc = kind == 0 ? cell.k : cell.n;
          bool aligned = bc % 4 == 0;
          for (const auto& n : lv[l]) aligned = aligned && aligned16(n.src) && n.ld % 4 == 0;
          const int width = tree_width(L, aligned);
          // The top operand read once; of each S / T block of level l + j,
          // the 3^(L-1-j) cells that the levels below read as views.
          double cells = (double)(1 << (2 * L));
          for (int j = 0; j < L; ++j) {
            double seen = 1.0;
            for (int i = 0; i < L - 1 - j; ++i) seen *= 3.0;
            cells += (double)pow7(j) * 4.0 * seen;
          }
          for (int64_t x = 0; x < (int64_t)lv[l].size(); ++x) {
            TreeNode tn{};
            tn.src = lv[l][x].src;
            tn.ld = lv[l][x].ld;
            tn.vrows = lv[l][x].top_rows + lv[l][x].bot_rows;
            tn.vcols = lv[l][x].left_cols + lv[l][x].right_cols;
            for (int j = 0; j < L; ++j) tn.dst[j] = base[l + j];
            tn.node = x;
            tn.br = (int32_t)br;
            tn.bc = (int32_t)bc;
            add_tree(kind, l, L, width, tn);
          }
          s.add_bytes += (double)lv[l].size() * cells * 4.0 * (double)br * (double)bc;
        }
      }
    };
    if (!p.a_tree_ready) pre_side(0, lvA, Sb, byA, s.preA);
    if (!p.b_tree_ready) pre_side(1, lvB, Tb, byB, s.preB);
    // Product buffers P[l] (l = 1..d), 7^l blocks of m_l x n_l (the leaves'
    // own, P[d], not when they write into their nodes' results).
    std::vector<float*> P(d + 1, nullptr);
    for (int l = 1; l <= d; ++l)
      if (!(s.fused_post && l == d)) P[l] = carve((size_t)pow7(l) * dims[l].m * dims[l].n);
    // Leaves.
    const Dims lf = dims[d];
    const int64_t nleaves = pow7(d);
    const TileShape ts = tile_shape(p.tile);
    const size_t leaf_base = s.leaf[p.tile].size();
    const bool split = p.tile == kTileBf16x3 || p.tile == kTileFp16x3;
    const int64_t packed = split ? leaf_packed_bytes(lf.m, lf.n, lf.k) : 0;
    char* packs = split ? reinterpret_cast<char*>(carve((size_t)(nleaves * packed / 4))) : nullptr;
    const int64_t scale_ints = leaf_scale_bytes(lf.m, lf.n, lf.k) / 4;
    int32_t* exps = p.tile == kTileFp16x3
                        ? reinterpret_cast<int32_t*>(carve((size_t)(nleaves * scale_ints)))
                        : nullptr;
    for (int64_t x = 0; x < nleaves; ++x) {
      GemmDesc g{};
      if (packs) {
        g.pa = packs + x * packed;
        g.pb = packs + x * packed + leaf_packed_a_bytes(lf.m, lf.k);
      }
      if (exps) {
        g.ea = exps + x * scale_ints;
        g.eb = g.ea + lf.m;
      }
      g.A = Av[x].p;
      g.lda = Av[x].ld;
      g.B = Bv[x].p;
      g.ldb = Bv[x].ld;
      g.a_rows = (int32_t)Av[x].vrows;
      g.b_cols = (int32_t)Bv[x].vcols;
      g.kmax = (int32_t)std::min(Av[x].vcols, Bv[x].vrows);
      if (d == 0) {
        g.C = p.C;
        g.ldc = p.ldc;
        g.c_rows = (int32_t)p.cr();
        g.c_cols = (int32_t)p.cc();
      } else if (s.fused_post) {
        // Product i of node x / 7 of the last level, straight into the
        // node's result (the root's C, clipped, or a level d-1 product).
        const int i = (int)(x % 7);
        const int64_t nd = x / 7;
        const bool root = d == 1;
        const int64_t rows = root ? p.cr() : dims[d - 1].m, cols = root ? p.cc() : dims[d - 1].n;
        g.E = root ? p.C : P[d - 1] + nd * dims[d - 1].m * dims[d - 1].n;
        g.e_ld = root ? p.ldc : dims[d - 1].n;
        g.e_bot_off = lf.m * g.e_ld;
        g.e_right_off = (int32_t)lf.n;
        g.e_rows[0] = clamp_extent(rows, lf.m);
        g.e_rows[1] = clamp_extent(rows - lf.m, lf.m);
        g.e_cols[0] = clamp_extent(cols, lf.n);
        g.e_cols[1] = clamp_extent(cols - lf.n, lf.n);
        g.e_mask = kFusedMask[i];
        g.e_first = kFusedFirst[i];
        g.e_sub = kFusedSub[i];
        g.C = g.E;
        g.ldc = g.e_ld;
        g.c_rows = (int32_t)lf.m;
        g.c_cols = (int32_t)lf.n;
      } else {
        g.C = P[d] + x * lf.m * lf.n;
        g.ldc = lf.n;
        g.c_rows = (int32_t)lf.m;
        g.c_cols = (int32_t)lf.n;
      }
      g.tiles_n = (g.c_cols + ts.bn - 1) / ts.bn;
      s.leaf[p.tile].push_back(g);
    }
    // Fused nodes: the seven leaves of node x are leaf_base + 7 x + i.
    for (const Fused& f : fused) {
      PackNode na{}, nb{};
      na.q = f.a;
      nb.q = f.b;
      na.tiles = (int32_t)((lf.m + 127) / 128);
      nb.tiles = (int32_t)((lf.n + 127) / 128);
      for (int i = 0; i < 7; ++i) {
        GemmDesc& g = s.leaf[p.tile][leaf_base + 7 * f.x + i];
        g.prepacked = 1;
        na.dst[i] = g.pa;
        nb.dst[i] = g.pb;
        na.e[i] = g.ea;
        nb.e[i] = g.eb;
        na.rows[i] = g.a_rows;
        nb.rows[i] = g.b_cols;
        na.kmax[i] = nb.kmax[i] = g.kmax;
        na.slabs[i] = nb.slabs[i] = (g.kmax + 31) / 32;
        na.max_slabs = std::max(na.max_slabs, na.slabs[i]);
      }
      nb.max_slabs = na.max_slabs;
      s.pack[fmt][0].push_back(na);
      s.pack[fmt][1].push_back(nb);
      // 7 packed outputs instead of 4 FP32 ones (same bytes per element)
      const Dims& c = dims[d];
      s.add_bytes += 12.0 * c.m * c.k + 12.0 * c.k * c.n;
    }
    s.leaves += nleaves;
    s.leaf_flops += (double)nleaves * 2.0 * lf.m * lf.n * lf.k;
    s.leaf_dims = lf;
    // Post-additions, deepest level first.
    std::vector<std::vector<PostAddNode>> lvP(d);
    for (int l = d - 1; l >= 0; --l) {
      const Dims c = dims[l + 1];
      const int64_t nodes = pow7(l);
      for (int64_t x = 0; x < nodes; ++x) {
        const float* pin = P[l + 1] + x * 7 * c.m * c.n;
        if (l == 0)
          lvP[l].push_back(postadd_node(pin, c.m, c.n, p.C, p.ldc, p.cr(), p.cc()));
        else
          lvP[l].push_back(postadd_node(pin, c.m, c.n, P[l] + x * dims[l].m * dims[l].n,
                                        dims[l].n, dims[l].m, dims[l].n));
      }
    }
    // A clipped C (the root's product) keeps the root's level to itself.
    const bool c_clipped = d > 0 && (lvP[0][0].top_rows + lvP[0][0].bot_rows < 2 * lvP[0][0].h_r ||
                                     lvP[0][0].left_cols + lvP[0][0].right_cols < 2 * lvP[0][0].h_c);
    // With the last level fused into the leaves, the launches cover levels
    // 0 .. d-2 only.
    const int post_top = s.fused_post ? d - 1 : d;
    std::vector<int> gp = group_levels(post_top, [&](int l, int L) {
      return exact(l, l + L, 2) && !(l == 0 && c_clipped);
    });
    if (s.fused_post) {
      gp[d - 1] = 0;
      const Dims c = dims[d];
      s.add_bytes += (double)pow7(d - 1) * 96.0 * c.m * c.n;  // 24 reads or writes per node
    }
    for (int l = d - 1; l >= 0; --l) {
      const Dims c = dims[l + 1];
      if (gp[l] == 1) {
        s.post[l].insert(s.post[l].end(), lvP[l].begin(), lvP[l].end());
        s.add_bytes += (double)lvP[l].size() * 44.0 * c.m * c.n;
      } else if (gp[l] > 1) {
        // The node's 7^L bottom products in, its product out.
        const int L = gp[l];
        const Dims& cell = dims[l + L];
        const int64_t blocks = pow7(L);
        bool aligned = cell.n % 4 == 0;
        for (const auto& n : lvP[l]) aligned = aligned && aligned16(n.dst) && n.ld % 4 == 0;
        const int width = tree_width(L, aligned);
        for (int64_t x = 0; x < (int64_t)lvP[l].size(); ++x) {
          TreeNode tn{};
          tn.src = P[l + L] + x * blocks * cell.m * cell.n;
          tn.dst[0] = lvP[l][x].dst;
          tn.ld = lvP[l][x].ld;
          tn.vrows = lvP[l][x].top_rows + lvP[l][x].bot_rows;
          tn.vcols = lvP[l][x].left_cols + lvP[l][x].right_cols;
          tn.node = x;
          tn.br = (int32_t)cell.m;
          tn.bc = (int32_t)cell.n;
          add_tree(2, l, L, width, tn);
        }
        s.add_bytes += (double)lvP[l].size() * (double)(blocks + (1 << (2 * L))) * 4.0 *
                       (double)cell.m * (double)cell.n;
      }
    }
  }
  s.temp_bytes = off * sizeof(float);

  // Block / tile prefixes and the vector-path flags of every launch.
  s.vec_preA.assign(maxd, 1);
  s.vec_preB.assign(maxd, 1);
  s.vec_post.assign(maxd, 1);
  auto fix_pre = [](std::vector<PreAddNode>& v, char& vec) {
    int64_t b = 0;
    for (auto& n : v) {
      n.block_begin = (int32_t)b;
      b += add_blocks_for(n.h_r, n.h_c);
      if (!pre_vec_ok(n)) vec = 0;
    }
    if (b > INT32_MAX) throw Error(kNotSupported, "pre-addition launch too large");
    return (int)b;
  };
  for (int l = 0; l < maxd; ++l) {
    fix_pre(s.preA[l], s.vec_preA[l]);
    fix_pre(s.preB[l], s.vec_preB[l]);
    int64_t b = 0;
    for (auto& n : s.post[l]) {
      n.block_begin = (int32_t)b;
      b += add_blocks_for(n.h_r, n.h_c);
      if (!post_vec_ok(n)) s.vec_post[l] = 0;
    }
    if (b > INT32_MAX) throw Error(kNotSupported, "post-addition launch too large");
  }
  for (int fmt = 0; fmt < 2; ++fmt)
    for (int side = 0; side < 2; ++side) {
      int64_t u = 0;
      for (auto& n : s.pack[fmt][side]) {
        n.unit_begin = (int32_t)u;
        u += pack_node_units(n);
      }
      if (u > INT32_MAX) throw Error(kNotSupported, "fused pack launch too large");
      s.pack_units[fmt][side] = (int)u;
    }
  for (auto& t : s.trees) {
    int64_t b = 0;
    for (auto& n : t.nodes) {
      if (n.vrows < ((int64_t)n.br << t.levels) || n.vcols < ((int64_t)n.bc << t.levels)) t.clip = true;
      n.block_begin = (int32_t)b;
      b += tree_blocks_for(t.width, n.br, n.bc);
    }
    if (b > INT32_MAX) throw Error(kNotSupported, "multi-level addition launch too large");
    t.blocks = (int)b;
  }
  s.leaf_tiles_total.assign(kNumTiles, 0);
  for (int t = 0; t < kNumTiles; ++t) {
    s.vec_leaf[t] = true;
    const TileShape ts = tile_shape(t);
    // Leaves of different reduction lengths (a batch of uneven products):
    // dispatch the longest tiles first and deal tiles to the XCDs in small
    // round-robin runs, so that no XCD is left with the long tail.
    auto& lv = s.leaf[t];
    s.xcd_chunk[t] = 0;
    const bool phased = s.fused_post && t == kTile128x128;
    if (!phased)
      for (auto& g : lv)
        if (g.kmax != lv[0].kmax) s.xcd_chunk[t] = 8;
    if (s.xcd_chunk[t])
      std::stable_sort(lv.begin(), lv.end(),
                       [](const GemmDesc& a, const GemmDesc& b) { return a.kmax > b.kmax; });
    if (phased) {  // leaf x is product x % 7 of its node: group by launch
      std::vector<GemmDesc> by[7];
      for (size_t x = 0; x < lv.size(); ++x) by[x % 7].push_back(lv[x]);
      lv.clear();
      for (int j = 0; j < 7; ++j) {
        s.phase_begin[j] = (int)lv.size();
        lv.insert(lv.end(), by[kFusedPostOrder[j]].begin(), by[kFusedPostOrder[j]].end());
      }
      s.phase_begin[7] = (int)lv.size();
    }
    int64_t total = 0;
    int phase = 0;
    for (size_t x = 0; x < s.leaf[t].size(); ++x) {
      GemmDesc& g = s.leaf[t][x];
      if (phased) {
        while (phase < 7 && (int)x >= s.phase_begin[phase + 1]) ++phase;
        if ((int)x == s.phase_begin[phase]) total = 0;  // numbering restarts per launch
      }
      g.tile_begin = (int32_t)total;
      total += (int64_t)((g.c_rows + ts.bm - 1) / ts.bm) * g.tiles_n;
      // 16-byte loads need aligned rows and float4 groups that are either
      // wholly inside or wholly outside the valid extent.
      if (!(aligned16(g.A) && aligned16(g.B) && g.lda % 4 == 0 && g.ldb % 4 == 0 &&
            g.kmax % 4 == 0 && g.b_cols % 4 == 0))
        s.vec_leaf[t] = false;
      if (g.lda > kMaxLeadingDimA || g.ldb > kMaxLeadingDimB)
        throw Error(kNotSupported, "leading dimension too large for the leaf kernel");
      if (total > INT32_MAX) throw Error(kNotSupported, "leaf launch too large");
      if (phased) s.phase_tiles[phase] = (int)total;
    }
    s.leaf_tiles_total[t] = (int)total;
    if (phased) {
      int64_t all = 0;
      for (int j = 0; j < 7; ++j) all += s.phase_tiles[j];
      if (all > INT32_MAX) throw Error(kNotSupported, "leaf launch too large");
      s.leaf_tiles_total[t] = (int)all;
    }
  }
}

size_t schedule_desc_bytes(const Schedule& s) {
  size_t b = 0;
  for (int l = 0; l < s.max_depth; ++l) {
    b += align_up(s.preA[l].size() * sizeof(PreAddNode), 256);
    b += align_up(s.preB[l].size() * sizeof(PreAddNode), 256);
    b += align_up(s.post[l].size() * sizeof(PostAddNode), 256);
  }
  for (int t = 0; t < kNumTiles; ++t) b += align_up(s.leaf[t].size() * sizeof(GemmDesc), 256);
  for (const auto& t : s.trees) b += align_up(t.nodes.size() * sizeof(TreeNode), 256);
  for (int fmt = 0; fmt < 2; ++fmt)
    for (int side = 0; side < 2; ++side) b += align_up(s.pack[fmt][side].size() * sizeof(PackNode), 256);
  return b;
}

namespace {
int add_total_blocks(const std::vector<PreAddNode>& v) {
  if (v.empty()) return 0;
  return v.back().block_begin + (int)add_blocks_for(v.back().h_r, v.back().h_c);
}
int add_total_blocks(const std::vector<PostAddNode>& v) {
  if (v.empty()) return 0;
  return v.back().block_begin + (int)add_blocks_for(v.back().h_r, v.back().h_c);
}
}  // namespace

void upload_schedule(Library& L, Schedule& s, char* desc_dev, char* desc_host) {
  // Pack every descriptor array into one host block, upload it once.
  size_t off = 0;
  auto put = [&](const void* src, size_t bytes) {
    std::memcpy(desc_host + off, src, bytes);
    char* dev = desc_dev + off;
    off += align_up(bytes, 256);
    return dev;
  };
  s.d_preA.assign(s.max_depth, nullptr);
  s.d_preB.assign(s.max_depth, nullptr);
  s.d_post.assign(s.max_depth, nullptr);
  for (int l = 0; l < s.max_depth; ++l) {
    s.d_preA[l] = reinterpret_cast<const PreAddNode*>(put(s.preA[l].data(), s.preA[l].size() * sizeof(PreAddNode)));
    s.d_preB[l] = reinterpret_cast<const PreAddNode*>(put(s.preB[l].data(), s.preB[l].size() * sizeof(PreAddNode)));
    s.d_post[l] = reinterpret_cast<const PostAddNode*>(put(s.post[l].data(), s.post[l].size() * sizeof(PostAddNode)));
  }
  for (int t = 0; t < kNumTiles; ++t)
    s.d_leaf[t] = reinterpret_cast<const GemmDesc*>(put(s.leaf[t].data(), s.leaf[t].size() * sizeof(GemmDesc)));
  for (auto& t : s.trees)
    t.d_nodes = reinterpret_cast<const TreeNode*>(put(t.nodes.data(), t.nodes.size() * sizeof(TreeNode)));
  for (int fmt = 0; fmt < 2; ++fmt)
    for (int side = 0; side < 2; ++side)
      s.d_pack[fmt][side] = reinterpret_cast<const PackNode*>(
          put(s.pack[fmt][side].data(), s.pack[fmt][side].size() * sizeof(PackNode)));
  if (off) FASTMM_HIP(hipMemcpyAsync(desc_dev, desc_host, off, hipMemcpyHostToDevice, L.stream));
}

int launch_schedule(Library& L, Schedule& s, hipEvent_t leaf_begin, hipEvent_t leaf_end,
                    bool profile) {
  int launches = 0;
  if (profile) FASTMM_HIP(hipEventRecord(L.ev[1], L.stream));
  for (int l = 0; l < s.max_depth; ++l) {
    const int ba = add_total_blocks(s.preA[l]);
    const int bb = add_total_blocks(s.preB[l]);
    if (ba) { launch_preadd(0, s.d_preA[l], (int)s.preA[l].size(), ba, s.vec_preA[l], L.stream); ++launches; }
    if (bb) { launch_preadd(1, s.d_preB[l], (int)s.preB[l].size(), bb, s.vec_preB[l], L.stream); ++launches; }
    for (const auto& t : s.trees)
      if (t.kind < 2 && t.level == l && t.blocks > 0) {
        launch_tree_add(t.kind, t.levels, t.width, t.clip, t.d_nodes, (int)t.nodes.size(), t.blocks,
                        L.stream);
        ++launches;
      }
  }
  // Fused last-level pre-addition and pack of split-precision leaves; the
  // scaled FP16 form first takes its scale exponents from the same quadrants.
  if (!s.pack[1][0].empty()) {
    int max_rows = 0, max_cols = 0, max_kdim = 0;
    for (const auto& n : s.pack[1][0]) max_rows = std::max(max_rows, (int)n.q.h_r);
    for (const auto& n : s.pack[1][1]) {
      max_cols = std::max(max_cols, (int)n.q.h_c);
      max_kdim = std::max(max_kdim, (int)n.q.h_r);
    }
    launch_preadd_scale(s.d_pack[1][0], (int)s.pack[1][0].size(), s.d_pack[1][1],
                        (int)s.pack[1][1].size(), max_rows, max_cols, max_kdim, s.d_leaf[kTileFp16x3],
                        (int)s.leaf[kTileFp16x3].size(), L.stream);
    launches += 3;
  }
  for (int fmt = 0; fmt < 2; ++fmt)
    for (int side = 0; side < 2; ++side)
      if (s.pack_units[fmt][side] > 0) {
        launch_preadd_pack(side, s.d_pack[fmt][side], (int)s.pack[fmt][side].size(),
                           s.pack_units[fmt][side], fmt == 1, L.stream);
        ++launches;
      }
  if (profile) FASTMM_HIP(hipEventRecord(L.ev[2], L.stream));
  if (leaf_begin) FASTMM_HIP(hipEventRecord(leaf_begin, L.stream));
  for (int t = 0; t < kNumTiles; ++t) {
    if (s.leaf_tiles_total[t] <= 0) continue;
    if (t == kTileBf16x3 || t == kTileFp16x3) {
      LeafExtents ext;
      for (const auto& g : s.leaf[t]) {
        ext.max_a_rows = std::max(ext.max_a_rows, (int)g.a_rows);
        ext.max_b_cols = std::max(ext.max_b_cols, (int)g.b_cols);
        ext.max_c_rows = std::max(ext.max_c_rows, (int)g.c_rows);
        ext.max_c_cols = std::max(ext.max_c_cols, (int)g.c_cols);
        ext.max_slabs = std::max(ext.max_slabs, (int)((g.kmax + 31) / 32));
        ext.max_kmax = std::max(ext.max_kmax, (int)g.kmax);
      }
      ext.any_unpacked = false;
      for (const auto& g : s.leaf[t])
        if (!g.prepacked) ext.any_unpacked = true;
      launch_leaf_packed(t, s.d_leaf[t], (int)s.leaf[t].size(), s.leaf_tiles_total[t], s.vec_leaf[t],
                         L.stream, s.xcd_chunk[t], ext);
      // scale passes (FP16), the pack pass unless every operand is prepacked, the leaf
      launches += (t == kTileFp16x3 ? 2 : 0) + (ext.any_unpacked ? 1 : 0) + 1;
    } else if (s.fused_post && t == kTile128x128) {
      for (int j = 0; j < 7; ++j) {
        const int n = s.phase_begin[j + 1] - s.phase_begin[j];
        if (n <= 0) continue;
        launch_leaf_gemm(t, s.d_leaf[t] + s.phase_begin[j], n, s.phase_tiles[j], s.vec_leaf[t], L.stream,
                         0, nullptr, true);
        ++launches;
      }
    } else {
      launch_leaf_gemm(t, s.d_leaf[t], (int)s.leaf[t].size(), s.leaf_tiles_total[t], s.vec_leaf[t],
                       L.stream, s.xcd_chunk[t], s.persistent ? L.leaf_queue : nullptr);
      ++launches;
    }
  }
  if (leaf_end) FASTMM_HIP(hipEventRecord(leaf_end, L.stream));
  if (profile) FASTMM_HIP(hipEventRecord(L.ev[3], L.stream));
  for (int l = s.max_depth - 1; l >= 0; --l) {
    const int bp = add_total_blocks(s.post[l]);
    if (bp) { launch_postadd(s.d_post[l], (int)s.post[l].size(), bp, s.vec_post[l], L.stream); ++launches; }
    for (const auto& t : s.trees)
      if (t.kind == 2 && t.level == l && t.blocks > 0) {
        launch_tree_add(2, t.levels, t.width, false, t.d_nodes, (int)t.nodes.size(), t.blocks, L.stream);
        ++launches;
      }
  }
  if (profile) FASTMM_HIP(hipEventRecord(L.ev[4], L.stream));
  s.launches = launches;
  return launches;
}

int enqueue_schedule(Library& L, Schedule& s, char* desc_dev, char* desc_host,
                     hipEvent_t leaf_begin, hipEvent_t leaf_end) {
  upload_schedule(L, s, desc_dev, desc_host);
  return launch_schedule(L, s, leaf_begin, leaf_end, L.profiling);
}

// ---------------------------------------------------------------------------
// Argument checks shared by the single and batched paths.

namespace {

enum Residency { kHost = 0, kDevice = 1 };

Residency classify(const void* p) {
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return kHost;  // unknown to HIP: pageable host memory
  }
  if (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged) return kDevice;
  return kHost;
}

struct Range {
  uintptr_t lo, hi;
};

Range span(const void* p, int64_t rows, int64_t cols, int64_t ld) {
  if (rows <= 0 || cols <= 0 || p == nullptr) return {0, 0};
  const uintptr_t lo = reinterpret_cast<uintptr_t>(p);
  return {lo, lo + (uintptr_t)(((rows - 1) * ld + cols) * (int64_t)sizeof(float))};
}

bool overlaps(Range a, Range b) { return a.lo < a.hi && b.lo < b.hi && a.lo < b.hi && b.lo < a.hi; }

}  // namespace

void validate_gemm_args(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                        const float* B, int64_t ldb, const float* C, int64_t ldc, int depth) {
  if (M < 0 || N < 0 || K < 0) throw Error(kInvalidValue, "negative dimension");
  // K and N leave room for the staging's rounding up to a multiple of 4.
  if (M > INT32_MAX || N > INT32_MAX - 3 || K > INT32_MAX - 3)
    throw Error(kNotSupported, "dimension above 2^31-1 (K or N above 2^31-4)");
  if (lda < std::max<int64_t>(1, K)) throw Error(kInvalidValue, "lda < max(1, K)");
  if (ldb < std::max<int64_t>(1, N)) throw Error(kInvalidValue, "ldb < max(1, N)");
  if (ldc < std::max<int64_t>(1, N)) throw Error(kInvalidValue, "ldc < max(1, N)");
  if (depth > 16) throw Error(kInvalidValue, "depth > 16");
  if (lda > kMaxLeadingDimA || ldb > kMaxLeadingDimB)
    throw Error(kNotSupported, "lda above 2^21 or ldb above 2^24 is not supported");
  if (M > 0 && N > 0 && C == nullptr) throw Error(kInvalidValue, "C is NULL");
  if (M > 0 && K > 0 && A == nullptr) throw Error(kInvalidValue, "A is NULL");
  if (K > 0 && N > 0 && B == nullptr) throw Error(kInvalidValue, "B is NULL");
  const Range rc = span(C, M, N, ldc);
  if (overlaps(rc, span(A, M, K, lda)) || overlaps(rc, span(B, K, N, ldb)))
    throw Error(kInvalidValue, "C overlaps A or B");
}

// Residency of a product's operands: true = device.  Mixed -> error.
bool operands_on_device(int64_t M, int64_t N, int64_t K, const float* A, const float* B,
                        const float* C) {
  int dev = 0, host = 0;
  auto see = [&](const void* p, bool used) {
    if (!used) return;
    if (classify(p) == kDevice) ++dev; else ++host;
  };
  see(C, M > 0 && N > 0);
  see(A, M > 0 && K > 0);
  see(B, K > 0 && N > 0);
  if (dev && host)
    throw Error(kNotSupported, "A, B and C must be all device memory or all host memory");
  return dev > 0;
}

namespace {

double ev_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return -1.0;
  }
  return ms;
}

}  // namespace

// ---------------------------------------------------------------------------
// Workspace scheduler: level-wise when the whole tree's temporaries fit the
// budget, otherwise depth-first at the top: one level's S, T and P blocks are
// kept and the seven sub-products run one after another in the remaining
// space (each again level-wise if it fits, else depth-first), as the paper's
// recursion fits each call to the device capacity it finds (Section 3.3).

namespace {

size_t placeholder_desc_bytes(const Problem& p) {
  Problem q = p;
  q.A = q.B = reinterpret_cast<const float*>(256);
  q.C = const_cast<float*>(q.A);
  Schedule s;
  build_schedule({q}, reinterpret_cast<char*>(256), s);
  return align_up(schedule_desc_bytes(s), 256) + 256;
}

size_t bfs_need(const Problem& p) {
  return align_up(problem_temp_bytes(p), 256) + placeholder_desc_bytes(p);
}

size_t top_need(const Problem& p) {
  const int64_t m2 = split_at(p.M, p.depth), k2 = split_at(p.K, p.depth), n2 = split_at(p.N, p.depth);
  return align_up((size_t)4 * m2 * k2 * 4, 256) + align_up((size_t)4 * k2 * n2 * 4, 256) +
         align_up((size_t)7 * m2 * n2 * 4, 256) + 3 * 256;
}

// Sub-product i (P1..P7 = 0..6) of p, with p's S, T and P blocks at S, T, P.
Problem child_problem(const Problem& p, int i, float* S, float* T, float* P) {
  const int64_t m2 = split_at(p.M, p.depth), k2 = split_at(p.K, p.depth), n2 = split_at(p.N, p.depth);
  const View a{p.A, p.lda, p.ar(), p.ac()}, b{p.B, p.ldb, p.br(), p.bc()};
  auto sv = [&](int j) { return View{S + j * m2 * k2, k2, m2, k2}; };
  auto tv = [&](int j) { return View{T + j * k2 * n2, n2, k2, n2}; };
  const View ca[7] = {quadrant(a, 0, 0, m2, k2), quadrant(a, 0, 1, m2, k2), sv(3),
                      quadrant(a, 1, 1, m2, k2), sv(0), sv(1), sv(2)};
  const View cb[7] = {quadrant(b, 0, 0, k2, n2), quadrant(b, 1, 0, k2, n2),
                      quadrant(b, 1, 1, k2, n2), tv(3), tv(0), tv(1), tv(2)};
  Problem c;
  c.M = m2;
  c.K = k2;
  c.N = n2;
  c.A = ca[i].p;
  c.lda = ca[i].ld;
  c.a_rows = ca[i].vrows;
  c.a_cols = ca[i].vcols;
  c.B = cb[i].p;
  c.ldb = cb[i].ld;
  c.b_rows = cb[i].vrows;
  c.b_cols = cb[i].vcols;
  c.C = P + i * m2 * n2;
  c.ldc = n2;
  c.depth = p.depth - 1;
  c.tile = p.tile;
  return c;
}

// Smallest workspace the product can run in (level-wise or depth-first).
size_t min_need(const Problem& p) {
  const size_t b = bfs_need(p);
  if (p.depth == 0) return b;
  return std::min(b, top_need(p) + min_need(child_problem(p, 0, nullptr, nullptr, nullptr)));
}

struct RunTotals {
  int64_t leaves = 0;
  double leaf_flops = 0, add_bytes = 0;
  int launches = 0, leaf_launches = 0, schedules = 0;
  Dims leaf_dims{0, 0, 0};
};

// Enqueue p inside [ws, ws + bytes).  Each level-wise piece is followed by a
// stream synchronisation, so the one pinned descriptor buffer can be reused.
void run_within(Library& L, const Problem& p, char* ws, size_t bytes, RunTotals& rt) {
  const size_t need = bfs_need(p);
  if (need <= bytes) {
    const size_t t = align_up(problem_temp_bytes(p), 256);
    char* host = ensure_pinned(L, need - t);
    Schedule s;
    build_schedule({p}, ws, s);
    rt.launches += enqueue_schedule(L, s, ws + t, host);
    FASTMM_HIP(hipStreamSynchronize(L.stream));
    rt.leaves += s.leaves;
    rt.leaf_flops += s.leaf_flops;
    rt.add_bytes += s.add_bytes;
    rt.leaf_dims = s.leaf_dims;
    for (int k = 0; k < kNumTiles; ++k) rt.leaf_launches += s.leaf_tiles_total[k] > 0 ? 1 : 0;
    ++rt.schedules;
    return;
  }
  if (p.depth == 0 || top_need(p) >= bytes)
    throw Error(kOutOfMemory, "workspace budget too small even for depth-first execution");
  const int64_t m2 = split_at(p.M, p.depth), k2 = split_at(p.K, p.depth), n2 = split_at(p.N, p.depth);
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = ws + off;
    off += align_up(b, 256);
    return q;
  };
  float* S = reinterpret_cast<float*>(take((size_t)4 * m2 * k2 * 4));
  float* T = reinterpret_cast<float*>(take((size_t)4 * k2 * n2 * 4));
  float* P = reinterpret_cast<float*>(take((size_t)7 * m2 * n2 * 4));
  char* dnodes = take(3 * 256);
  char* host = ensure_pinned(L, 3 * 256);
  const PreAddNode na = preadd_node(p.A, p.lda, p.ar(), p.ac(), m2, k2, S);
  const PreAddNode nb = preadd_node(p.B, p.ldb, p.br(), p.bc(), k2, n2, T);
  const PostAddNode np = postadd_node(P, m2, n2, p.C, p.ldc, p.cr(), p.cc());
  std::memcpy(host, &na, sizeof(na));
  std::memcpy(host + 256, &nb, sizeof(nb));
  std::memcpy(host + 512, &np, sizeof(np));
  FASTMM_HIP(hipMemcpyAsync(dnodes, host, 3 * 256, hipMemcpyHostToDevice, L.stream));
  launch_preadd(0, reinterpret_cast<const PreAddNode*>(dnodes), 1,
                (int)add_blocks_for(m2, k2), pre_vec_ok(na), L.stream);
  launch_preadd(1, reinterpret_cast<const PreAddNode*>(dnodes + 256), 1,
                (int)add_blocks_for(k2, n2), pre_vec_ok(nb), L.stream);
  FASTMM_HIP(hipStreamSynchronize(L.stream));  // the pinned block is reused below
  rt.launches += 2;
  for (int i = 0; i < 7; ++i) run_within(L, child_problem(p, i, S, T, P), ws + off, bytes - off, rt);
  // A child may have grown (reallocated) the pinned block for its own
  // descriptors: take its current address again.
  host = ensure_pinned(L, 3 * 256);
  std::memcpy(host + 512, &np, sizeof(np));
  FASTMM_HIP(hipMemcpyAsync(dnodes + 512, host + 512, sizeof(np), hipMemcpyHostToDevice, L.stream));
  launch_postadd(reinterpret_cast<const PostAddNode*>(dnodes + 512), 1,
                 (int)add_blocks_for(m2, n2), post_vec_ok(np), L.stream);
  FASTMM_HIP(hipStreamSynchronize(L.stream));
  rt.launches += 1;
  rt.add_bytes += 32.0 * m2 * k2 + 32.0 * k2 * n2 + 44.0 * m2 * n2;
}

// Device memory the library may use: FASTMM_WORKSPACE_LIMIT if set, else the
// free memory plus the current workspace, less a safety margin.
size_t workspace_budget(Library& L) {
  if (const char* s = std::getenv("FASTMM_WORKSPACE_LIMIT")) return std::strtoull(s, nullptr, 10);
  size_t free_b = 0, total_b = 0;
  FASTMM_HIP(hipMemGetInfo(&free_b, &total_b));
  const size_t avail = free_b + L.arena_bytes;
  const size_t margin = std::min<size_t>(avail / 16, size_t(2) << 30);
  return avail - margin;
}

}  // namespace

Staging plan_staging(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
                     int64_t ldb, bool on_dev) {
  Staging g;
  g.K4 = (K + 3) / 4 * 4;
  g.N4 = (N + 3) / 4 * 4;
  if (g.K4 > INT32_MAX || g.N4 > INT32_MAX)
    throw Error(kNotSupported, "K or N within 3 of 2^31: no room for the 16-byte padding");
  g.a = !on_dev || !(aligned16(A) && lda % 4 == 0 && K % 4 == 0);
  g.b = !on_dev || !(aligned16(B) && ldb % 4 == 0 && N % 4 == 0 && K % 4 == 0);
  g.a_bytes = (g.a && K > 0) ? align_up((size_t)M * g.K4 * 4, 256) : 0;
  g.b_bytes = (g.b && K > 0) ? align_up((size_t)g.K4 * g.N4 * 4, 256) : 0;
  return g;
}

void stage_operands(const Staging& g, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                    const float* B, int64_t ldb, float* dA, float* dB, hipStream_t sm) {
  if (K == 0) return;
  const int64_t K4 = g.K4, N4 = g.N4;
  if (g.a) {
    if (K4 > K) FASTMM_HIP(hipMemset2DAsync(dA + K, K4 * 4, 0, (K4 - K) * 4, M, sm));
    FASTMM_HIP(hipMemcpy2DAsync(dA, K4 * 4, A, lda * 4, K * 4, M, hipMemcpyDefault, sm));
  }
  if (g.b) {
    if (N4 > N) FASTMM_HIP(hipMemset2DAsync(dB + N, N4 * 4, 0, (N4 - N) * 4, K, sm));
    if (K4 > K) FASTMM_HIP(hipMemsetAsync(dB + K * N4, 0, (K4 - K) * N4 * 4, sm));
    FASTMM_HIP(hipMemcpy2DAsync(dB, N4 * 4, B, ldb * 4, N * 4, K, hipMemcpyDefault, sm));
  }
}

void gemm_impl(Library& L, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
               const float* B, int64_t ldb, float* C, int64_t ldc, int depth, int64_t leaf,
               int tile) {
  validate_gemm_args(M, N, K, A, lda, B, ldb, C, ldc, depth);
  if (tile >= kNumTiles) throw Error(kInvalidValue, "unknown tile id");
  ensure_init(L);
  fastmm_stats_t st{};
  st.h2d_ms = st.preadd_ms = st.leaf_ms = st.postadd_ms = st.d2h_ms = st.total_ms = -1.0;
  if (M == 0 || N == 0) {
    L.stats = st;
    return;
  }
  const bool on_dev = operands_on_device(M, N, K, A, B, C);

  if (depth < 0 || tile < 0) {
    fastmm_plan_t pl{};
    int rc = plan_choose(L, M, N, K, L.plan_mode, &pl);
    if (rc != kSuccess) throw Error(rc, "planner failed");
    if (depth < 0) {
      depth = pl.depth;
      leaf = pl.leaf;
      // Host operands: below this extent the transfers bound the call, and
      // the plain product's pipeline ends sooner than the Winograd one,
      // whose last pieces (P2, P3) and result blocks wait for the last
      // input blocks (pinned, repeated calls, median of 6: n = 4096 3.5
      // against 3.9 ms at the planner's depth 1, n = 6144 7.4 against 7.9 ms
      // at depth 2; from n = 7168 on Winograd leads, 10.8 against 11.6 ms,
      // except at 8192, 13.7 against 13.1 ms).
      constexpr int64_t kHostPlainBelow = 6656;
      if (!on_dev && std::min(std::min(M, N), K) < kHostPlainBelow) depth = 0;
    }
    if (tile < 0) tile = pl.tile;
  }

  Problem p;
  p.M = M;
  p.N = N;
  p.K = K;
  p.depth = (K == 0) ? 0 : effective_depth(M, N, K, depth, leaf);
  p.tile = tile;

  const char* pipe = std::getenv("FASTMM_PIPELINE");
  const bool pipelined = !(pipe && pipe[0] == '0');
  if (!on_dev && pipelined && std::min(std::min(M, N), K) >= 2 &&
      pipelined_need(M, N, K, p.depth, tile) <= workspace_budget(L)) {
    try {
      gemm_host_pipelined(L, M, N, K, A, lda, B, ldb, C, ldc, p.depth, tile, st);
    } catch (...) {
      // Work already queued on the staged path's streams must not outlive
      // the call: the next one reuses the workspace it reads and writes.
      for (hipStream_t x : {L.stream, L.aux_stream, L.h2d_stream, L.d2h_stream})
        if (x) (void)hipStreamSynchronize(x);
      (void)hipGetLastError();
      throw;
    }
    if (!L.profiling) {
      st.h2d_ms = st.preadd_ms = st.leaf_ms = st.postadd_ms = st.d2h_ms = st.total_ms = -1.0;
    }
    L.stats = st;
    return;
  }

  // Staging (plan_staging): host operands, and device operands the leaf's
  // 16-byte load path cannot read, go to padded buffers in the workspace;
  // the product then runs on the padded extents and C keeps N columns.
  const Staging sg = plan_staging(M, N, K, A, lda, B, ldb, on_dev);
  const bool stage_a = sg.a, stage_b = sg.b;
  const int64_t lda_s = stage_a ? sg.K4 : lda, ldb_s = stage_b ? sg.N4 : ldb;
  p.K = sg.K4;  // K4 > K only when both operands are staged
  p.N = sg.N4;  // N4 > N only when B is staged
  p.c_cols = N;

  // Workspace: [staged A | staged B | staged C | temporaries | descriptors].
  const size_t a_bytes = sg.a_bytes;
  const size_t b_bytes = sg.b_bytes;
  const size_t c_bytes = on_dev ? 0 : align_up((size_t)M * N * 4, 256);
  const size_t t_bytes = align_up(problem_temp_bytes(p), 256);
  auto stage_in = [&](float* dA, float* dB, hipStream_t sm) {
    stage_operands(sg, M, N, K, A, lda, B, ldb, dA, dB, sm);
  };

  // Over budget: depth-first execution of the top levels.
  if (K > 0 && p.depth > 0) {
    const size_t stage = a_bytes + b_bytes + c_bytes;
    const size_t budget = workspace_budget(L);
    if (stage + bfs_need(p) > budget) {
      const size_t need = stage + min_need(p);
      if (need > budget)
        throw Error(kOutOfMemory, "workspace of " + std::to_string(need) +
                                      " bytes (depth-first) exceeds the budget of " +
                                      std::to_string(budget) + " (FASTMM_WORKSPACE_LIMIT or free memory)");
      char* ws = ensure_arena(L, budget);
      float* dA = stage_a ? reinterpret_cast<float*>(ws) : const_cast<float*>(A);
      float* dB = stage_b ? reinterpret_cast<float*>(ws + a_bytes) : const_cast<float*>(B);
      float* dC = on_dev ? C : reinterpret_cast<float*>(ws + a_bytes + b_bytes);
      stage_in(dA, dB, L.stream);
      p.A = dA;
      p.B = dB;
      p.C = dC;
      p.lda = lda_s;
      p.ldb = ldb_s;
      p.ldc = on_dev ? ldc : N;
      RunTotals rt;
      run_within(L, p, ws + stage, budget - stage, rt);
      if (!on_dev)
        FASTMM_HIP(hipMemcpy2DAsync(C, ldc * 4, dC, N * 4, N * 4, M, hipMemcpyDeviceToHost, L.stream));
      FASTMM_HIP(hipStreamSynchronize(L.stream));
      st.depth = p.depth;
      st.tile = tile;
      st.leaves = rt.leaves;
      st.leaf_m = rt.leaf_dims.m;
      st.leaf_k = rt.leaf_dims.k;
      st.leaf_n = rt.leaf_dims.n;
      st.leaf_flops = rt.leaf_flops;
      st.add_bytes = rt.add_bytes;
      st.transfer_bytes = on_dev ? 0.0 : 4.0 * ((double)M * K + (double)K * N + (double)M * N);
      st.launches = rt.launches;
      st.leaf_launches = rt.leaf_launches;
      st.workspace_bytes = L.arena_bytes;
      L.stats = st;
      return;
    }
  }

  // Schedule with temporaries at a placeholder base to size the descriptors.
  Schedule s;
  {
    Problem q = p;
    q.A = reinterpret_cast<const float*>(256);
    q.B = q.A;
    q.C = const_cast<float*>(q.A);
    q.lda = lda_s;
    q.ldb = ldb_s;
    q.ldc = on_dev ? ldc : N;
    build_schedule({q}, reinterpret_cast<char*>(256), s);
  }
  const size_t d_bytes = align_up(schedule_desc_bytes(s), 256) + 256;
  char* ws = ensure_arena(L, a_bytes + b_bytes + c_bytes + t_bytes + d_bytes);
  char* desc_host = ensure_pinned(L, d_bytes);

  float* dA = stage_a ? reinterpret_cast<float*>(ws) : const_cast<float*>(A);
  float* dB = stage_b ? reinterpret_cast<float*>(ws + a_bytes) : const_cast<float*>(B);
  float* dC = on_dev ? C : reinterpret_cast<float*>(ws + a_bytes + b_bytes);
  p.A = dA;
  p.B = dB;
  p.C = dC;
  p.lda = lda_s;
  p.ldb = ldb_s;
  p.ldc = on_dev ? ldc : N;
  char* temps = ws + a_bytes + b_bytes + c_bytes;
  char* desc_dev = temps + t_bytes;

  hipStream_t sm = L.stream;
  if (L.profiling) FASTMM_HIP(hipEventRecord(L.ev[0], sm));
  // Step (1) of the paper's leaf call (operands to the device), or the
  // alignment staging of device operands.
  stage_in(dA, dB, sm);
  if (L.profiling) FASTMM_HIP(hipEventRecord(L.ev[5], sm));
  int launches = 0;
  if (K == 0) {
    FASTMM_HIP(hipMemset2DAsync(dC, p.ldc * 4, 0, N * 4, M, sm));
  } else {
    build_schedule({p}, temps, s);
    launches = enqueue_schedule(L, s, desc_dev, desc_host);
  }
  if (L.profiling) FASTMM_HIP(hipEventRecord(L.ev[6], sm));
  if (!on_dev) {
    // Step (3): the result back to the host.
    FASTMM_HIP(hipMemcpy2DAsync(C, ldc * 4, dC, N * 4, N * 4, M, hipMemcpyDeviceToHost, sm));
  }
  if (L.profiling) FASTMM_HIP(hipEventRecord(L.ev[7], sm));
  FASTMM_HIP(hipStreamSynchronize(sm));

  st.depth = p.depth;
  st.tile = tile;
  st.leaves = s.leaves;
  st.leaf_m = s.leaf_dims.m;
  st.leaf_k = s.leaf_dims.k;
  st.leaf_n = s.leaf_dims.n;
  st.leaf_flops = s.leaf_flops;
  st.add_bytes = s.add_bytes;
  st.transfer_bytes = on_dev ? 0.0 : 4.0 * ((double)M * K + (double)K * N + (double)M * N);
  st.launches = launches;
  st.workspace_bytes = L.arena_bytes;
  st.leaf_launches = 0;
  for (int t = 0; t < kNumTiles; ++t) st.leaf_launches += s.leaf_tiles_total[t] > 0 ? 1 : 0;
  if (L.profiling && K > 0) {
    st.h2d_ms = ev_ms(L.ev[0], L.ev[5]);
    st.preadd_ms = ev_ms(L.ev[1], L.ev[2]);
    st.leaf_ms = ev_ms(L.ev[2], L.ev[3]);
    st.postadd_ms = ev_ms(L.ev[3], L.ev[4]);
    st.d2h_ms = ev_ms(L.ev[6], L.ev[7]);
    st.total_ms = ev_ms(L.ev[0], L.ev[7]);
  }
  L.stats = st;
}

namespace {

template <typename F>
int guarded(F&& f) {
  try {
    t_last_error.clear();
    f();
    return kSuccess;
  } catch (const Error& e) {
    t_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    t_last_error = "host allocation failed";
    return kOutOfMemory;
  } catch (const std::exception& e) {
    t_last_error = e.what();
    return kDeviceError;
  } catch (...) {
    t_last_error = "unknown error";
    return kDeviceError;
  }
}

}  // namespace

int run_guarded(const std::function<void()>& f) { return guarded(f); }

}  // namespace fastmm

using namespace fastmm;

extern "C" {

int fastmm_gemm_ex(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
                   int64_t ldb, float* C, int64_t ldc, int depth, int64_t leaf, int tile) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return guarded([&] { gemm_impl(L, M, N, K, A, lda, B, ldb, C, ldc, depth, leaf, tile); });
}

int fastmm_gemm(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
                int64_t ldb, float* C, int64_t ldc, int depth, int64_t leaf) {
  const int tile = depth < 0 ? -1 : kTile128x128;
  return fastmm_gemm_ex(M, N, K, A, lda, B, ldb, C, ldc, depth, leaf, tile);
}

int fastmm_set_stream(void* hip_stream) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return guarded([&] {
    ensure_init(L);
    FASTMM_HIP(hipStreamSynchronize(L.stream));
    L.stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : L.own_stream;
  });
}

int fastmm_set_profiling(int on) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  L.profiling = (on != 0);
  return kSuccess;
}

int fastmm_get_stats(fastmm_stats_t* out) {
  if (!out) {
    t_last_error = "out is NULL";
    return kInvalidValue;
  }
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  *out = L.stats;
  return kSuccess;
}

const char* fastmm_get_last_error(void) { return t_last_error.c_str(); }

int fastmm_preadd(int side, int64_t rows, int64_t cols, const float* X, int64_t ldx, float* out) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return guarded([&] {
    if (side != 0 && side != 1) throw Error(kInvalidValue, "side must be 0 (A) or 1 (B)");
    if (rows < 0 || cols < 0 || rows > INT32_MAX || cols > INT32_MAX)
      throw Error(kInvalidValue, "bad extent");
    if (ldx < std::max<int64_t>(1, cols)) throw Error(kInvalidValue, "ldx < max(1, cols)");
    if (rows == 0 || cols == 0) return;
    if (!X || !out) throw Error(kInvalidValue, "NULL pointer");
    ensure_init(L);
    if (classify(X) != kDevice || classify(out) != kDevice)
      throw Error(kNotSupported, "fastmm_preadd takes device pointers");
    PreAddNode n = preadd_node(X, ldx, rows, cols, half_up(rows), half_up(cols), out);
    const bool vec = pre_vec_ok(n);
    char* dev = ensure_arena(L, 256);
    char* host = ensure_pinned(L, sizeof(n));
    std::memcpy(host, &n, sizeof(n));
    FASTMM_HIP(hipMemcpyAsync(dev, host, sizeof(n), hipMemcpyHostToDevice, L.stream));
    launch_preadd(side, reinterpret_cast<const PreAddNode*>(dev), 1,
                  (int)add_blocks_for(n.h_r, n.h_c), vec, L.stream);
    FASTMM_HIP(hipStreamSynchronize(L.stream));
  });
}

int fastmm_postadd(int64_t h_r, int64_t h_c, const float* P, float* C, int64_t ldc, int64_t rows,
                   int64_t cols) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return guarded([&] {
    if (h_r < 0 || h_c < 0 || h_r > INT32_MAX / 2 || h_c > INT32_MAX / 2)
      throw Error(kInvalidValue, "bad extent");
    if (rows < 0 || cols < 0 || rows > 2 * h_r || cols > 2 * h_c)
      throw Error(kInvalidValue, "rows/cols must lie in [0, 2 h]");
    if (ldc < std::max<int64_t>(1, cols)) throw Error(kInvalidValue, "ldc < max(1, cols)");
    if (h_r == 0 || h_c == 0 || rows == 0 || cols == 0) return;
    if (!P || !C) throw Error(kInvalidValue, "NULL pointer");
    ensure_init(L);
    if (classify(P) != kDevice || classify(C) != kDevice)
      throw Error(kNotSupported, "fastmm_postadd takes device pointers");
    PostAddNode n = postadd_node(P, h_r, h_c, C, ldc, rows, cols);
    const bool vec = post_vec_ok(n);
    char* dev = ensure_arena(L, 256);
    char* host = ensure_pinned(L, sizeof(n));
    std::memcpy(host, &n, sizeof(n));
    FASTMM_HIP(hipMemcpyAsync(dev, host, sizeof(n), hipMemcpyHostToDevice, L.stream));
    launch_postadd(reinterpret_cast<const PostAddNode*>(dev), 1, (int)add_blocks_for(h_r, h_c), vec,
                   L.stream);
    FASTMM_HIP(hipStreamSynchronize(L.stream));
  });
}

void fastmm_finalize(void) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  if (!L.initialised) return;
  (void)hipStreamSynchronize(L.stream);
  if (L.h2d_stream) (void)hipStreamSynchronize(L.h2d_stream);
  if (L.d2h_stream) (void)hipStreamSynchronize(L.d2h_stream);
  if (L.aux_stream) (void)hipStreamSynchronize(L.aux_stream);
  destroy_graphs();
  if (L.arena) (void)hipFree(L.arena);
  if (L.pinned) (void)hipHostFree(L.pinned);
  for (auto& e : L.ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : L.sync_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : L.leaf_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : L.tune_ev)
    if (e) (void)hipEventDestroy(e);
  if (L.h2d_stream) (void)hipStreamDestroy(L.h2d_stream);
  if (L.d2h_stream) (void)hipStreamDestroy(L.d2h_stream);
  if (L.aux_stream) (void)hipStreamDestroy(L.aux_stream);
  L.h2d_stream = L.d2h_stream = L.aux_stream = nullptr;
  for (auto& e : L.sync_ev) e = nullptr;
  for (auto& e : L.leaf_ev) e = nullptr;
  for (auto& e : L.tune_ev) e = nullptr;
  if (L.own_stream) (void)hipStreamDestroy(L.own_stream);
  L.leaf_queue = nullptr;  // static device memory: nothing to free
  L.arena = nullptr;
  L.arena_bytes = 0;
  L.pinned = nullptr;
  L.pinned_bytes = 0;
  L.own_stream = nullptr;
  L.stream = nullptr;
  for (auto& e : L.ev) e = nullptr;
  L.initialised = false;
}

}  // extern "C"
