// Recursion engine: turns one or many products into a level-wise schedule of
// grouped launches (pre-additions per level, one grouped leaf launch per tile
// shape, post-additions per level) over a single device workspace.
#pragma once

#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fastmm.h"
#include "common.h"

namespace fastmm {

// Extents (m, k, n) of the nodes of one recursion level.
struct Dims {
  int64_t m, k, n;
};

// Half extent of equation (1): quadrant 0 takes ceil(m/2).
inline int64_t half_up(int64_t m) { return (m + 1) / 2; }

// One step of the ceil(m/2) chain, rounded up to a multiple of 4 once it
// reaches 64 (16-byte aligned rows and quadrant offsets; the extra rows or
// columns are virtual zeros, quadrant 1 keeps m minus this, at least 61).
// The stop rule's depth is decided on this chain, and the classic recursion
// splits at it; the Winograd engine splits at split_at below.
inline int64_t split_half(int64_t m) {
  const int64_t h = (m + 1) / 2;
  return h >= 64 ? (h + 3) / 4 * 4 : h;
}

// Leaf extent of a d-level split of m: ceil(m / 2^d), rounded up just
// enough that every level's extent (2^j leaf extents) of 64 or more is a
// multiple of 4: to a multiple of 4 from 64 on, to an even number from 32 on
// when the level above it exists.  (The top level's bottom quadrant keeps
// m - 2^(d-1) x leaf >= 1 rows.)
inline int64_t leaf_extent(int64_t m, int d) {
  const int64_t leaf = (m + (int64_t(1) << d) - 1) >> d;
  const int64_t g = leaf >= 64 ? 4 : (d >= 2 && leaf >= 32) ? 2 : 1;
  return (leaf + g - 1) / g * g;
}

// Quadrant extent at which the engine splits m when d levels remain
// (d >= 1): 2^(d-1) leaf extents.  Every level below is then exactly twice
// the next, so only the quadrants of the operands at the top of the
// recursion can be clipped (their missing rows and columns are virtual
// zeros), and several levels of additions can share one pass.  For d = 1
// this is split_half(m); where repeated split_half is exact at every level
// the two rules agree.
inline int64_t split_at(int64_t m, int d) { return d <= 0 ? m : leaf_extent(m, d) << (d - 1); }

// Stop rule: split iff levels remain and floor(min(m,k,n)/2) >= max(leaf,1).
inline bool splits(int64_t m, int64_t k, int64_t n, int levels_left, int64_t leaf) {
  int64_t mn = m < k ? m : k;
  mn = mn < n ? mn : n;
  return levels_left > 0 && mn / 2 >= (leaf > 1 ? leaf : 1);
}

int effective_depth(int64_t M, int64_t N, int64_t K, int depth, int64_t leaf);

// One product as the engine sees it, operands already device-resident.
// M, N, K are the (virtual) extents; each operand may hold fewer valid rows
// or columns (the rest reads as zero), which is how a quadrant of an odd
// extent enters the recursion.  C is written over c_rows x c_cols.
struct Problem {
  int64_t M = 0, N = 0, K = 0;
  const float* A = nullptr;
  int64_t lda = 0;
  int64_t a_rows = -1, a_cols = -1;  // -1: M, K
  const float* B = nullptr;
  int64_t ldb = 0;
  int64_t b_rows = -1, b_cols = -1;  // -1: K, N
  float* C = nullptr;
  int64_t ldc = 0;
  int64_t c_rows = -1, c_cols = -1;  // -1: M, N
  int depth = 0;  // effective depth
  int tile = 0;
  // Optional home of the B-side temporaries (the T blocks of every level,
  // b_tree_bytes of them) outside the schedule's workspace, so that several
  // products with the same right operand can share them; with
  // b_tree_ready they are taken as already computed and no B-side
  // pre-additions are issued.
  float* b_tree = nullptr;
  bool b_tree_ready = false;
  // The same for the A-side temporaries (the S blocks of every level,
  // a_tree_bytes of them), for products that share their left operand.
  float* a_tree = nullptr;
  bool a_tree_ready = false;
  int64_t ar() const { return a_rows < 0 ? M : a_rows; }
  int64_t ac() const { return a_cols < 0 ? K : a_cols; }
  int64_t br() const { return b_rows < 0 ? K : b_rows; }
  int64_t bc() const { return b_cols < 0 ? N : b_cols; }
  int64_t cr() const { return c_rows < 0 ? M : c_rows; }
  int64_t cc() const { return c_cols < 0 ? N : c_cols; }
};

// A level-wise schedule over a set of problems.
struct Schedule {
  std::vector<std::vector<PreAddNode>> preA, preB;  // per level
  std::vector<std::vector<PostAddNode>> post;       // per level
  std::vector<GemmDesc> leaf[kNumTiles];
  std::vector<int> leaf_tiles_total;                // per tile id
  std::vector<char> vec_preA, vec_preB, vec_post;   // per level
  // Device addresses of the uploaded descriptor arrays (upload_schedule).
  std::vector<const PreAddNode*> d_preA, d_preB;
  std::vector<const PostAddNode*> d_post;
  const GemmDesc* d_leaf[kNumTiles] = {};
  // Split-precision leaves: fused last-level pre-addition and pack nodes,
  // [format: 0 split BF16, 1 scaled split FP16][side: 0 A, 1 B], their
  // workgroup totals and device copies.
  std::vector<PackNode> pack[2][2];
  int pack_units[2][2] = {};
  const PackNode* d_pack[2][2] = {};
  // Multi-level additions (subtrees that split exactly at every level):
  // one launch per kind (0 A-side pre, 1 B-side pre, 2 post), top level and
  // number of levels; pre launches run with the level-wise ones of their
  // top level, post launches with the post-additions of their top level.
  struct TreeLaunch {
    int kind = 0, level = 0, levels = 0, width = 1, blocks = 0;
    bool clip = false;  // some top operand is clipped (pre-additions only)
    std::vector<TreeNode> nodes;
    const TreeNode* d_nodes = nullptr;
  };
  std::vector<TreeLaunch> trees;
  bool vec_leaf[kNumTiles] = {};  // set in build_schedule
  // Last-level post-additions fused into the leaf epilogue
  // (FASTMM_FUSED_POST=1, one problem of depth >= 1, 128x128 tiles): its
  // leaves run in seven launches, launch j holding product kFusedPostOrder[j]
  // of every last-level node (s.leaf[kTile128x128][phase_begin[j] ..
  // phase_begin[j + 1]), tile numbers restarting at 0, phase_tiles[j] tiles).
  bool fused_post = false;
  int phase_begin[8] = {};
  int phase_tiles[7] = {};
  int xcd_chunk[kNumTiles] = {};  // leaf launch tile -> XCD mapping (leaf_tile_of_block)
  bool persistent = false;        // leaf launches take tiles from L.leaf_queue
  int max_depth = 0;
  size_t temp_bytes = 0;  // bytes of S, T and P temporaries
  // statistics
  int64_t leaves = 0;
  double leaf_flops = 0.0;
  double add_bytes = 0.0;
  int launches = 0;
  Dims leaf_dims{0, 0, 0};
};

// Bytes of temporaries a problem needs in the schedule's workspace (no
// allocation; without the B-side blocks when p.b_tree is set, nor the A-side
// ones when p.a_tree is).
size_t problem_temp_bytes(const Problem& p);
// Bytes of the B-side (A-side) temporaries of a product with these extents
// and depth.
size_t b_tree_bytes(int64_t M, int64_t K, int64_t N, int depth);
size_t a_tree_bytes(int64_t M, int64_t K, int64_t N, int depth);

// Builds the schedule; temporaries are carved from `ws` (device), which must
// hold at least the sum of problem_temp_bytes.
void build_schedule(const std::vector<Problem>& probs, char* ws, Schedule& s);

// Library state (one per process).
struct Library {
  std::mutex mu;
  bool initialised = false;
  int device = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;  // stream in use
  char* arena = nullptr;         // device workspace
  size_t arena_bytes = 0;
  char* pinned = nullptr;        // host staging for descriptors
  size_t pinned_bytes = 0;
  bool profiling = false;
  hipEvent_t ev[8] = {};
  hipStream_t h2d_stream = nullptr;  // host->device staging copies
  hipStream_t d2h_stream = nullptr;  // device->host result copies
  hipStream_t aux_stream = nullptr;  // second compute stream of the staged path
  static constexpr int kSyncEvents = 512;
  hipEvent_t sync_ev[kSyncEvents] = {};  // ordering between the streams
  static constexpr int kLeafEvents = 256;
  hipEvent_t leaf_ev[kLeafEvents] = {};  // timing of leaf launches
  hipEvent_t tune_ev[2] = {};            // planner's candidate timing
  int* leaf_queue = nullptr;             // two counters for persistent leaf launches
  fastmm_stats_t stats{};
  size_t limit = 0;              // workspace cap (0: none)
  int plan_mode = FASTMM_PLAN_DEFAULT;
  uint64_t arena_generation = 0;  // bumped whenever the workspace moves
};

Library& lib();
void ensure_init(Library& L);
// Device address of the statically allocated workspace on `device` (looked
// up once per device with that device current; noalloc.cpp), and the bytes
// at its head that hold the persistent leaf launches' counters.
char* bind_static_scratch(int device);
size_t static_queue_bytes();
char* ensure_arena(Library& L, size_t bytes);
char* ensure_pinned(Library& L, size_t bytes);

// Uploads every descriptor array of `s` (one copy) and enqueues all launches
// on L.stream.  Returns the number of launches.  Events ev[1..4] bracket
// pre-additions, leaves and post-additions when profiling is on.
int enqueue_schedule(Library& L, Schedule& s, char* desc_dev, char* desc_host,
                     hipEvent_t leaf_begin = nullptr, hipEvent_t leaf_end = nullptr);
// The two halves of enqueue_schedule: copy the descriptor arrays to the
// device (stream-ordered), then issue the launches.  Only the launches are
// captured into a graph by the batched path.
void upload_schedule(Library& L, Schedule& s, char* desc_dev, char* desc_host);
int launch_schedule(Library& L, Schedule& s, hipEvent_t leaf_begin, hipEvent_t leaf_end,
                    bool profile);
size_t schedule_desc_bytes(const Schedule& s);

// Host-resident operands: stage quadrants in, run the top level of the
// recursion product by product as the quadrants arrive, and stream result
// quadrants out as they complete (pipeline.cpp).
// Workspace bytes the pipelined path needs for this product.
size_t pipelined_need(int64_t M, int64_t N, int64_t K, int depth, int tile);
void gemm_host_pipelined(Library& L, int64_t M, int64_t N, int64_t K, const float* A,
                         int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc,
                         int depth, int tile, fastmm_stats_t& st);

// Staging of one product's operands.  The leaf kernels' 16-byte load path
// (slabs straight into LDS) needs 16-byte aligned rows and K, N multiples of
// 4; without it every leaf of the launch takes the 4-byte path (23-30%
// slower).  Host operands are always staged; device operands that miss
// those conditions are copied once.  Staged A is M x K4 (lda K4), staged B
// K4 x N4 (ldb N4), with K4, N4 = K, N rounded up to 4 and zeros beyond K
// and N, so the product can run on the padded extents.
struct Staging {
  bool a = false, b = false;  // operand staged
  int64_t K4 = 0, N4 = 0;
  size_t a_bytes = 0, b_bytes = 0;  // workspace bytes of the staged copies
};
Staging plan_staging(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
                     int64_t ldb, bool on_dev);
// Enqueues the staging copies and zero padding (memsets: not for graphs).
void stage_operands(const Staging& g, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                    const float* B, int64_t ldb, float* dA, float* dB, hipStream_t sm);

// The single-product path behind fastmm_gemm_ex (caller holds L.mu).
void gemm_impl(Library& L, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
               const float* B, int64_t ldb, float* C, int64_t ldc, int depth, int64_t leaf,
               int tile);

bool aligned16(const void* p);
bool pre_vec_ok(const PreAddNode& n);
bool post_vec_ok(const PostAddNode& n);

// Batched path's graph cache (batched.cpp).
void destroy_graphs();
int64_t graph_captures();
int64_t graph_replays();

// Planner hooks (planner.cpp).
int plan_choose(Library& L, int64_t M, int64_t N, int64_t K, int mode, fastmm_plan_t* out);
// The plan of one problem of a batched call (128x128 tiles; see planner.cpp).
int plan_choose_batched(Library& L, int64_t M, int64_t N, int64_t K, int mode, fastmm_plan_t* out);
int64_t default_leaf();
// Changes whenever the planner's timings or model change (so plans taken
// earlier may no longer be the planner's choice).
uint64_t planner_epoch();

void set_error(const std::string& msg);

// Runs f, turning exceptions into a status code and the thread's last error.
int run_guarded(const std::function<void()>& f);

// Argument checks (throw Error before anything is written).
void validate_gemm_args(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                        const float* B, int64_t ldb, const float* C, int64_t ldc, int depth);
// true: all used operands are device memory; false: all host; mixed: throws.
bool operands_on_device(int64_t M, int64_t N, int64_t K, const float* A, const float* B,
                        const float* C);

}  // namespace fastmm
