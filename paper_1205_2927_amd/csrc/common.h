// Shared types of the fastmm HIP library (gfx950 / CDNA4).
//
// A matrix operand anywhere in the recursion is a strided view with a
// "valid" extent: elements outside it read as zero.  That is how odd extents
// follow the paper's quadrant split (equation (1), Section 3.1: quadrant 0 is
// ceil(m/2) x ceil(n/2), quadrant 3 floor(m/2) x floor(n/2)) while every
// quadrant of one level keeps the same virtual shape (the engine places the
// split at or a little above ceil(m/2): split_at in engine.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>

namespace fastmm {

// One problem of a grouped leaf launch: C (c_rows x c_cols, ldc) =
// A (a_rows x kmax valid, lda) * B (kmax x b_cols valid, ldb).  Rows of C at
// or beyond a_rows and columns at or beyond b_cols come out zero.
struct GemmDesc {
  const float* A;
  const float* B;
  float* C;
  int64_t lda, ldb, ldc;
  int32_t a_rows, b_cols;   // valid rows of A, valid columns of B
  int32_t kmax;             // reduction length that can be non-zero
  int32_t c_rows, c_cols;   // extent of C that is written
  int32_t tiles_n;          // ceil(c_cols / BN) for the launch's tile shape
  int32_t tile_begin;       // first tile of this problem within the launch
  int32_t beta;             // 0: C = A B; 1: C += A B
  int32_t prepacked;        // split-precision leaves: pa / pb already written
  // Split-precision leaves only (else unused): the packed hi/lo operands
  // (leaf_packed_bytes in all, B's part from pa + leaf_packed_a_bytes) and,
  // for the scaled FP16 form, power-of-two exponents of the a_rows rows of A
  // and the b_cols columns of B, eb followed by ceil(kmax / 256) x b_cols
  // floats of scratch (leaf_scale_bytes in all).
  void* pa;
  void* pb;
  int32_t* ea;
  int32_t* eb;
  // Last-level post-additions fused into the epilogue (FP32 leaves, 128x128
  // tiles, FASTMM_FUSED_POST=1; else e_mask = 0): the leaf is product P_i of
  // a node whose result (E, leading dimension e_ld; C21 / C22 at e_bot_off,
  // C12 / C22 at e_right_off from C11 / C21) it writes into directly.  Bit
  // q of e_mask (C11, C12, C21, C22) marks the quadrants this product enters:
  // stored where e_first has the bit, subtracted where e_sub has it, else
  // added.  Valid rows of the top / bottom quadrants e_rows[0 / 1], valid
  // columns of the left / right ones e_cols[0 / 1].
  float* E;
  int64_t e_ld, e_bot_off;
  int32_t e_right_off, e_mask, e_first, e_sub;
  int32_t e_rows[2], e_cols[2];
};

// One node of a pre-addition launch: reads the four quadrants of a parent
// operand (or a band of rows or of columns of each) and writes four h_r x h_c
// results.  Quadrant X11 starts at src, X12 at src + right_off, X21 at
// src + bot_off and X22 at src + bot_off + right_off, all with leading
// dimension ld (right_off = h_c for whole quadrants); rows / columns beyond
// the valid counts read as zero.  Output q (0..3) starts at
// dst + q * out_stride with leading dimension h_c.
struct PreAddNode {
  const float* src;
  float* dst;
  int64_t ld;
  int64_t bot_off;
  int64_t out_stride;
  int32_t top_rows, bot_rows;     // valid rows of the top / bottom quadrants
  int32_t left_cols, right_cols;  // valid columns of the left / right quadrants
  int32_t h_r, h_c;               // rows of this node, quadrant width
  int32_t block_begin;            // first workgroup of this node within the launch
  int32_t mask;                   // outputs to write (bit q-1 for S_q / T_q); 0 = all
  int32_t right_off;              // offset of the right quadrants from the left ones
  int32_t pad_;
};

// One node of a fused pre-addition and pack launch (split-BF16 leaves, last
// level of the recursion): the parent operand's quadrants (geometry as in
// PreAddNode; dst, out_stride and mask unused) are combined into S1..S4
// (T1..T4) in FP32 exactly as the pre-addition kernel does, and the seven
// leaf operands of the node -- A side: A11, A12, S4, A22, S1, S2, S3; B side:
// B11, B21, B22, T4, T1, T2, T3 -- are written straight in the packed layout
// of the split-precision leaf (leaf_pack_kernel's), never as FP32.
struct PackNode {
  PreAddNode q;
  void* dst[7];         // packed operand of leaf i of the node
  int32_t* e[7];        // scaled FP16 only: the leaf's e_A (A side) or e_B (B side)
  int32_t rows[7];      // its valid rows of A (A side) or columns of B (B side)
  int32_t kmax[7];      // its reduction length
  int32_t slabs[7];     // its K-slabs of 32: ceil(kmax / 32)
  int32_t tiles;        // 128-row (A) or 128-column (B) tiles of every output
  int32_t max_slabs;    // largest of slabs[]
  int32_t unit_begin;   // first workgroup of this node within the launch
  int32_t pad_;
};

// Quadrants (bit 0 = X11, 1 = X12, 2 = X21, 3 = X22) that pre-addition
// outputs read: side 0 (S1..S4 from A), side 1 (T1..T4 from B).
inline unsigned preadd_inputs(int side, unsigned outputs) {
  static const unsigned a_need[4] = {0xC, 0xD, 0x5, 0xF};  // S1: A21 A22; S2: +A11; S3: A11 A21; S4: all
  static const unsigned b_need[4] = {0x3, 0xB, 0xA, 0xF};  // T1: B11 B12; T2: +B22; T3: B12 B22; T4: all
  unsigned q = 0;
  for (int i = 0; i < 4; ++i)
    if (outputs & (1u << i)) q |= (side == 0 ? a_need[i] : b_need[i]);
  return q;
}

// One node of a post-addition launch: reads seven h_r x h_c products (P_i at
// P + i * p_stride, leading dimension h_c) and writes the result quadrants
// (or a band of rows or of columns of each): C11 at dst, C12 at
// dst + right_off, C21 at dst + bot_off, C22 at dst + bot_off + right_off
// (leading dimension ld; right_off = h_c for whole quadrants), each clipped
// to its valid rows / columns.
struct PostAddNode {
  const float* P;
  float* dst;
  int64_t ld;
  int64_t p_stride;
  int64_t bot_off;
  int32_t top_rows, bot_rows;
  int32_t left_cols, right_cols;
  int32_t h_r, h_c;
  int32_t block_begin;
  int32_t right_off;  // offset of C12 / C22 from C11 / C21
};

// One node of a multi-level addition launch: L consecutive levels of the
// recursion (L = 2 or 3) in one pass, for subtrees in which every level is
// exactly twice the next (the engine's split rule makes them so below the
// top of the recursion).  The top node's operand (or product) is then a
// 2^L x 2^L grid of equal cells of br x bc elements -- virtually: only its
// first vrows x vcols elements exist, the rest read as zero and are not
// written -- and every S, T and P of the levels in between is a dense grid
// of the same cells, so one thread can follow one element position through
// all L levels.
//   pre-additions: src = the top node's operand (leading dimension ld,
//     vrows x vcols valid); dst[j] = the S (T) blocks of level l0 + j, all
//     nodes of that level, node-major, four dense blocks per node (the
//     level-wise layout); node = index of the top node within level l0.
//   post-additions: src = the 7^L products of level l0 + L under this node
//     (consecutive dense br x bc blocks); dst[0] = the node's product
//     (leading dimension ld), never clipped: vrows x vcols is the whole grid.
struct TreeNode {
  const float* src;
  float* dst[3];
  int64_t ld;
  int64_t node;
  int32_t br, bc;
  int32_t vrows, vcols;
  int32_t block_begin;
  int32_t pad_;
};

inline int32_t clamp_extent(int64_t v, int64_t hi) {
  return (int32_t)(v < 0 ? 0 : (v > hi ? hi : v));
}

// Pre-additions of a whole parent operand (vrows x vcols valid) whose
// quadrants are h_r x h_c, into four dense blocks at dst.
inline PreAddNode preadd_node(const float* src, int64_t ld, int64_t vrows, int64_t vcols,
                              int64_t h_r, int64_t h_c, float* dst) {
  PreAddNode n{};
  n.src = src;
  n.dst = dst;
  n.ld = ld;
  n.bot_off = h_r * ld;
  n.out_stride = h_r * h_c;
  n.top_rows = clamp_extent(vrows, h_r);
  n.bot_rows = clamp_extent(vrows - h_r, h_r);
  n.left_cols = clamp_extent(vcols, h_c);
  n.right_cols = clamp_extent(vcols - h_c, h_c);
  n.h_r = (int32_t)h_r;
  n.h_c = (int32_t)h_c;
  n.right_off = (int32_t)h_c;
  return n;
}

// Post-additions of seven dense h_r x h_c products at P into a result of
// rows x cols (leading dimension ld) at dst.
inline PostAddNode postadd_node(const float* P, int64_t h_r, int64_t h_c, float* dst, int64_t ld,
                                int64_t rows, int64_t cols) {
  PostAddNode n{};
  n.P = P;
  n.dst = dst;
  n.ld = ld;
  n.p_stride = h_r * h_c;
  n.bot_off = h_r * ld;
  n.top_rows = clamp_extent(rows, h_r);
  n.bot_rows = clamp_extent(rows - h_r, h_r);
  n.left_cols = clamp_extent(cols, h_c);
  n.right_cols = clamp_extent(cols - h_c, h_c);
  n.h_r = (int32_t)h_r;
  n.h_c = (int32_t)h_c;
  n.right_off = (int32_t)h_c;
  return n;
}

// Work of one add workgroup: kAddChunk float4 groups of one node, one per
// thread (measured: many small workgroups stream best, 5.6-5.8 TB/s on the
// largest quadrants against 5.3 with four groups per thread).
constexpr int kAddThreadsPerBlock = 256;
constexpr int kAddChunk = kAddThreadsPerBlock * 1;

inline int64_t add_blocks_for(int64_t h_r, int64_t h_c) {
  const int64_t groups = h_r * ((h_c + 3) / 4);
  return (groups + kAddChunk - 1) / kAddChunk;
}

// Status codes of the C ABI (mirrors include/fastmm.h).
enum Status {
  kSuccess = 0,
  kInvalidValue = -1,
  kOutOfMemory = -2,
  kDeviceError = -3,
  kNotSupported = -4,
};

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    int code = (e == hipErrorOutOfMemory) ? kOutOfMemory : kDeviceError;
    throw Error(code, std::string(what) + ": " + hipGetErrorString(e));
  }
}

#define FASTMM_HIP(call) ::fastmm::hip_check((call), #call)

// The leaf kernels address a tile's slab with 32-bit byte offsets relative
// to the slab: at most 256 rows of A (255 * 2^21 * 4 < 2^31) and 32 rows of
// B (31 * 2^24 * 4 < 2^31).  These bounds keep every offset and every slab
// extent below 2^31.
constexpr int64_t kMaxLeadingDimA = int64_t(1) << 21;
constexpr int64_t kMaxLeadingDimB = int64_t(1) << 24;

// Leaf tile shapes (ids are part of the ABI: fastmm_plan_t.tile).
enum TileId {
  kTile128x128 = 0,
  kTile256x128 = 1,
  kTile128x64 = 2,
  kTile64x64 = 3,
  kTile128x128k32 = 4,  // K-slab of 32
  kTile256x128w8 = 5,   // 8 wavefronts
  kTile256x256w8 = 6,   // 8 wavefronts
  kTile128x256 = 7,
  kTileBf16x3 = 8,      // 128x128, split-BF16 arithmetic (precision form)
  kTileFp16x3 = 9,      // 128x128, scaled split-FP16 arithmetic (precision form)
  kNumTiles = 10,
};

struct TileShape {
  int bm, bn;
};

// Macro tile and wavefront grid of the split-precision leaves on packed
// operands (tile ids kTileBf16x3 and kTileFp16x3 of the level-wise engine).
constexpr int kSplitTileM = 256, kSplitTileN = 256;
constexpr int kSplitWavesM = 4, kSplitWavesN = 4;

inline TileShape tile_shape(int id) {
  switch (id) {
    case kTile128x128: return {128, 128};
    case kTile256x128: return {256, 128};
    case kTile128x64: return {128, 64};
    case kTile64x64: return {64, 64};
    case kTile128x128k32: return {128, 128};
    case kTile256x128w8: return {256, 128};
    case kTile256x256w8: return {256, 256};
    case kTile128x256: return {128, 256};
    case kTileBf16x3: return {kSplitTileM, kSplitTileN};
    case kTileFp16x3: return {kSplitTileM, kSplitTileN};
    default: throw Error(kInvalidValue, "unknown tile id " + std::to_string(id));
  }
}

// Workgroup id -> logical tile of a grouped leaf launch.  The dispatcher
// deals workgroups round-robin over the 8 XCDs (XCD = id % 8), each with its
// own L2.  chunk == 0: each XCD gets one contiguous run of logical tiles (the
// most L2 reuse, right when every tile costs the same).  chunk > 0: runs of
// `chunk` consecutive tiles are dealt round-robin over the XCDs, so that
// when tile costs differ (uneven products, ordered longest first) every XCD
// gets the same mix, in the same order; ids past the last whole round keep
// their own index.
__device__ __forceinline__ int leaf_tile_of_block(int bid, int nblocks, int chunk) {
  if (chunk <= 0) {
    const int xcd = bid & 7;
    const int q = nblocks >> 3;
    const int r = nblocks & 7;
    return xcd * q + (xcd < r ? xcd : r) + (bid >> 3);
  }
  const int span = 8 * chunk;
  if (bid >= nblocks / span * span) return bid;
  const int j = bid >> 3;
  return ((j / chunk) * 8 + (bid & 7)) * chunk + j % chunk;
}

// Kernel launchers (stream-ordered, no synchronisation).  xcd_chunk: see
// leaf_tile_of_block.  queue: two zeroed ints in device memory for a
// persistent launch (workgroups take tiles from a counter; the kernel leaves
// the counters zeroed), or nullptr for one workgroup per tile.
void launch_leaf_gemm(int tile, const GemmDesc* d_descs, int ndesc, int total_tiles, bool vec,
                      hipStream_t stream, int xcd_chunk = 0, int* queue = nullptr,
                      bool fused_post = false);
void launch_leaf_bf16x3(const GemmDesc* d_descs, int ndesc, int total_tiles, bool vec,
                        hipStream_t stream, int xcd_chunk = 0);
// Split-precision leaves on packed operands (tile kTileBf16x3 or
// kTileFp16x3): for FP16 a scale pass (each descriptor's ea / eb hold a_rows
// / b_cols ints), then a pass that packs both operands of every descriptor
// into pa / pb, then the leaf.  ext: largest extents over the descriptors.
struct LeafExtents {
  int max_a_rows = 0, max_b_cols = 0, max_c_rows = 0, max_c_cols = 0, max_slabs = 0, max_kmax = 0;
  bool any_unpacked = true;  // some descriptor still needs the pack pass
};
// Workgroups of a fused pre-addition and pack node (4 K-slabs per workgroup).
int pack_node_units(const PackNode& n);
// side 0: A operands, 1: B operands; nodes with unit_begin prefixes.  fp16:
// scaled split FP16 (the node's scale exponents must be in place).
void launch_preadd_pack(int side, const PackNode* d_nodes, int nnodes, int total_units, bool fp16,
                        hipStream_t stream);
// Scaled FP16 leaves: the fused nodes' scale exponents, from the parent
// quadrants (rows of the seven A-side operands; column maxima of the seven
// B-side operands in 256-row parts, then reduced per leaf over d_descs).
// max_rows / max_kdim: largest node rows (A side) / reduction extent (B
// side); max_cols: largest node columns (B side) and leaf b_cols.
void launch_preadd_scale(const PackNode* d_a, int na, const PackNode* d_b, int nb, int max_rows,
                         int max_cols, int max_kdim, const GemmDesc* d_descs, int ndesc,
                         hipStream_t stream);
// Bytes of the FP16 scale exponents and scratch of a rows x k by k x cols leaf.
int64_t leaf_scale_bytes(int64_t rows, int64_t cols, int64_t k);
// Bytes of the packed operands of a rows x k by k x cols leaf (A's part first).
int64_t leaf_packed_bytes(int64_t rows, int64_t cols, int64_t k);
int64_t leaf_packed_a_bytes(int64_t rows, int64_t k);
void launch_leaf_packed(int tile, const GemmDesc* d_descs, int ndesc, int total_tiles, bool vec,
                        hipStream_t stream, int xcd_chunk, const LeafExtents& ext);
void launch_preadd(int side, const PreAddNode* d_nodes, int nnodes, int total_blocks, bool vec,
                   hipStream_t stream);
// quad < 0: all four result quadrants; 0..3: only C11, C12, C21 or C22
// (each by the same chain of operations as in the fused form).
void launch_postadd(const PostAddNode* d_nodes, int nnodes, int total_blocks, bool vec,
                    hipStream_t stream, int quad = -1);

// Multi-level additions over TreeNode descriptors.  kind 0: A-side
// pre-additions, 1: B-side pre-additions, 2: post-additions; levels 2 or 3.
// Each thread takes `width` consecutive elements of a cell: four (16-byte
// accesses; two levels, aligned rows and cells only) or one (three levels,
// whose 64 inputs (pre) or 64 outputs (post) per element already fill the
// registers, and any misaligned case).
constexpr int kMaxTreeLevels = 3;
inline int tree_width(int levels, bool aligned) { return levels == 2 && aligned ? 4 : 1; }
inline int64_t tree_blocks_for(int width, int64_t br, int64_t bc) {
  const int64_t groups = br * (bc / width);
  return (groups + kAddThreadsPerBlock - 1) / kAddThreadsPerBlock;
}
// clip: some top operand of a pre-addition launch is clipped (post-addition
// launches never are).
void launch_tree_add(int kind, int levels, int width, bool clip, const TreeNode* d_nodes, int nnodes,
                     int total_blocks, hipStream_t stream);

}  // namespace fastmm
