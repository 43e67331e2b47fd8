// Shared types of the fastmm HIP library (gfx950 / CDNA4).
//
// A matrix operand anywhere in the recursion is a strided view with a
// "valid" extent: elements outside it read as zero.  That is how odd extents
// follow the paper's quadrant split (equation (1), Section 3.1: quadrant 0 is
// ceil(m/2) x ceil(n/2), quadrant 3 floor(m/2) x floor(n/2)) while every
// quadrant of one level keeps the same ceil-sized virtual shape.
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
  int32_t pad_;
};

// One node of a pre-addition launch: reads the four quadrants of a parent
// operand view and writes four dense (h_r x h_c, ld = h_c) results.
struct PreAddNode {
  const float* src;
  float* dst;               // 4 consecutive h_r*h_c blocks
  int64_t ld;
  int32_t vrows, vcols;     // valid extent of the parent view
  int32_t h_r, h_c;         // quadrant extents
  int32_t block_begin;      // first workgroup of this node within the launch
  int32_t pad_;
};

// One node of a post-addition launch: reads seven dense products (h_r x h_c)
// and writes the four result quadrants into dst, clipped to rows x cols.
struct PostAddNode {
  const float* P;           // 7 consecutive h_r*h_c blocks
  float* dst;
  int64_t ld;
  int32_t rows, cols;
  int32_t h_r, h_c;
  int32_t block_begin;
  int32_t pad_;
};

// Work of one add workgroup: kAddChunk float4 groups of one node.
constexpr int kAddThreadsPerBlock = 256;
constexpr int kAddChunk = kAddThreadsPerBlock * 4;

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

// The leaf kernel addresses a tile's slab with 32-bit byte offsets relative
// to the slab (at most 256 rows of A, 16 rows of B): these bounds keep every
// offset below 2^31.
constexpr int64_t kMaxLeadingDimA = int64_t(1) << 21;
constexpr int64_t kMaxLeadingDimB = int64_t(1) << 26;

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
  kNumTiles = 8,
};

struct TileShape {
  int bm, bn;
};

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
    default: throw Error(kInvalidValue, "unknown tile id " + std::to_string(id));
  }
}

// Kernel launchers (stream-ordered, no synchronisation).
void launch_leaf_gemm(int tile, const GemmDesc* d_descs, int ndesc, int total_tiles, bool vec,
                      hipStream_t stream);
void launch_preadd(int side, const PreAddNode* d_nodes, int nnodes, int total_blocks, bool vec,
                   hipStream_t stream);
// quad < 0: all four result quadrants; 0..3: only C11, C12, C21 or C22
// (each by the same chain of operations as in the fused form).
void launch_postadd(const PostAddNode* d_nodes, int nnodes, int total_blocks, bool vec,
                    hipStream_t stream, int quad = -1);

}  // namespace fastmm
