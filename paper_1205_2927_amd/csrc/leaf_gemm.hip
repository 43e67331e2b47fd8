// Leaf product of the recursion: classic FP32 GEMM on the CDNA4 matrix cores.
//
// Each leaf computes c_ij = sum_k a_ik b_kj (equation (6), Section 3.3) for
// one of the 7^d sub-products; the paper hands this step to a GPU kernel that
// owns a 32x32 tile of C (Section 3.3).  Here one workgroup owns a BM x BN
// macro tile, four wavefronts (2 x 2) each own a (BM/2) x (BN/2) sub-tile made
// of 32x32 blocks, and every block is accumulated by
// v_mfma_f32_32x32x2_f32 (FP32 inputs, FP32 accumulation).
//
// Grouped launch: all leaves of a level (and of every problem of a batch) are
// one grid.  Workgroup ids are first remapped so that consecutive logical
// tiles stay on one XCD (the dispatcher deals workgroups round-robin over the
// 8 XCDs, each with its own L2), then tiles of a problem are walked in groups
// of 8 tile-rows so that neighbours share A row-panels and B column-panels.
//
// Data path per K-slab of BK:
//   global -> registers (float4, prefetched one slab ahead)
//   registers -> LDS (double buffered; A as [m][k], B as [k][n])
//   LDS -> MFMA operands: lane l of a 32x32x2 step supplies A[row l%32][k]
//   and B[k][col l%32] with k chosen by the lane half l/32.  Over a slab the
//   two halves take the k-indices 8g+4h+s (s = 0..3); the sum over k does not
//   depend on the order the indices are visited in.
#include <hip/hip_runtime.h>

#include "common.h"

namespace fastmm {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;  // 4 wavefronts of 64

__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  // Blocks bid, bid+8, ... run on XCD bid%8; give each XCD a contiguous run
  // of logical tiles.
  const int xcd = bid & 7;
  const int q = nblocks >> 3;
  const int r = nblocks & 7;
  return xcd * q + (xcd < r ? xcd : r) + (bid >> 3);
}

template <int BM, int BN, int BK, bool VEC>
__global__ void __launch_bounds__(kThreads)
leaf_gemm_kernel(const GemmDesc* __restrict__ descs, int ndesc, int total_tiles) {
  constexpr int WM = BM / 2, WN = BN / 2;   // wave sub-tile
  constexpr int FM = WM / 32, FN = WN / 32; // 32x32 blocks per wave
  constexpr int LDA = BK + 4;               // LDS row stride of A ([m][k])
  constexpr int LDB = BN + 8;               // LDS row stride of B ([k][n])
  constexpr int A_F4 = BM * BK / 4 / kThreads;  // float4 loads per thread
  constexpr int B_F4 = BK * BN / 4 / kThreads;
  static_assert(A_F4 >= 1 && B_F4 >= 1, "tile too small for 256 threads");
  static_assert(BK % 8 == 0, "BK must be a multiple of 8");

  __shared__ __attribute__((aligned(16))) float As[2][BM * LDA];
  __shared__ __attribute__((aligned(16))) float Bs[2][BK * LDB];

  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  if (logical >= total_tiles) return;

  // Which problem owns this tile (tile_begin is ascending).
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_begin <= logical) lo = mid; else hi = mid - 1;
  }
  const GemmDesc& d = descs[lo];
  const float* __restrict__ A = d.A;
  const float* __restrict__ B = d.B;
  float* __restrict__ C = d.C;
  const int64_t lda = d.lda, ldb = d.ldb, ldc = d.ldc;
  const int a_rows = d.a_rows, b_cols = d.b_cols, kmax = d.kmax;
  const int c_rows = d.c_rows, c_cols = d.c_cols;
  const int tiles_n = d.tiles_n;
  const int tiles_m = (c_rows + BM - 1) / BM;

  // Grouped walk: 8 tile-rows at a time, column-major inside a group.
  const int lt = logical - d.tile_begin;
  constexpr int GROUP = 8;
  const int group_tiles = GROUP * tiles_n;
  const int g = lt / group_tiles;
  const int first_m = g * GROUP;
  const int gm = min(tiles_m - first_m, GROUP);
  const int in_g = lt - g * group_tiles;
  const int tm = (first_m + in_g % gm) * BM;
  const int tn = (in_g / gm) * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * WM;
  const int wn = (wave & 1) * WN;
  const int lr = lane & 31;
  const int lh = lane >> 5;

  // Global -> register mapping.
  int a_r[A_F4], a_c[A_F4], b_r[B_F4], b_c[B_F4];
#pragma unroll
  for (int i = 0; i < A_F4; ++i) {
    const int f = tid + kThreads * i;
    a_r[i] = f / (BK / 4);
    a_c[i] = (f % (BK / 4)) * 4;
  }
#pragma unroll
  for (int i = 0; i < B_F4; ++i) {
    const int f = tid + kThreads * i;
    b_r[i] = f / (BN / 4);
    b_c[i] = (f % (BN / 4)) * 4;
  }

  float4 ra[A_F4], rb[B_F4];
  const bool rows_in = (tm + BM <= a_rows);
  const bool cols_in = (tn + BN <= b_cols);

  auto load_slab = [&](int k0) {
    const bool k_in = (k0 + BK <= kmax);
#pragma unroll
    for (int i = 0; i < A_F4; ++i) {
      const int r = tm + a_r[i];
      const int c = k0 + a_c[i];
      const float* p = A + (int64_t)r * lda + c;
      if (VEC && rows_in && k_in) {
        ra[i] = *reinterpret_cast<const float4*>(p);
      } else if (VEC && r < a_rows && c + 3 < kmax) {
        ra[i] = *reinterpret_cast<const float4*>(p);
      } else {
        const bool rv = r < a_rows;
        ra[i].x = (rv && c + 0 < kmax) ? p[0] : 0.f;
        ra[i].y = (rv && c + 1 < kmax) ? p[1] : 0.f;
        ra[i].z = (rv && c + 2 < kmax) ? p[2] : 0.f;
        ra[i].w = (rv && c + 3 < kmax) ? p[3] : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < B_F4; ++i) {
      const int r = k0 + b_r[i];
      const int c = tn + b_c[i];
      const float* p = B + (int64_t)r * ldb + c;
      if (VEC && cols_in && k_in) {
        rb[i] = *reinterpret_cast<const float4*>(p);
      } else if (VEC && r < kmax && c + 3 < b_cols) {
        rb[i] = *reinterpret_cast<const float4*>(p);
      } else {
        const bool rv = r < kmax;
        rb[i].x = (rv && c + 0 < b_cols) ? p[0] : 0.f;
        rb[i].y = (rv && c + 1 < b_cols) ? p[1] : 0.f;
        rb[i].z = (rv && c + 2 < b_cols) ? p[2] : 0.f;
        rb[i].w = (rv && c + 3 < b_cols) ? p[3] : 0.f;
      }
    }
  };

  auto store_slab = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_F4; ++i)
      *reinterpret_cast<float4*>(&As[buf][a_r[i] * LDA + a_c[i]]) = ra[i];
#pragma unroll
    for (int i = 0; i < B_F4; ++i)
      *reinterpret_cast<float4*>(&Bs[buf][b_r[i] * LDB + b_c[i]]) = rb[i];
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int nk = (kmax + BK - 1) / BK;
  if (nk > 0) {
    load_slab(0);
    store_slab(0);
    __syncthreads();
  }
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = (kt + 1 < nk);
    if (more) load_slab((kt + 1) * BK);
    const float* as = As[cur];
    const float* bs = Bs[cur];
#pragma unroll
    for (int g8 = 0; g8 < BK / 8; ++g8) {
      const int kb = g8 * 8 + lh * 4;
      float4 af[FM];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        af[i] = *reinterpret_cast<const float4*>(&as[(wm + 32 * i + lr) * LDA + kb]);
      float bf[FN][4];
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int s = 0; s < 4; ++s) bf[j][s] = bs[(kb + s) * LDB + wn + 32 * j + lr];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          const float a = (s == 0) ? af[i].x : (s == 1) ? af[i].y : (s == 2) ? af[i].z : af[i].w;
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bf[j][s], acc[i][j], 0, 0, 0);
        }
    }
    if (more) store_slab(cur ^ 1);
    __syncthreads();
  }

  // Epilogue: register r of block (i, j) holds row 8*(r/4) + 4*(lane/32) + r%4
  // and column lane%32 of that 32x32 block.
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = tn + wn + 32 * j + lr;
      if (col >= c_cols) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = tm + wm + 32 * i + 8 * (r >> 2) + 4 * lh + (r & 3);
        if (row < c_rows) C[(int64_t)row * ldc + col] = acc[i][j][r];
      }
    }
}

template <int BM, int BN, int BK>
static void launch_t(const GemmDesc* d, int ndesc, int total, bool vec, hipStream_t s) {
  if (total <= 0) return;
  dim3 grid(total), block(kThreads);
  if (vec)
    hipLaunchKernelGGL((leaf_gemm_kernel<BM, BN, BK, true>), grid, block, 0, s, d, ndesc, total);
  else
    hipLaunchKernelGGL((leaf_gemm_kernel<BM, BN, BK, false>), grid, block, 0, s, d, ndesc, total);
  FASTMM_HIP(hipGetLastError());
}

void launch_leaf_gemm(int tile, const GemmDesc* d_descs, int ndesc, int total_tiles, bool vec,
                      hipStream_t stream) {
  switch (tile) {
    case kTile128x128: launch_t<128, 128, 16>(d_descs, ndesc, total_tiles, vec, stream); break;
    case kTile256x128: launch_t<256, 128, 16>(d_descs, ndesc, total_tiles, vec, stream); break;
    case kTile128x64: launch_t<128, 64, 16>(d_descs, ndesc, total_tiles, vec, stream); break;
    case kTile64x64: launch_t<64, 64, 16>(d_descs, ndesc, total_tiles, vec, stream); break;
    default: throw Error(kInvalidValue, "unknown tile id");
  }
}

}  // namespace fastmm
