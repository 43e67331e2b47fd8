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
// one grid.  Workgroup ids are first mapped to logical tiles with the XCDs in
// mind (the dispatcher deals workgroups round-robin over the 8 XCDs, each with
// its own L2; see leaf_tile_of_block), then tiles of a problem are walked in
// groups of 8 tile-rows so that neighbours share A row-panels and B
// column-panels.
//
// Data path per K-slab of BK (double-buffered in LDS, one slab ahead):
//   16-byte vector tiles with BK = 16: global -> LDS directly (buffer loads
//   with the LDS bit), A as [m][k] and B as [k][n], unpadded and swizzled;
//   otherwise global -> registers -> LDS (A padded or swizzled, B padded).
//   LDS -> MFMA operands: lane l of a 32x32x2 step supplies A[row l%32][k]
//   and B[k][col l%32] with k chosen by the lane half l/32.  Over a slab the
//   two halves take the k-indices 8g+4h+s (s = 0..3); the sum over k does not
//   depend on the order the indices are visited in.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace fastmm {

typedef float f32x16 __attribute__((ext_vector_type(16)));


// Buffer resource over [p, p + bytes).  Both values are the same in every
// lane; readfirstlane states that, so the resource lives in scalar registers
// (a resource the compiler thinks may differ per lane costs a loop per load).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const float* p, int bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  float* q = reinterpret_cast<float*>(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, __builtin_amdgcn_readfirstlane(bytes),
                                           0x00020000);
}

// Occupancy: waves whose accumulators fit in 64 registers are asked to fit
// four per SIMD (all operands in 128 registers), which hides the per-slab
// barrier better than the three the register allocator would otherwise give.
// (The element-wise load variant needs a few more registers and is left to
// the allocator.)
template <int BM, int BN, int WGM, int WGN, bool VEC>
constexpr int leaf_waves_per_simd() {
  return VEC && (BM / WGM / 32) * (BN / WGN / 32) <= 4 ? 4 : 1;
}

template <int BM, int BN, int BK, int WGM, int WGN, bool VEC, bool PERSIST, bool EPI = false>
__global__ void __launch_bounds__(64 * WGM * WGN, (leaf_waves_per_simd<BM, BN, WGM, WGN, VEC>()))
leaf_gemm_kernel(const GemmDesc* __restrict__ descs, int ndesc, int total_tiles, int xcd_chunk,
                 int* __restrict__ queue) {
  constexpr int kThreads = 64 * WGM * WGN;  // WGM x WGN wavefronts of 64
  constexpr int WM = BM / WGM, WN = BN / WGN;  // wave sub-tile
  constexpr int FM = WM / 32, FN = WN / 32; // 32x32 blocks per wave
  // A in LDS as [m][k].  With BK = 16 rows are unpadded and the 16-byte
  // group g of row r is stored at group g ^ ((r >> 2) & 3): both the stores
  // (16 lanes write 4 rows x 4 groups) and the fragment reads (16 lanes read
  // 16 rows, one group) then touch 64 distinct banks.  Other BK: rows padded
  // by 4 floats.
  constexpr bool SWZ = BK == 16;
  constexpr int LDA = SWZ ? BK : BK + 4;    // LDS row stride of A
  // DTL: the vector path with BK = 16 loads both slabs straight into LDS
  // (buffer loads with the LDS bit: each wave instruction fills 1 KB of LDS,
  // lane i at byte 16 i), with no register staging and no LDS stores.  B is
  // then kept unpadded as [k][n] with column bit 5 flipped on rows whose
  // (k >> 2) is odd, so the two lane halves of a fragment read (rows k and
  // k + 4) fall on different banks.
  constexpr int kWaves = kThreads / 64;
  constexpr bool DTL = VEC && SWZ && (BM / 16) % kWaves == 0 && (BN / 16) % kWaves == 0 &&
                       BN >= 64 && 256 % BN == 0;
  constexpr int LDB = DTL ? BN : BN + 8;    // LDS row stride of B ([k][n])
  constexpr int A_F4 = BM * BK / 4 / kThreads;  // float4 loads per thread
  constexpr int B_F4 = BK * BN / 4 / kThreads;
  static_assert(A_F4 >= 1 && B_F4 >= 1, "tile too small for 256 threads");
  static_assert(BK % 8 == 0, "BK must be a multiple of 8");

  // Double-buffered slabs as four separate arrays.  With DTL the K loop is
  // unrolled by two so that every access names its buffer statically: the
  // compiler then knows that slab k + 1 landing in one buffer cannot alias
  // the reads of slab k from the other, and does not wait for the in-flight
  // loads before those reads.
  __shared__ __attribute__((aligned(16))) float As0[BM * LDA], As1[BM * LDA];
  __shared__ __attribute__((aligned(16))) float Bs0[BK * LDB], Bs1[BK * LDB];

  // Without a queue each workgroup owns one tile.  With one (a persistent
  // launch of about one workgroup per slot), workgroups take tiles in
  // logical order from queue[0] until it passes total_tiles; every workgroup
  // then counts itself out in queue[1], and the last one clears both, so the
  // queue is ready for the next launch (also on a graph replay) without a
  // memset.  No workgroup ever waits for another.
  __shared__ int next_tile;
  int logical = PERSIST ? 0 : leaf_tile_of_block(blockIdx.x, gridDim.x, xcd_chunk);
  for (;;) {
  if (PERSIST) {
    if (threadIdx.x == 0) next_tile = atomicAdd(&queue[0], 1);
    __syncthreads();
    logical = next_tile;
    __syncthreads();
  }
  if (logical >= total_tiles) break;

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
  const int beta = d.beta;
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
  const int wm = (wave / WGN) * WM;
  const int wn = (wave % WGN) * WN;
  const int lr = lane & 31;
  const int lh = lane >> 5;

  // Global -> register mapping (fixed per thread).
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

  // Loads are branch-free raw buffer loads: a slab's resource covers exactly
  // its valid extent, and lanes outside it use an out-of-range offset, for
  // which the hardware returns zero.  This is the zero padding of the
  // recursion's odd quadrants and of ragged tiles, with no divergent code
  // around the loads (which would force a wait right after each one).
  const int rv = min(BM, a_rows - tm);  // valid rows of A in this tile
  const int cv = min(BN, b_cols - tn);  // valid columns of B in this tile
  const float* a_tile = A + (int64_t)tm * lda;
  const float* b_tile = B + tn;
  constexpr int kOOB = 0x7FFFFFF0;

  float4 ra[DTL ? 1 : A_F4], rb[DTL ? 1 : B_F4];

  // Direct-to-LDS slab load into one buffer pair (DTL only).
  auto load_slab_lds = [&](int k0, float* __restrict__ as_dst, float* __restrict__ bs_dst) {
    const int kv = min(BK, kmax - k0);
    const uint32_t a_bytes =
        (rv > 0 && kv > 0) ? (uint32_t)(((int64_t)(rv - 1) * lda + kv) * 4) : 0u;
    const uint32_t b_bytes =
        (cv > 0 && kv > 0) ? (uint32_t)(((int64_t)(kv - 1) * ldb + cv) * 4) : 0u;
    const __amdgpu_buffer_rsrc_t ar = make_rsrc(a_tile + k0, (int)a_bytes);
    const __amdgpu_buffer_rsrc_t br = make_rsrc(b_tile + (int64_t)k0 * ldb, (int)b_bytes);
#pragma unroll
    for (int j = 0; j < BM / 16 / kWaves; ++j) {
      const int q = j * kWaves + wave;            // 1 KB chunk: rows 16 q .. 16 q + 15
      const int row = q * 16 + (lane >> 2);
      const int g = (lane & 3) ^ ((row >> 2) & 3);  // global 16-byte group of this slot
      const int off = (row < rv && 4 * g < kv) ? (row * (int)lda + 4 * g) * 4 : kOOB;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          ar, (__attribute__((address_space(3))) void*)&as_dst[q * 256], 16, off, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < BN / 16 / kWaves; ++j) {
      const int q = j * kWaves + wave;            // 1 KB chunk: 256 / BN rows of B
      const int k = q * (256 / BN) + lane / (BN / 4);
      const int g = (lane % (BN / 4)) ^ (((k >> 2) & 1) << 3);
      const int off = (k < kv && 4 * g < cv) ? (k * (int)ldb + 4 * g) * 4 : kOOB;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          br, (__attribute__((address_space(3))) void*)&bs_dst[q * 256], 16, off, 0, 0, 0);
    }
  };

  auto load_slab = [&](int k0) {
    const int kv = min(BK, kmax - k0);  // valid k in this slab
    const uint32_t a_bytes =
        (rv > 0 && kv > 0) ? (uint32_t)(((int64_t)(rv - 1) * lda + kv) * 4) : 0u;
    const uint32_t b_bytes =
        (cv > 0 && kv > 0) ? (uint32_t)(((int64_t)(kv - 1) * ldb + cv) * 4) : 0u;
    const __amdgpu_buffer_rsrc_t ar = make_rsrc(a_tile + k0, (int)a_bytes);
    const __amdgpu_buffer_rsrc_t br = make_rsrc(b_tile + (int64_t)k0 * ldb, (int)b_bytes);
#pragma unroll
    for (int i = 0; i < A_F4; ++i) {
      const int base = (a_r[i] * (int)lda + a_c[i]) * 4;
      const bool rok = a_r[i] < rv;
      if (VEC) {
        const int off = (rok && a_c[i] < kv) ? base : kOOB;
        ra[i] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(ar, off, 0, 0));
      } else {
        float e[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int off = (rok && a_c[i] + q < kv) ? base + 4 * q : kOOB;
          e[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ar, off, 0, 0));
        }
        ra[i] = make_float4(e[0], e[1], e[2], e[3]);
      }
    }
#pragma unroll
    for (int i = 0; i < B_F4; ++i) {
      const int base = (b_r[i] * (int)ldb + b_c[i]) * 4;
      const bool kok = b_r[i] < kv;
      if (VEC) {
        const int off = (kok && b_c[i] < cv) ? base : kOOB;
        rb[i] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(br, off, 0, 0));
      } else {
        float e[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int off = (kok && b_c[i] + q < cv) ? base + 4 * q : kOOB;
          e[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(br, off, 0, 0));
        }
        rb[i] = make_float4(e[0], e[1], e[2], e[3]);
      }
    }
  };

  auto a_slot = [&](int r, int c) {  // float offset of A[r][c..c+3] in a buffer
    return r * LDA + (SWZ ? (((c >> 2) ^ ((r >> 2) & 3)) << 2) : c);
  };
  auto store_slab = [&](float* __restrict__ as_dst, float* __restrict__ bs_dst) {
#pragma unroll
    for (int i = 0; i < A_F4; ++i)
      *reinterpret_cast<float4*>(&as_dst[a_slot(a_r[i], a_c[i])]) = ra[i];
#pragma unroll
    for (int i = 0; i < B_F4; ++i)
      *reinterpret_cast<float4*>(&bs_dst[b_r[i] * LDB + b_c[i]]) = rb[i];
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
    if (DTL) {
      load_slab_lds(0, As0, Bs0);
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the slab is in LDS
    } else {
      load_slab(0);
      store_slab(As0, Bs0);
    }
    __syncthreads();
  }
  // One K-slab: prefetch slab kt + 1 into the other buffers, multiply slab kt.
  auto step = [&](const float* __restrict__ as, const float* __restrict__ bs,
                  float* __restrict__ as_next, float* __restrict__ bs_next, int kt) {
    const bool more = (kt + 1 < nk);
    if (more) {
      if (DTL) load_slab_lds((kt + 1) * BK, as_next, bs_next);
      else load_slab((kt + 1) * BK);
    }
#pragma unroll
    for (int g8 = 0; g8 < BK / 8; ++g8) {
      const int kb = g8 * 8 + lh * 4;
      float4 af[FM];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        af[i] = *reinterpret_cast<const float4*>(&as[a_slot(wm + 32 * i + lr, kb)]);
      float bf[FN][4];
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = kb + s, n = wn + 32 * j + lr;
          bf[j][s] = bs[k * LDB + (DTL ? (n ^ (((k >> 2) & 1) << 5)) : n)];
        }
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
    if (more) {
      if (DTL) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      else store_slab(as_next, bs_next);
    }
    __syncthreads();
  };
  if constexpr (DTL) {
    for (int kt = 0; kt < nk; kt += 2) {
      step(As0, Bs0, As1, Bs1, kt);
      if (kt + 1 < nk) step(As1, Bs1, As0, Bs0, kt + 1);
    }
  } else {  // register staging: the stores wait for the loads anyway
    for (int kt = 0; kt < nk; ++kt) {
      const bool odd = kt & 1;
      step(odd ? As1 : As0, odd ? Bs1 : Bs0, odd ? As0 : As1, odd ? Bs0 : Bs1, kt);
    }
  }

  // Epilogue: register r of block (i, j) holds row 8*(r/4) + 4*(lane/32) + r%4
  // and column lane%32 of that 32x32 block.
  if constexpr (EPI) {
    // Fused post-additions: this product's element enters up to three
    // quadrants of its node's result, each by the next operation of that
    // quadrant's chain (the launches run the node's products in an order
    // that makes every chain the post-addition kernel's).
    const int emask = d.e_mask, efirst = d.e_first, esub = d.e_sub;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!((emask >> q) & 1)) continue;
      float* __restrict__ Eq = d.E + ((q >> 1) ? d.e_bot_off : 0) + ((q & 1) ? d.e_right_off : 0);
      const int vr = d.e_rows[q >> 1], vc = d.e_cols[q & 1];
      const bool first = (efirst >> q) & 1, neg = (esub >> q) & 1;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int col = tn + wn + 32 * j + lr;
          if (col >= vc) continue;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = tm + wm + 32 * i + 8 * (r >> 2) + 4 * lh + (r & 3);
            if (row < vr) {
              float* cp = Eq + (int64_t)row * d.e_ld + col;
              *cp = first ? acc[i][j][r] : (neg ? *cp - acc[i][j][r] : *cp + acc[i][j][r]);
            }
          }
        }
    }
  } else {
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = tn + wn + 32 * j + lr;
      if (col >= c_cols) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = tm + wm + 32 * i + 8 * (r >> 2) + 4 * lh + (r & 3);
        if (row < c_rows) {
          float* cp = C + (int64_t)row * ldc + col;
          *cp = beta ? *cp + acc[i][j][r] : acc[i][j][r];
        }
      }
    }
  }
  if (!PERSIST) break;
  }
  if (PERSIST && threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&queue[1], 1) == (int)gridDim.x - 1) {
      atomicExch(&queue[0], 0);
      atomicExch(&queue[1], 0);
    }
  }
}

template <int BM, int BN, int BK, int WGM, int WGN>
static void launch_t(const GemmDesc* d, int ndesc, int total, bool vec, hipStream_t s, int xc,
                     int* queue) {
  if (total <= 0) return;
  constexpr int kThreads = 64 * WGM * WGN;
  // Persistent launches are built for the 128-wide and smaller tiles only.
  constexpr bool kCanPersist = BM <= 128 && BN <= 128 && BK == 16;
  if (!kCanPersist) queue = nullptr;
  auto kv = queue ? leaf_gemm_kernel<BM, BN, BK, WGM, WGN, true, kCanPersist>
                  : leaf_gemm_kernel<BM, BN, BK, WGM, WGN, true, false>;
  auto ks = queue ? leaf_gemm_kernel<BM, BN, BK, WGM, WGN, false, kCanPersist>
                  : leaf_gemm_kernel<BM, BN, BK, WGM, WGN, false, false>;
  int blocks = total;
  if (queue) {  // persistent: one workgroup per slot the device can hold at once
    static int slots[2] = {0, 0};
    int& sl = slots[vec ? 1 : 0];
    if (!sl) {
      int dev = 0, cus = 0, per_cu = 0;
      FASTMM_HIP(hipGetDevice(&dev));
      FASTMM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      FASTMM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(vec ? kv : ks), kThreads, 0));
      sl = std::max(1, cus * per_cu);
    }
    blocks = std::min(total, sl);
  }
  dim3 grid(blocks), block(kThreads);
  if (vec)
    hipLaunchKernelGGL(kv, grid, block, 0, s, d, ndesc, total, xc, queue);
  else
    hipLaunchKernelGGL(ks, grid, block, 0, s, d, ndesc, total, xc, queue);
  FASTMM_HIP(hipGetLastError());
}

void launch_leaf_gemm(int tile, const GemmDesc* d_descs, int ndesc, int total_tiles, bool vec,
                      hipStream_t stream, int xcd_chunk, int* queue, bool fused_post) {
  if (fused_post) {  // 128x128 tiles, one workgroup per tile
    if (tile != kTile128x128 || queue) throw Error(kNotSupported, "fused post-additions need 128x128 tiles");
    if (total_tiles <= 0) return;
    dim3 grid(total_tiles), block(256);
    if (vec)
      hipLaunchKernelGGL((leaf_gemm_kernel<128, 128, 16, 2, 2, true, false, true>), grid, block, 0, stream,
                         d_descs, ndesc, total_tiles, xcd_chunk, nullptr);
    else
      hipLaunchKernelGGL((leaf_gemm_kernel<128, 128, 16, 2, 2, false, false, true>), grid, block, 0,
                         stream, d_descs, ndesc, total_tiles, xcd_chunk, nullptr);
    FASTMM_HIP(hipGetLastError());
    return;
  }
  switch (tile) {
    case kTile128x128: launch_t<128, 128, 16, 2, 2>(d_descs, ndesc, total_tiles, vec, stream, xcd_chunk, queue); break;
    case kTile256x128: launch_t<256, 128, 16, 2, 2>(d_descs, ndesc, total_tiles, vec, stream, xcd_chunk, queue); break;
    case kTile128x64: launch_t<128, 64, 16, 2, 2>(d_descs, ndesc, total_tiles, vec, stream, xcd_chunk, queue); break;
    case kTile64x64: launch_t<64, 64, 16, 2, 2>(d_descs, ndesc, total_tiles, vec, stream, xcd_chunk, queue); break;
    case kTile128x128k32: launch_t<128, 128, 32, 2, 2>(d_descs, ndesc, total_tiles, vec, stream, xcd_chunk, queue); break;
    case kTile256x128w8: launch_t<256, 128, 16, 4, 2>(d_descs, ndesc, total_tiles, vec, stream, xcd_chunk, queue); break;
    case kTile256x256w8: launch_t<256, 256, 16, 2, 4>(d_descs, ndesc, total_tiles, vec, stream, xcd_chunk, queue); break;
    case kTile128x256: launch_t<128, 256, 16, 2, 2>(d_descs, ndesc, total_tiles, vec, stream, xcd_chunk, queue); break;
    case kTileBf16x3: launch_leaf_bf16x3(d_descs, ndesc, total_tiles, vec, stream, xcd_chunk); break;
    case kTileFp16x3:  // needs packed-operand storage and the operand extents
      throw Error(kInvalidValue, "the scaled FP16 leaf is launched by launch_leaf_packed");
    default: throw Error(kInvalidValue, "unknown tile id");
  }
}

}  // namespace fastmm
