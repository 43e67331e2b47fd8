// Leaf products in split 16-bit arithmetic on the 16-bit matrix cores: the
// precision forms of the leaf, selected explicitly, never substituted for
// the FP32 leaf.
//
// Each FP32 operand element x is split into two 16-bit numbers, hi = r(x)
// and lo = r(x - hi) (round to nearest even), and the product a*b is taken
// as hi_a*hi_b + hi_a*lo_b + lo_a*hi_b (lo*lo dropped) with every term
// accumulated in FP32 by a 32x32x16 MFMA.
//
// * Split BF16 ("bf16x3"; Henry, Tang and Heinecke, "Leveraging the bfloat16
//   Artificial Intelligence Datatype For Higher-Precision Computations",
//   ARITH 2019): hi and lo are BF16, so x = hi + lo to a relative 2^-17 and
//   each product is good to about 2^-16.  BF16 has FP32's exponent range: no
//   scaling is needed.
// * Scaled split FP16 ("fp16x3"; the hi/lo FP16 split of Ootomo and Yokota,
//   "Recovering single precision accuracy from Tensor Cores while
//   surpassing the FP32 theoretical peak performance", IJHPCA 2022): hi and
//   lo are FP16 (11-bit significands), so x = hi + lo to a relative 2^-22,
//   but FP16 spans only 2^-24..2^16.  Every row r of the leaf's A operand and
//   every column c of its B operand therefore carries a power-of-two scale:
//   leaf_scale_kernel stores exponents e_A[r], e_B[c] that bring the row's
//   (column's) largest magnitude into [2^14, 2^15), the tile splits
//   x * 2^-e instead of x, and the epilogue multiplies the accumulated sum by
//   2^(e_A[r] + e_B[c]).  Powers of two factor out of the sum over k, so the
//   scaling itself is exact.  With the largest element at 2^14..2^15, a lo
//   part can only become subnormal (or vanish) for elements more than 2^17
//   below their row's (column's) largest one, whose contribution to a
//   product is below 2^-39 of the row-times-column bound: Ootomo and Yokota's
//   extra 2^11 factor on lo, and the second accumulator it needs, buy
//   nothing here, and one FP32 accumulator holds all three terms.
//
// The level-wise engine packs every leaf's operands once (leaf_pack_kernel,
// after leaf_scale_kernel for FP16) and runs leaf_packed_kernel, 256x256
// tiles that copy pre-split slabs straight into LDS.  At the last level of a
// recursion the packed operands come instead straight from the parent
// quadrants (preadd_pack_a/b_kernel, after preadd_scale_a/b_kernel for
// FP16), which form S1..S4 / T1..T4 as the pre-addition kernel does and
// write all seven leaf operands of a node packed.  The classic recursion, which
// has no workspace for packed operands, runs split BF16 on
// leaf_split_kernel: 128x128 tiles (4 wavefronts of 64x64, the FP32 leaf's
// descriptors and XCD-aware walk) with K-slabs of 32 whose FP32 loads
// (branch-free buffer loads, zero outside the valid extent) are split in
// registers and stored to LDS as hi and lo arrays with k contiguous ([m][k]
// for A, [n][k] for B).  In both, one 16-byte LDS read gives the 8
// consecutive k a lane supplies to a 32x32x16 step.
#include <hip/hip_runtime.h>

#include "common.h"

namespace fastmm {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

namespace {

enum SplitFormat { kSplitBf16 = 0, kSplitFp16 = 1 };

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc16(const float* p, int bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  float* q = reinterpret_cast<float*>(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, __builtin_amdgcn_readfirstlane(bytes),
                                           0x00020000);
}

// BF16 bits of x rounded to nearest even (finite inputs).
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float((uint32_t)h << 16);
}

// hi and lo halves of four values; for FP16 the values are first scaled by
// 2^-e (e = 0 for BF16).
template <int FMT>
__device__ __forceinline__ void split4(float4 v, int e, u16x4& hi, u16x4& lo) {
  const float x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if constexpr (FMT == kSplitBf16) {
      const unsigned short h = bf16_rne(x[i]);
      hi[i] = h;
      lo[i] = bf16_rne(x[i] - bf16_to_f32(h));
    } else {
      const float y = __builtin_ldexpf(x[i], -e);
      const _Float16 h = (_Float16)y;
      hi[i] = __builtin_bit_cast(unsigned short, h);
      lo[i] = __builtin_bit_cast(unsigned short, (_Float16)(y - (float)h));
    }
  }
}

template <int FMT>
__device__ __forceinline__ f32x16 mfma16(u16x8 a, u16x8 b, f32x16 c) {
  if constexpr (FMT == kSplitBf16)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// Exponent e with m * 2^-e in [2^14, 2^15); 0 for a zero, NaN or infinite m
// (non-finite inputs then stay non-finite through the split).
__device__ __forceinline__ int scale_exponent(float m) {
  if (!(m > 0.f) || !(m <= 3.402823466e38f)) return 0;
  return __builtin_amdgcn_frexp_expf(m) - 15;
}

__device__ __forceinline__ float wave_max(float m) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  return m;
}

constexpr int kScaleRowsPerBlock = 4;    // one row of A per wavefront
constexpr int kScaleColsPerBlock = 256;  // one column of B per thread
constexpr int kScaleRowsPerPart = 256;   // rows of B per partial column maximum

}  // namespace

// Scale exponents of the FP16 form, one block range per descriptor.
// Blocks [0, a_blocks) take 4 rows of A each, one per wavefront (max over
// the kmax reduction columns), and store e_A.  Blocks [a_blocks, per_desc)
// take 256 columns of B by 256 rows each and store the partial maxima in the
// scratch after e_B (ceil(kmax / 256) x b_cols floats); leaf_scale_b_kernel
// then reduces them to e_B.  Splitting B's reduction keeps enough loads in
// flight: one thread per column walking all kmax rows is latency-bound.
template <bool VEC>
__global__ void __launch_bounds__(256)
leaf_scale_kernel(const GemmDesc* __restrict__ descs, int a_blocks, int per_desc) {
  const GemmDesc& d = descs[blockIdx.x / per_desc];
  if (d.prepacked) return;  // scaled by the fused pass
  const int blk = blockIdx.x % per_desc;
  const int kmax = d.kmax;
  const int tid = threadIdx.x;
  if (blk < a_blocks) {
    const int lane = tid & 63, wave = tid >> 6;
    const int r = blk * kScaleRowsPerBlock + wave;
    if (r >= d.a_rows) return;
    const float* a = d.A + (int64_t)r * d.lda;
    float m0 = 0.f, m1 = 0.f;
    if (VEC) {
      int k = 4 * lane;
      for (; k + 256 < kmax; k += 512) {
        const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(a + k));
        const f32x4 w = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(a + k + 256));
        m0 = fmaxf(m0, fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))));
        m1 = fmaxf(m1, fmaxf(fmaxf(fabsf(w[0]), fabsf(w[1])), fmaxf(fabsf(w[2]), fabsf(w[3]))));
      }
      if (k < kmax) {
        const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(a + k));
        m0 = fmaxf(m0, fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))));
      }
    } else {
      for (int k = lane; k < kmax; k += 64) m0 = fmaxf(m0, fabsf(a[k]));
    }
    const float m = wave_max(fmaxf(m0, m1));
    if (lane == 0) d.ea[r] = scale_exponent(m);
  } else {
    const int parts = (kmax + kScaleRowsPerPart - 1) / kScaleRowsPerPart;
    const int col_blocks = (d.b_cols + kScaleColsPerBlock - 1) / kScaleColsPerBlock;
    const int u = blk - a_blocks;
    if (u >= col_blocks * parts) return;
    const int p = u / col_blocks;
    const int c = (u - p * col_blocks) * kScaleColsPerBlock + tid;
    if (c >= d.b_cols) return;
    const int k0 = p * kScaleRowsPerPart;
    const int k1 = min(kmax, k0 + kScaleRowsPerPart);
    const int64_t ldb = d.ldb;
    const float* b = d.B + (int64_t)k0 * ldb + c;
    float m[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int k = 0;
    const int n = k1 - k0;
    for (; k + 8 <= n; k += 8)
#pragma unroll
      for (int i = 0; i < 8; ++i) m[i] = fmaxf(m[i], fabsf(b[(int64_t)(k + i) * ldb]));
    for (; k < n; ++k) m[0] = fmaxf(m[0], fabsf(b[(int64_t)k * ldb]));
    const float mx = fmaxf(fmaxf(fmaxf(m[0], m[1]), fmaxf(m[2], m[3])), fmaxf(fmaxf(m[4], m[5]), fmaxf(m[6], m[7])));
    reinterpret_cast<float*>(d.eb + d.b_cols)[(int64_t)p * d.b_cols + c] = mx;
  }
}

// e_B[c] from the partial column maxima of leaf_scale_kernel (descriptors
// with prepacked == which; the fused pass writes its own partials).
__global__ void __launch_bounds__(256)
leaf_scale_b_kernel(const GemmDesc* __restrict__ descs, int per_desc, int which) {
  const GemmDesc& d = descs[blockIdx.x / per_desc];
  if (d.prepacked != which) return;
  const int c = (blockIdx.x % per_desc) * 256 + threadIdx.x;
  if (c >= d.b_cols) return;
  const int parts = (d.kmax + kScaleRowsPerPart - 1) / kScaleRowsPerPart;
  const float* part = reinterpret_cast<const float*>(d.eb + d.b_cols);
  float m = 0.f;
  for (int p = 0; p < parts; ++p) m = fmaxf(m, part[(int64_t)p * d.b_cols + c]);
  d.eb[c] = scale_exponent(m);
}

template <int FMT, bool VEC>
__global__ void __launch_bounds__(256)
leaf_split_kernel(const GemmDesc* __restrict__ descs, int ndesc, int total_tiles, int xcd_chunk) {
  constexpr int BM = 128, BN = 128, BK = 32;
  constexpr int WM = 64, WN = 64, FM = 2, FN = 2;
  constexpr int LDK = BK + 8;  // 16-bit elements per LDS row (80 bytes: conflict-free 16-byte reads)
  constexpr bool kScaled = FMT == kSplitFp16;

  __shared__ __attribute__((aligned(16))) unsigned short Ah[2][BM * LDK], Al[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) unsigned short Bh[2][BN * LDK], Bl[2][BN * LDK];

  // Tile of this workgroup: the same XCD mapping and grouped walk as the FP32 leaf.
  const int logical = leaf_tile_of_block(blockIdx.x, gridDim.x, xcd_chunk);
  if (logical >= total_tiles) return;
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
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  const int lr = lane & 31, lh = lane >> 5;

  // A: thread loads rows a_r + 32 i (i = 0..3), columns a_c..a_c+3.
  const int a_r = tid / 8, a_c = (tid % 8) * 4;
  // B: thread loads column b_n, k-rows b_k..b_k+15 (4-byte loads, coalesced
  // across the wave), and writes them as one row of the [n][k] arrays: the
  // lanes of a store then write consecutive rows, which fall on distinct
  // LDS banks (four columns per thread gave 8-way bank conflicts).
  const int b_n = tid & (BN - 1), b_k = (tid / BN) * 16;

  const int rv = min(BM, a_rows - tm);
  const int cv = min(BN, b_cols - tn);
  const float* a_tile = A + (int64_t)tm * lda;
  const float* b_tile = B + tn;
  constexpr int kOOB = 0x7FFFFFF0;

  // Scale exponents of the rows and the column this thread splits.
  int ea_ld[4] = {0, 0, 0, 0};
  int eb_ld = 0;
  if constexpr (kScaled) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (a_r + 32 * i < rv) ea_ld[i] = d.ea[tm + a_r + 32 * i];
    if (b_n < cv) eb_ld = d.eb[tn + b_n];
  }

  float4 ra[4];
  float rb[16];
  auto load_slab = [&](int k0) {
    const int kv = min(BK, kmax - k0);
    const uint32_t a_bytes =
        (rv > 0 && kv > 0) ? (uint32_t)(((int64_t)(rv - 1) * lda + kv) * 4) : 0u;
    const uint32_t b_bytes =
        (cv > 0 && kv > 0) ? (uint32_t)(((int64_t)(kv - 1) * ldb + cv) * 4) : 0u;
    const __amdgpu_buffer_rsrc_t ar = make_rsrc16(a_tile + k0, (int)a_bytes);
    const __amdgpu_buffer_rsrc_t br = make_rsrc16(b_tile + (int64_t)k0 * ldb, (int)b_bytes);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = a_r + 32 * i;
      const int base = (r * (int)lda + a_c) * 4;
      if (VEC) {
        const int off = (r < rv && a_c < kv) ? base : kOOB;
        ra[i] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(ar, off, 0, 0));
      } else {
        float e[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int off = (r < rv && a_c + q < kv) ? base + 4 * q : kOOB;
          e[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ar, off, 0, 0));
        }
        ra[i] = make_float4(e[0], e[1], e[2], e[3]);
      }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int k = b_k + i;
      const int off = (k < kv && b_n < cv) ? (k * (int)ldb + b_n) * 4 : kOOB;
      rb[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(br, off, 0, 0));
    }
  };

  auto store_slab = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      u16x4 h, l;
      split4<FMT>(ra[i], ea_ld[i], h, l);
      const int o = (a_r + 32 * i) * LDK + a_c;
      *reinterpret_cast<u16x4*>(&Ah[buf][o]) = h;
      *reinterpret_cast<u16x4*>(&Al[buf][o]) = l;
    }
    // B: the 16 k of column b_n go to row b_n of the [n][k] arrays, 8 at a
    // time (16-byte stores).
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      u16x4 h0, l0, h1, l1;
      split4<FMT>(make_float4(rb[8 * q], rb[8 * q + 1], rb[8 * q + 2], rb[8 * q + 3]), eb_ld, h0, l0);
      split4<FMT>(make_float4(rb[8 * q + 4], rb[8 * q + 5], rb[8 * q + 6], rb[8 * q + 7]), eb_ld, h1, l1);
      const u16x8 h = {h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3]};
      const u16x8 l = {l0[0], l0[1], l0[2], l0[3], l1[0], l1[1], l1[2], l1[3]};
      const int o = b_n * LDK + b_k + 8 * q;
      *reinterpret_cast<u16x8*>(&Bh[buf][o]) = h;
      *reinterpret_cast<u16x8*>(&Bl[buf][o]) = l;
    }
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
    const bool more = kt + 1 < nk;
    if (more) load_slab((kt + 1) * BK);
#pragma unroll
    for (int g16 = 0; g16 < BK / 16; ++g16) {
      // Lane half h supplies k = 16 g16 + 8 h + e (e = 0..7) for both operands.
      const int kb = g16 * 16 + lh * 8;
      u16x8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int o = (wm + 32 * i + lr) * LDK + kb;
        ah[i] = *reinterpret_cast<const u16x8*>(&Ah[cur][o]);
        al[i] = *reinterpret_cast<const u16x8*>(&Al[cur][o]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int o = (wn + 32 * j + lr) * LDK + kb;
        bh[j] = *reinterpret_cast<const u16x8*>(&Bh[cur][o]);
        bl[j] = *reinterpret_cast<const u16x8*>(&Bl[cur][o]);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acc[i][j] = mfma16<FMT>(al[i], bh[j], acc[i][j]);
          acc[i][j] = mfma16<FMT>(ah[i], bl[j], acc[i][j]);
          acc[i][j] = mfma16<FMT>(ah[i], bh[j], acc[i][j]);
        }
    }
    if (more) store_slab(cur ^ 1);
    __syncthreads();
  }

  // Epilogue: register r of block (i, j) holds row 8*(r/4) + 4*(lane/32) + r%4
  // and column lane%32 of that 32x32 block.  The FP16 form undoes the row
  // and column scales here.
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = tn + wn + 32 * j + lr;
      if (col >= c_cols) continue;
      int ec = 0;
      if constexpr (kScaled) ec = col < b_cols ? d.eb[col] : 0;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = tm + wm + 32 * i + 8 * (r >> 2) + 4 * lh + (r & 3);
        if (row < c_rows) {
          float v = acc[i][j][r];
          if constexpr (kScaled) v = __builtin_ldexpf(v, ec + (row < a_rows ? d.ea[row] : 0));
          float* cp = C + (int64_t)row * ldc + col;
          *cp = beta ? *cp + v : v;
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Packed form.  A pass over every leaf's operands (leaf_pack_kernel) writes
// them once as hi/lo 16-bit tiles, in exactly the order the leaf's LDS holds
// them, so that the leaf (leaf_packed_kernel) copies slabs straight into LDS
// and runs nothing but MFMAs: the register-split kernel above splits each A
// slab once per column of tiles and each B slab once per row of tiles, about
// as many VALU cycles as MFMA cycles.
//
// Packed layout of one leaf operand (A, or B read as B^T): blocks of 128 rows
// of A (columns of B) by 32 k, zero beyond the valid extent; block (t, s) of
// tile t and slab s at byte (t * slabs + s) * 16384, slabs = ceil(kmax / 32).
// In a block the hi half (8 KB) comes first, then the lo half, each 128 rows
// of 64 bytes; row r keeps k = 8c..8c+7 (16 bytes) in 16-byte slot
// c ^ ((r >> 2) & 3), which makes the 16-byte fragment reads of the MFMA
// loop free of LDS bank conflicts.
namespace {
constexpr int kPackRows = 128;
constexpr int kPackK = 32;
constexpr int kPackHalfBytes = kPackRows * kPackK * 2;   // 8 KB
constexpr int kPackBlockBytes = 2 * kPackHalfBytes;      // 16 KB
constexpr int kPackSlabsPerGroup = 4;                    // slabs per pack workgroup

__device__ __forceinline__ int pack_slot(int r, int c) { return r * 64 + ((c ^ ((r >> 2) & 3)) << 4); }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc_bytes(const void* p, int bytes) {
  return make_rsrc16(reinterpret_cast<const float*>(p), bytes);
}
}  // namespace

// One workgroup per (operand side, tile, group of 4 slabs) of a descriptor:
// units [0, a_units) of a descriptor's range pack A, [a_units, per_desc)
// pack B.  Each thread splits 8 consecutive k of one row (column) per step.
template <int FMT, bool VEC>
__global__ void __launch_bounds__(256)
leaf_pack_kernel(const GemmDesc* __restrict__ descs, int a_units, int per_desc) {
  const GemmDesc& d = descs[blockIdx.x / per_desc];
  if (d.prepacked) return;  // written by the fused pre-addition and pack pass
  int u = blockIdx.x % per_desc;
  const int kmax = d.kmax;
  const int slabs = (kmax + kPackK - 1) / kPackK;
  const int groups = (slabs + kPackSlabsPerGroup - 1) / kPackSlabsPerGroup;
  const bool side_a = u < a_units;
  if (!side_a) u -= a_units;
  const int tiles = side_a ? (d.c_rows + kPackRows - 1) / kPackRows : (d.c_cols + kPackRows - 1) / kPackRows;
  if (u >= tiles * groups) return;
  const int t = u / groups;
  const int s0 = (u - t * groups) * kPackSlabsPerGroup;
  const int s1 = min(s0 + kPackSlabsPerGroup, slabs);
  char* out = reinterpret_cast<char*>(side_a ? d.pa : d.pb) + (int64_t)t * slabs * kPackBlockBytes;
  const int tid = threadIdx.x;
  if (side_a) {
    const int rv = min(kPackRows, d.a_rows - t * kPackRows);
    const float* a = d.A + (int64_t)t * kPackRows * d.lda;
    for (int s = s0; s < s1; ++s) {
      const int k0 = s * kPackK;
      const int kv = min(kPackK, kmax - k0);
      char* blk = out + (int64_t)s * kPackBlockBytes;
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const int q = it * 256 + tid;
        const int r = q >> 2, c = q & 3;
        float4 x0 = make_float4(0.f, 0.f, 0.f, 0.f), x1 = x0;
        int e = 0;
        if (r < rv) {
          const float* src = a + (int64_t)r * d.lda + k0 + 8 * c;
          if (VEC && 8 * c + 8 <= kv) {
            x0 = *reinterpret_cast<const float4*>(src);
            x1 = *reinterpret_cast<const float4*>(src + 4);
          } else {
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = (8 * c + i < kv) ? src[i] : 0.f;
            x0 = make_float4(v[0], v[1], v[2], v[3]);
            x1 = make_float4(v[4], v[5], v[6], v[7]);
          }
          if constexpr (FMT == kSplitFp16) e = d.ea[t * kPackRows + r];
        }
        u16x4 h0, l0, h1, l1;
        split4<FMT>(x0, e, h0, l0);
        split4<FMT>(x1, e, h1, l1);
        const int o = pack_slot(r, c);
        *reinterpret_cast<u16x8*>(blk + o) = u16x8{h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3]};
        *reinterpret_cast<u16x8*>(blk + kPackHalfBytes + o) =
            u16x8{l0[0], l0[1], l0[2], l0[3], l1[0], l1[1], l1[2], l1[3]};
      }
    }
  } else {
    const int cv = min(kPackRows, d.b_cols - t * kPackRows);
    const int64_t ldb = d.ldb;
    const float* b = d.B + (int64_t)t * kPackRows;
    if constexpr (VEC) {
      // Transposed through LDS: 16-byte loads along rows of B, then each
      // thread gathers 8 k of one column and the wavefront writes 1 KB of
      // packed rows at once (column-wise global writes ran at 3 TB/s).  Row
      // k of the slab keeps column n at n ^ (8 * (k / 8)), which makes the
      // gathers (lanes: 8 columns x 4 chunks) free of bank conflicts.
      __shared__ __attribute__((aligned(16))) float bt[kPackK * kPackRows];
      int e = 0;
      for (int s = s0; s < s1; ++s) {
        const int k0 = s * kPackK;
        const int kv = min(kPackK, kmax - k0);
        char* blk = out + (int64_t)s * kPackBlockBytes;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int kr = (tid >> 5) + 8 * i, n4 = 4 * (tid & 31);
          float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
          if (kr < kv && n4 < cv) x = *reinterpret_cast<const float4*>(b + (int64_t)(k0 + kr) * ldb + n4);
          *reinterpret_cast<float4*>(&bt[kr * kPackRows + (n4 ^ (8 * (kr >> 3)))]) = x;
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < 2; ++it) {
          const int q = it * 256 + tid;
          const int n = q >> 2, c = q & 3;  // lanes: 16 columns x 4 chunks per wavefront
          float v[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) v[i] = bt[(8 * c + i) * kPackRows + (n ^ (8 * c))];
          if constexpr (FMT == kSplitFp16) e = n < cv ? d.eb[t * kPackRows + n] : 0;
          u16x4 h0, l0, h1, l1;
          split4<FMT>(make_float4(v[0], v[1], v[2], v[3]), e, h0, l0);
          split4<FMT>(make_float4(v[4], v[5], v[6], v[7]), e, h1, l1);
          const int o = pack_slot(n, c);
          *reinterpret_cast<u16x8*>(blk + o) = u16x8{h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3]};
          *reinterpret_cast<u16x8*>(blk + kPackHalfBytes + o) =
              u16x8{l0[0], l0[1], l0[2], l0[3], l1[0], l1[1], l1[2], l1[3]};
        }
        __syncthreads();
      }
      return;
    }
    for (int s = s0; s < s1; ++s) {
      const int k0 = s * kPackK;
      const int kv = min(kPackK, kmax - k0);
      char* blk = out + (int64_t)s * kPackBlockBytes;
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const int q = it * 256 + tid;
        const int n = q & (kPackRows - 1), c = q >> 7;  // lanes take consecutive columns
        float v[8];
        int e = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
          v[i] = (n < cv && 8 * c + i < kv) ? b[(int64_t)(k0 + 8 * c + i) * ldb + n] : 0.f;
        if constexpr (FMT == kSplitFp16) e = n < cv ? d.eb[t * kPackRows + n] : 0;
        u16x4 h0, l0, h1, l1;
        split4<FMT>(make_float4(v[0], v[1], v[2], v[3]), e, h0, l0);
        split4<FMT>(make_float4(v[4], v[5], v[6], v[7]), e, h1, l1);
        const int o = pack_slot(n, c);
        *reinterpret_cast<u16x8*>(blk + o) = u16x8{h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3]};
        *reinterpret_cast<u16x8*>(blk + kPackHalfBytes + o) =
            u16x8{l0[0], l0[1], l0[2], l0[3], l1[0], l1[1], l1[2], l1[3]};
      }
    }
  }
}

// Eight consecutive floats of a quadrant row, zero outside the valid extent
// (ok: row valid; c: first column; vcols: valid columns).
__device__ __forceinline__ void load8(const float* p, bool ok, int c, int vcols, float* v) {
  if (ok && c + 7 < vcols) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    const float4 b = *reinterpret_cast<const float4*>(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (ok && c + e < vcols) ? p[e] : 0.f;
  }
}

__device__ __forceinline__ float4 load4q(const float* p, bool ok, int c, int vcols) {
  if (ok && c + 3 < vcols) return *reinterpret_cast<const float4*>(p);
  return make_float4((ok && c < vcols) ? p[0] : 0.f, (ok && c + 1 < vcols) ? p[1] : 0.f,
                     (ok && c + 2 < vcols) ? p[2] : 0.f, (ok && c + 3 < vcols) ? p[3] : 0.f);
}

// Split 8 values (FP16: scaled by 2^-e) and store them as the hi and lo
// 16-byte slots of a packed block.
template <int FMT>
__device__ __forceinline__ void store_packed8(char* blk, int slot, const float* v, int e) {
  u16x4 h0, l0, h1, l1;
  split4<FMT>(make_float4(v[0], v[1], v[2], v[3]), e, h0, l0);
  split4<FMT>(make_float4(v[4], v[5], v[6], v[7]), e, h1, l1);
  *reinterpret_cast<u16x8*>(blk + slot) = u16x8{h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3]};
  *reinterpret_cast<u16x8*>(blk + kPackHalfBytes + slot) =
      u16x8{l0[0], l0[1], l0[2], l0[3], l1[0], l1[1], l1[2], l1[3]};
}

template <typename Node>
__device__ __forceinline__ int find_unit_node(const Node* __restrict__ nodes, int nnodes, int b) {
  int lo = 0, hi = nnodes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (nodes[mid].unit_begin <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Fused last-level pre-addition and pack, A side: a workgroup takes 128 rows
// of the node's quadrants by 4 K-slabs of 32; each thread reads 8 consecutive
// k of one row from the four quadrants, forms S1..S4 with the pre-addition
// kernel's FP32 chains (so the values are those the unfused path would
// store), and writes all seven leaf operands' hi/lo slots.
template <int FMT>
__global__ void __launch_bounds__(256) preadd_pack_a_kernel(const PackNode* __restrict__ nodes, int nnodes) {
  const PackNode& n = nodes[find_unit_node(nodes, nnodes, blockIdx.x)];
  const PreAddNode& q = n.q;
  const int groups = (n.max_slabs + kPackSlabsPerGroup - 1) / kPackSlabsPerGroup;
  const int u = blockIdx.x - n.unit_begin;
  const int t = u / groups;
  const int s0 = (u - t * groups) * kPackSlabsPerGroup;
  const int s1 = min(s0 + kPackSlabsPerGroup, n.max_slabs);
  const int tid = threadIdx.x;
  // FP16: the exponents of the thread's two rows, for all seven operands.
  int ex[2][7] = {};
  if constexpr (FMT == kSplitFp16) {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int row = t * kPackRows + ((it * 256 + tid) >> 2);
#pragma unroll
      for (int i = 0; i < 7; ++i) ex[it][i] = row < n.rows[i] ? n.e[i][row] : 0;
    }
  }
  for (int s = s0; s < s1; ++s) {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int qi = it * 256 + tid;
      const int r = qi >> 2, c = qi & 3;
      const int row = t * kPackRows + r;
      const int col = s * kPackK + 8 * c;
      const float* top = q.src + (int64_t)row * q.ld;
      const float* bot = q.src + q.bot_off + (int64_t)row * q.ld;
      float x11[8], x12[8], x21[8], x22[8];
      load8(top + col, row < q.top_rows, col, q.left_cols, x11);
      load8(top + q.h_c + col, row < q.top_rows, col, q.right_cols, x12);
      load8(bot + col, row < q.bot_rows, col, q.left_cols, x21);
      load8(bot + q.h_c + col, row < q.bot_rows, col, q.right_cols, x22);
      float s1v[8], s2v[8], s3v[8], s4v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        // S1 = A21 + A22; S2 = S1 - A11; S3 = A11 - A21; S4 = A12 - S2
        s1v[e] = x21[e] + x22[e];
        s2v[e] = s1v[e] - x11[e];
        s3v[e] = x11[e] - x21[e];
        s4v[e] = x12[e] - s2v[e];
      }
      const float* outs[7] = {x11, x12, s4v, x22, s1v, s2v, s3v};
      const int slot = pack_slot(r, c);
#pragma unroll
      for (int i = 0; i < 7; ++i)
        if (s < n.slabs[i]) {
          store_packed8<FMT>(reinterpret_cast<char*>(n.dst[i]) + ((int64_t)t * n.slabs[i] + s) * kPackBlockBytes,
                             slot, outs[i], ex[it][i]);
        }
    }
  }
}

// Fused last-level pre-addition and pack, B side: a workgroup takes 128
// columns of the node's quadrants by 4 K-slabs of 32.  Each slab of the four
// quadrants goes through LDS (16-byte row loads, XOR-swizzled rows as in the
// pack pass); each thread then gathers 8 consecutive k of one column from
// all four, forms T1..T4 with the pre-addition kernel's FP32 chains and
// writes all seven leaf operands' hi/lo slots.
template <int FMT>
__global__ void __launch_bounds__(256) preadd_pack_b_kernel(const PackNode* __restrict__ nodes, int nnodes) {
  __shared__ __attribute__((aligned(16))) float bt[4][kPackK * kPackRows];
  const PackNode& n = nodes[find_unit_node(nodes, nnodes, blockIdx.x)];
  const PreAddNode& q = n.q;
  const int groups = (n.max_slabs + kPackSlabsPerGroup - 1) / kPackSlabsPerGroup;
  const int u = blockIdx.x - n.unit_begin;
  const int t = u / groups;
  const int s0 = (u - t * groups) * kPackSlabsPerGroup;
  const int s1 = min(s0 + kPackSlabsPerGroup, n.max_slabs);
  const int tid = threadIdx.x;
  // FP16: the exponents of the thread's two columns, for all seven operands.
  int ex[2][7] = {};
  if constexpr (FMT == kSplitFp16) {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int gcol = t * kPackRows + ((it * 256 + tid) >> 2);
#pragma unroll
      for (int i = 0; i < 7; ++i) ex[it][i] = gcol < n.rows[i] ? n.e[i][gcol] : 0;
    }
  }
  for (int s = s0; s < s1; ++s) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kr = (tid >> 5) + 8 * i, n4 = 4 * (tid & 31);
      const int row = s * kPackK + kr, col = t * kPackRows + n4;
      const float* top = q.src + (int64_t)row * q.ld;
      const float* bot = q.src + q.bot_off + (int64_t)row * q.ld;
      const int o = kr * kPackRows + (n4 ^ (8 * (kr >> 3)));
      *reinterpret_cast<float4*>(&bt[0][o]) = load4q(top + col, row < q.top_rows, col, q.left_cols);
      *reinterpret_cast<float4*>(&bt[1][o]) = load4q(top + q.h_c + col, row < q.top_rows, col, q.right_cols);
      *reinterpret_cast<float4*>(&bt[2][o]) = load4q(bot + col, row < q.bot_rows, col, q.left_cols);
      *reinterpret_cast<float4*>(&bt[3][o]) = load4q(bot + q.h_c + col, row < q.bot_rows, col, q.right_cols);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int qi = it * 256 + tid;
      const int col = qi >> 2, c = qi & 3;
      float x11[8], x12[8], x21[8], x22[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int o = (8 * c + e) * kPackRows + (col ^ (8 * c));
        x11[e] = bt[0][o];
        x12[e] = bt[1][o];
        x21[e] = bt[2][o];
        x22[e] = bt[3][o];
      }
      float t1[8], t2[8], t3[8], t4[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        // T1 = B12 - B11; T2 = B22 - T1; T3 = B22 - B12; T4 = T2 - B21
        t1[e] = x12[e] - x11[e];
        t2[e] = x22[e] - t1[e];
        t3[e] = x22[e] - x12[e];
        t4[e] = t2[e] - x21[e];
      }
      const float* outs[7] = {x11, x21, x22, t4, t1, t2, t3};
      const int slot = pack_slot(col, c);
#pragma unroll
      for (int i = 0; i < 7; ++i)
        if (s < n.slabs[i])
          store_packed8<FMT>(reinterpret_cast<char*>(n.dst[i]) + ((int64_t)t * n.slabs[i] + s) * kPackBlockBytes,
                             slot, outs[i], ex[it][i]);
    }
    __syncthreads();
  }
}

// Scale exponents of the fused nodes (scaled FP16), A side: one wavefront
// per row of a node streams the row of all four quadrants (16-byte loads),
// forms S1..S4 as the pre-addition kernel does, and keeps the largest
// magnitude of each of the seven leaf operands over that leaf's reduction
// length; e_A of leaf i for the row follows.
__global__ void __launch_bounds__(256) preadd_scale_a_kernel(const PackNode* __restrict__ nodes, int per_node) {
  const PackNode& n = nodes[blockIdx.x / per_node];
  const PreAddNode& q = n.q;
  const int lane = threadIdx.x & 63;
  const int row = (blockIdx.x % per_node) * 4 + (threadIdx.x >> 6);
  if (row >= q.h_r) return;
  const float* top = q.src + (int64_t)row * q.ld;
  const float* bot = q.src + q.bot_off + (int64_t)row * q.ld;
  const bool rt = row < q.top_rows, rb = row < q.bot_rows;
  float m[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int k = 4 * lane; k < q.h_c; k += 256) {
    const float4 a11 = load4q(top + k, rt, k, q.left_cols);
    const float4 a12 = load4q(top + q.h_c + k, rt, k, q.right_cols);
    const float4 a21 = load4q(bot + k, rb, k, q.left_cols);
    const float4 a22 = load4q(bot + q.h_c + k, rb, k, q.right_cols);
    const float x11[4] = {a11.x, a11.y, a11.z, a11.w}, x12[4] = {a12.x, a12.y, a12.z, a12.w};
    const float x21[4] = {a21.x, a21.y, a21.z, a21.w}, x22[4] = {a22.x, a22.y, a22.z, a22.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float s1 = x21[e] + x22[e], s2 = s1 - x11[e], s3 = x11[e] - x21[e], s4 = x12[e] - s2;
      const float v[7] = {x11[e], x12[e], s4, x22[e], s1, s2, s3};
#pragma unroll
      for (int i = 0; i < 7; ++i)
        if (k + e < n.kmax[i]) m[i] = fmaxf(m[i], fabsf(v[i]));
    }
  }
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    const float mx = wave_max(m[i]);
    if (lane == 0 && row < n.rows[i]) n.e[i][row] = scale_exponent(mx);
  }
}

// B side: one thread per column of a node, over one 256-row part of the
// reduction; the seven leaf operands' partial column maxima go to each
// leaf's scratch after e_B (as leaf_scale_kernel's do) and
// leaf_scale_b_kernel reduces them.
__global__ void __launch_bounds__(256) preadd_scale_b_kernel(const PackNode* __restrict__ nodes, int per_node,
                                                             int col_blocks) {
  const PackNode& n = nodes[blockIdx.x / per_node];
  const PreAddNode& q = n.q;
  const int u = blockIdx.x % per_node;
  const int p = u / col_blocks;
  const int col = (u - p * col_blocks) * 256 + threadIdx.x;
  if (col >= q.h_c) return;
  const int k0 = p * kScaleRowsPerPart;
  const int k1 = min(q.h_r, k0 + kScaleRowsPerPart);
  if (k0 >= k1) return;
  const bool cl = col < q.left_cols, cr = col < q.right_cols;
  float m[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int k = k0; k < k1; ++k) {
    const float* top = q.src + (int64_t)k * q.ld;
    const float* bot = q.src + q.bot_off + (int64_t)k * q.ld;
    const bool rt = k < q.top_rows, rb = k < q.bot_rows;
    const float x11 = (rt && cl) ? top[col] : 0.f, x12 = (rt && cr) ? top[q.h_c + col] : 0.f;
    const float x21 = (rb && cl) ? bot[col] : 0.f, x22 = (rb && cr) ? bot[q.h_c + col] : 0.f;
    const float t1 = x12 - x11, t2 = x22 - t1, t3 = x22 - x12, t4 = t2 - x21;
    const float v[7] = {x11, x21, x22, t4, t1, t2, t3};
#pragma unroll
    for (int i = 0; i < 7; ++i)
      if (k < n.kmax[i]) m[i] = fmaxf(m[i], fabsf(v[i]));
  }
#pragma unroll
  for (int i = 0; i < 7; ++i)
    if (col < n.rows[i] && k0 < n.kmax[i])
      reinterpret_cast<float*>(n.e[i] + n.rows[i])[(int64_t)p * n.rows[i] + col] = m[i];
}

// Leaf on packed operands: TM x TN tiles on WGM x WGN wavefronts, K-slabs
// of 32 double-buffered in LDS (the slab's A blocks, then its B blocks, 16 KB
// per 128 rows or columns), each slab copied straight from the packed blocks
// into LDS by buffer loads with the LDS bit (1 KB per wavefront
// instruction).  A tile reaching past the last packed block of an operand
// reads zeros there (empty buffer range).  The two 64 KB slab buffers of a
// 256x256 tile take the CU's LDS, so one workgroup runs per CU; 16
// wavefronts of 64x64 (four per SIMD) hide the fragment reads far better than
// 8 of 64x128 (the waves of one workgroup meet at every slab barrier):
// +8-9% at n = 19456.
template <int FMT, int TM, int TN, int WGM, int WGN>
__global__ void __launch_bounds__(64 * WGM * WGN, WGM * WGN / 4)  // one workgroup per CU
leaf_packed_kernel(const GemmDesc* __restrict__ descs, int ndesc, int total_tiles, int xcd_chunk) {
  constexpr int BK = kPackK;
  constexpr int kWaves = WGM * WGN;
  constexpr int WM = TM / WGM, WN = TN / WGN, FM = WM / 32, FN = WN / 32;
  constexpr int kABlocks = TM / kPackRows, kBBlocks = TN / kPackRows;
  constexpr int kStageBytes = (kABlocks + kBBlocks) * kPackBlockBytes;
  constexpr int kChunks = kStageBytes / 1024;
  static_assert(kChunks % kWaves == 0, "slab chunks must divide among the wavefronts");
  constexpr bool kScaled = FMT == kSplitFp16;
  __shared__ __attribute__((aligned(1024))) char lds0[kStageBytes];
  __shared__ __attribute__((aligned(1024))) char lds1[kStageBytes];

  const int logical = leaf_tile_of_block(blockIdx.x, gridDim.x, xcd_chunk);
  if (logical >= total_tiles) return;
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_begin <= logical) lo = mid; else hi = mid - 1;
  }
  const GemmDesc& d = descs[lo];
  float* __restrict__ C = d.C;
  const int64_t ldc = d.ldc;
  const int a_rows = d.a_rows, b_cols = d.b_cols, kmax = d.kmax;
  const int c_rows = d.c_rows, c_cols = d.c_cols;
  const int tiles_n = d.tiles_n;
  const int beta = d.beta;
  const int tiles_m = (c_rows + TM - 1) / TM;
  const int lt = logical - d.tile_begin;
  constexpr int GROUP = 8;
  const int group_tiles = GROUP * tiles_n;
  const int g = lt / group_tiles;
  const int first_m = g * GROUP;
  const int gm = min(tiles_m - first_m, GROUP);
  const int in_g = lt - g * group_tiles;
  const int tm = (first_m + in_g % gm) * TM;
  const int tn = (in_g / gm) * TN;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WGN) * WM, wn = (wave % WGN) * WN;
  const int lr = lane & 31, lh = lane >> 5;

  const int slabs = (kmax + BK - 1) / BK;
  const int pack_m = (c_rows + kPackRows - 1) / kPackRows;  // packed blocks of A per slab column
  const int pack_n = (c_cols + kPackRows - 1) / kPackRows;
  const char* pa = reinterpret_cast<const char*>(d.pa);
  const char* pb = reinterpret_cast<const char*>(d.pb);

  auto load_slab = [&](int s, char* __restrict__ dst) {
#pragma unroll
    for (int j = 0; j < kChunks / kWaves; ++j) {
      const int q = j * kWaves + wave;  // 1 KB chunk of the stage (wavefront-uniform)
      const int blk = q / 16;           // packed block of the stage: A blocks, then B blocks
      const bool is_a = blk < kABlocks;
      const int t = is_a ? tm / kPackRows + blk : tn / kPackRows + (blk - kABlocks);
      const bool there = t < (is_a ? pack_m : pack_n);
      const char* src = (is_a ? pa : pb) + ((int64_t)t * slabs + s) * kPackBlockBytes;
      const __amdgpu_buffer_rsrc_t r = make_rsrc_bytes(src, there ? kPackBlockBytes : 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          r, (__attribute__((address_space(3))) void*)(dst + q * 1024), 16, (q % 16) * 1024 + lane * 16,
          0, 0, 0);
    }
  };
  // Byte offset of the 16-byte fragment (row R of the stage's A rows, or
  // column R of its B columns, k-chunk c) in a stage.
  auto a_frag = [](int R, int c) { return (R / kPackRows) * kPackBlockBytes + pack_slot(R % kPackRows, c); };
  auto b_frag = [](int R, int c) {
    return (kABlocks + R / kPackRows) * kPackBlockBytes + pack_slot(R % kPackRows, c);
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  auto step = [&](const char* __restrict__ cur, char* __restrict__ next, int s) {
    const bool more = s + 1 < slabs;
    if (more) load_slab(s + 1, next);
#pragma unroll
    for (int g16 = 0; g16 < BK / 16; ++g16) {
      const int c = g16 * 2 + lh;  // lane half h supplies k = 16 g16 + 8 h + 0..7
      u16x8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int o = a_frag(wm + 32 * i + lr, c);
        ah[i] = *reinterpret_cast<const u16x8*>(cur + o);
        al[i] = *reinterpret_cast<const u16x8*>(cur + kPackHalfBytes + o);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int o = b_frag(wn + 32 * j + lr, c);
        bh[j] = *reinterpret_cast<const u16x8*>(cur + o);
        bl[j] = *reinterpret_cast<const u16x8*>(cur + kPackHalfBytes + o);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acc[i][j] = mfma16<FMT>(al[i], bh[j], acc[i][j]);
          acc[i][j] = mfma16<FMT>(ah[i], bl[j], acc[i][j]);
          acc[i][j] = mfma16<FMT>(ah[i], bh[j], acc[i][j]);
        }
    }
    if (more) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the next slab is in LDS
    __syncthreads();
  };

  if (slabs > 0) {
    load_slab(0, lds0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
  }
  for (int s = 0; s < slabs; s += 2) {
    step(lds0, lds1, s);
    if (s + 1 < slabs) step(lds1, lds0, s + 1);
  }

  // Epilogue: register r of block (i, j) holds row 8*(r/4) + 4*(lane/32) + r%4
  // and column lane%32 of that 32x32 block.
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = tn + wn + 32 * j + lr;
      if (col >= c_cols) continue;
      int ec = 0;
      if constexpr (kScaled) ec = col < b_cols ? d.eb[col] : 0;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = tm + wm + 32 * i + 8 * (r >> 2) + 4 * lh + (r & 3);
        if (row < c_rows) {
          float v = acc[i][j][r];
          if constexpr (kScaled) v = __builtin_ldexpf(v, ec + (row < a_rows ? d.ea[row] : 0));
          float* cp = C + (int64_t)row * ldc + col;
          *cp = beta ? *cp + v : v;
        }
      }
    }
}

void launch_leaf_bf16x3(const GemmDesc* d_descs, int ndesc, int total_tiles, bool vec,
                        hipStream_t stream, int xcd_chunk) {
  if (total_tiles <= 0) return;
  dim3 grid(total_tiles), block(256);
  if (vec)
    hipLaunchKernelGGL((leaf_split_kernel<kSplitBf16, true>), grid, block, 0, stream, d_descs, ndesc,
                       total_tiles, xcd_chunk);
  else
    hipLaunchKernelGGL((leaf_split_kernel<kSplitBf16, false>), grid, block, 0, stream, d_descs, ndesc,
                       total_tiles, xcd_chunk);
  FASTMM_HIP(hipGetLastError());
}

int64_t leaf_packed_bytes(int64_t rows, int64_t cols, int64_t k) {
  const int64_t slabs = (k + kPackK - 1) / kPackK;
  return ((rows + kPackRows - 1) / kPackRows + (cols + kPackRows - 1) / kPackRows) * slabs *
         kPackBlockBytes;
}

int64_t leaf_scale_bytes(int64_t rows, int64_t cols, int64_t k) {
  return 4 * (rows + cols + (k + kScaleRowsPerPart - 1) / kScaleRowsPerPart * cols);
}

int64_t leaf_packed_a_bytes(int64_t rows, int64_t k) {
  return (rows + kPackRows - 1) / kPackRows * ((k + kPackK - 1) / kPackK) * kPackBlockBytes;
}

int pack_node_units(const PackNode& n) {
  return n.tiles * ((n.max_slabs + kPackSlabsPerGroup - 1) / kPackSlabsPerGroup);
}

void launch_preadd_pack(int side, const PackNode* d_nodes, int nnodes, int total_units, bool fp16,
                        hipStream_t stream) {
  if (total_units <= 0 || nnodes <= 0) return;
  dim3 grid(total_units), block(256);
  if (side == 0) {
    if (fp16) hipLaunchKernelGGL(preadd_pack_a_kernel<kSplitFp16>, grid, block, 0, stream, d_nodes, nnodes);
    else hipLaunchKernelGGL(preadd_pack_a_kernel<kSplitBf16>, grid, block, 0, stream, d_nodes, nnodes);
  } else {
    if (fp16) hipLaunchKernelGGL(preadd_pack_b_kernel<kSplitFp16>, grid, block, 0, stream, d_nodes, nnodes);
    else hipLaunchKernelGGL(preadd_pack_b_kernel<kSplitBf16>, grid, block, 0, stream, d_nodes, nnodes);
  }
  FASTMM_HIP(hipGetLastError());
}

void launch_preadd_scale(const PackNode* d_a, int na, const PackNode* d_b, int nb, int max_rows,
                         int max_cols, int max_kdim, const GemmDesc* d_descs, int ndesc,
                         hipStream_t stream) {
  if (na > 0 && max_rows > 0) {
    const int64_t per_node = (max_rows + 3) / 4;
    if (per_node * na > INT32_MAX) throw Error(kNotSupported, "scale launch too large");
    hipLaunchKernelGGL(preadd_scale_a_kernel, dim3((unsigned)(per_node * na)), dim3(256), 0, stream, d_a,
                       (int)per_node);
    FASTMM_HIP(hipGetLastError());
  }
  if (nb > 0 && max_cols > 0 && max_kdim > 0) {
    const int64_t col_blocks = (max_cols + 255) / 256;
    const int64_t per_node = col_blocks * ((max_kdim + kScaleRowsPerPart - 1) / kScaleRowsPerPart);
    if (per_node * nb > INT32_MAX || col_blocks * ndesc > INT32_MAX)
      throw Error(kNotSupported, "scale launch too large");
    hipLaunchKernelGGL(preadd_scale_b_kernel, dim3((unsigned)(per_node * nb)), dim3(256), 0, stream, d_b,
                       (int)per_node, (int)col_blocks);
    FASTMM_HIP(hipGetLastError());
    hipLaunchKernelGGL(leaf_scale_b_kernel, dim3((unsigned)(col_blocks * ndesc)), dim3(256), 0, stream,
                       d_descs, (int)col_blocks, 1);
    FASTMM_HIP(hipGetLastError());
  }
}

void launch_leaf_packed(int tile, const GemmDesc* d_descs, int ndesc, int total_tiles, bool vec,
                        hipStream_t stream, int xcd_chunk, const LeafExtents& ext) {
  if (total_tiles <= 0) return;
  const bool fp16 = tile == kTileFp16x3;
  if (!fp16 && tile != kTileBf16x3) throw Error(kInvalidValue, "not a split-precision tile");
  // 1. FP16 only: scale exponents of the valid rows of A and columns of B.
  if (fp16 && ext.any_unpacked) {
    const int a_blocks = (ext.max_a_rows + kScaleRowsPerBlock - 1) / kScaleRowsPerBlock;
    const int64_t parts = (ext.max_kmax + kScaleRowsPerPart - 1) / kScaleRowsPerPart;
    const int64_t col_blocks = (ext.max_b_cols + kScaleColsPerBlock - 1) / kScaleColsPerBlock;
    const int64_t per_desc = a_blocks + col_blocks * parts;
    if (per_desc * ndesc > INT32_MAX || col_blocks * ndesc > INT32_MAX)
      throw Error(kNotSupported, "scale launch too large");
    if (per_desc > 0) {
      dim3 grid((unsigned)(per_desc * ndesc)), block(256);
      if (vec)
        hipLaunchKernelGGL((leaf_scale_kernel<true>), grid, block, 0, stream, d_descs, a_blocks, (int)per_desc);
      else
        hipLaunchKernelGGL((leaf_scale_kernel<false>), grid, block, 0, stream, d_descs, a_blocks, (int)per_desc);
      FASTMM_HIP(hipGetLastError());
    }
    if (col_blocks > 0) {
      dim3 grid((unsigned)(col_blocks * ndesc)), block(256);
      hipLaunchKernelGGL(leaf_scale_b_kernel, grid, block, 0, stream, d_descs, (int)col_blocks, 0);
      FASTMM_HIP(hipGetLastError());
    }
  }
  // 2. Pack both operands of every leaf.
  const int64_t groups = (ext.max_slabs + kPackSlabsPerGroup - 1) / kPackSlabsPerGroup;
  const int64_t a_units = (int64_t)((ext.max_c_rows + kPackRows - 1) / kPackRows) * groups;
  const int64_t b_units = (int64_t)((ext.max_c_cols + kPackRows - 1) / kPackRows) * groups;
  const int64_t per_desc = a_units + b_units;
  if (per_desc * ndesc > INT32_MAX) throw Error(kNotSupported, "pack launch too large");
  if (per_desc > 0 && ext.any_unpacked) {
    dim3 grid((unsigned)(per_desc * ndesc)), block(256);
    if (fp16) {
      if (vec)
        hipLaunchKernelGGL((leaf_pack_kernel<kSplitFp16, true>), grid, block, 0, stream, d_descs, (int)a_units, (int)per_desc);
      else
        hipLaunchKernelGGL((leaf_pack_kernel<kSplitFp16, false>), grid, block, 0, stream, d_descs, (int)a_units, (int)per_desc);
    } else {
      if (vec)
        hipLaunchKernelGGL((leaf_pack_kernel<kSplitBf16, true>), grid, block, 0, stream, d_descs, (int)a_units, (int)per_desc);
      else
        hipLaunchKernelGGL((leaf_pack_kernel<kSplitBf16, false>), grid, block, 0, stream, d_descs, (int)a_units, (int)per_desc);
    }
    FASTMM_HIP(hipGetLastError());
  }
  // 3. The leaf itself.
  constexpr int TM = kSplitTileM, TN = kSplitTileN, WGM = kSplitWavesM, WGN = kSplitWavesN;
  dim3 grid(total_tiles), block(64 * WGM * WGN);
  if (fp16)
    hipLaunchKernelGGL((leaf_packed_kernel<kSplitFp16, TM, TN, WGM, WGN>), grid, block, 0, stream, d_descs,
                       ndesc, total_tiles, xcd_chunk);
  else
    hipLaunchKernelGGL((leaf_packed_kernel<kSplitBf16, TM, TN, WGM, WGN>), grid, block, 0, stream, d_descs,
                       ndesc, total_tiles, xcd_chunk);
  FASTMM_HIP(hipGetLastError());
}

}  // namespace fastmm
