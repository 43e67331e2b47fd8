// Fused quadrant additions of Winograd's variant of Strassen's recursion.
//
// The paper leaves the fast recursion with GPU leaves as future work
// (Section 4.3, closing remarks) and never prints the schedule; the one used
// here is Winograd's standard 7-product form with 8 pre-additions and 7
// post-additions per level:
//   S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2
//   T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21
//   C11 = P1 + P2,  U2 = P1 + P6,  U3 = U2 + P7,   U4 = U2 + P5
//   C12 = U4 + P3,  C21 = U3 - P4, C22 = U3 + P5
// Each output element is one fixed chain of FP32 operations in exactly this
// order (no fused multiply-add can form: there are no products), so results
// are reproducible bit for bit against any IEEE FP32 evaluation of the chain.
//
// The kernels are HBM-bound streams: every launch covers all nodes of one
// recursion level, every input quadrant is read once and every output written
// once, four consecutive floats per thread (16-byte accesses, consecutive
// threads on consecutive addresses).  Quadrants use the split of equation (1)
// with virtual zero padding: reads outside a parent's valid extent give 0.
#include <hip/hip_runtime.h>

#include "common.h"

namespace fastmm {

// Every element is read once and written once, so the 16-byte accesses are
// marked non-temporal (streamed past the caches): +4-12% bandwidth on these
// kernels.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
constexpr int kAddThreads = kAddThreadsPerBlock;
constexpr int kItems = kAddChunk / kAddThreads;  // float4 groups per thread

__device__ __forceinline__ float4 load4(const float* p, bool vec, bool rv, int c, int vcols) {
  float4 v;
  if (vec && rv && c + 3 < vcols) {
    const nt_f4 t = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
    v = make_float4(t.x, t.y, t.z, t.w);
  } else {
    v.x = (rv && c + 0 < vcols) ? p[0] : 0.f;
    v.y = (rv && c + 1 < vcols) ? p[1] : 0.f;
    v.z = (rv && c + 2 < vcols) ? p[2] : 0.f;
    v.w = (rv && c + 3 < vcols) ? p[3] : 0.f;
  }
  return v;
}

__device__ __forceinline__ void store4(float* p, float4 v, bool vec, bool rv, int c, int cols) {
  if (!rv) return;
  if (vec && c + 3 < cols) {
    const nt_f4 t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, reinterpret_cast<nt_f4*>(p));
  } else {
    if (c + 0 < cols) p[0] = v.x;
    if (c + 1 < cols) p[1] = v.y;
    if (c + 2 < cols) p[2] = v.z;
    if (c + 3 < cols) p[3] = v.w;
  }
}

// Node owning workgroup b (block_begin ascending; one search per workgroup).
template <typename Node>
__device__ __forceinline__ int find_node(const Node* __restrict__ nodes, int nnodes, int b) {
  int lo = 0, hi = nnodes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (nodes[mid].block_begin <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// side 0: A operand -> S1..S4.  side 1: B operand -> T1..T4.
template <int SIDE, bool VEC>
__global__ void __launch_bounds__(kAddThreads)
preadd_kernel(const PreAddNode* __restrict__ nodes, int nnodes) {
  const PreAddNode nd = nodes[find_node(nodes, nnodes, blockIdx.x)];
  const int h_r = nd.h_r, h_c = nd.h_c;
  const unsigned out_q = nd.mask ? (unsigned)nd.mask : 0xFu;
  // Quadrants read by the requested outputs (see preadd_inputs).
  unsigned in_q = 0;
  if (SIDE == 0) {
    if (out_q & 1u) in_q |= 0xCu;
    if (out_q & 2u) in_q |= 0xDu;
    if (out_q & 4u) in_q |= 0x5u;
    if (out_q & 8u) in_q |= 0xFu;
  } else {
    if (out_q & 1u) in_q |= 0x3u;
    if (out_q & 2u) in_q |= 0xBu;
    if (out_q & 4u) in_q |= 0xAu;
    if (out_q & 8u) in_q |= 0xFu;
  }
  const int c4n = (h_c + 3) >> 2;
  const int64_t groups = (int64_t)h_r * c4n;
  const int64_t g0 = (int64_t)(blockIdx.x - nd.block_begin) * kAddChunk;
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t gidx = g0 + it * kAddThreads + threadIdx.x;
    if (gidx >= groups) break;
    const int r = (int)(gidx / c4n);
    const int c = (int)(gidx - (int64_t)r * c4n) * 4;
    const float* top = nd.src + (int64_t)r * nd.ld;
    const float* bot = nd.src + nd.bot_off + (int64_t)r * nd.ld;
    // Quadrants the requested outputs do not need are never read (they may
    // not have been copied in yet); they enter as zero.
    const bool rt = r < nd.top_rows;
    const bool rb = r < nd.bot_rows;
    const float4 x11 = load4(top + c, VEC, rt && (in_q & 1u), c, nd.left_cols);
    const float4 x12 = load4(top + nd.right_off + c, VEC, rt && (in_q & 2u), c, nd.right_cols);
    const float4 x21 = load4(bot + c, VEC, rb && (in_q & 4u), c, nd.left_cols);
    const float4 x22 = load4(bot + nd.right_off + c, VEC, rb && (in_q & 8u), c, nd.right_cols);
    float4 o1, o2, o3, o4;
    if (SIDE == 0) {
      // S1 = A21 + A22; S2 = S1 - A11; S3 = A11 - A21; S4 = A12 - S2
      o1.x = x21.x + x22.x; o1.y = x21.y + x22.y; o1.z = x21.z + x22.z; o1.w = x21.w + x22.w;
      o2.x = o1.x - x11.x;  o2.y = o1.y - x11.y;  o2.z = o1.z - x11.z;  o2.w = o1.w - x11.w;
      o3.x = x11.x - x21.x; o3.y = x11.y - x21.y; o3.z = x11.z - x21.z; o3.w = x11.w - x21.w;
      o4.x = x12.x - o2.x;  o4.y = x12.y - o2.y;  o4.z = x12.z - o2.z;  o4.w = x12.w - o2.w;
    } else {
      // T1 = B12 - B11; T2 = B22 - T1; T3 = B22 - B12; T4 = T2 - B21
      o1.x = x12.x - x11.x; o1.y = x12.y - x11.y; o1.z = x12.z - x11.z; o1.w = x12.w - x11.w;
      o2.x = x22.x - o1.x;  o2.y = x22.y - o1.y;  o2.z = x22.z - o1.z;  o2.w = x22.w - o1.w;
      o3.x = x22.x - x12.x; o3.y = x22.y - x12.y; o3.z = x22.z - x12.z; o3.w = x22.w - x12.w;
      o4.x = o2.x - x21.x;  o4.y = o2.y - x21.y;  o4.z = o2.z - x21.z;  o4.w = o2.w - x21.w;
    }
    float* out = nd.dst + (int64_t)r * h_c + c;
    if (out_q & 1u) store4(out, o1, VEC, true, c, h_c);
    if (out_q & 2u) store4(out + nd.out_stride, o2, VEC, true, c, h_c);
    if (out_q & 4u) store4(out + 2 * nd.out_stride, o3, VEC, true, c, h_c);
    if (out_q & 8u) store4(out + 3 * nd.out_stride, o4, VEC, true, c, h_c);
  }
}

template <bool VEC, int QUAD>
__global__ void __launch_bounds__(kAddThreads)
postadd_kernel(const PostAddNode* __restrict__ nodes, int nnodes) {
  const PostAddNode nd = nodes[find_node(nodes, nnodes, blockIdx.x)];
  const int h_r = nd.h_r, h_c = nd.h_c;
  const int c4n = (h_c + 3) >> 2;
  const int64_t groups = (int64_t)h_r * c4n;
  const int64_t g0 = (int64_t)(blockIdx.x - nd.block_begin) * kAddChunk;
  // Products each quadrant reads (P1..P7 = bit 0..6).
  constexpr unsigned kNeed = QUAD < 0 ? 0x7Fu
                           : QUAD == 0 ? 0x03u                 // C11: P1 P2
                           : QUAD == 1 ? (0x01u | 0x20u | 0x10u | 0x04u)  // C12: P1 P6 P5 P3
                           : QUAD == 2 ? (0x01u | 0x20u | 0x40u | 0x08u)  // C21: P1 P6 P7 P4
                                       : (0x01u | 0x20u | 0x40u | 0x10u); // C22: P1 P6 P7 P5
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t gidx = g0 + it * kAddThreads + threadIdx.x;
    if (gidx >= groups) break;
    const int r = (int)(gidx / c4n);
    const int c = (int)(gidx - (int64_t)r * c4n) * 4;
    const float* p = nd.P + (int64_t)r * h_c + c;
    float4 P[7];
#pragma unroll
    for (int i = 0; i < 7; ++i)
      P[i] = (kNeed >> i) & 1u ? load4(p + i * nd.p_stride, VEC, true, c, h_c)
                               : make_float4(0.f, 0.f, 0.f, 0.f);
    float4 c11, c12, c21, c22, u2, u3, u4;
    // C11 = P1 + P2; U2 = P1 + P6; U3 = U2 + P7; U4 = U2 + P5
    // C12 = U4 + P3; C21 = U3 - P4; C22 = U3 + P5
    c11.x = P[0].x + P[1].x; c11.y = P[0].y + P[1].y; c11.z = P[0].z + P[1].z; c11.w = P[0].w + P[1].w;
    u2.x = P[0].x + P[5].x;  u2.y = P[0].y + P[5].y;  u2.z = P[0].z + P[5].z;  u2.w = P[0].w + P[5].w;
    u3.x = u2.x + P[6].x;    u3.y = u2.y + P[6].y;    u3.z = u2.z + P[6].z;    u3.w = u2.w + P[6].w;
    u4.x = u2.x + P[4].x;    u4.y = u2.y + P[4].y;    u4.z = u2.z + P[4].z;    u4.w = u2.w + P[4].w;
    c12.x = u4.x + P[2].x;   c12.y = u4.y + P[2].y;   c12.z = u4.z + P[2].z;   c12.w = u4.w + P[2].w;
    c21.x = u3.x - P[3].x;   c21.y = u3.y - P[3].y;   c21.z = u3.z - P[3].z;   c21.w = u3.w - P[3].w;
    c22.x = u3.x + P[4].x;   c22.y = u3.y + P[4].y;   c22.z = u3.z + P[4].z;   c22.w = u3.w + P[4].w;
    float* top = nd.dst + (int64_t)r * nd.ld;
    float* bot = nd.dst + nd.bot_off + (int64_t)r * nd.ld;
    const bool rt = r < nd.top_rows;
    const bool rb = r < nd.bot_rows;
    if (QUAD < 0 || QUAD == 0) store4(top + c, c11, VEC, rt, c, nd.left_cols);
    if (QUAD < 0 || QUAD == 1) store4(top + nd.right_off + c, c12, VEC, rt, c, nd.right_cols);
    if (QUAD < 0 || QUAD == 2) store4(bot + c, c21, VEC, rb, c, nd.left_cols);
    if (QUAD < 0 || QUAD == 3) store4(bot + nd.right_off + c, c22, VEC, rb, c, nd.right_cols);
  }
}

// ---------------------------------------------------------------------------
// Several levels in one pass.  Where a subtree splits exactly at each of L
// levels, one element position of the bottom cell grid meets the same
// position of every S, T and P block in it: a thread loads the 4^L values of
// its position in the top operand, forms the S (T) blocks of every level in
// registers and writes each once; a post-addition thread loads its
// position in the 7^L bottom products and writes the 4^L results.  The chains
// are the single-level ones, operand for operand, so results are bit for bit
// those of the level-by-level launches; what disappears is the traffic of
// the levels in between (each S or T block of an inner level read back, each
// inner product written and read back), and the writes of the S / T cells
// that only the sums of the next level inside the subtree need.

template <int W>
struct Vw {
  float v[W];
};
typedef float nt_f2 __attribute__((ext_vector_type(2)));

template <int W>
__device__ __forceinline__ Vw<W> ldw(const float* p) {
  Vw<W> r;
  if constexpr (W == 4) {
    const nt_f4 t = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
    r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
  } else if constexpr (W == 2) {
    const nt_f2 t = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
    r.v[0] = t.x; r.v[1] = t.y;
  } else {
    r.v[0] = __builtin_nontemporal_load(p);
  }
  return r;
}

template <int W>
__device__ __forceinline__ void stw(float* p, const Vw<W>& x) {
  if constexpr (W == 4) {
    const nt_f4 t = {x.v[0], x.v[1], x.v[2], x.v[3]};
    __builtin_nontemporal_store(t, reinterpret_cast<nt_f4*>(p));
  } else if constexpr (W == 2) {
    const nt_f2 t = {x.v[0], x.v[1]};
    __builtin_nontemporal_store(t, reinterpret_cast<nt_f2*>(p));
  } else {
    __builtin_nontemporal_store(x.v[0], p);
  }
}

// Loads of a clipped top operand: elements outside the valid rows / columns
// read as zero.
template <int W>
__device__ __forceinline__ Vw<W> ldw_valid(const float* p, bool rv, int64_t col, int64_t vcols) {
  if (rv && col + W <= vcols) return ldw<W>(p);
  Vw<W> r;
#pragma unroll
  for (int i = 0; i < W; ++i) r.v[i] = (rv && col + i < vcols) ? p[i] : 0.f;
  return r;
}

template <int W>
__device__ __forceinline__ Vw<W> vadd(const Vw<W>& a, const Vw<W>& b) {
  Vw<W> r;
#pragma unroll
  for (int i = 0; i < W; ++i) r.v[i] = a.v[i] + b.v[i];
  return r;
}

template <int W>
__device__ __forceinline__ Vw<W> vsub(const Vw<W>& a, const Vw<W>& b) {
  Vw<W> r;
#pragma unroll
  for (int i = 0; i < W; ++i) r.v[i] = a.v[i] - b.v[i];
  return r;
}

// One pre-addition level of a subtree.  X: the node's operand as a 2^J x 2^J
// grid (this thread's element of each cell).  Writes S1..S4 (T1..T4) of the
// node -- level base dst[REL], node index `node` -- and recurses into the
// seven children's operands in product order (A side: A11, A12, S4, A22,
// S1, S2, S3; B side: B11, B21, B22, T4, T1, T2, T3).
template <int SIDE, int J, int REL, int W>
__device__ __forceinline__ void tree_pre(const Vw<W> (&X)[1 << J][1 << J], const TreeNode& nd,
                                         int64_t node, int r, int c) {
  constexpr int H = 1 << (J - 1);
  Vw<W> S[4][H][H];
#pragma unroll
  for (int u = 0; u < H; ++u)
#pragma unroll
    for (int v = 0; v < H; ++v) {
      const Vw<W>& x11 = X[u][v];
      const Vw<W>& x12 = X[u][v + H];
      const Vw<W>& x21 = X[u + H][v];
      const Vw<W>& x22 = X[u + H][v + H];
      if constexpr (SIDE == 0) {
        // S1 = A21 + A22; S2 = S1 - A11; S3 = A11 - A21; S4 = A12 - S2
        S[0][u][v] = vadd(x21, x22);
        S[1][u][v] = vsub(S[0][u][v], x11);
        S[2][u][v] = vsub(x11, x21);
        S[3][u][v] = vsub(x12, S[1][u][v]);
      } else {
        // T1 = B12 - B11; T2 = B22 - T1; T3 = B22 - B12; T4 = T2 - B21
        S[0][u][v] = vsub(x12, x11);
        S[1][u][v] = vsub(x22, S[0][u][v]);
        S[2][u][v] = vsub(x22, x12);
        S[3][u][v] = vsub(S[1][u][v], x21);
      }
    }
  // Blocks of this level: (H br) x (H bc), dense.  Below this level each
  // block is read only through the children that are quadrant views (A11,
  // A12, A22 / B11, B21, B22) -- the other quadrant enters the sums done
  // here in registers -- and in full only at the bottom of the subtree (by
  // the leaves, the pack pass or the next launch, all of which read views
  // within their valid extents).  So cell (u, v) is written only if every
  // level of its path is a view quadrant: no bit of u set where v's is
  // clear (A side), or the reverse (B side).
  const int64_t ldo = (int64_t)H * nd.bc;
  const int64_t blk = (int64_t)H * nd.br * ldo;
  float* base = nd.dst[REL] + node * 4 * blk + (int64_t)r * ldo + c;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int u = 0; u < H; ++u)
#pragma unroll
      for (int v = 0; v < H; ++v)
        if ((SIDE == 0 ? (u & ~v) : (v & ~u)) == 0)
          stw(base + i * blk + (int64_t)u * nd.br * ldo + (int64_t)v * nd.bc, S[i][u][v]);
  if constexpr (J > 1) {
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      Vw<W> Ch[H][H];
#pragma unroll
      for (int u = 0; u < H; ++u)
#pragma unroll
        for (int v = 0; v < H; ++v) {
          if constexpr (SIDE == 0) {
            Ch[u][v] = i == 0 ? X[u][v] : i == 1 ? X[u][v + H] : i == 2 ? S[3][u][v]
                     : i == 3 ? X[u + H][v + H] : S[i - 4][u][v];
          } else {
            Ch[u][v] = i == 0 ? X[u][v] : i == 1 ? X[u + H][v] : i == 2 ? X[u + H][v + H]
                     : i == 3 ? S[3][u][v] : S[i - 4][u][v];
          }
        }
      tree_pre<SIDE, J - 1, REL + 1, W>(Ch, nd, node * 7 + i, r, c);
    }
  }
}

// CLIP: some top node of the launch is clipped (reads outside its valid
// extent give zero); without it every read is a plain one.
template <int SIDE, int L, int W, bool CLIP>
__global__ void __launch_bounds__(kAddThreads)
tree_preadd_kernel(const TreeNode* __restrict__ nodes, int nnodes) {
  const TreeNode nd = nodes[find_node(nodes, nnodes, blockIdx.x)];
  const int cw = nd.bc / W;
  const int64_t g = (int64_t)(blockIdx.x - nd.block_begin) * kAddThreads + threadIdx.x;
  if (g >= (int64_t)nd.br * cw) return;
  const int r = (int)(g / cw);
  const int c = (int)(g - (int64_t)r * cw) * W;
  Vw<W> X[1 << L][1 << L];
#pragma unroll
  for (int u = 0; u < (1 << L); ++u)
#pragma unroll
    for (int v = 0; v < (1 << L); ++v)
      X[u][v] = CLIP ? ldw_valid<W>(nd.src + ((int64_t)u * nd.br + r) * nd.ld + (int64_t)v * nd.bc + c,
                                    (int64_t)u * nd.br + r < nd.vrows, (int64_t)v * nd.bc + c, nd.vcols)
                     : ldw<W>(nd.src + ((int64_t)u * nd.br + r) * nd.ld + (int64_t)v * nd.bc + c);
  tree_pre<SIDE, L, 0, W>(X, nd, nd.node, r, c);
}

__host__ __device__ constexpr int64_t pow7c(int j) { return j == 0 ? 1 : 7 * pow7c(j - 1); }

// The product of a subtree of J levels as a 2^J x 2^J grid (this thread's
// element of each cell), from its 7^J bottom products starting at block t.
// Children are taken in the order that keeps the fewest grids alive; every
// result is the single-level chain of the same operands.
template <int J, int W>
__device__ __forceinline__ void tree_post(Vw<W> (&G)[1 << J][1 << J], const float* __restrict__ P,
                                          int64_t t, int64_t cell, int64_t off) {
  if constexpr (J == 0) {
    G[0][0] = ldw<W>(P + t * cell + off);
  } else {
    constexpr int H = 1 << (J - 1);
    constexpr int64_t s7 = pow7c(J - 1);
    Vw<W> p1[H][H], p2[H][H], u2[H][H], u3[H][H], q[H][H];
    tree_post<J - 1, W>(p1, P, t + 0 * s7, cell, off);
    tree_post<J - 1, W>(p2, P, t + 1 * s7, cell, off);
#pragma unroll
    for (int u = 0; u < H; ++u)
#pragma unroll
      for (int v = 0; v < H; ++v) G[u][v] = vadd(p1[u][v], p2[u][v]);  // C11 = P1 + P2
    tree_post<J - 1, W>(q, P, t + 5 * s7, cell, off);  // P6
#pragma unroll
    for (int u = 0; u < H; ++u)
#pragma unroll
      for (int v = 0; v < H; ++v) u2[u][v] = vadd(p1[u][v], q[u][v]);  // U2 = P1 + P6
    tree_post<J - 1, W>(q, P, t + 6 * s7, cell, off);  // P7
#pragma unroll
    for (int u = 0; u < H; ++u)
#pragma unroll
      for (int v = 0; v < H; ++v) u3[u][v] = vadd(u2[u][v], q[u][v]);  // U3 = U2 + P7
    tree_post<J - 1, W>(q, P, t + 4 * s7, cell, off);  // P5
#pragma unroll
    for (int u = 0; u < H; ++u)
#pragma unroll
      for (int v = 0; v < H; ++v) {
        u2[u][v] = vadd(u2[u][v], q[u][v]);            // U4 = U2 + P5
        G[u + H][v + H] = vadd(u3[u][v], q[u][v]);     // C22 = U3 + P5
      }
    tree_post<J - 1, W>(q, P, t + 2 * s7, cell, off);  // P3
#pragma unroll
    for (int u = 0; u < H; ++u)
#pragma unroll
      for (int v = 0; v < H; ++v) G[u][v + H] = vadd(u2[u][v], q[u][v]);  // C12 = U4 + P3
    tree_post<J - 1, W>(q, P, t + 3 * s7, cell, off);  // P4
#pragma unroll
    for (int u = 0; u < H; ++u)
#pragma unroll
      for (int v = 0; v < H; ++v) G[u + H][v] = vsub(u3[u][v], q[u][v]);  // C21 = U3 - P4
  }
}

// Every product below the root is a dense block, so a grouped launch never
// writes a clipped product: the root's post-additions, when C is clipped,
// stay with the single-level kernel.  (Masked stores here made the compiler
// hoist all 7^L loads: 256 registers and spills for L = 3.)
template <int L, int W>
__global__ void __launch_bounds__(kAddThreads)
tree_postadd_kernel(const TreeNode* __restrict__ nodes, int nnodes) {
  const TreeNode nd = nodes[find_node(nodes, nnodes, blockIdx.x)];
  const int cw = nd.bc / W;
  const int64_t g = (int64_t)(blockIdx.x - nd.block_begin) * kAddThreads + threadIdx.x;
  if (g >= (int64_t)nd.br * cw) return;
  const int r = (int)(g / cw);
  const int c = (int)(g - (int64_t)r * cw) * W;
  Vw<W> G[1 << L][1 << L];
  tree_post<L, W>(G, nd.src, 0, (int64_t)nd.br * nd.bc, (int64_t)r * nd.bc + c);
  float* out = nd.dst[0];
#pragma unroll
  for (int u = 0; u < (1 << L); ++u)
#pragma unroll
    for (int v = 0; v < (1 << L); ++v)
      stw<W>(out + ((int64_t)u * nd.br + r) * nd.ld + (int64_t)v * nd.bc + c, G[u][v]);
}

template <int L, int W, bool CLIP>
static void launch_tree_kind(int kind, dim3 grid, dim3 block, hipStream_t stream, const TreeNode* d,
                             int n) {
  if (kind == 0) hipLaunchKernelGGL((tree_preadd_kernel<0, L, W, CLIP>), grid, block, 0, stream, d, n);
  else if (kind == 1) hipLaunchKernelGGL((tree_preadd_kernel<1, L, W, CLIP>), grid, block, 0, stream, d, n);
  else hipLaunchKernelGGL((tree_postadd_kernel<L, W>), grid, block, 0, stream, d, n);
}

void launch_tree_add(int kind, int levels, int width, bool clip, const TreeNode* d_nodes, int nnodes,
                     int total_blocks, hipStream_t stream) {
  if (nnodes <= 0 || total_blocks <= 0) return;
  if (kind < 0 || kind > 2 || (kind == 2 && clip)) throw Error(kInvalidValue, "bad multi-level addition launch");
  dim3 grid(total_blocks), block(kAddThreads);
  const int key = levels * 10 + width;
  switch (key) {
    case 24:
      clip ? launch_tree_kind<2, 4, true>(kind, grid, block, stream, d_nodes, nnodes)
           : launch_tree_kind<2, 4, false>(kind, grid, block, stream, d_nodes, nnodes);
      break;
    case 21:
      clip ? launch_tree_kind<2, 1, true>(kind, grid, block, stream, d_nodes, nnodes)
           : launch_tree_kind<2, 1, false>(kind, grid, block, stream, d_nodes, nnodes);
      break;
    case 31:
      clip ? launch_tree_kind<3, 1, true>(kind, grid, block, stream, d_nodes, nnodes)
           : launch_tree_kind<3, 1, false>(kind, grid, block, stream, d_nodes, nnodes);
      break;
    default: throw Error(kInvalidValue, "bad multi-level addition launch");
  }
  FASTMM_HIP(hipGetLastError());
}

void launch_preadd(int side, const PreAddNode* d_nodes, int nnodes, int total_blocks, bool vec,
                   hipStream_t stream) {
  if (nnodes <= 0 || total_blocks <= 0) return;
  dim3 grid(total_blocks), block(kAddThreads);
  if (side == 0) {
    if (vec) hipLaunchKernelGGL((preadd_kernel<0, true>), grid, block, 0, stream, d_nodes, nnodes);
    else hipLaunchKernelGGL((preadd_kernel<0, false>), grid, block, 0, stream, d_nodes, nnodes);
  } else {
    if (vec) hipLaunchKernelGGL((preadd_kernel<1, true>), grid, block, 0, stream, d_nodes, nnodes);
    else hipLaunchKernelGGL((preadd_kernel<1, false>), grid, block, 0, stream, d_nodes, nnodes);
  }
  FASTMM_HIP(hipGetLastError());
}

template <int QUAD>
static void launch_post_q(const PostAddNode* d, int n, int blocks, bool vec, hipStream_t s) {
  dim3 grid(blocks), block(kAddThreads);
  if (vec) hipLaunchKernelGGL((postadd_kernel<true, QUAD>), grid, block, 0, s, d, n);
  else hipLaunchKernelGGL((postadd_kernel<false, QUAD>), grid, block, 0, s, d, n);
}

void launch_postadd(const PostAddNode* d_nodes, int nnodes, int total_blocks, bool vec,
                    hipStream_t stream, int quad) {
  if (nnodes <= 0 || total_blocks <= 0) return;
  switch (quad) {
    case -1: launch_post_q<-1>(d_nodes, nnodes, total_blocks, vec, stream); break;
    case 0: launch_post_q<0>(d_nodes, nnodes, total_blocks, vec, stream); break;
    case 1: launch_post_q<1>(d_nodes, nnodes, total_blocks, vec, stream); break;
    case 2: launch_post_q<2>(d_nodes, nnodes, total_blocks, vec, stream); break;
    case 3: launch_post_q<3>(d_nodes, nnodes, total_blocks, vec, stream); break;
    default: throw Error(kInvalidValue, "bad quadrant");
  }
  FASTMM_HIP(hipGetLastError());
}

}  // namespace fastmm
