// The paper's classic recursion (Table 1), kept as a comparator for the
// Winograd path: C = A B by eight sub-products per level,
//   C0 = A0 B0, C1 = A0 B1, C2 = A2 B0, C3 = A2 B1,
//   C0 += A1 B2, C1 += A1 B3, C2 += A3 B2, C3 += A3 B3,
// over the quadrant split of equation (1) (quadrant 0 ceil x ceil), with the
// same stop rule as the Winograd path.  Unrolled, depth d is a product of
// 2^d x 2^d result blocks, each the sum over 2^d reduction chunks taken in
// Table 1's order (chunk 0 overwrites, later chunks accumulate).  Here every
// chunk index is one grouped launch of the MFMA leaf kernel over all result
// blocks (the first with C = A B, the rest with C += A B), so a depth-d
// product costs 2^d launches.  It performs all 2MNK flops: the comparison
// with the Winograd path isolates what the seven-product recursion saves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "engine.h"

namespace fastmm {
namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Span {
  int64_t off, len;
};

// 2^levels consecutive spans of [0, n), halving with the larger part first
// (split_half: ceil(n/2), rounded up to a multiple of 4 from 64 on).
void split_spans(int64_t off, int64_t n, int levels, std::vector<Span>& out) {
  if (levels == 0) {
    out.push_back({off, n});
    return;
  }
  const int64_t h = split_half(n);
  split_spans(off, h, levels - 1, out);
  split_spans(off + h, n - h, levels - 1, out);
}

void rmul_impl(Library& L, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
               const float* B, int64_t ldb, float* C, int64_t ldc, int depth, int64_t leaf,
               int tile) {
  validate_gemm_args(M, N, K, A, lda, B, ldb, C, ldc, depth);
  if (depth < 0) throw Error(kInvalidValue, "depth must be >= 0 for the classic recursion");
  if (tile < 0 || tile >= kNumTiles) throw Error(kInvalidValue, "unknown tile id");
  if (tile == kTileFp16x3)
    throw Error(kNotSupported, "the scaled FP16 leaf is not available in the classic recursion");
  ensure_init(L);
  fastmm_stats_t st{};
  st.h2d_ms = st.preadd_ms = st.leaf_ms = st.postadd_ms = st.d2h_ms = st.total_ms = -1.0;
  if (M == 0 || N == 0) {
    L.stats = st;
    return;
  }
  const bool on_dev = operands_on_device(M, N, K, A, B, C);
  const int d = K == 0 ? 0 : effective_depth(M, N, K, depth, leaf);
  // Staging as in the Winograd path (plan_staging).  The spans follow M, K
  // and N; the last span of K (of N) also reads the staged zero padding up
  // to K4 (N4), so that its extent stays a multiple of 4.
  const Staging sg = plan_staging(M, N, K, A, lda, B, ldb, on_dev);
  std::vector<Span> rs, ks, cs;
  split_spans(0, M, d, rs);
  split_spans(0, K, d, ks);
  split_spans(0, N, d, cs);
  auto padded = [](const Span& sp, int64_t n, int64_t n4) {
    return sp.off + sp.len == n ? sp.len + (n4 - n) : sp.len;
  };
  const int nb = 1 << d;
  // Split-BF16 leaves run here on the register-split kernel (128x128 tiles,
  // no packed operands).
  const TileShape ts = tile == kTileBf16x3 ? TileShape{128, 128} : tile_shape(tile);

  const size_t a_bytes = sg.a_bytes;
  const size_t b_bytes = sg.b_bytes;
  const size_t c_bytes = on_dev ? 0 : align_up((size_t)M * N * 4, 256);
  const size_t phase_desc = align_up((size_t)nb * nb * sizeof(GemmDesc), 256);
  const size_t d_bytes = phase_desc * nb;
  char* ws = ensure_arena(L, a_bytes + b_bytes + c_bytes + d_bytes);
  char* host = ensure_pinned(L, d_bytes);
  float* dA = sg.a ? reinterpret_cast<float*>(ws) : const_cast<float*>(A);
  float* dB = sg.b ? reinterpret_cast<float*>(ws + a_bytes) : const_cast<float*>(B);
  float* dC = on_dev ? C : reinterpret_cast<float*>(ws + a_bytes + b_bytes);
  const int64_t la = sg.a ? std::max<int64_t>(sg.K4, 1) : lda, lb = sg.b ? sg.N4 : ldb,
                lc = on_dev ? ldc : N;
  char* ddesc = ws + a_bytes + b_bytes + c_bytes;
  hipStream_t sm = L.stream;
  stage_operands(sg, M, N, K, A, lda, B, ldb, dA, dB, sm);
  // One descriptor array per reduction chunk p: every non-empty result block
  // (i, j) with A block (i, p), B block (p, j); chunk 0 overwrites.
  std::vector<int> totals(nb, 0), counts(nb, 0);
  std::vector<char> vecs(nb, 1);
  for (int p = 0; p < nb; ++p) {
    std::vector<GemmDesc> v;
    int64_t total = 0;
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j) {
        if (rs[i].len == 0 || cs[j].len == 0) continue;
        GemmDesc g{};
        g.A = dA + rs[i].off * la + ks[p].off;
        g.lda = la;
        g.B = dB + ks[p].off * lb + cs[j].off;
        g.ldb = lb;
        g.C = dC + rs[i].off * lc + cs[j].off;
        g.ldc = lc;
        g.a_rows = (int32_t)rs[i].len;
        g.b_cols = (int32_t)padded(cs[j], N, sg.N4);
        g.kmax = (int32_t)padded(ks[p], K, sg.K4);
        g.c_rows = (int32_t)rs[i].len;
        g.c_cols = (int32_t)cs[j].len;
        g.tiles_n = (g.c_cols + ts.bn - 1) / ts.bn;
        g.tile_begin = (int32_t)total;
        g.beta = p > 0 ? 1 : 0;
        total += (int64_t)((g.c_rows + ts.bm - 1) / ts.bm) * g.tiles_n;
        if (!(aligned16(g.A) && aligned16(g.B) && g.lda % 4 == 0 && g.ldb % 4 == 0 &&
              g.kmax % 4 == 0 && g.b_cols % 4 == 0))
          vecs[p] = 0;
        st.leaf_flops += 2.0 * g.c_rows * g.c_cols * ks[p].len;
        v.push_back(g);
      }
    if (total > INT32_MAX) throw Error(kNotSupported, "leaf launch too large");
    totals[p] = (int)total;
    counts[p] = (int)v.size();
    st.leaves += (int64_t)v.size();
    if (!v.empty()) std::memcpy(host + p * phase_desc, v.data(), v.size() * sizeof(GemmDesc));
  }
  st.leaf_m = rs[0].len;
  st.leaf_k = ks[0].len;
  st.leaf_n = cs[0].len;
  FASTMM_HIP(hipMemcpyAsync(ddesc, host, d_bytes, hipMemcpyHostToDevice, sm));
  if (K == 0) {
    FASTMM_HIP(hipMemset2DAsync(dC, lc * 4, 0, N * 4, M, sm));
  } else {
    for (int p = 0; p < nb; ++p)
      if (totals[p] > 0) {
        launch_leaf_gemm(tile, reinterpret_cast<const GemmDesc*>(ddesc + p * phase_desc),
                         counts[p], totals[p], vecs[p], sm);
        ++st.launches;
      }
  }
  if (!on_dev)
    FASTMM_HIP(hipMemcpy2DAsync(C, ldc * 4, dC, N * 4, N * 4, M, hipMemcpyDeviceToHost, sm));
  FASTMM_HIP(hipStreamSynchronize(sm));
  st.depth = d;
  st.tile = tile;
  st.leaf_launches = st.launches;
  st.transfer_bytes = on_dev ? 0.0 : 4.0 * ((double)M * K + (double)K * N + (double)M * N);
  st.workspace_bytes = L.arena_bytes;
  L.stats = st;
}

}  // namespace
}  // namespace fastmm

using namespace fastmm;

extern "C" int fastmm_rmul(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                           const float* B, int64_t ldb, float* C, int64_t ldc, int depth,
                           int64_t leaf, int tile) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return run_guarded([&] { rmul_impl(L, M, N, K, A, lda, B, ldb, C, ldc, depth, leaf, tile); });
}
