// Host-resident operands: overlap the PCIe transfers with the recursion.
//
// The paper's leaf call moves the operands to the device, computes and moves
// the result back, one step after the other (Section 3.3), and it observes
// that transfers, not kernels, cap its throughput on large problems
// (Section 4.2).  On MI355X the same holds in proportion: at n = 19456 the
// copies of A, B and C take about as long as the whole Winograd product.
//
// Here the top level of the recursion runs as a sequence of pieces,
// alternating between two compute streams, while one copy stream brings
// operand blocks in and a second copy stream sends result blocks back as
// soon as they are final.  The top quadrants are cut into row bands (A
// side; four where the rows hold at least two leaf-tile units per band,
// else two) and, where B's quadrants are at least 4096 wide, two column
// bands (B side): piece (i, r, c) of top-level product i,
// P_i[r, c] = L_i[r] R_i[:, c], needs only row band r of its left operand
// and column band c of its right operand, and is itself a Winograd product
// of depth d - 1.  The pieces of one product and row band (column band)
// share the inner recursion's A-side (B-side) temporaries, computed by the
// first of them.
//
// Input order.  Every product needs a different subset of the eight
// quadrants (P1: A11 B11; P7: A11 A21 B12 B22; P5: A21 A22 B11 B12; P6: A11
// A21 A22 B11 B12 B22; P2: A12 B21; P4: A22 and all of B; P3: all of A and
// B22).  Each band layout has a fixed order of its band blocks (found by
// simulating the copies and the pieces at n = 19456, searching over orders,
// and measuring): it starts with bands of B11 and A11 and leaves A12 and
// B21 for the end, so that the first piece waits for a small part of the
// data and only P2 and P3 wait for the end of the transfer.  Pieces run
// greedily in order of estimated readiness.  Pre-additions compute only the
// S / T outputs of a band whose inputs have arrived (a later pass adds the
// rest), and each result block C_q[r, c] is formed and sent out as soon as
// its four products (C11: P1 P2; C12: P1 P6 P5 P3; C21: P1 P6 P7 P4; C22: P1
// P6 P7 P5) are done, so one block of one quadrant (under 1 ms of copy at
// n = 19456) remains after the last piece.
//
// A plain product (depth 0) streams A's rows and B's columns in two to five
// bands by size, alternately, and computes each block C[r, c] as a piece
// once its two bands are in.
//
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "engine.h"

namespace fastmm {
namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Copy rows [r0, r0 + rows) x cols [c0, c0 + cols) of a host matrix into the
// same block of a dense device matrix (or back).
void h2d_block(float* dev, int64_t ld_dev, const float* host, int64_t ld_host, int64_t r0,
               int64_t c0, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  FASTMM_HIP(hipMemcpy2DAsync(dev + r0 * ld_dev + c0, ld_dev * 4, host + r0 * ld_host + c0,
                              ld_host * 4, cols * 4, rows, hipMemcpyHostToDevice, s));
}

void d2h_block(float* host, int64_t ld_host, const float* dev, int64_t ld_dev, int64_t r0,
               int64_t c0, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  FASTMM_HIP(hipMemcpy2DAsync(host + r0 * ld_host + c0, ld_host * 4, dev + r0 * ld_dev + c0,
                              ld_dev * 4, cols * 4, rows, hipMemcpyDeviceToHost, s));
}

double ev_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return -1.0;
  }
  return ms;
}

// A group of sub-products launched as one level-wise schedule.
struct Group {
  std::vector<Problem> probs;
  Schedule s;
  size_t desc_off = 0, desc_bytes = 0;
  int x = 0;  // compute stream (index)
};

// Row bands [r0, r0 + rows) of the top quadrants (rows of the bottom
// quadrants in the band: bot).
struct Band {
  int64_t r0, rows, bot;
};

// Also column bands of the left quadrants' n2 columns (r0, rows: first
// column and width; bot: valid columns of the right quadrants' band).  Two
// bands split at a multiple of `align` near the middle, else of 4 (16-byte
// aligned band starts), else the middle.  More bands (where m2 holds at
// least one unit of `align` per band): whole units each, the first bands
// one unit longer where the units do not divide evenly, the last band also
// taking the rows beyond the last whole unit.
std::vector<Band> make_bands(int64_t m2, int64_t mb, int nb, int64_t align) {
  std::vector<int64_t> starts{0};
  if (nb >= 3 && align > 0 && m2 / align >= nb) {
    const int64_t units = m2 / align, base = units / nb, rem = units % nb;
    int64_t r = 0;
    for (int i = 0; i + 1 < nb; ++i) {
      r += (base + (i < rem ? 1 : 0)) * align;
      starts.push_back(r);
    }
  } else if (nb >= 2 && m2 >= 2) {
    int64_t split = (m2 / 2 + align / 2) / align * align;
    if (split <= 0 || split >= m2) split = (m2 / 2 + 3) / 4 * 4;
    if (split <= 0 || split >= m2) split = (m2 + 1) / 2;
    starts.push_back(split);
  }
  std::vector<Band> v;
  for (size_t i = 0; i < starts.size(); ++i) {
    const int64_t r0 = starts[i], r1 = i + 1 < starts.size() ? starts[i + 1] : m2;
    v.push_back({r0, r1 - r0, std::max<int64_t>(0, std::min(r1 - r0, mb - r0))});
  }
  return v;
}

// Input orders of the Winograd pipeline per band layout (row bands x column
// bands), each block as {matrix (0: A, 1: B), quadrant (0: X11, 1: X12, 2:
// X21, 3: X22), band}.  Found by simulating the copies (at the PCIe rate)
// and the pieces (at the leaf rate) for n = 19456 and searching over orders.
struct Recipe {
  int nr, nc;
  std::vector<std::array<int, 3>> items;
};

const std::vector<Recipe>& recipes() {
  static const std::vector<Recipe> r = {
      // Two row and two column bands: B quadrants before A ones within a
      // pair, the first row and column bands of the X11 quadrants first, A12
      // last.
      {2, 2, {{1, 0, 0}, {0, 0, 0}, {1, 0, 1}, {0, 0, 1}, {1, 1, 1}, {0, 2, 1}, {1, 3, 1}, {0, 3, 1},
              {1, 1, 0}, {1, 3, 0}, {1, 2, 0}, {0, 3, 0}, {0, 1, 0}, {0, 2, 0}, {1, 2, 1}, {0, 1, 1}}},
      // Whole B quadrants (one column band): A11[r0] B11 A22[r0] A11[r1]
      // A21[r0] B12 B22 B21 A22[r1] A21[r1] A12[r0] A12[r1].
      {2, 1, {{0, 0, 0}, {1, 0, 0}, {0, 3, 0}, {0, 0, 1}, {0, 2, 0}, {1, 1, 0}, {1, 3, 0}, {1, 2, 0},
              {0, 3, 1}, {0, 2, 1}, {0, 1, 0}, {0, 1, 1}}},
      // Finer layouts (the same search, pieces priced at the two-stream rate).
      {4, 2, {{1, 0, 0}, {0, 0, 1}, {1, 0, 1}, {0, 2, 3}, {0, 0, 3}, {0, 0, 2}, {1, 3, 1}, {0, 0, 0},
              {1, 1, 1}, {0, 3, 3}, {0, 2, 1}, {0, 3, 1}, {0, 2, 0}, {0, 1, 3}, {0, 1, 1}, {0, 3, 0},
              {1, 1, 0}, {1, 3, 0}, {1, 2, 0}, {0, 2, 2}, {0, 3, 2}, {0, 1, 0}, {0, 1, 2}, {1, 2, 1}}},
      {6, 2, {{0, 2, 3}, {1, 0, 1}, {0, 0, 3}, {0, 0, 1}, {0, 0, 0}, {1, 0, 0}, {0, 0, 2}, {0, 0, 5},
              {0, 0, 4}, {1, 1, 1}, {0, 3, 3}, {1, 3, 1}, {0, 2, 4}, {0, 3, 4}, {0, 2, 5}, {0, 2, 0},
              {0, 3, 0}, {0, 3, 5}, {0, 1, 4}, {0, 1, 0}, {1, 1, 0}, {0, 1, 2}, {1, 2, 0}, {0, 1, 1},
              {1, 3, 0}, {0, 3, 1}, {0, 3, 2}, {1, 2, 1}, {0, 2, 2}, {0, 2, 1}, {0, 1, 3}, {0, 1, 5}}},
      {8, 2, {{0, 0, 6}, {1, 0, 1}, {0, 0, 3}, {0, 3, 5}, {0, 0, 7}, {1, 0, 0}, {0, 0, 4}, {0, 0, 1},
              {0, 0, 5}, {0, 0, 0}, {1, 1, 1}, {0, 2, 5}, {0, 0, 2}, {1, 3, 1}, {0, 2, 2}, {0, 3, 2},
              {0, 2, 3}, {0, 1, 4}, {0, 2, 7}, {0, 3, 7}, {0, 2, 6}, {0, 3, 4}, {0, 3, 3}, {0, 2, 4},
              {0, 2, 0}, {0, 3, 0}, {0, 1, 0}, {0, 1, 2}, {1, 2, 1}, {0, 1, 1}, {0, 2, 1}, {1, 2, 0},
              {0, 3, 6}, {1, 3, 0}, {1, 1, 0}, {0, 1, 7}, {0, 1, 3}, {0, 1, 6}, {0, 3, 1}, {0, 1, 5}}},
      {3, 2, {{0, 0, 2}, {1, 0, 1}, {1, 0, 0}, {0, 0, 1}, {0, 2, 1}, {0, 3, 1}, {0, 0, 0}, {1, 1, 1},
              {1, 3, 1}, {0, 2, 2}, {0, 2, 0}, {0, 3, 0}, {0, 1, 2}, {0, 3, 2}, {1, 3, 0}, {0, 1, 0},
              {1, 2, 1}, {1, 1, 0}, {1, 2, 0}, {0, 1, 1}}},
      {5, 2, {{0, 2, 4}, {0, 0, 3}, {1, 0, 0}, {1, 0, 1}, {0, 0, 2}, {0, 0, 0}, {0, 0, 1}, {0, 3, 4},
              {1, 1, 1}, {0, 0, 4}, {1, 3, 1}, {0, 2, 1}, {0, 2, 2}, {0, 3, 2}, {0, 1, 2}, {0, 3, 1},
              {1, 2, 1}, {0, 3, 3}, {0, 1, 3}, {1, 1, 0}, {1, 3, 0}, {0, 1, 0}, {0, 2, 3}, {0, 1, 1},
              {0, 3, 0}, {1, 2, 0}, {0, 2, 0}, {0, 1, 4}}},
      {4, 3, {{1, 2, 1}, {0, 1, 3}, {1, 2, 2}, {0, 1, 2}, {0, 1, 0}, {0, 0, 2}, {1, 2, 0}, {0, 1, 1},
              {0, 0, 0}, {1, 0, 1}, {0, 0, 1}, {1, 0, 0}, {1, 1, 2}, {0, 0, 3}, {1, 0, 2}, {0, 2, 3},
              {1, 3, 2}, {0, 3, 3}, {0, 3, 1}, {0, 2, 1}, {0, 2, 0}, {0, 2, 2}, {1, 3, 0}, {0, 3, 0},
              {0, 3, 2}, {1, 3, 1}, {1, 1, 0}, {1, 1, 1}}},
      {4, 4, {{1, 2, 0}, {0, 1, 3}, {1, 2, 1}, {1, 2, 3}, {0, 1, 2}, {0, 1, 0}, {0, 1, 1}, {1, 2, 2},
              {0, 0, 1}, {1, 0, 3}, {0, 0, 2}, {1, 0, 2}, {0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 0, 3},
              {1, 0, 1}, {0, 2, 3}, {1, 3, 0}, {0, 3, 3}, {0, 3, 1}, {0, 2, 1}, {1, 1, 2}, {0, 2, 0},
              {0, 3, 0}, {0, 2, 2}, {1, 3, 1}, {0, 3, 2}, {1, 3, 2}, {1, 1, 1}, {1, 3, 3}, {1, 1, 3}}},
  };
  return r;
}

const Recipe* find_recipe(int nr, int nc) {
  for (const auto& r : recipes())
    if (r.nr == nr && r.nc == nc) return &r;
  return nullptr;
}

constexpr int kMaxBands = 8;

}  // namespace

namespace {
size_t g_dry_need = 0;
}

size_t pipelined_need(int64_t M, int64_t N, int64_t K, int depth, int tile) {
  // The need depends on the shape, the plan and the layout switches only:
  // kept per key, so that repeated calls skip the sizing pass.
  auto env = [](const char* n) {
    const char* e = std::getenv(n);
    return std::string(e ? e : "-");
  };
  const std::string key = std::to_string(M) + ',' + std::to_string(N) + ',' + std::to_string(K) + ',' +
                          std::to_string(depth) + ',' + std::to_string(tile) + ',' +
                          env("FASTMM_PIPE_ROWBANDS") + ',' + env("FASTMM_PIPE_COLBANDS") + ',' +
                          env("FASTMM_PIPE_STREAMS") + ',' + env("FASTMM_PIPE_PLAINBANDS");
  static std::map<std::string, size_t> cache;  // calls are serialised by the library lock
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  Library dummy;
  fastmm_stats_t st{};
  g_dry_need = 0;
  gemm_host_pipelined(dummy, M, N, K, nullptr, 0, nullptr, 0, nullptr, 0, depth, tile, st);
  if (cache.size() >= 64) cache.clear();
  cache.emplace(key, g_dry_need);
  return g_dry_need;
}

// With L.initialised false (pipelined_need), only sizes the workspace.
void gemm_host_pipelined(Library& L, int64_t M, int64_t N, int64_t K, const float* A,
                         int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc,
                         int depth, int tile, fastmm_stats_t& st) {
  // The device copies are padded as in plan_staging: A is M x K4 (ld K4),
  // B is K4 x N4 and C is M x N4, zero beyond K and N, so that every leaf
  // operand keeps 16-byte aligned rows.  The split and all device-side
  // extents use K4 and N4; the copies move the K and N valid columns.
  const int64_t K4 = (K + 3) / 4 * 4, N4 = (N + 3) / 4 * 4;
  // The top split: where the recursion continues below it, at the extent
  // that keeps every lower level exactly halved (split_at).
  const bool wino = depth >= 1;
  auto top = [&](int64_t x) { return wino ? split_at(x, depth) : split_half(x); };
  const int64_t m2 = top(M), k2 = top(K4), n2 = top(N4);
  const int64_t mb = M - m2, kb = K4 - k2, nb = N4 - n2;
  const int64_t kb_v = std::max<int64_t>(0, K - k2), nb_v = std::max<int64_t>(0, N - n2);
  const TileShape ts = tile_shape(tile);
  // Compute streams of the pieces: the caller's stream and the library's
  // second one, the pieces alternating between them (each stream with its
  // own temporaries), so that one piece's additions and leaf launch fill the
  // partial last round of workgroups of the previous piece's leaf launch
  // (FASTMM_PIPE_STREAMS=1: the caller's stream alone).
  int ncs = 2;
  if (const char* e = std::getenv("FASTMM_PIPE_STREAMS"))
    if (e[0] == '1') ncs = 1;

  // ---- workspace layout (byte offsets into the arena)
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes, 256);
    return o;
  };
  const size_t oA = take((size_t)M * K4 * 4), oB = take((size_t)K4 * N4 * 4),
               oC = take((size_t)M * N4 * 4);

  // ---- bands.  Winograd: row bands of the top quadrants' rows (m2) and
  // column bands of their columns (n2); a band of the bottom (right)
  // quadrants keeps only its valid rows (columns).  Plain product: A's rows
  // and B's columns in two to five bands by size.
  std::vector<Band> bands, cbands;
  if (wino) {
    // Column bands only where B's quadrants are wide: for narrow ones (one
    // GPU's column panel of a sharded product, 19456 x 19456 x 2432) they
    // bring no earlier start worth the smaller leaf launches (33.9 against
    // 38.4 ms for that panel, 25.1 against 28.9 ms for a 9728 x 19456 x
    // 4864 block).  With column bands, four row bands where the top rows
    // hold at least two leaf-tile units per band.  FASTMM_PIPE_ROWBANDS and
    // FASTMM_PIPE_COLBANDS choose another layout that has an input order of
    // its own (2 x 1, 2 x 2, 3 x 2, 4 x 2, 5 x 2, 6 x 2, 8 x 2, 4 x 3,
    // 4 x 4).
    const int64_t ra = (int64_t)ts.bm << (depth - 1), ca = (int64_t)ts.bn << (depth - 1);
    const bool colb = n2 >= 4096;
    int nrb = colb && m2 / ra >= 8 ? 4 : 2, ncb = colb ? 2 : 1;
    if (const char* e = std::getenv("FASTMM_PIPE_ROWBANDS")) nrb = std::atoi(e);
    if (const char* e = std::getenv("FASTMM_PIPE_COLBANDS")) ncb = std::atoi(e);
    if (!find_recipe(nrb, ncb) || (nrb > 2 && m2 / ra < nrb) || (ncb > 2 && n2 / ca < ncb) ||
        (ncb > 1 && !colb)) {
      nrb = 2;
      ncb = colb ? 2 : 1;
    }
    bands = make_bands(m2, mb, nrb, ra);
    cbands = make_bands(n2, nb, ncb, ca);
  } else {
    // A's rows and B's columns (the padded width N4) in np parts each, from
    // measurements of the plain product on this path (best of 5 interleaved
    // calls): halves where neither extent exceeds 4608 (3.6 against 4.7 ms
    // in quarters at n = 4096; 12.5 against 16.6 ms for 4096 x 4096 x
    // 16384), thirds up to 7168 (7.3 against 8.1 ms at n = 6144), fifths
    // where both hold at least 10240 (the first piece starts sooner: 123
    // against 129 ms at n = 19456, 71.7 against 73.4 ms at 19456 x 12288 x
    // 16384), else quarters (13.3 ms at n = 8192 against 14.8 in thirds and
    // 15.4 in fifths; 28.3 ms for 9728 x 4864 x 19456 against 29.5 and 31.1).
    // Few bands delay the first piece, many bands make pieces too small to
    // fill the device and copies of short rows slow.  FASTMM_PIPE_PLAINBANDS:
    // 1 to 8 parts instead.  Parts are rounded up to whole tiles where the
    // extent allows, so that there are at most np bands; column bands start
    // at multiples of 4, so that B's and C's rows in a band stay 16-byte
    // aligned.
    const int64_t lo_ext = std::min(M, N4), hi_ext = std::max(M, N4);
    int np = hi_ext <= 4608 ? 2 : hi_ext <= 7168 ? 3 : lo_ext >= 10240 ? 5 : 4;
    if (const char* e = std::getenv("FASTMM_PIPE_PLAINBANDS")) np = std::min(8, std::max(1, std::atoi(e)));
    auto parts = [np](int64_t x, int64_t t, int64_t a) {
      std::vector<Band> v;
      int64_t q = (x + np - 1) / np;
      if (q >= t) q = (q + t - 1) / t * t;
      q = (q + a - 1) / a * a;
      for (int64_t r0 = 0; r0 < x; r0 += q) v.push_back({r0, std::min(q, x - r0), 0});
      return v;
    };
    bands = parts(M, ts.bm, 1);
    cbands = parts(N4, ts.bn, 4);
  }
  const int nband = (int)bands.size(), ncband = (int)cbands.size();
  // Valid host columns of a column band of B (plain product) or of the right
  // quadrants (Winograd).
  auto plain_valid = [&](const Band& c) { return std::max<int64_t>(0, std::min(c.rows, N - c.r0)); };
  auto right_valid = [&](const Band& c) {
    return std::max<int64_t>(0, std::min(c.rows, nb_v - c.r0));
  };

  // Winograd temporaries: S (four m2 x k2 blocks; a row band is a row range
  // of each), T per column band (four dense k2 x cols blocks), and the seven
  // products of each (row band, column band) block, dense rows x cols each.
  size_t oS = 0, oT = 0, oP = 0;
  std::vector<size_t> t_off(ncband), p_off((size_t)nband * ncband);
  if (wino) {
    oS = take((size_t)4 * m2 * k2 * 4);
    size_t t = 0;
    for (int c = 0; c < ncband; ++c) {
      t_off[c] = t;
      t += (size_t)4 * k2 * cbands[c].rows;
    }
    oT = take(t * 4);
    size_t q = 0;
    for (int r = 0; r < nband; ++r)
      for (int c = 0; c < ncband; ++c) {
        p_off[(size_t)r * ncband + c] = q;
        q += (size_t)7 * bands[r].rows * cbands[c].rows;
      }
    oP = take(q * 4);
  }
  // A piece (i, r, c) -- top-level product i restricted to row band r and
  // column band c -- is a Winograd product of depth d - 1.  The pieces of one
  // product and row band share their left operand, those of one product and
  // column band their right operand, so the inner recursion's A-side (B-side)
  // temporaries are computed by the first such piece and reused by the
  // others: one region per (product, row band) and per (product, column
  // band), outside the temporaries the pieces take in turn.
  const bool trees = wino && depth >= 2;
  std::vector<size_t> at_off((size_t)7 * std::max(nband, 1)), bt_off((size_t)7 * std::max(ncband, 1));
  size_t oAT = 0, oBT = 0;
  if (trees) {
    size_t a = 0, b = 0;
    for (int i = 0; i < 7; ++i) {
      for (int r = 0; r < nband; ++r) {
        at_off[(size_t)i * nband + r] = a;
        a += align_up(a_tree_bytes(bands[r].rows, k2, 1, depth - 1), 256);
      }
      for (int c = 0; c < ncband; ++c) {
        bt_off[(size_t)i * ncband + c] = b;
        b += align_up(b_tree_bytes(1, k2, cbands[c].rows, depth - 1), 256);
      }
    }
    oAT = take(a);
    oBT = take(b);
  }
  char* tree_base = reinterpret_cast<char*>(256);  // placeholder until allocation

  // Placeholder device pointers for sizing (real ones set after allocation).
  char* ws = nullptr;
  float *dA = nullptr, *dB = nullptr, *dC = nullptr, *S = nullptr, *T = nullptr, *P = nullptr;
  const int64_t ma = m2 * k2;

  struct V {
    const float* p;
    int64_t ld, r, c;
  };
  // Left operand of top-level product i (0..6), row band b.
  auto left = [&](int i, const Band& b) -> V {
    switch (i) {
      case 0: return {dA + b.r0 * K4, K4, b.rows, k2};               // A11
      case 1: return {dA + b.r0 * K4 + k2, K4, b.rows, kb};          // A12
      case 2: return {S + 3 * ma + b.r0 * k2, k2, b.rows, k2};       // S4
      case 3: return {dA + (m2 + b.r0) * K4 + k2, K4, b.bot, kb};    // A22
      case 4: return {S + 0 * ma + b.r0 * k2, k2, b.rows, k2};       // S1
      case 5: return {S + 1 * ma + b.r0 * k2, k2, b.rows, k2};       // S2
      default: return {S + 2 * ma + b.r0 * k2, k2, b.rows, k2};      // S3
    }
  };
  // Right operand of product i, column band c.
  auto right = [&](int i, int ci) -> V {
    const Band& c = cbands[ci];
    float* Tc = T + t_off[ci];
    const int64_t tb = k2 * c.rows;
    switch (i) {
      case 0: return {dB + c.r0, N4, k2, c.rows};                    // B11
      case 1: return {dB + k2 * N4 + c.r0, N4, kb, c.rows};          // B21
      case 2: return {dB + k2 * N4 + n2 + c.r0, N4, kb, c.bot};      // B22
      case 3: return {Tc + 3 * tb, c.rows, k2, c.rows};              // T4
      case 4: return {Tc + 0 * tb, c.rows, k2, c.rows};              // T1
      case 5: return {Tc + 1 * tb, c.rows, k2, c.rows};              // T2
      default: return {Tc + 2 * tb, c.rows, k2, c.rows};             // T3
    }
  };
  auto wino_piece = [&](int i, int ri, int ci) {
    const Band& b = bands[ri];
    const Band& c = cbands[ci];
    Problem p;
    const V l = left(i, b), r = right(i, ci);
    p.M = b.rows;
    p.K = k2;
    p.N = c.rows;
    p.A = l.p;
    p.lda = l.ld;
    p.a_rows = l.r;
    p.a_cols = l.c;
    p.B = r.p;
    p.ldb = r.ld;
    p.b_rows = r.r;
    p.b_cols = r.c;
    p.C = P + p_off[(size_t)ri * ncband + ci] + (int64_t)i * b.rows * c.rows;
    p.ldc = c.rows;
    p.depth = depth - 1;
    p.tile = tile;
    if (trees) {
      // tree_base is the arena at oAT; the B-side regions follow at oBT.
      p.a_tree = reinterpret_cast<float*>(tree_base + at_off[(size_t)i * nband + ri]);
      p.b_tree = reinterpret_cast<float*>(tree_base + (oBT - oAT) + bt_off[(size_t)i * ncband + ci]);
    }
    return p;
  };
  auto plain_problem = [&](const Band& b, const Band& c) {
    Problem p;
    p.M = b.rows;
    p.K = K4;
    p.N = c.rows;
    p.A = dA + b.r0 * K4;
    p.lda = K4;
    p.B = dB + c.r0;
    p.ldb = N4;
    p.C = dC + b.r0 * N4 + c.r0;
    p.ldc = N4;
    p.depth = 0;
    p.tile = tile;
    return p;
  };

  // The step list is built twice: once with placeholder pointers (sizes),
  // once with the real ones.  Each group's temporaries share one region.
  std::vector<Group> groups;
  // Input blocks: A quadrant q of row band b (mat 0), B quadrant q of column
  // band b (mat 1).
  struct Item {
    int mat, q, band;
  };
  std::vector<Item> items;
  struct Piece {
    int i, r, c;
  };
  std::vector<Piece> order;  // pieces in compute order
  std::vector<int> plain_ready;  // plain product: last input item each piece needs
  int a_item[4][kMaxBands], b_item[4][kMaxBands];  // input item of quadrant q, band
  for (int q = 0; q < 4; ++q)
    for (int b = 0; b < kMaxBands; ++b) a_item[q][b] = b_item[q][b] = -1;
  // Quadrants each product reads (bit 0 = X11, 1 = X12, 2 = X21, 3 = X22).
  static const unsigned kNeedA[7] = {0x1, 0x2, 0xF, 0x8, 0xC, 0xD, 0x5};
  static const unsigned kNeedB[7] = {0x1, 0x4, 0x8, 0xF, 0x3, 0xB, 0xA};
  if (wino) {
    // Input order: the layout's own (recipes()).
    // (A layout with a single row band takes the two-band order, its
    // missing band's blocks skipped.)
    const Recipe* rc = find_recipe(nband, ncband);
    if (!rc) rc = find_recipe(2, ncband > 1 ? 2 : 1);
    if (!rc || nband > kMaxBands || ncband > kMaxBands)
      throw Error(kDeviceError, "no input order for this band layout");
    const auto& recipe = rc->items;
    for (const auto& x : recipe) {
      const int mat = x[0], q = x[1], band = x[2];
      if (band >= (mat == 0 ? nband : ncband)) continue;
      items.push_back({mat, q, band});
      (mat == 0 ? a_item : b_item)[q][band] = (int)items.size() - 1;
    }
    // Estimated arrival times (bytes at the PCIe rate) and piece costs
    // (flops at the leaf rate); only the order matters.
    std::vector<double> t_arrive(items.size());
    double t = 0.0;
    for (size_t k = 0; k < items.size(); ++k) {
      const Item& it = items[k];
      const Band& b = it.mat == 0 ? bands[it.band] : cbands[it.band];
      double rows, cols;
      if (it.mat == 0) {
        rows = (double)(it.q / 2 ? b.bot : b.rows);
        cols = (double)(it.q % 2 ? kb : k2);
      } else {
        rows = (double)(it.q / 2 ? kb : k2);
        cols = (double)(it.q % 2 ? b.bot : b.rows);
      }
      t += rows * cols * 4.0 / 56e9;
      t_arrive[k] = t;
    }
    auto ready_item = [&](const Piece& pc) {
      int last = -1;
      for (int q = 0; q < 4; ++q) {
        if (kNeedA[pc.i] & (1u << q)) last = std::max(last, a_item[q][pc.r]);
        if (kNeedB[pc.i] & (1u << q)) last = std::max(last, b_item[q][pc.c]);
      }
      return last;
    };
    std::vector<Piece> pending;
    for (int r = 0; r < nband; ++r)
      for (int c = 0; c < ncband; ++c)
        for (int i = 0; i < 7; ++i) pending.push_back({i, r, c});
    double tc = 0.0;
    while (!pending.empty()) {
      size_t best = 0;
      double best_start = 1e300, best_ready = 1e300;
      for (size_t k = 0; k < pending.size(); ++k) {
        const double r = t_arrive[ready_item(pending[k])];
        const double st = std::max(r, tc);
        if (st < best_start - 1e-12 || (std::abs(st - best_start) <= 1e-12 && r < best_ready)) {
          best = k;
          best_start = st;
          best_ready = r;
        }
      }
      const Piece pc = pending[best];
      pending.erase(pending.begin() + best);
      tc = best_start + 2.0 * bands[pc.r].rows * k2 * cbands[pc.c].rows / 120e12;
      order.push_back(pc);
    }
  } else {
    // Plain product: B's first column band and A's first row band, then A's
    // and B's further bands in turn, so that every band that arrives
    // completes a row or column of pieces; pieces in order of the later of
    // their two bands.
    const int nmax = std::max(nband, ncband);
    for (int i = 0; i < nmax; ++i) {
      if (i == 0) {
        items.push_back({1, 0, 0});
        items.push_back({0, 0, 0});
        continue;
      }
      if (i < nband) items.push_back({0, 0, i});
      if (i < ncband) items.push_back({1, 0, i});
    }
    std::vector<int> ia(nband), ib(ncband);
    for (size_t k = 0; k < items.size(); ++k) (items[k].mat == 0 ? ia : ib)[items[k].band] = (int)k;
    for (int r = 0; r < nband; ++r)
      for (int c = 0; c < ncband; ++c) order.push_back({0, r, c});
    std::stable_sort(order.begin(), order.end(), [&](const Piece& x, const Piece& y) {
      return std::max(ia[x.r], ib[x.c]) < std::max(ia[y.r], ib[y.c]);
    });
    plain_ready.resize(order.size());
    for (size_t g = 0; g < order.size(); ++g) plain_ready[g] = std::max(ia[order[g].r], ib[order[g].c]);
  }
  auto build_groups = [&]() {
    groups.clear();
    if (wino) {
      std::vector<char> a_seen((size_t)7 * nband, 0), b_seen((size_t)7 * ncband, 0);
      for (const Piece& pc : order) {
        Problem p = wino_piece(pc.i, pc.r, pc.c);
        char& as = a_seen[(size_t)pc.i * nband + pc.r];
        char& bs = b_seen[(size_t)pc.i * ncband + pc.c];
        p.a_tree_ready = trees && as;
        p.b_tree_ready = trees && bs;
        as = bs = 1;
        groups.push_back({{p}});
      }
    } else {
      for (const Piece& pc : order) groups.push_back({{plain_problem(bands[pc.r], cbands[pc.c])}});
    }
    // Pieces alternate between the compute streams.  The last piece follows
    // the one before it on the same stream: the result blocks that one
    // completes are then formed and on their way out while the last piece
    // runs, instead of waiting for workgroup slots behind its leaf launch.
    for (size_t g = 0; g < groups.size(); ++g)
      groups[g].x = (int)(std::min(g, groups.size() >= 2 ? groups.size() - 2 : 0) % ncs);
  };
  build_groups();
  // Descriptor slots: pre-addition passes (at most 4 per row band for S and
  // 4 per column band for T), one post-addition node per block; then the
  // product schedules.
  const size_t nslots = (size_t)4 * nband + 4 * std::max(ncband, 1) + (size_t)nband * std::max(ncband, 1) + 8;
  size_t temp_max = 0, desc_total = 256 * nslots;
  for (auto& g : groups) {
    size_t t = 0;
    for (auto& p : g.probs) t += align_up(problem_temp_bytes(p), 256);
    temp_max = std::max(temp_max, t);
    std::vector<Problem> q = g.probs;
    for (auto& x : q) {  // any non-null placeholder: only counts matter here
      x.A = x.B = reinterpret_cast<const float*>(256);
      x.C = const_cast<float*>(x.A);
    }
    Schedule tmp;
    build_schedule(q, reinterpret_cast<char*>(256), tmp);
    g.desc_bytes = align_up(schedule_desc_bytes(tmp), 256) + 256;
    g.desc_off = desc_total;
    desc_total += g.desc_bytes;
  }
  const size_t temp_stride = align_up(temp_max, 256);
  const size_t oTemp = take(temp_stride * ncs);
  const size_t oDesc = take(desc_total);
  if (!L.initialised) {  // sizing only
    g_dry_need = off;
    return;
  }

  ws = ensure_arena(L, off);
  char* host = ensure_pinned(L, desc_total);
  dA = reinterpret_cast<float*>(ws + oA);
  dB = reinterpret_cast<float*>(ws + oB);
  dC = reinterpret_cast<float*>(ws + oC);
  S = reinterpret_cast<float*>(ws + oS);
  T = reinterpret_cast<float*>(ws + oT);
  P = reinterpret_cast<float*>(ws + oP);
  tree_base = ws + oAT;
  char* temps = ws + oTemp;
  char* ddesc = ws + oDesc;
  hipStream_t cs = L.stream, hs = L.h2d_stream, ds = L.d2h_stream;
  hipStream_t xs[2] = {cs, ncs > 1 ? L.aux_stream : cs};
  int ev_next = 1;
  auto next_event = [&]() {
    if (ev_next >= Library::kSyncEvents) throw Error(kDeviceError, "pipeline event pool exhausted");
    return L.sync_ev[ev_next++];
  };
  FASTMM_HIP(hipEventRecord(L.ev[0], cs));
  FASTMM_HIP(hipEventRecord(L.sync_ev[0], cs));
  FASTMM_HIP(hipStreamWaitEvent(hs, L.sync_ev[0], 0));
  FASTMM_HIP(hipStreamWaitEvent(ds, L.sync_ev[0], 0));
  // Zero padding of the device copies, ahead of the copies on their stream.
  if (K4 > K) {
    FASTMM_HIP(hipMemset2DAsync(dA + K, K4 * 4, 0, (K4 - K) * 4, M, hs));
    FASTMM_HIP(hipMemsetAsync(dB + K * N4, 0, (K4 - K) * N4 * 4, hs));
  }
  if (N4 > N) FASTMM_HIP(hipMemset2DAsync(dB + N, N4 * 4, 0, (N4 - N) * 4, K, hs));
  auto arrive = [&]() {  // event after the copies queued so far
    hipEvent_t e = next_event();
    FASTMM_HIP(hipEventRecord(e, hs));
    return e;
  };
  auto a_band = [&](int qr, int qc, const Band& b) {
    const int64_t rows = qr ? b.bot : b.rows;
    h2d_block(dA, K4, A, lda, (qr ? m2 : 0) + b.r0, qc ? k2 : 0, rows, qc ? kb_v : k2, hs);
  };
  auto b_band = [&](int qr, int qc, const Band& c) {
    h2d_block(dB, N4, B, ldb, qr ? k2 : 0, (qc ? n2 : 0) + c.r0, qr ? kb_v : k2,
              qc ? right_valid(c) : c.rows, hs);
  };

  // ---- inputs, in the order of `items`, queued before the schedules are
  // built so that the host's work overlaps the first copies
  std::vector<hipEvent_t> ev_item(items.size());  // after each input item's copy
  for (size_t k = 0; k < items.size(); ++k) {
    const Item& it = items[k];
    if (wino) {
      if (it.mat == 0) a_band(it.q / 2, it.q % 2, bands[it.band]);
      else b_band(it.q / 2, it.q % 2, cbands[it.band]);
    } else if (it.mat == 0) {
      const Band& b = bands[it.band];
      h2d_block(dA, K4, A, lda, b.r0, 0, b.rows, K, hs);
    } else {
      const Band& c = cbands[it.band];
      h2d_block(dB, N4, B, ldb, 0, c.r0, K, plain_valid(c), hs);
    }
    ev_item[k] = arrive();
  }
  FASTMM_HIP(hipEventRecord(L.ev[5], hs));

  // ---- the pieces' schedules and the top-level post-addition nodes
  {
    std::vector<size_t> doff, dbytes;
    for (auto& g : groups) {
      doff.push_back(g.desc_off);
      dbytes.push_back(g.desc_bytes);
    }
    build_groups();
    for (size_t i = 0; i < groups.size(); ++i) {
      groups[i].desc_off = doff[i];
      groups[i].desc_bytes = dbytes[i];
      build_schedule(groups[i].probs, temps + groups[i].x * temp_stride, groups[i].s);
    }
  }
  size_t slot = 0;
  auto next_slot = [&]() {
    if (slot >= nslots) throw Error(kDeviceError, "descriptor slots exhausted");
    return 256 * slot++;
  };
  // Top-level post-addition nodes, one per (row band, column band) block (the
  // quadrant is chosen at launch).  Pre-addition nodes are written as they
  // are issued (their output masks depend on what has arrived).
  std::vector<const PostAddNode*> d_post((size_t)nband * std::max(ncband, 1));
  std::vector<char> vec_post(d_post.size());
  if (wino) {
    for (int bi = 0; bi < nband; ++bi)
      for (int ci = 0; ci < ncband; ++ci) {
        const Band& b = bands[bi];
        const Band& c = cbands[ci];
        PostAddNode np{};
        np.P = P + p_off[(size_t)bi * ncband + ci];
        np.dst = dC + b.r0 * N4 + c.r0;
        np.ld = N4;
        np.p_stride = b.rows * c.rows;
        np.bot_off = m2 * N4;
        np.right_off = (int32_t)n2;
        np.top_rows = (int32_t)b.rows;
        np.bot_rows = (int32_t)b.bot;
        np.left_cols = (int32_t)c.rows;
        np.right_cols = (int32_t)c.bot;
        np.h_r = (int32_t)b.rows;
        np.h_c = (int32_t)c.rows;
        const size_t o = next_slot();
        std::memcpy(host + o, &np, sizeof(np));
        d_post[(size_t)bi * ncband + ci] = reinterpret_cast<const PostAddNode*>(ddesc + o);
        vec_post[(size_t)bi * ncband + ci] = post_vec_ok(np);
      }
  }
  if (slot) FASTMM_HIP(hipMemcpyAsync(ddesc, host, 256 * slot, hipMemcpyHostToDevice, cs));
  if (ncs > 1) {  // the second stream starts after the caller's work and that upload
    hipEvent_t e = next_event();
    FASTMM_HIP(hipEventRecord(e, cs));
    FASTMM_HIP(hipStreamWaitEvent(xs[1], e, 0));
  }

  int launches = 0, nleaf = 0;
  auto run_group = [&](Group& g) {
    if (2 * nleaf + 1 >= Library::kLeafEvents) throw Error(kDeviceError, "leaf event pool exhausted");
    hipEvent_t b = L.leaf_ev[2 * nleaf], e = L.leaf_ev[2 * nleaf + 1];
    ++nleaf;
    // enqueue_schedule launches on L.stream: point it at the group's stream.
    const hipStream_t keep = L.stream;
    L.stream = xs[g.x];
    try {
      launches += enqueue_schedule(L, g.s, ddesc + g.desc_off, host + g.desc_off, b, e);
    } catch (...) {
      L.stream = keep;
      throw;
    }
    L.stream = keep;
  };
  auto wait = [&](int x, hipEvent_t e) { FASTMM_HIP(hipStreamWaitEvent(xs[x], e, 0)); };
  int waited[2] = {-1, -1};  // per compute stream: inputs 0..waited are on the device
  auto wait_item = [&](int x, int k) {
    if (k > waited[x]) {
      wait(x, ev_item[k]);
      waited[x] = k;
    }
  };

  if (wino) {
    // ---- compute
    unsigned s_done[kMaxBands] = {}, t_done[kMaxBands] = {};  // outputs computed so far, per band
    // Which stream computed each S / T output, and the event after its pass.
    struct Made {
      hipEvent_t e = nullptr;
      int x = -1;
    };
    Made s_made[kMaxBands][4], t_made[kMaxBands][4];
    auto after = [&](int x, const Made& m) {
      if (m.x >= 0 && m.x != x) wait(x, m.e);
    };
    auto have = [&](int x, int mat, int q, int band) {
      return (mat == 0 ? a_item[q][band] : b_item[q][band]) <= waited[x];
    };
    // Issue, on stream x, one pre-addition pass for every output of this
    // operand's band whose inputs are all on the device and that is not
    // computed yet.
    auto preadd_pass = [&](int x, int side, int bi) {
      unsigned& done = side == 0 ? s_done[bi] : t_done[bi];
      unsigned mask = 0;
      for (int j = 0; j < 4; ++j) {
        if (done & (1u << j)) continue;
        const unsigned in = preadd_inputs(side, 1u << j);
        bool ok = true;
        for (int q = 0; q < 4; ++q)
          if ((in & (1u << q)) && !have(x, side, q, bi)) ok = false;
        if (ok) mask |= 1u << j;
      }
      if (!mask) return;
      PreAddNode n{};
      if (side == 0) {  // row band of A's quadrants -> rows of S1..S4
        const Band& b = bands[bi];
        n.src = dA + b.r0 * K4;
        n.dst = S + b.r0 * k2;
        n.ld = K4;
        n.bot_off = m2 * K4;
        n.out_stride = ma;
        n.top_rows = (int32_t)b.rows;
        n.bot_rows = (int32_t)b.bot;
        n.left_cols = (int32_t)k2;
        n.right_cols = (int32_t)kb;
        n.h_r = (int32_t)b.rows;
        n.h_c = (int32_t)k2;
        n.right_off = (int32_t)k2;
      } else {  // column band of B's quadrants -> the band's own T1..T4
        const Band& c = cbands[bi];
        n.src = dB + c.r0;
        n.dst = T + t_off[bi];
        n.ld = N4;
        n.bot_off = k2 * N4;
        n.out_stride = k2 * c.rows;
        n.top_rows = (int32_t)k2;
        n.bot_rows = (int32_t)kb;
        n.left_cols = (int32_t)c.rows;
        n.right_cols = (int32_t)c.bot;
        n.h_r = (int32_t)k2;
        n.h_c = (int32_t)c.rows;
        n.right_off = (int32_t)n2;
      }
      n.mask = (int32_t)mask;
      const size_t o = next_slot();
      std::memcpy(host + o, &n, sizeof(n));
      FASTMM_HIP(hipMemcpyAsync(ddesc + o, host + o, sizeof(n), hipMemcpyHostToDevice, xs[x]));
      launch_preadd(side, reinterpret_cast<const PreAddNode*>(ddesc + o), 1,
                    (int)add_blocks_for(n.h_r, n.h_c), pre_vec_ok(n), xs[x]);
      ++launches;
      done |= mask;
      if (ncs > 1) {
        const Made m{next_event(), x};
        FASTMM_HIP(hipEventRecord(m.e, xs[x]));
        for (int j = 0; j < 4; ++j)
          if (mask & (1u << j)) (side == 0 ? s_made : t_made)[bi][j] = m;
      }
    };
    // Left / right operand: which S / T output product i reads (0 = none).
    static const int kLeftS[7] = {0, 0, 4, 0, 1, 2, 3};   // P3: S4, P5: S1, P6: S2, P7: S3
    static const int kRightT[7] = {0, 0, 0, 4, 1, 2, 3};  // P4: T4, P5: T1, P6: T2, P7: T3
    static const int kQuadP[4][4] = {{0, 1, -1, -1}, {0, 5, 4, 2}, {0, 5, 6, 3}, {0, 5, 6, 4}};
    std::vector<int> pgi((size_t)7 * nband * ncband, -1);  // piece -> its position in `order`
    std::vector<char> sent((size_t)4 * nband * ncband, 0);
    auto pidx = [&](int i, int r, int c) { return ((size_t)r * ncband + c) * 7 + i; };
    // Per piece: its first leaf event (recorded once its pre-additions, the
    // shared inner temporaries included, are done) and, with two streams, an
    // event after its last launch.  First piece of each (product, row band)
    // and (product, column band): the one that computes the shared
    // temporaries.
    std::vector<int> piece_leaf(order.size(), -1);
    std::vector<hipEvent_t> piece_end(order.size(), nullptr);
    std::vector<int> a_first((size_t)7 * nband, -1), b_first((size_t)7 * ncband, -1);
    for (size_t gi = 0; gi < order.size(); ++gi) {
      const Piece& pc = order[gi];
      const int x = groups[gi].x;
      int last = -1;
      for (int q = 0; q < 4; ++q) {
        if (kNeedA[pc.i] & (1u << q)) last = std::max(last, a_item[q][pc.r]);
        if (kNeedB[pc.i] & (1u << q)) last = std::max(last, b_item[q][pc.c]);
      }
      wait_item(x, last);
      if (kLeftS[pc.i]) {
        const int j = kLeftS[pc.i] - 1;
        if (!(s_done[pc.r] & (1u << j))) preadd_pass(x, 0, pc.r);
        else after(x, s_made[pc.r][j]);
      }
      if (kRightT[pc.i]) {
        const int j = kRightT[pc.i] - 1;
        if (!(t_done[pc.c] & (1u << j))) preadd_pass(x, 1, pc.c);
        else after(x, t_made[pc.c][j]);
      }
      int& af = a_first[(size_t)pc.i * nband + pc.r];
      int& bf = b_first[(size_t)pc.i * ncband + pc.c];
      if (trees && af >= 0 && groups[af].x != x) wait(x, L.leaf_ev[2 * piece_leaf[af]]);
      if (trees && bf >= 0 && groups[bf].x != x) wait(x, L.leaf_ev[2 * piece_leaf[bf]]);
      if (af < 0) af = (int)gi;
      if (bf < 0) bf = (int)gi;
      piece_leaf[gi] = nleaf;
      run_group(groups[gi]);
      if (ncs > 1) {
        piece_end[gi] = next_event();
        FASTMM_HIP(hipEventRecord(piece_end[gi], xs[x]));
      }
      pgi[pidx(pc.i, pc.r, pc.c)] = (int)gi;
      // Result blocks whose four (two for C11) products are now all done:
      // form them and send them out.
      for (int q = 0; q < 4; ++q) {
        char& sq = sent[((size_t)pc.r * ncband + pc.c) * 4 + q];
        if (sq) continue;
        bool ok = true;
        for (int k = 0; k < 4; ++k)
          if (kQuadP[q][k] >= 0 && pgi[pidx(kQuadP[q][k], pc.r, pc.c)] < 0) ok = false;
        if (!ok) continue;
        for (int k = 0; k < 4; ++k) {  // products finished on the other stream
          if (kQuadP[q][k] < 0) continue;
          const int j = pgi[pidx(kQuadP[q][k], pc.r, pc.c)];
          if (groups[j].x != x) wait(x, piece_end[j]);
        }
        const Band& b = bands[pc.r];
        const Band& c = cbands[pc.c];
        const size_t blk = (size_t)pc.r * ncband + pc.c;
        launch_postadd(d_post[blk], 1, (int)add_blocks_for(b.rows, c.rows), vec_post[blk], xs[x], q);
        ++launches;
        const int qr = q / 2, qc = q % 2;
        hipEvent_t e = next_event();
        FASTMM_HIP(hipEventRecord(e, xs[x]));
        FASTMM_HIP(hipStreamWaitEvent(ds, e, 0));
        d2h_block(C, ldc, dC, N4, (qr ? m2 : 0) + b.r0, (qc ? n2 : 0) + c.r0, qr ? b.bot : b.rows,
                  qc ? right_valid(c) : c.rows, ds);
        sq = 1;
      }
    }
  } else {
    // Plain product: each piece C[r, c] once its two bands are in, each
    // result block sent out once computed.
    for (size_t gi = 0; gi < order.size(); ++gi) {
      const int x = groups[gi].x;
      const Band& b = bands[order[gi].r];
      const Band& c = cbands[order[gi].c];
      wait_item(x, plain_ready[gi]);
      run_group(groups[gi]);
      hipEvent_t e = next_event();
      FASTMM_HIP(hipEventRecord(e, xs[x]));
      FASTMM_HIP(hipStreamWaitEvent(ds, e, 0));
      d2h_block(C, ldc, dC, N4, b.r0, c.r0, b.rows, plain_valid(c), ds);
    }
  }
  FASTMM_HIP(hipEventRecord(L.ev[7], ds));
  // Every stream of the call has drained when it returns.  (The second
  // compute stream is joined on the host: a final wait of the caller's
  // stream for it would leave that stream reporting unfinished work to the
  // first query after the return.)
  FASTMM_HIP(hipStreamSynchronize(ds));
  if (ncs > 1) FASTMM_HIP(hipStreamSynchronize(xs[1]));
  FASTMM_HIP(hipStreamSynchronize(cs));
  FASTMM_HIP(hipStreamSynchronize(hs));

  // ---- statistics
  st.depth = depth;
  st.tile = tile;
  st.leaves = 0;
  st.leaf_flops = 0;
  st.add_bytes = 0;
  for (auto& g : groups) {
    st.leaves += g.s.leaves;
    st.leaf_flops += g.s.leaf_flops;
    st.add_bytes += g.s.add_bytes;
  }
  st.leaf_m = groups[0].s.leaf_dims.m;
  st.leaf_k = groups[0].s.leaf_dims.k;
  st.leaf_n = groups[0].s.leaf_dims.n;
  if (wino)  // top level: 8 pre-addition blocks in and out, 14 product reads + 4 writes out
    st.add_bytes += 32.0 * m2 * k2 + 32.0 * k2 * n2 + 72.0 * m2 * n2;
  st.transfer_bytes = 4.0 * ((double)M * K + (double)K * N + (double)M * N);
  st.launches = launches;
  st.workspace_bytes = L.arena_bytes;
  // Leaf time: the union of the leaf launches' intervals (the launches of
  // the two compute streams overlap).
  double leaf = 0.0;
  std::vector<std::pair<double, double>> iv;
  for (int i = 0; i < nleaf; ++i) {
    const double a = ev_ms(L.ev[0], L.leaf_ev[2 * i]), b = ev_ms(L.ev[0], L.leaf_ev[2 * i + 1]);
    if (a < 0 || b < 0) {
      leaf = -1.0;
      break;
    }
    iv.push_back({a, b});
  }
  if (leaf >= 0) {
    std::sort(iv.begin(), iv.end());
    double end = -1.0;
    for (const auto& x : iv) {
      if (x.second <= end) continue;
      leaf += x.second - std::max(x.first, end);
      end = x.second;
    }
  }
  st.leaf_ms = leaf;
  st.h2d_ms = ev_ms(L.ev[0], L.ev[5]);
  st.total_ms = ev_ms(L.ev[0], L.ev[7]);
  st.preadd_ms = st.postadd_ms = st.d2h_ms = -1.0;
  st.leaf_launches = nleaf;
}

}  // namespace fastmm
