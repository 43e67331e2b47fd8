// Host-resident operands: overlap the PCIe transfers with the recursion.
//
// The paper's leaf call moves the operands to the device, computes and moves
// the result back, one step after the other (Section 3.3), and it observes
// that transfers, not kernels, cap its throughput on large problems
// (Section 4.2).  On MI355X the same holds in proportion: at n = 19456 the
// copies of A, B and C take about as long as the whole Winograd product.
// Here the top level of the recursion is run product by product on a compute
// stream while a copy stream brings the operand quadrants in, in the order
// the products need them, and a second copy stream sends each result
// quadrant back as soon as its post-addition is done:
//
//   in:   A11 B11 | A12 B21 | B12 B22 A22 | A21
//   run:  P1 = A11 B11, P2 = A12 B21        -> C11 = P1 + P2        -> out
//         T1..T4, P4 = A22 T4; S1..S4, P6, P7 -> C21 = U3 - P4      -> out
//         P5                                 -> C22 = U3 + P5       -> out
//         P3                                 -> C12 = U4 + P3       -> out
//
// Each product Pi is itself a level-wise Winograd product of depth d - 1
// (one grouped leaf launch).  Each result quadrant is formed by the same
// chain of FP32 operations as the fused post-addition, so the result is bit
// for bit the one of the unpipelined path.  With no Winograd level (plain
// SGEMM) the same overlap is used on the 2 x 2 block product
// C_ij = A_i B_j (row halves of A, column halves of B).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "engine.h"

namespace fastmm {
namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Copy rows [r0, r0 + rows) x cols [c0, c0 + cols) of a host matrix into the
// same block of a dense device matrix.
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

struct Child {
  Problem p;
  Schedule s;
  char* desc_dev = nullptr;
  char* desc_host = nullptr;
};

double ev_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return -1.0;
  }
  return ms;
}

}  // namespace

void gemm_host_pipelined(Library& L, int64_t M, int64_t N, int64_t K, const float* A,
                         int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc,
                         int depth, int tile, fastmm_stats_t& st) {
  const int64_t m2 = half_up(M), k2 = half_up(K), n2 = half_up(N);
  const int64_t mb = M - m2, kb = K - k2, nb = N - n2;
  const bool wino = depth >= 1;

  // ---- workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes, 256);
    return o;
  };
  const size_t oA = take((size_t)M * K * 4), oB = take((size_t)K * N * 4),
               oC = take((size_t)M * N * 4);
  size_t oS = 0, oT = 0, oP = 0;
  if (wino) {
    oS = take((size_t)4 * m2 * k2 * 4);
    oT = take((size_t)4 * k2 * n2 * 4);
    oP = take((size_t)7 * m2 * n2 * 4);
  }
  // Children: 7 sub-products (depth - 1 each) or 4 block products (depth 0).
  const int nchild = wino ? 7 : 4;
  std::vector<Child> ch(nchild);
  for (int i = 0; i < nchild; ++i) {
    Problem& p = ch[i].p;
    p.tile = tile;
    if (wino) {
      p.M = m2;
      p.K = k2;
      p.N = n2;
      p.depth = depth - 1;
    } else {
      const int bi = i / 2, bj = i % 2;
      p.M = bi == 0 ? m2 : mb;
      p.N = bj == 0 ? n2 : nb;
      p.K = K;
      p.depth = 0;
    }
  }
  const size_t child_temp = align_up(problem_temp_bytes(ch[0].p), 256);
  const size_t oTemp = take(child_temp);
  // Descriptor regions: one per child plus one for the top-level additions.
  std::vector<size_t> desc_size(nchild);
  for (int i = 0; i < nchild; ++i) {
    Problem q = ch[i].p;
    q.A = q.B = reinterpret_cast<const float*>(256);
    q.C = const_cast<float*>(q.A);
    q.lda = std::max<int64_t>(q.K, 1);
    q.ldb = q.ldc = std::max<int64_t>(q.N, 1);
    Schedule tmp;
    build_schedule({q}, reinterpret_cast<char*>(256), tmp);
    desc_size[i] = align_up(schedule_desc_bytes(tmp), 256) + 256;
  }
  const size_t top_desc = 6 * 256;  // preA, preB and four post-addition nodes
  size_t desc_total = top_desc;
  for (auto d : desc_size) desc_total += d;
  const size_t oDesc = take(desc_total);

  char* ws = ensure_arena(L, off);
  char* host = ensure_pinned(L, desc_total);
  float* dA = reinterpret_cast<float*>(ws + oA);
  float* dB = reinterpret_cast<float*>(ws + oB);
  float* dC = reinterpret_cast<float*>(ws + oC);
  float* S = reinterpret_cast<float*>(ws + oS);
  float* T = reinterpret_cast<float*>(ws + oT);
  float* P = reinterpret_cast<float*>(ws + oP);
  char* temps = ws + oTemp;
  char* ddesc = ws + oDesc;

  // ---- operand views of the children (device staging buffers, dense).
  if (wino) {
    const int64_t ma = m2 * k2, tb = k2 * n2, pc = m2 * n2;
    struct V {
      const float* p;
      int64_t ld, r, c;
    };
    const V a11{dA, K, m2, k2}, a12{dA + k2, K, m2, kb}, a22{dA + m2 * K + k2, K, mb, kb};
    const V b11{dB, N, k2, n2}, b21{dB + k2 * N, N, kb, n2}, b22{dB + k2 * N + n2, N, kb, nb};
    auto sv = [&](int i) { return V{S + i * ma, k2, m2, k2}; };
    auto tv = [&](int i) { return V{T + i * tb, n2, k2, n2}; };
    // P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4, P5 = S1 T1,
    // P6 = S2 T2, P7 = S3 T3.
    const V ca[7] = {a11, a12, sv(3), a22, sv(0), sv(1), sv(2)};
    const V cb[7] = {b11, b21, b22, tv(3), tv(0), tv(1), tv(2)};
    for (int i = 0; i < 7; ++i) {
      Problem& p = ch[i].p;
      p.A = ca[i].p;
      p.lda = ca[i].ld;
      p.a_rows = ca[i].r;
      p.a_cols = ca[i].c;
      p.B = cb[i].p;
      p.ldb = cb[i].ld;
      p.b_rows = cb[i].r;
      p.b_cols = cb[i].c;
      p.C = P + i * pc;
      p.ldc = n2;
    }
  } else {
    for (int i = 0; i < 4; ++i) {
      const int bi = i / 2, bj = i % 2;
      Problem& p = ch[i].p;
      p.A = dA + bi * m2 * K;
      p.lda = K;
      p.B = dB + bj * n2;
      p.ldb = N;
      p.C = dC + bi * m2 * N + bj * n2;
      p.ldc = N;
    }
  }
  // Schedules and descriptor blocks (host side, before anything is queued).
  size_t doff = top_desc;
  for (int i = 0; i < nchild; ++i) {
    build_schedule({ch[i].p}, temps, ch[i].s);
    ch[i].desc_dev = ddesc + doff;
    ch[i].desc_host = host + doff;
    doff += desc_size[i];
  }
  PreAddNode na{dA, S, K, (int32_t)M, (int32_t)K, (int32_t)m2, (int32_t)k2, 0, 0};
  PreAddNode nbn{dB, T, N, (int32_t)K, (int32_t)N, (int32_t)k2, (int32_t)n2, 0, 0};
  PostAddNode pn{P, dC, N, (int32_t)M, (int32_t)N, (int32_t)m2, (int32_t)n2, 0, 0};
  std::memcpy(host, &na, sizeof(na));
  std::memcpy(host + 256, &nbn, sizeof(nbn));
  std::memcpy(host + 512, &pn, sizeof(pn));
  const PreAddNode* d_na = reinterpret_cast<const PreAddNode*>(ddesc);
  const PreAddNode* d_nb = reinterpret_cast<const PreAddNode*>(ddesc + 256);
  const PostAddNode* d_pn = reinterpret_cast<const PostAddNode*>(ddesc + 512);
  const bool vec_a = K % 4 == 0 && k2 % 4 == 0;
  const bool vec_b = N % 4 == 0 && n2 % 4 == 0;
  const bool vec_p = N % 4 == 0 && n2 % 4 == 0;

  hipStream_t cs = L.stream, hs = L.h2d_stream, ds = L.d2h_stream;
  hipEvent_t* E = L.sync_ev;  // E[0] start, E[1..4] inputs, E[5..8] outputs
  FASTMM_HIP(hipEventRecord(L.ev[0], cs));
  FASTMM_HIP(hipEventRecord(E[0], cs));
  FASTMM_HIP(hipStreamWaitEvent(hs, E[0], 0));
  FASTMM_HIP(hipStreamWaitEvent(ds, E[0], 0));

  // ---- inputs, in the order the products consume them
  if (wino) {
    h2d_block(dA, K, A, lda, 0, 0, m2, k2, hs);    // A11
    h2d_block(dB, N, B, ldb, 0, 0, k2, n2, hs);    // B11
    FASTMM_HIP(hipEventRecord(E[1], hs));
    h2d_block(dA, K, A, lda, 0, k2, m2, kb, hs);   // A12
    h2d_block(dB, N, B, ldb, k2, 0, kb, n2, hs);   // B21
    FASTMM_HIP(hipEventRecord(E[2], hs));
    h2d_block(dB, N, B, ldb, 0, n2, k2, nb, hs);   // B12
    h2d_block(dB, N, B, ldb, k2, n2, kb, nb, hs);  // B22
    h2d_block(dA, K, A, lda, m2, k2, mb, kb, hs);  // A22
    FASTMM_HIP(hipEventRecord(E[3], hs));
    h2d_block(dA, K, A, lda, m2, 0, mb, k2, hs);   // A21
    FASTMM_HIP(hipEventRecord(E[4], hs));
  } else {
    h2d_block(dA, K, A, lda, 0, 0, m2, K, hs);     // A top
    h2d_block(dB, N, B, ldb, 0, 0, K, n2, hs);     // B left
    FASTMM_HIP(hipEventRecord(E[1], hs));
    h2d_block(dB, N, B, ldb, 0, n2, K, nb, hs);    // B right
    FASTMM_HIP(hipEventRecord(E[2], hs));
    h2d_block(dA, K, A, lda, m2, 0, mb, K, hs);    // A bottom
    FASTMM_HIP(hipEventRecord(E[3], hs));
    FASTMM_HIP(hipEventRecord(E[4], hs));
  }
  FASTMM_HIP(hipEventRecord(L.ev[5], hs));

  // ---- compute
  FASTMM_HIP(hipMemcpyAsync(ddesc, host, top_desc, hipMemcpyHostToDevice, cs));
  int launches = 0, nleaf = 0;
  auto run_child = [&](int i) {
    hipEvent_t b = L.leaf_ev[2 * nleaf], e = L.leaf_ev[2 * nleaf + 1];
    ++nleaf;
    launches += enqueue_schedule(L, ch[i].s, ch[i].desc_dev, ch[i].desc_host, b, e);
  };
  // Result quadrant q (0 = C11, 1 = C12, 2 = C21, 3 = C22) out to the host.
  auto send = [&](int q, hipEvent_t ev) {
    const int qr = q / 2, qc = q % 2;
    FASTMM_HIP(hipEventRecord(ev, cs));
    FASTMM_HIP(hipStreamWaitEvent(ds, ev, 0));
    d2h_block(C, ldc, dC, N, qr ? m2 : 0, qc ? n2 : 0, qr ? mb : m2, qc ? nb : n2, ds);
  };
  auto post = [&](int q) {
    launch_postadd(d_pn, 1, (int)add_blocks_for(m2, n2), vec_p, cs, q);
    ++launches;
  };
  // Each child's schedule uploads its own descriptor block on this stream
  // (distinct host and device regions), ahead of its launches.
  if (wino) {
    FASTMM_HIP(hipStreamWaitEvent(cs, E[1], 0));
    run_child(0);                                   // P1
    FASTMM_HIP(hipStreamWaitEvent(cs, E[2], 0));
    run_child(1);                                   // P2
    post(0);                                        // C11 = P1 + P2
    send(0, E[5]);
    FASTMM_HIP(hipStreamWaitEvent(cs, E[3], 0));
    launch_preadd(1, d_nb, 1, (int)add_blocks_for(k2, n2), vec_b, cs);  // T1..T4
    ++launches;
    run_child(3);                                   // P4 = A22 T4
    FASTMM_HIP(hipStreamWaitEvent(cs, E[4], 0));
    launch_preadd(0, d_na, 1, (int)add_blocks_for(m2, k2), vec_a, cs);  // S1..S4
    ++launches;
    run_child(5);                                   // P6 = S2 T2
    run_child(6);                                   // P7 = S3 T3
    post(2);                                        // C21 = U3 - P4
    send(2, E[6]);
    run_child(4);                                   // P5 = S1 T1
    post(3);                                        // C22 = U3 + P5
    send(3, E[7]);
    run_child(2);                                   // P3 = S4 B22
    post(1);                                        // C12 = U4 + P3
    send(1, E[8]);
  } else {
    FASTMM_HIP(hipStreamWaitEvent(cs, E[1], 0));
    run_child(0);                                   // C11 = A_top B_left
    send(0, E[5]);
    FASTMM_HIP(hipStreamWaitEvent(cs, E[2], 0));
    run_child(1);                                   // C12 = A_top B_right
    send(1, E[6]);
    FASTMM_HIP(hipStreamWaitEvent(cs, E[3], 0));
    run_child(2);                                   // C21 = A_bottom B_left
    send(2, E[7]);
    run_child(3);                                   // C22 = A_bottom B_right
    send(3, E[8]);
  }
  FASTMM_HIP(hipEventRecord(L.ev[7], ds));
  FASTMM_HIP(hipStreamSynchronize(ds));
  FASTMM_HIP(hipStreamSynchronize(cs));
  FASTMM_HIP(hipStreamSynchronize(hs));

  // ---- statistics
  st.depth = depth;
  st.tile = tile;
  st.leaves = 0;
  st.leaf_flops = 0;
  st.add_bytes = 0;
  for (auto& c : ch) {
    st.leaves += c.s.leaves;
    st.leaf_flops += c.s.leaf_flops;
    st.add_bytes += c.s.add_bytes;
  }
  st.leaf_m = ch[0].s.leaf_dims.m;
  st.leaf_k = ch[0].s.leaf_dims.k;
  st.leaf_n = ch[0].s.leaf_dims.n;
  if (wino)  // top level: 8 pre-addition blocks in and out, 14 product reads + 4 writes out
    st.add_bytes += 32.0 * m2 * k2 + 32.0 * k2 * n2 + 72.0 * m2 * n2;
  st.transfer_bytes = 4.0 * ((double)M * K + (double)K * N + (double)M * N);
  st.launches = launches;
  st.workspace_bytes = L.arena_bytes;
  double leaf = 0.0;
  for (int i = 0; i < nleaf; ++i) {
    const double t = ev_ms(L.leaf_ev[2 * i], L.leaf_ev[2 * i + 1]);
    if (t < 0) {
      leaf = -1.0;
      break;
    }
    leaf += t;
  }
  st.leaf_ms = leaf;
  st.h2d_ms = ev_ms(L.ev[0], L.ev[5]);
  st.total_ms = ev_ms(L.ev[0], L.ev[7]);
  st.preadd_ms = st.postadd_ms = st.d2h_ms = -1.0;
  st.leaf_launches = nleaf;
}

}  // namespace fastmm
