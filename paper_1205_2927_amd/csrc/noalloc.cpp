// fastmm_gemm_noalloc: the single-product path without device allocation,
// for callers that cannot allocate (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// The recursion's temporaries (S, T and P blocks of every level) and the
// uploaded descriptor arrays live in one statically allocated device array,
// `scratch`, of kStaticScratchBytes.  The loader reserves it on every GPU the
// library's code object is loaded on, and it stays there until the process
// ends.  Its first kQueueBytes also hold the two counters of the persistent
// leaf launches of the batched path, so the library's initialisation itself
// allocates no device memory.
//
// In host code `scratch` names a host-side stand-in, not the device array:
// the device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and only that address is ever passed to kernels or
// copies.
//
// Every call on a GPU shares that GPU's array and leaves its last
// temporaries in it.  Nothing in it has to start at zero: every temporary is
// written by the schedule before it is read, and the persistent-launch
// counters are left at zero by the kernel that uses them.  Calls are
// serialised by the library lock and return only when their work is done, so
// two calls of one process never overlap; work that overlapped a call on the
// same GPU while using the array would race with it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "engine.h"

namespace fastmm {
namespace {

constexpr size_t kStaticScratchBytes = size_t(FASTMM_NOALLOC_WORKSPACE_BYTES);
constexpr size_t kQueueBytes = 256;
// Host staging of the descriptor upload: a file-scope array, so the upload
// needs no pinned allocation either (a copy from pageable memory, complete
// before the call returns).
constexpr size_t kStaticDescBytes = size_t(2) << 20;

__device__ __align__(256) char scratch[kStaticScratchBytes];

alignas(256) char g_desc_host[kStaticDescBytes];

constexpr int kMaxDevices = 64;
char* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

__global__ void zero_matrix_kernel(float* C, int64_t ldc, int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x)
    C[(i / cols) * ldc + i % cols] = 0.f;
}

}  // namespace

char* bind_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error(kNotSupported, "device id out of range");
  if (!g_scratch_dev[device]) {
    int cur = -1;
    FASTMM_HIP(hipGetDevice(&cur));
    if (cur != device) throw Error(kDeviceError, "static workspace bound with another device current");
    void* p = nullptr;
    FASTMM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(kDeviceError, "hipGetSymbolAddress returned no address for the static workspace");
    g_scratch_dev[device] = static_cast<char*>(p);
  }
  return g_scratch_dev[device];
}

size_t static_queue_bytes() { return kQueueBytes; }

namespace {

void gemm_noalloc_impl(Library& L, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                       const float* B, int64_t ldb, float* C, int64_t ldc, int depth, int64_t leaf) {
  validate_gemm_args(M, N, K, A, lda, B, ldb, C, ldc, depth);
  ensure_init(L);
  int cur = -1;
  FASTMM_HIP(hipGetDevice(&cur));
  if (cur != L.device)
    throw Error(kNotSupported, "fastmm_gemm_noalloc: the current device is not the library's device");
  char* base = bind_static_scratch(cur);
  fastmm_stats_t st{};
  st.h2d_ms = st.preadd_ms = st.leaf_ms = st.postadd_ms = st.d2h_ms = st.total_ms = -1.0;
  if (M == 0 || N == 0) {
    L.stats = st;
    return;
  }
  if (!operands_on_device(M, N, K, A, B, C))
    throw Error(kNotSupported, "fastmm_gemm_noalloc takes device operands only (host operands need "
                               "staging buffers: use fastmm_gemm)");
  const Staging sg = plan_staging(M, N, K, A, lda, B, ldb, true);
  if (sg.a || sg.b)
    throw Error(kNotSupported, "fastmm_gemm_noalloc needs 16-byte aligned rows of A and B, lda and ldb "
                               "multiples of 4 and K, N multiples of 4 (other operands need staging "
                               "copies: use fastmm_gemm)");
  hipStream_t sm = L.stream;
  if (K == 0) {
    hipLaunchKernelGGL(zero_matrix_kernel, dim3(1024), dim3(256), 0, sm, C, ldc, M, N);
    FASTMM_HIP(hipGetLastError());
    FASTMM_HIP(hipStreamSynchronize(sm));
    L.stats = st;
    return;
  }
  int tile = kTile128x128;
  if (depth < 0) {  // the fixed rule: host arithmetic only
    fastmm_plan_t pl{};
    const int rc = plan_choose(L, M, N, K, FASTMM_PLAN_DEFAULT, &pl);
    if (rc != kSuccess) throw Error(rc, "planner failed");
    depth = pl.depth;
    leaf = pl.leaf;
    tile = pl.tile;
  }
  Problem p;
  p.M = M;
  p.N = N;
  p.K = K;
  p.depth = effective_depth(M, N, K, depth, leaf);
  p.tile = tile;
  p.A = A;
  p.lda = lda;
  p.B = B;
  p.ldb = ldb;
  p.C = C;
  p.ldc = ldc;

  // Size the temporaries and the descriptors before anything is written.
  const size_t t_bytes = align_up(problem_temp_bytes(p), 256);
  Schedule s;
  {
    Problem q = p;
    q.A = reinterpret_cast<const float*>(256);
    q.B = q.A;
    q.C = const_cast<float*>(q.A);
    build_schedule({q}, reinterpret_cast<char*>(256), s);
  }
  const size_t d_bytes = align_up(schedule_desc_bytes(s), 256);
  const size_t need = kQueueBytes + t_bytes + d_bytes;
  if (need > kStaticScratchBytes || d_bytes > kStaticDescBytes)
    throw Error(kOutOfMemory,
                "fastmm_gemm_noalloc: depth " + std::to_string(p.depth) + " needs " +
                    std::to_string(need) + " bytes of workspace, the static workspace holds " +
                    std::to_string(kStaticScratchBytes) +
                    " (use a smaller depth, or fastmm_gemm, which allocates)");
  char* temps = base + kQueueBytes;
  char* desc_dev = temps + t_bytes;
  build_schedule({p}, temps, s);
  const int launches = enqueue_schedule(L, s, desc_dev, g_desc_host);
  FASTMM_HIP(hipStreamSynchronize(sm));

  st.depth = p.depth;
  st.tile = tile;
  st.leaves = s.leaves;
  st.leaf_m = s.leaf_dims.m;
  st.leaf_k = s.leaf_dims.k;
  st.leaf_n = s.leaf_dims.n;
  st.leaf_flops = s.leaf_flops;
  st.add_bytes = s.add_bytes;
  st.launches = launches;
  st.workspace_bytes = need;
  for (int t = 0; t < kNumTiles; ++t) st.leaf_launches += s.leaf_tiles_total[t] > 0 ? 1 : 0;
  L.stats = st;
}

}  // namespace
}  // namespace fastmm

using namespace fastmm;

extern "C" int fastmm_gemm_noalloc(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                                   const float* B, int64_t ldb, float* C, int64_t ldc, int depth,
                                   int64_t leaf) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return run_guarded([&] { gemm_noalloc_impl(L, M, N, K, A, lda, B, ldb, C, ldc, depth, leaf); });
}
