// Cost-model network of the planner: forward, backward and Adam on the GPU.
//
// The paper chooses its leaf engine by problem size against thresholds found
// by hand (Table 2; K0 = 400 and K1 ~ 3000, Section 3.2).  The planner here
// learns a cost model instead: a 5 -> 64 -> 64 -> 1 ReLU network maps the
// features of a candidate plan (log extents, depth, leaf tile) to its
// predicted log run time, and is trained on timings the library itself
// measures.  These kernels are that network's training and inference.
//
// Layout: X is batch x 5 row-major; W is (fan_in x fan_out) row-major; the
// flat parameter vector is [W1 (5x64), b1 (64), W2 (64x64), b2 (64),
// W3 (64x1), b3 (1)].  Loss: mean over the batch of (y - t)^2.  Adam with
// bias correction.  All sums over the batch run in sample order, so results
// are reproducible run to run.
#include <hip/hip_runtime.h>

#include <cstring>

#include "engine.h"

namespace fastmm {

constexpr int kIn = 5, kH1 = 64, kH2 = 64;
constexpr int oW1 = 0, ob1 = oW1 + kIn * kH1, oW2 = ob1 + kH1, ob2 = oW2 + kH1 * kH2,
              oW3 = ob2 + kH2, ob3 = oW3 + kH2, kParams = ob3 + 1;
static_assert(kParams == FASTMM_MLP_PARAMS, "parameter count");

// One wavefront per sample; lane j owns hidden unit j of both layers.
// cache (optional): z1 (batch x 64) then z2 (batch x 64).
__global__ void __launch_bounds__(256)
mlp_forward_kernel(int batch, const float* __restrict__ p, const float* __restrict__ X,
                   float* __restrict__ y, float* __restrict__ cache) {
  __shared__ float h1s[4][kH1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + wave;
  const bool live = b < batch;
  float z1 = 0.f;
  if (live) {
    z1 = p[ob1 + lane];
    for (int i = 0; i < kIn; ++i) z1 += X[b * kIn + i] * p[oW1 + i * kH1 + lane];
  }
  h1s[wave][lane] = z1 > 0.f ? z1 : 0.f;
  __syncthreads();
  float z2 = 0.f;
  if (live) {
    z2 = p[ob2 + lane];
    for (int i = 0; i < kH1; ++i) z2 += h1s[wave][i] * p[oW2 + i * kH2 + lane];
  }
  const float h2 = z2 > 0.f ? z2 : 0.f;
  // y = b3 + sum_j h2_j W3_j: butterfly sum over the 64 lanes.
  float v = h2 * p[oW3 + lane];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (live) {
    if (lane == 0) y[b] = v + p[ob3];
    if (cache) {
      cache[(size_t)b * kH1 + lane] = z1;
      cache[(size_t)batch * kH1 + (size_t)b * kH2 + lane] = z2;
    }
  }
}

// Per-sample backward: dy = 2 (y - t) / batch, dz2 = dy W3 * [z2 > 0],
// dz1 = (W2 dz2) * [z1 > 0].  Writes dy (batch), dz1, dz2 (batch x 64).
__global__ void __launch_bounds__(256)
mlp_backward_sample_kernel(int batch, const float* __restrict__ p, const float* __restrict__ y,
                           const float* __restrict__ t, const float* __restrict__ cache,
                           float* __restrict__ dy_out, float* __restrict__ dz1_out,
                           float* __restrict__ dz2_out) {
  __shared__ float dz2s[4][kH2];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + wave;
  const bool live = b < batch;
  float dy = 0.f, dz2 = 0.f;
  if (live) {
    dy = 2.f * (y[b] - t[b]) / (float)batch;
    const float z2 = cache[(size_t)batch * kH1 + (size_t)b * kH2 + lane];
    dz2 = z2 > 0.f ? dy * p[oW3 + lane] : 0.f;
  }
  dz2s[wave][lane] = dz2;
  __syncthreads();
  if (!live) return;
  // dh1_i = sum_j W2[i][j] dz2_j; lane i computes unit i.
  float dh1 = 0.f;
  for (int j = 0; j < kH2; ++j) dh1 += p[oW2 + lane * kH2 + j] * dz2s[wave][j];
  const float z1 = cache[(size_t)b * kH1 + lane];
  dz1_out[(size_t)b * kH1 + lane] = z1 > 0.f ? dh1 : 0.f;
  dz2_out[(size_t)b * kH2 + lane] = dz2;
  if (lane == 0) dy_out[b] = dy;
}

// Parameter gradients: one thread per parameter, summing its per-sample
// contributions in sample order (no atomics).
__global__ void __launch_bounds__(256)
mlp_backward_param_kernel(int batch, const float* __restrict__ X, const float* __restrict__ cache,
                          const float* __restrict__ dy, const float* __restrict__ dz1,
                          const float* __restrict__ dz2, float* __restrict__ grad) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kParams) return;
  float g = 0.f;
  const float* z1 = cache;
  const float* z2 = cache + (size_t)batch * kH1;
  if (q < ob1) {  // W1[i][j] = sum_b X_bi dz1_bj
    const int i = q / kH1, j = q % kH1;
    for (int b = 0; b < batch; ++b) g += X[b * kIn + i] * dz1[(size_t)b * kH1 + j];
  } else if (q < oW2) {  // b1[j]
    const int j = q - ob1;
    for (int b = 0; b < batch; ++b) g += dz1[(size_t)b * kH1 + j];
  } else if (q < ob2) {  // W2[i][j] = sum_b h1_bi dz2_bj
    const int i = (q - oW2) / kH2, j = (q - oW2) % kH2;
    for (int b = 0; b < batch; ++b) {
      const float h1 = z1[(size_t)b * kH1 + i];
      g += (h1 > 0.f ? h1 : 0.f) * dz2[(size_t)b * kH2 + j];
    }
  } else if (q < oW3) {  // b2[j]
    const int j = q - ob2;
    for (int b = 0; b < batch; ++b) g += dz2[(size_t)b * kH2 + j];
  } else if (q < ob3) {  // W3[j] = sum_b h2_bj dy_b
    const int j = q - oW3;
    for (int b = 0; b < batch; ++b) {
      const float h2 = z2[(size_t)b * kH2 + j];
      g += (h2 > 0.f ? h2 : 0.f) * dy[b];
    }
  } else {  // b3
    for (int b = 0; b < batch; ++b) g += dy[b];
  }
  grad[q] = g;
}

// Loss = (1/batch) sum_b (y_b - t_b)^2, one block, fixed reduction order.
__global__ void __launch_bounds__(256)
mlp_loss_kernel(int batch, const float* __restrict__ y, const float* __restrict__ t,
                float* __restrict__ loss) {
  __shared__ float part[256];
  float s = 0.f;
  for (int b = threadIdx.x; b < batch; b += 256) {
    const float d = y[b] - t[b];
    s += d * d;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = part[0] / (float)batch;
}

__global__ void __launch_bounds__(256)
mlp_adam_kernel(const float* __restrict__ g, float* __restrict__ p, float* __restrict__ m,
                float* __restrict__ v, float lr, float b1, float b2, float eps, float c1,
                float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kParams) return;
  const float mq = b1 * m[q] + (1.f - b1) * g[q];
  const float vq = b2 * v[q] + (1.f - b2) * g[q] * g[q];
  m[q] = mq;
  v[q] = vq;
  const float mhat = mq / c1, vhat = vq / c2;
  p[q] -= lr * mhat / (sqrtf(vhat) + eps);
}

// ---- host launchers (stream-ordered), shared with the planner's trainer

size_t mlp_scratch_floats(int batch) { return (size_t)batch * (kH1 + kH2) * 2 + 2 * (size_t)batch + 64; }

void mlp_forward(int batch, const float* p, const float* X, float* y, float* cache,
                 hipStream_t s) {
  if (batch <= 0) return;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((batch + 3) / 4), dim3(256), 0, s, batch, p, X, y,
                     cache);
  FASTMM_HIP(hipGetLastError());
}

// scratch: mlp_scratch_floats(batch) floats of device memory.
void mlp_backward(int batch, const float* p, const float* X, const float* t, float* grad,
                  float* loss, float* scratch, hipStream_t s) {
  if (batch <= 0) return;
  float* cache = scratch;                                 // z1, z2
  float* y = cache + (size_t)batch * (kH1 + kH2);
  float* dy = y + batch;
  float* dz1 = dy + batch;
  float* dz2 = dz1 + (size_t)batch * kH1;
  mlp_forward(batch, p, X, y, cache, s);
  hipLaunchKernelGGL(mlp_backward_sample_kernel, dim3((batch + 3) / 4), dim3(256), 0, s, batch,
                     p, y, t, cache, dy, dz1, dz2);
  hipLaunchKernelGGL(mlp_backward_param_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s,
                     batch, X, cache, dy, dz1, dz2, grad);
  if (loss) hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(256), 0, s, batch, y, t, loss);
  FASTMM_HIP(hipGetLastError());
}

void mlp_adam(const float* g, float* p, float* m, float* v, int step, float lr, float b1,
              float b2, float eps, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step);
  const float c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, g, p, m, v,
                     lr, b1, b2, eps, c1, c2);
  FASTMM_HIP(hipGetLastError());
}

}  // namespace fastmm

using namespace fastmm;

namespace {
bool is_device_ptr(const void* p) {
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}
}  // namespace

extern "C" {

int fastmm_mlp_forward(int batch, const float* params, const float* X, float* y) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return run_guarded([&] {
    if (batch < 0) throw Error(kInvalidValue, "batch < 0");
    if (batch == 0) return;
    if (!params || !X || !y) throw Error(kInvalidValue, "NULL pointer");
    ensure_init(L);
    if (!is_device_ptr(params) || !is_device_ptr(X) || !is_device_ptr(y))
      throw Error(kNotSupported, "fastmm_mlp_forward takes device pointers");
    mlp_forward(batch, params, X, y, nullptr, L.stream);
    FASTMM_HIP(hipStreamSynchronize(L.stream));
  });
}

int fastmm_mlp_backward(int batch, const float* params, const float* X, const float* t,
                        float* grad, float* loss_out) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return run_guarded([&] {
    if (batch <= 0) throw Error(kInvalidValue, "batch must be positive");
    if (!params || !X || !t || !grad) throw Error(kInvalidValue, "NULL pointer");
    ensure_init(L);
    if (!is_device_ptr(params) || !is_device_ptr(X) || !is_device_ptr(t) || !is_device_ptr(grad) ||
        (loss_out && !is_device_ptr(loss_out)))
      throw Error(kNotSupported, "fastmm_mlp_backward takes device pointers");
    float* scratch = reinterpret_cast<float*>(ensure_arena(L, mlp_scratch_floats(batch) * 4));
    mlp_backward(batch, params, X, t, grad, loss_out, scratch, L.stream);
    FASTMM_HIP(hipStreamSynchronize(L.stream));
  });
}

int fastmm_mlp_adam(const float* grad, float* params, float* m, float* v, int step, float lr,
                    float beta1, float beta2, float eps) {
  Library& L = lib();
  std::lock_guard<std::mutex> g(L.mu);
  return run_guarded([&] {
    if (step < 1) throw Error(kInvalidValue, "step counts from 1");
    if (!grad || !params || !m || !v) throw Error(kInvalidValue, "NULL pointer");
    ensure_init(L);
    if (!is_device_ptr(grad) || !is_device_ptr(params) || !is_device_ptr(m) || !is_device_ptr(v))
      throw Error(kNotSupported, "fastmm_mlp_adam takes device pointers");
    mlp_adam(grad, params, m, v, step, lr, beta1, beta2, eps, L.stream);
    FASTMM_HIP(hipStreamSynchronize(L.stream));
  });
}

}  // extern "C"
