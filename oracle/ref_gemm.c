/* ORACLE -- test infrastructure only.  Plain, slow, obviously correct CPU code
 * for the classic matrix product, used to check the GPU library.  Nothing in
 * the product path links or calls this file.
 *
 * Definition followed: c_ij = sum_k a_ik * b_kj (Section 3.3, the per-element
 * row-by-column formula, equation (6)).  Every sum runs over k in ascending
 * order and accumulates in IEEE double; FP32 inputs widen to double exactly.
 * Parallelism (OpenMP over rows of C) does not change any entry's sum order.
 */
#include <omp.h>
#include <stdint.h>

/* C (M x N, ldc) = A (M x K, lda) * B (K x N, ldb), all double, row-major. */
void ref_gemm_f64(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                  const double* B, int64_t ldb, double* C, int64_t ldc) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < M; ++i) {
    double* c = C + i * ldc;
    for (int64_t j = 0; j < N; ++j) c[j] = 0.0;
    for (int64_t k = 0; k < K; ++k) {
      const double a = A[i * lda + k];
      const double* b = B + k * ldb;
      for (int64_t j = 0; j < N; ++j) c[j] += a * b[j];
    }
  }
}

/* Same product, FP32 inputs (widened exactly to double), FP64 accumulation. */
void ref_gemm_f32in(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                    const float* B, int64_t ldb, double* C, int64_t ldc) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < M; ++i) {
    double* c = C + i * ldc;
    for (int64_t j = 0; j < N; ++j) c[j] = 0.0;
    for (int64_t k = 0; k < K; ++k) {
      const double a = (double)A[i * lda + k];
      const float* b = B + k * ldb;
      for (int64_t j = 0; j < N; ++j) c[j] += a * (double)b[j];
    }
  }
}

/* Selected rows of the same product: out[r, :] = row rows[r] of A*B. */
void ref_gemm_rows_f32in(int64_t nrows, const int64_t* rows, int64_t N, int64_t K,
                         const float* A, int64_t lda, const float* B, int64_t ldb,
                         double* out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = rows[r];
    double* c = out + r * N;
    for (int64_t j = 0; j < N; ++j) c[j] = 0.0;
    for (int64_t k = 0; k < K; ++k) {
      const double a = (double)A[i * lda + k];
      const float* b = B + k * ldb;
      for (int64_t j = 0; j < N; ++j) c[j] += a * (double)b[j];
    }
  }
}

/* y (M) = X (M x N, ldx, FP32 widened) * v (N, double): used by Freivalds'
 * check, which compares C*v with A*(B*v). */
void ref_gemv_f32in(int64_t M, int64_t N, const float* X, int64_t ldx, const double* v,
                    double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < M; ++i) {
    double s = 0.0;
    const float* x = X + i * ldx;
    for (int64_t j = 0; j < N; ++j) s += (double)x[j] * v[j];
    y[i] = s;
  }
}

/* Integer product with exact int64 accumulation (inputs small integers). */
void ref_gemm_i64(int64_t M, int64_t N, int64_t K, const int64_t* A, int64_t lda,
                  const int64_t* B, int64_t ldb, int64_t* C, int64_t ldc) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < M; ++i) {
    int64_t* c = C + i * ldc;
    for (int64_t j = 0; j < N; ++j) c[j] = 0;
    for (int64_t k = 0; k < K; ++k) {
      const int64_t a = A[i * lda + k];
      const int64_t* b = B + k * ldb;
      for (int64_t j = 0; j < N; ++j) c[j] += a * b[j];
    }
  }
}

/* Threads OpenMP will use for the loops above. */
int ref_num_threads(void) { return omp_get_max_threads(); }
