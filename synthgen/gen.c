/* Host filler for the seeded synthetic inputs (SplitMix64, counter-based).
 * Holds no arithmetic of the matrix-multiplication method.  The value maps
 * are defined in synthgen/__init__.py; this file restates them in C so that
 * multi-gigabyte inputs can be written straight into (pinned) host buffers.
 * Element (r, c) uses logical index i = r * cols + c, whatever the ld. */
#include <stdint.h>
#include <math.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t at(uint64_t seed, uint64_t i) { return mix64(seed + (i + 1) * GAMMA); }

void synth_uniform_pm1_f32(uint64_t seed, int64_t rows, int64_t cols, int64_t ld, float* out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r)
    for (int64_t c = 0; c < cols; ++c) {
      uint64_t z = at(seed, (uint64_t)(r * cols + c));
      int64_t k = (int64_t)(z >> 40) - (1 << 23);
      out[r * ld + c] = (float)((double)k * 0x1p-23);
    }
}

void synth_int_range_f32(uint64_t seed, int64_t rows, int64_t cols, int64_t ld, int32_t lo,
                         int32_t hi, float* out) {
  uint64_t span = (uint64_t)((int64_t)hi - lo + 1);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r)
    for (int64_t c = 0; c < cols; ++c) {
      uint64_t z = at(seed, (uint64_t)(r * cols + c));
      out[r * ld + c] = (float)((int64_t)((z >> 32) % span) + lo);
    }
}

void synth_loguniform_f32(uint64_t seed, int64_t rows, int64_t cols, int64_t ld, int32_t emin,
                          int32_t emax, float* out) {
  uint64_t span = (uint64_t)((int64_t)emax - emin);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r)
    for (int64_t c = 0; c < cols; ++c) {
      uint64_t z = at(seed, (uint64_t)(r * cols + c));
      int octave = (int)((z >> 32) % span) + emin;
      double frac = (double)((z >> 8) & ((1u << 23) - 1)) * 0x1p-23;
      double v = ldexp(1.0 + frac, octave);
      out[r * ld + c] = (float)((z & 1) ? -v : v);
    }
}
