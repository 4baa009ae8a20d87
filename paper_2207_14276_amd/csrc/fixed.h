// 64-bit fixed-point accumulators with 2^-32 resolution.  Force-like sums in
// LDS and in the force buffers use them: integer atomics are fast on this
// hardware where float LDS atomics are not, and integer sums are exact, so a
// sum does not depend on the order of its terms.
#pragma once

#include <math.h>

namespace nnp {

constexpr float kFix = 4294967296.0f;              // 2^32
constexpr float kUnfix = 2.3283064365386963e-10f;  // 2^-32
constexpr float kFixLoMax = 4294967040.0f;         // largest float below 2^32

// floor(v * 2^32) as a 64-bit integer, for |v| < 2^31, built from two 32-bit
// halves: hi = floor(v) (exact) and lo = (v - hi) * 2^32.  The difference
// v - hi is exact for v >= 0 and for v <= -1; for -1 < v < 0 it is 1 + v
// rounded to float, so lo may be off by up to 2^8 units (6e-8 absolute) and
// may round up to 2^32 itself, which is clamped to the largest float below
// it so that the conversion stays in range.  The result is a function of v
// alone (no dependence on summation order).
__host__ __device__ inline long long to_fix(float v) {
  const float hi = floorf(v);
  const float f = fminf((v - hi) * kFix, kFixLoMax);
  const unsigned lo = (unsigned)f;
  return (long long)(((unsigned long long)(unsigned)(int)hi << 32) | lo);
}
__host__ __device__ inline float from_fix(long long v) { return (float)v * kUnfix; }

}  // namespace nnp
