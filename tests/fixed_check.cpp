// Host check of the fixed-point conversion used by the force accumulators:
// every value of a sweep converts in range, and the result is floor(v 2^32)
// exactly for v >= 0 and v <= -1, within 2^8 units for -1 < v < 0.
#define __host__
#define __device__
#include "../paper_2207_14276_amd/csrc/fixed.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

static long long exact_fix(float v) { return (long long)std::floor((double)v * 4294967296.0); }

int main() {
  std::vector<float> vals;
  // tiny negative values, where 1 + v rounds to 1
  for (double v = -3e-8; v < 0; v += 1e-10) vals.push_back((float)v);
  for (int k = 0; k < 200; ++k) vals.push_back(-std::ldexp(1.0f, -k / 4 - 1));
  // just below and above integers, both signs
  for (int n = -5000; n <= 5000; n += 7)
    for (int u = -3; u <= 3; ++u) vals.push_back(std::nextafter((float)n, u < 0 ? -1e9f : 1e9f) + 0.0f * u);
  for (int n = -2000; n <= 2000; ++n) {
    float x = (float)n;
    vals.push_back(std::nextafter(x, -1e30f));
    vals.push_back(x);
    vals.push_back(std::nextafter(x, 1e30f));
  }
  std::mt19937 g(7);
  std::uniform_real_distribution<float> U(-1.f, 1.f);
  for (int k = 0; k < 200000; ++k) vals.push_back(U(g) * std::ldexp(1.0f, (int)(g() % 60) - 40));
  vals.push_back(2147483520.0f);   // largest float below 2^31
  vals.push_back(-2147483648.0f);  // -2^31
  long long worst_neg = 0;
  int bad = 0;
  for (float v : vals) {
    if (!(std::fabs(v) < 2147483648.0f) && v != -2147483648.0f) continue;
    const long long got = nnp::to_fix(v), want = exact_fix(v);
    const long long err = std::llabs(got - want);
    if (v >= 0.f || v <= -1.f) {
      if (err != 0) {
        if (bad++ < 10) std::printf("inexact at %.9g: got %lld want %lld\n", v, got, want);
      }
    } else {
      if (err > worst_neg) worst_neg = err;
      if (err > 256) {
        if (bad++ < 10) std::printf("error %lld units at %.9g\n", err, v);
      }
    }
    // the round trip stays within float rounding of v
    const float back = nnp::from_fix(got);
    if (std::fabs((double)back - (double)v) > 1e-7 * std::fabs((double)v) + 6e-8) {
      if (bad++ < 10) std::printf("round trip %.9g -> %.9g\n", v, back);
    }
  }
  std::printf("values %zu worst error on (-1, 0): %lld units; failures %d\n", vals.size(), worst_neg, bad);
  return bad ? 1 : 0;
}
