// The immersed-boundary stencil shared by every kernel that spreads or
// interpolates (Sec. 2.3): Peskin's 4-point function, its derivative (for
// the reverse sweep), the weight of stencil position k, and periodic index
// wrapping.  Stencil nodes of a vertex at x are floor(x) - 1 .. floor(x) + 2
// (4-point) or floor(x), floor(x) + 1 (the 2-point linear hat).
#pragma once

#include "common.h"

namespace hc {

// p mod n in [0, n).  Positions within one period of the range, which is
// every stencil position of a vertex near the lattice, take one compare and
// add; others the exact remainder.
__host__ __device__ inline int wrap(int p, int n) {
  int q = p < 0 ? p + n : (p >= n ? p - n : p);
  if (q < 0 || q >= n) {
    q = p % n;
    q = q < 0 ? q + n : q;
  }
  return q;
}

// floor(a / n) for 0 <= a < 2^31 and a quotient below 2^20, from a float
// reciprocal r of n (within one ulp): the float quotient is then within a
// quarter unit, so one exact correction makes it right.
__device__ inline int div_small(int a, int n, float r) {
  int q = (int)((float)a * r);
  const int m = a - q * n;
  q += m >= n ? 1 : 0;
  q -= m < 0 ? 1 : 0;
  return q;
}

__device__ inline float phi4(float r) {
  r = fabsf(r);
  if (r <= 1.f) return 0.125f * (3.f - 2.f * r + sqrtf(1.f + 4.f * r - 4.f * r * r));
  if (r < 2.f) return 0.125f * (5.f - 2.f * r - sqrtf(-7.f + 12.f * r - 4.f * r * r));
  return 0.f;
}

// d phi4 / dr.
__device__ inline float dphi4(float r) {
  const float a = fabsf(r), s = r < 0.f ? -1.f : 1.f;
  if (a <= 1.f) return s * 0.25f * (-1.f + (1.f - 2.f * a) / sqrtf(1.f + 4.f * a - 4.f * a * a));
  if (a < 2.f) return s * 0.25f * (-1.f - (3.f - 2.f * a) / sqrtf(-7.f + 12.f * a - 4.f * a * a));
  return 0.f;
}

// Weight of stencil position k (0..K-1) for fractional position f in [0, 1).
template <int K>
__device__ inline float stencil_w(float f, int k) {
  if (K == 4) return phi4(f + 1.f - (float)k);
  return k == 0 ? 1.f - f : f;
}

// A vertex coordinate held as the unevaluated sum hi + lo of two floats, moved
// by d.  hi + a is formed with its exact rounding error (Knuth's TwoSum), which
// becomes the new lo: a float position alone drops up to half an ulp per move,
// and when a vertex creeps at nearly constant speed the same rounding repeats
// every step, a drift that grows linearly with the step count.  Readers of the
// position use hi (within half an ulp of hi + lo).
__device__ __forceinline__ void move_compensated(float& hi, float& lo, float d) {
  const float a = d + lo;
  const float s = hi + a;
  const float bp = s - hi;
  lo = (hi - (s - bp)) + (a - bp);
  hi = s;
}

}  // namespace hc
