// Scalar and forward-mode dual arithmetic shared by the membrane force code.
// A Dual carries a value and its directional derivative; evaluating the
// membrane forces on Duals whose tangents are a vertex field t gives the
// forces and, in the tangent parts, the product of the force Jacobian with t.
#pragma once

#include <hip/hip_runtime.h>

namespace hc {

struct Dual {
  float v, d;
};

__device__ inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ inline Dual operator/(Dual a, Dual b) {
  const float r = 1.f / b.v;
  return {a.v * r, (a.d - a.v * r * b.d) * r};
}
__device__ inline Dual operator+(Dual a, float b) { return {a.v + b, a.d}; }
__device__ inline Dual operator-(Dual a, float b) { return {a.v - b, a.d}; }
__device__ inline Dual operator-(float a, Dual b) { return {a - b.v, -b.d}; }
__device__ inline Dual operator*(float a, Dual b) { return {a * b.v, a * b.d}; }
__device__ inline Dual operator*(Dual a, float b) { return {a.v * b, a.d * b}; }
__device__ inline Dual operator/(Dual a, float b) { return {a.v / b, a.d / b}; }
__device__ inline Dual operator/(float a, Dual b) { return {a / b.v, -a * b.d / (b.v * b.v)}; }

// Quotient in the force formulas: for floats the hardware reciprocal (1 ulp)
// and a product, within 2 ulp of the rounded quotient (the correctly
// rounded division costs about ten instructions), for duals the quotient
// above.
__device__ inline float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ inline Dual quot(Dual a, Dual b) { return a / b; }
__device__ inline Dual quot(Dual a, float b) { return a / b; }

__device__ inline float val(float a) { return a; }
__device__ inline float val(Dual a) { return a.v; }
__device__ inline float tan_(float) { return 0.f; }
__device__ inline float tan_(Dual a) { return a.d; }

__device__ inline float sqrt_(float a) { return sqrtf(a); }
__device__ inline Dual sqrt_(Dual a) {
  const float s = sqrtf(a.v);
  return {s, 0.5f * a.d / s};
}
__device__ inline float rsqrt_(float a) { return rsqrtf(a); }
__device__ inline Dual rsqrt_(Dual a) {
  const float r = rsqrtf(a.v);
  return {r, -0.5f * a.d * r * r * r};
}
__device__ inline float atan2_(float y, float x) { return atan2f(y, x); }
__device__ inline Dual atan2_(Dual y, Dual x) {
  return {atan2f(y.v, x.v), (x.v * y.d - y.v * x.d) / (x.v * x.v + y.v * y.v)};
}

template <class T>
struct V3 {
  T x, y, z;
};
template <class T>
__device__ inline V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T>
__device__ inline V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T, class S>
__device__ inline V3<T> operator*(S s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T>
__device__ inline T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T>
__device__ inline V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

}  // namespace hc
