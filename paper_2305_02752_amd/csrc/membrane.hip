// Membrane constitutive forces, one wavefront per cell (Sec. 2.3:
// F_total = F_link + F_bend + F_area + F_volume, linear at small and strongly
// non-linear at large deformation, relative to the stress-free rest shape).
//
// Forms (the paper defers them to a reference it does not reproduce; these
// are minus the gradients of the energies below):
//   link   k_l L0 [s^2/2 - ln(1 - s^2/3^2)/2],          s = (L - L0)/L0
//   bend   k_b [d^2/2 - ln(1 - d^2/(pi/6)^2)/2],         d = theta - theta0
//   area   k_a A0 a^2/2,  a = (A - A0)/A0  (cell area)
//   volume k_v V0 v^2/2,  v = (V - V0)/V0  (cell volume)
// plus a pole traction +-F/32 on the 32 rest-frame x-extreme vertices.
// Non-linear arguments are clamped to +-0.99 of their poles.
//
// Layout of the work in the wave:
//  1. the cell's vertex offsets are staged in LDS;
//  2. per triangle: float32 normal into LDS, and the cell area and volume
//     accumulated in float64 (volume is a sum of 1280 signed terms whose
//     relative change of 1e-4..1e-2 drives F_volume) with a fixed-order
//     wave reduction;
//  3. per hinge: dihedral angle and bending magnitude into LDS;
//  4. per vertex: deterministic gather of link, area, volume and bending
//     terms over the vertex's own adjacency lists -- no atomics.
#include "common.h"

namespace hc {
namespace {

constexpr float kTauLink = 3.0f;
constexpr float kTauBend = 0.52359877559829887f;  // pi / 6
constexpr float kClamp = 0.99f;

struct f3 {
  float x, y, z;
};
__device__ inline f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline f3 operator*(float s, f3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline f3 cross(f3 a, f3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline f3 ld3(const float* p, int i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }

__device__ inline float nonlin(float s, float lim) {
  const float m = kClamp * lim;
  s = fminf(fmaxf(s, -m), m);
  return s + s / (lim * lim - s * s);
}

__global__ __launch_bounds__(64) void k_membrane(Cells C, Mesh M) {
  extern __shared__ float lds[];
  float* sp = lds;                 // [nv][3] positions (cell-local offsets)
  float* sN = sp + 3 * M.nv;       // [nt][3] unnormalised triangle normals
  float* sm = sN + 3 * M.nt;       // [nh]    bending magnitude -k_b g_b(d)
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const float* off = C.off + (int64_t)c * M.nv * 3;
  for (int i = lane; i < 3 * M.nv; i += kWave) sp[i] = off[i];
  __syncthreads();

  double A = 0.0, V = 0.0;
  for (int t = lane; t < M.nt; t += kWave) {
    const int a = M.tri[3 * t], b = M.tri[3 * t + 1], d = M.tri[3 * t + 2];
    const f3 xa = ld3(sp, a), xb = ld3(sp, b), xc = ld3(sp, d);
    const f3 n = cross(xb - xa, xc - xa);
    sN[3 * t] = n.x;
    sN[3 * t + 1] = n.y;
    sN[3 * t + 2] = n.z;
    const double ax = xa.x, ay = xa.y, az = xa.z, bx = xb.x, by = xb.y, bz = xb.z;
    const double cx = xc.x, cy = xc.y, cz = xc.z;
    const double ux = bx - ax, uy = by - ay, uz = bz - az, vx = cx - ax, vy = cy - ay, vz = cz - az;
    const double nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
    A += 0.5 * sqrt(nx * nx + ny * ny + nz * nz);
    V += (ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx)) / 6.0;
  }
  for (int m = kWave / 2; m > 0; m >>= 1) {
    A += __shfl_xor(A, m);
    V += __shfl_xor(V, m);
  }
  if (lane == 0) {
    C.area[c] = A;
    C.volume[c] = V;
  }
  const float kl = C.k[4 * c + 0], kb = C.k[4 * c + 1], ka = C.k[4 * c + 2], kv = C.k[4 * c + 3];
  const float ca = -ka * (float)((A - M.A0) / M.A0);        // force = ca * dA/dx
  const float cv = -kv * (float)((V - M.V0) / M.V0) / 6.f;  // force = cv * 6 dV/dx
  __syncthreads();

  for (int h = lane; h < M.nh; h += kWave) {
    const int i = M.hinge_v[4 * h], j = M.hinge_v[4 * h + 1];
    const f3 n1 = ld3(sN, M.hinge_t[2 * h]), n2 = ld3(sN, M.hinge_t[2 * h + 1]);
    const f3 e = ld3(sp, j) - ld3(sp, i);
    const float r1 = rsqrtf(dot(n1, n1)), r2 = rsqrtf(dot(n2, n2)), re = rsqrtf(dot(e, e));
    const float sn = dot(cross(r1 * n1, r2 * n2), re * e);
    const float cs = dot(r1 * n1, r2 * n2);
    const float theta = atan2f(sn, cs);
    sm[h] = -kb * nonlin(theta - M.theta0[h], kTauBend);
  }
  __syncthreads();

  const float* trac = C.traction ? C.traction + 3 * c : nullptr;
  for (int v = lane; v < M.nv; v += kWave) {
    const f3 xv = ld3(sp, v);
    f3 F = {0.f, 0.f, 0.f};
    for (int q = M.vlink_ptr[v]; q < M.vlink_ptr[v + 1]; ++q) {
      const f3 d = ld3(sp, M.vlink_j[q]) - xv;
      const float L = sqrtf(dot(d, d));
      const float L0 = M.vlink_L0[q];
      F = F + (kl * nonlin((L - L0) / L0, kTauLink) / L) * d;
    }
    for (int q = M.vtri_ptr[v]; q < M.vtri_ptr[v + 1]; ++q) {
      const int t = M.vtri[3 * q], j = M.vtri[3 * q + 1], k = M.vtri[3 * q + 2];
      const f3 xj = ld3(sp, j), xk = ld3(sp, k), n = ld3(sN, t);
      const float rn = rsqrtf(dot(n, n));
      F = F + (0.5f * ca * rn) * cross(n, xk - xj);
      F = F + cv * cross(xj, xk);
    }
    for (int q = M.vhinge_ptr[v]; q < M.vhinge_ptr[v + 1]; ++q) {
      const int h = M.vhinge[q] >> 2, role = M.vhinge[q] & 3;
      const int i = M.hinge_v[4 * h], j = M.hinge_v[4 * h + 1];
      const int k = M.hinge_v[4 * h + 2], l = M.hinge_v[4 * h + 3];
      const f3 xi = ld3(sp, i), e = ld3(sp, j) - xi;
      const f3 n1 = ld3(sN, M.hinge_t[2 * h]), n2 = ld3(sN, M.hinge_t[2 * h + 1]);
      const float el2 = dot(e, e), el = sqrtf(el2);
      const f3 gk = (-el / dot(n1, n1)) * n1;
      const f3 gl = (-el / dot(n2, n2)) * n2;
      f3 g;
      if (role == 2) {
        g = gk;
      } else if (role == 3) {
        g = gl;
      } else {
        const float ak = dot(ld3(sp, k) - xi, e) / el2;
        const float al = dot(ld3(sp, l) - xi, e) / el2;
        g = role == 0 ? (-(1.f - ak)) * gk + (-(1.f - al)) * gl : (-ak) * gk + (-al) * gl;
      }
      F = F + sm[h] * g;
    }
    if (trac) {
      const float p = M.pole[v] * M.inv_npole;
      F = F + p * f3{trac[0], trac[1], trac[2]};
    }
    float* out = C.force + ((int64_t)c * M.nv + v) * 3;
    out[0] = F.x;
    out[1] = F.y;
    out[2] = F.z;
  }
}

}  // namespace

hipError_t launch_membrane(const Cells& c, const Mesh& m, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  const size_t lds = (size_t)(3 * m.nv + 3 * m.nt + m.nh) * sizeof(float);
  hipLaunchKernelGGL(k_membrane, dim3(c.n), dim3(kWave), lds, s, c, m);
  return hipGetLastError();
}

}  // namespace hc
