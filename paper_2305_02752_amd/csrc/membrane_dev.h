// Membrane constitutive forces (Sec. 2.3: F_total = F_link + F_bend +
// F_area + F_volume, linear at small and strongly non-linear at large
// deformation, relative to the stress-free rest shape).
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
// The per-element force formulas are templates over the scalar type: float
// for the forward step, Dual for the Jacobian-vector products of the adjoint.
//
// Work per cell, element-parallel with no per-vertex table walks:
//  1. the cell's vertex offsets are staged in LDS;
//  2. per triangle: cell area and volume accumulated in float64 (the volume
//     is a sum of 1280 signed terms whose relative change of 1e-4..1e-2
//     drives F_volume) and reduced across threads in a fixed order;
//  3. per triangle, edge and hinge: force contributions to its vertices
//     added to a per-vertex LDS accumulator in 2^-40 fixed point -- integer
//     addition is associative, so the forces are bitwise reproducible;
//  4. per vertex: accumulator + traction written out.
#pragma once

#include "common.h"
#include "dual.h"

namespace hc {
namespace mem {

constexpr float kTauLink = 3.0f;
constexpr float kTauBend = 0.52359877559829887f;  // pi / 6
constexpr float kClamp = 0.99f;

using f3 = V3<float>;
__device__ inline f3 ld3(const float* p, int i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }

// g(s) = s + s / (lim^2 - s^2), argument clamped to +-0.99 lim (constant,
// zero derivative, beyond the clamp).
__device__ inline float nonlin(float s, float lim) {
  const float m = kClamp * lim;
  s = fminf(fmaxf(s, -m), m);
  return s + quot(s, lim * lim - s * s);
}
__device__ inline Dual nonlin(Dual s, float lim) {
  const float m = kClamp * lim;
  if (s.v > m || s.v < -m) return {nonlin(s.v, lim), 0.f};
  return s + s / (lim * lim - s * s);
}

// Link force on i (the force on j is its negative).
template <class T>
__device__ inline V3<T> link_force(V3<T> xi, V3<T> xj, float L0, float kl) {
  const V3<T> d = xj - xi;
  const T L = sqrt_(dot(d, d));
  return quot(kl * nonlin(quot(L - L0, L0), kTauLink), L) * d;
}

// Area and volume forces on the three vertices of triangle (a, b, c):
// for (v, j, k), dA/dx_v = n_hat x (x_k - x_j) / 2 and 6 dV/dx_v = x_j x x_k.
template <class T>
__device__ inline void tri_forces(V3<T> xa, V3<T> xb, V3<T> xc, T ca, T cv, V3<T>& fa, V3<T>& fb,
                                  V3<T>& fc) {
  const V3<T> n = cross(xb - xa, xc - xa);
  const T h = 0.5f * ca * rsqrt_(dot(n, n));
  fa = h * cross(n, xc - xb) + cv * cross(xb, xc);
  fb = h * cross(n, xa - xc) + cv * cross(xc, xa);
  fc = h * cross(n, xb - xa) + cv * cross(xa, xb);
}

// Bending forces of hinge (i, j, k, l): edge i->j in (i, j, k), j->i in
// (j, i, l).  theta = atan2((n1 x n2).e, n1.n2) is positive on a convex fold;
// d theta/dx moves the wings along their face normals and gives the edge
// vertices the complementary shares, so the four gradients sum to zero.
template <class T>
__device__ inline void hinge_forces(V3<T> xi, V3<T> xj, V3<T> xk, V3<T> xl, float theta0, float kb,
                                    V3<T>& fi, V3<T>& fj, V3<T>& fk, V3<T>& fl) {
  const V3<T> e = xj - xi;
  const V3<T> n1 = cross(e, xk - xi);
  const V3<T> n2 = cross(xi - xj, xl - xj);
  const T n1s = dot(n1, n1), n2s = dot(n2, n2), el2 = dot(e, e);
  const T r1 = rsqrt_(n1s), r2 = rsqrt_(n2s), re = rsqrt_(el2);
  const T theta = atan2_(dot(cross(r1 * n1, r2 * n2), re * e), r1 * r2 * dot(n1, n2));
  const T m = -kb * nonlin(theta - theta0, kTauBend);
  const T el = el2 * re;
  const V3<T> gk = quot(-el, n1s) * n1;
  const V3<T> gl = quot(-el, n2s) * n2;
  const T ak = quot(dot(xk - xi, e), el2), al = quot(dot(xl - xi, e), el2);
  fk = m * gk;
  fl = m * gl;
  fi = m * ((ak - 1.f) * gk + (al - 1.f) * gl);
  fj = m * ((-ak) * gk + (-al) * gl);
}

__device__ inline void add_force(long long* acc, int v, f3 f) {
  fix_add3(&acc[3 * v], &acc[3 * v + 1], &acc[3 * v + 2], f.x * kFixScaleF, f.y * kFixScaleF,
           f.z * kFixScaleF);
}

// Area and volume terms of triangle t (FP64): the triangle's area and its
// signed volume with the origin.
__device__ inline void tri_area_volume(const Mesh& M, const float* sp, int t, double& a, double& v) {
  const f3 xa = ld3(sp, M.tri[3 * t]), xb = ld3(sp, M.tri[3 * t + 1]), xc = ld3(sp, M.tri[3 * t + 2]);
  const double ax = xa.x, ay = xa.y, az = xa.z, bx = xb.x, by = xb.y, bz = xb.z;
  const double cx = xc.x, cy = xc.y, cz = xc.z;
  const double ux = bx - ax, uy = by - ay, uz = bz - az, vx = cx - ax, vy = cy - ay, vz = cz - az;
  const double nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
  a = 0.5 * sqrt(nx * nx + ny * ny + nz * nz);
  v = (ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx)) / 6.0;
}

// Forces on one cell with `nthr` cooperating threads (thread `tid`).
// acc: LDS [nv][3] int64, sp: LDS [nv][3] float (red: unused).  Writes
// area/volume (float64) and the per-vertex forces.  With off == nullptr the
// caller has already staged the offsets in sp.
__device__ inline void membrane_cell(const Mesh& M, const float* __restrict__ off,
                                     const float* __restrict__ k4, const float* trac,
                                     float* __restrict__ out, double* area, double* volume,
                                     long long* acc, float* sp, double* red, int tid, int nthr) {
  (void)red;
  if (off)
    for (int i = tid; i < 3 * M.nv; i += nthr) sp[i] = off[i];
  __syncthreads();
  // 1. Area and volume (FP64) over chunks of 64 triangles: lane i of a wave
  //    takes triangle 64 c + i of chunk c, the chunk is reduced by a fixed
  //    butterfly, and the chunk sums are added in chunk order, so the result
  //    does not depend on how many threads share the cell (the per-cell
  //    kernel widens its work-group when the cells are few).  The chunk sums
  //    are parked in the accumulator, free until the forces accumulate.
  double* cs = reinterpret_cast<double*>(acc);
  const int lane = tid & (kWave - 1), wv = tid / kWave, nw = nthr > kWave ? nthr / kWave : 1;
  const int nchunk = (M.nt + kWave - 1) / kWave;
  for (int ch = wv; ch < nchunk; ch += nw) {
    double a = 0.0, v = 0.0;
    if (ch * kWave + lane < M.nt) tri_area_volume(M, sp, ch * kWave + lane, a, v);
    for (int m = kWave / 2; m > 0; m >>= 1) {
      a += __shfl_xor(a, m);
      v += __shfl_xor(v, m);
    }
    if (lane == 0) {
      cs[2 * ch] = a;
      cs[2 * ch + 1] = v;
    }
  }
  __syncthreads();
  double A = 0.0, V = 0.0;
  for (int ch = 0; ch < nchunk; ++ch) {
    A += cs[2 * ch];
    V += cs[2 * ch + 1];
  }
  if (tid == 0) {
    *area = A;
    *volume = V;
  }
  __syncthreads();   // every thread has read the chunk sums
  for (int i = tid; i < 3 * M.nv; i += nthr) acc[i] = 0;
  __syncthreads();
  const float kl = k4[0], kb = k4[1], ka = k4[2], kv = k4[3];
  const float ca = -ka * (float)((A - M.A0) / M.A0);        // F_area = ca * dA/dx
  const float cv = -kv * (float)((V - M.V0) / M.V0) / 6.f;  // F_vol  = cv * 6 dV/dx
  // 2. One pass over the hinges (one per edge, same index): the edge's link
  //    force, the bending forces of its two triangles, and the area/volume
  //    forces of the triangle(s) it evaluates (each triangle with exactly
  //    one hinge); the four vertices' sums go to the fixed-point
  //    accumulator once each.
  for (int h = tid; h < M.nh; h += nthr) {
    const int p = M.hinge_v[4 * h], q = M.hinge_v[4 * h + 1];
    const int k = M.hinge_v[4 * h + 2], l = M.hinge_v[4 * h + 3];
    const f3 xp = ld3(sp, p), xq = ld3(sp, q), xk = ld3(sp, k), xl = ld3(sp, l);
    const f3 fe = link_force<float>(xp, xq, M.L0[h], kl);
    f3 Fp, Fq, Fk, Fl;
    hinge_forces<float>(xp, xq, xk, xl, M.theta0[h], kb, Fp, Fq, Fk, Fl);
    Fp = Fp + fe;
    Fq = Fq + -1.f * fe;
    const int own = M.hinge_own[h];
    if (own & 1) {
      f3 fa, fb, fc;
      tri_forces<float>(xp, xq, xk, ca, cv, fa, fb, fc);
      Fp = Fp + fa;
      Fq = Fq + fb;
      Fk = Fk + fc;
    }
    if (own & 2) {
      f3 fa, fb, fc;
      tri_forces<float>(xq, xp, xl, ca, cv, fa, fb, fc);
      Fq = Fq + fa;
      Fp = Fp + fb;
      Fl = Fl + fc;
    }
    add_force(acc, k, Fk);
    add_force(acc, l, Fl);
    add_force(acc, p, Fp);
    add_force(acc, q, Fq);
  }
  __syncthreads();

  for (int v = tid; v < M.nv; v += nthr) {
    f3 F = {(float)((double)acc[3 * v] * kFixInv), (float)((double)acc[3 * v + 1] * kFixInv),
            (float)((double)acc[3 * v + 2] * kFixInv)};
    if (trac) F = F + (M.pole[v] * M.inv_npole) * f3{trac[0], trac[1], trac[2]};
    out[3 * v] = F.x;
    out[3 * v + 1] = F.y;
    out[3 * v + 2] = F.z;
  }
}

}  // namespace mem
}  // namespace hc
