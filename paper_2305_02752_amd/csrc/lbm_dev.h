// D3Q19 BGK collision with Guo forcing for one node, shared by the
// single-lattice and batched kernels (Sec. 2.2: LBGK update, moments,
// second-order equilibrium; forcing after Guo, Zheng & Shi 2002).
//
// Populations are shifted, g_i = f_i - w_i.  Returns the post-collision
// shifted values, the density and the velocity (which carries half the
// force).
#pragma once

#include "common.h"

namespace hc {
namespace lbm {

__device__ constexpr int cx[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int cy[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int cz[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
// Lattice weights and the odd-part coefficients k = 3 w, as FP32 constants
// chosen so that the moment identities of the collision hold exactly for the
// stored values: w_0 + 6 w_1 + 12 w_2 = 1 (mass) and 2 (k_1 + 4 k_2) = 1
// (momentum).  Rounding 1/3, 1/18, 1/36 and 3 w one by one leaves both sums
// off by ~1e-8, and the same constants repeat that error at every node and
// step: a flow's momentum then grows or decays by that fraction per step, a
// drift that dominated the FP32 error of long runs (about 6x the rest after
// 2000 steps of a wall-driven flow).  Each value is within 2 ulp of the exact
// weight: w_2 = fl(1/36) - 1 ulp, w_1 = 2 w_2, w_0 = 1 - 24 w_2 (exact),
// k_2 = fl(1/12), k_1 = 1/2 - 4 k_2 (exact).  The values are HC_W0..HC_K2
// (common.h; the host's moving-wall coefficients use them too).
__device__ constexpr float wq[kQ] = {HC_W0, HC_W1, HC_W1, HC_W1, HC_W1, HC_W1, HC_W1,
                                     HC_W2, HC_W2, HC_W2, HC_W2, HC_W2, HC_W2,
                                     HC_W2, HC_W2, HC_W2, HC_W2, HC_W2, HC_W2};
__device__ constexpr float kq[kQ] = {0.f,   HC_K1, HC_K1, HC_K1, HC_K1, HC_K1, HC_K1,
                                     HC_K2, HC_K2, HC_K2, HC_K2, HC_K2, HC_K2,
                                     HC_K2, HC_K2, HC_K2, HC_K2, HC_K2, HC_K2};
__device__ constexpr int opp[kQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

// g: shifted populations in, post-collision shifted populations out.
//
// Directions come in opposite pairs (a, a + 1) for odd a, e_{a+1} = -e_a.
// Within a pair the equilibrium and the Guo source split into a part even
// in e (the same for both) and a part odd in e (opposite signs):
//   f_eq = w [drho - 3/2 rho u.u + 9/2 rho (e.u)^2] +- 3 w rho (e.u),
//   S    = (1 - omega/2) w [9 (e.u)(e.F) - 3 u.F] +- 3 (1 - omega/2) w (e.F),
// so each pair is relaxed from one even and one odd term.
__device__ inline void collide(float (&g)[kQ], float fx, float fy, float fz, float omega,
                               float& rho, float& ux, float& uy, float& uz) {
  float drho = g[0], jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int a = 1; a < kQ; a += 2) {
    const float d = g[a] - g[a + 1];
    drho += g[a] + g[a + 1];
    jx += cx[a] * d;
    jy += cy[a] * d;
    jz += cz[a] * d;
  }
  rho = 1.f + drho;
  const float inv = 1.f / rho;
  ux = (jx + 0.5f * fx) * inv;
  uy = (jy + 0.5f * fy) * inv;
  uz = (jz + 0.5f * fz) * inv;
  const float src = 1.f - 0.5f * omega, keep = 1.f - omega;
  const float uu = ux * ux + uy * uy + uz * uz;
  const float uF = ux * fx + uy * fy + uz * fz;
  const float c0 = drho - 1.5f * rho * uu;   // f_eq / w at e = 0
  const float omr = omega * rho;
  // each constant multiplies last, so no product of two constants (a rounded
  // coefficient shared by every node) enters the moments
  g[0] = keep * g[0] + wq[0] * (omega * c0 - 3.f * (src * uF));
#pragma unroll
  for (int a = 1; a < kQ; a += 2) {
    const float eu = cx[a] * ux + cy[a] * uy + cz[a] * uz;
    const float eF = cx[a] * fx + cy[a] * fy + cz[a] * fz;
    const float even = wq[a] * (omega * (c0 + 4.5f * rho * eu * eu) + src * (9.f * eu * eF - 3.f * uF));
    const float odd = kq[a] * (omr * eu + src * eF);
    g[a] = keep * g[a] + (even + odd);
    g[a + 1] = keep * g[a + 1] + (even - odd);
  }
}

// Where population i leaving node (x, y, z) lands.  Periodic axes wrap; on
// the wall axis a population leaving the fluid returns to its own node in
// the opposite direction (half-way bounce-back), and *dw receives Ladd's
// moving-wall correction -6 w_i rho (e_i . u_wall) to add to it.
// Returns the destination population index; *dst the destination node.
struct Walls {
  int axis;                 // -1: none
  float lo[3], hi[3];       // lower / upper wall velocity
};

__device__ inline int stream_target(int i, int x, int y, int z, int nx, int ny, int nz,
                                    const Walls& W, float rho, int64_t* dst, float* dw) {
  const int wall_axis = W.axis;
  int xt = x + cx[i], yt = y + cy[i], zt = z + cz[i];
  int crossed = 0;  // 0 none, 1 lower wall, 2 upper wall
  if (wall_axis == 0 && cx[i] != 0) crossed = xt < 0 ? 1 : (xt >= nx ? 2 : 0);
  if (wall_axis == 1 && cy[i] != 0) crossed = yt < 0 ? 1 : (yt >= ny ? 2 : 0);
  if (wall_axis == 2 && cz[i] != 0) crossed = zt < 0 ? 1 : (zt >= nz ? 2 : 0);
  if (crossed) {
    const float uw = crossed == 1 ? cx[i] * W.lo[0] + cy[i] * W.lo[1] + cz[i] * W.lo[2]
                                  : cx[i] * W.hi[0] + cy[i] * W.hi[1] + cz[i] * W.hi[2];
    *dw = -2.f * kq[i] * rho * uw;
    *dst = ((int64_t)z * ny + y) * nx + x;
    return opp[i];
  }
  xt = xt < 0 ? xt + nx : (xt >= nx ? xt - nx : xt);
  yt = yt < 0 ? yt + ny : (yt >= ny ? yt - ny : yt);
  zt = zt < 0 ? zt + nz : (zt >= nz ? zt - nz : zt);
  *dw = 0.f;
  *dst = ((int64_t)zt * ny + yt) * nx + xt;
  return i;
}

// Pull form of streaming on the tile-major lattice.  The stored state h
// holds post-collision values; population q at node x before the next
// collision is h_q(x - e_q), or, when x - e_q lies beyond the wall, the
// opposite population stored at x itself (half-way bounce-back, whose
// moving-wall term was added when it was stored).  Returns the slot in h;
// *qs the population index.
__host__ __device__ inline int64_t pull_source(const Lattice& L, int q, int x, int y, int z,
                                               int* qs) {
  constexpr int ex[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  constexpr int ey[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  constexpr int ez[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  constexpr int eo[kQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  int xs = x - ex[q], ys = y - ey[q], zs = z - ez[q];
  const int wa = L.wall_axis;
  if ((wa == 0 && (xs < 0 || xs >= L.nx)) || (wa == 1 && (ys < 0 || ys >= L.ny)) ||
      (wa == 2 && (zs < 0 || zs >= L.nz))) {
    *qs = eo[q];
    return site_of(L, x, y, z);
  }
  xs = xs < 0 ? xs + L.nx : (xs >= L.nx ? xs - L.nx : xs);
  ys = ys < 0 ? ys + L.ny : (ys >= L.ny ? ys - L.ny : ys);
  zs = zs < 0 ? zs + L.nz : (zs >= L.nz ? zs - L.nz : zs);
  *qs = q;
  return site_of(L, xs, ys, zs);
}

// Which wall population q leaving node (x, y, z) crosses: 0 none, 1 the
// lower, 2 the upper one (x + e_q beyond the wall axis' range).
__device__ inline int wall_crossed(const Lattice& L, int q, int x, int y, int z) {
  const int wa = L.wall_axis;
  if (wa < 0) return 0;
  const int e = wa == 0 ? cx[q] : (wa == 1 ? cy[q] : cz[q]);
  const int p = (wa == 0 ? x : (wa == 1 ? y : z)) + e;
  const int n = wa == 0 ? L.nx : (wa == 1 ? L.ny : L.nz);
  return p < 0 ? 1 : (p >= n ? 2 : 0);
}

// Moving-wall coefficient of population q leaving node (x, y, z): when it
// crosses a wall, the value stored for the bounce-back is post + c rho with
// c = -6 w_q (e_q . u_wall) (Ladd); otherwise c = 0.
__device__ inline float wall_coeff(const Lattice& L, int q, int x, int y, int z) {
  const int side = wall_crossed(L, q, x, y, z);
  if (side == 0) return 0.f;
  const float* uw = side == 1 ? L.ulo : L.uhi;
  return -2.f * kq[q] * (cx[q] * uw[0] + cy[q] * uw[1] + cz[q] * uw[2]);
}

// Population q arriving at boundary node (x, y, z) across the z boundary of
// a Lees-Edwards lattice, completing the streaming of the previous step (so
// with that step's displacement): from the image below (e_z > 0, node on z = 0) or
// above (e_z < 0, node on z = nz - 1), whose boundary row is displaced by
// -Delta or +Delta along x and moves with -U or +U.  The source point
// x - e_x +- Delta falls between two nodes: all 19 stored populations of
// both are interpolated linearly, and the transferred population gets the
// Galilean change f_eq(rho, u -+ U) - f_eq(rho, u) with the density and
// velocity of the interpolated set.  (Shifted populations: the weights
// cancel from both the interpolation and the velocity.)
__device__ inline float le_pull(const Lattice& L, const float* __restrict__ h, int q, int x, int y) {
  const int64_t NP = L.np;
  const int ez = cz[q];
  const int zs = ez > 0 ? L.nz - 1 : 0;
  const float sign = ez > 0 ? -1.f : 1.f;
  int ys = y - cy[q];
  ys = ys < 0 ? ys + L.ny : (ys >= L.ny ? ys - L.ny : ys);
  const float pos = (float)(x - cx[q]) - sign * L.le_pull_delta;
  const float fl = floorf(pos);
  const float s = pos - fl;
  int x0 = (int)fl % L.nx;
  x0 = x0 < 0 ? x0 + L.nx : x0;
  const int x1 = x0 + 1 == L.nx ? 0 : x0 + 1;
  const int64_t a = site_of(L, x0, ys, zs), b = site_of(L, x1, ys, zs);
  float hq = 0.f, drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int j = 0; j < kQ; ++j) {
    const float v = (1.f - s) * h[j * NP + a] + s * h[j * NP + b];
    drho += v;
    jx += cx[j] * v;
    jy += cy[j] * v;
    jz += cz[j] * v;
    if (j == q) hq = v;
  }
  const float rho = 1.f + drho, inv = 1.f / rho;
  const float ux = jx * inv, uy = jy * inv, uz = jz * inv;
  const float vx = ux + sign * L.le_u;
  const float eu = cx[q] * ux + cy[q] * uy + cz[q] * uz;
  const float ev = cx[q] * vx + cy[q] * uy + cz[q] * uz;
  const float uu = ux * ux + uy * uy + uz * uz, vv = vx * vx + uy * uy + uz * uz;
  return hq + wq[q] * rho * (3.f * (ev - eu) + 4.5f * (ev * ev - eu * eu) - 1.5f * (vv - uu));
}

}  // namespace lbm
}  // namespace hc
