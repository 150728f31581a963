// Hand-written reverse mode of the coupled step (cotangent "lam" of every
// state variable), used to differentiate a cell-shape loss with respect to
// the membrane stiffnesses and the relaxation time.
//
// The lattice state is the stored post-collision field h (pull form).  One
// forward step n maps (h^n, X^n) to (h^{n+1}, X^{n+1}) through
//   F_v = Fmem(X; k) + T                      (Sec. 2.3 force sum)
//   F(x) = g + sum_v F_v delta(x - X_v)       (Sec. 2.3 spreading)
//   f = pull(h^n)                             (streaming, bounce-back)
//   rho, u = moments(f, F)                    (Sec. 2.2, half force in u)
//   U_v = sum_x u(x) delta(x - X_v)           (Sec. 2.3 interpolation)
//   h^{n+1} = f - omega (f - f_eq) + (1 - omega/2) S(u, F) + c rho
//     (c: moving-wall coefficient of populations leaving through a wall)
//   X^{n+1} = X^n + U                          (Sec. 2.6 Euler)
// Its transpose, given lam_h^{n+1} and lam_X^{n+1}, is evaluated by:
//   spread of lam_U = lam_X^{n+1}        -> lam_u(x)        (k_spread, reused)
//   k_adj_collide: the collision VJP at each node from its own lam_h^{n+1}
//     -> lam_f, lam_F(x), and d/d omega partial sums (kept apart for the
//     sites inside cells, which relax at the interior rate); lam_f is then
//     scattered back to the pull sources (a bijection) as lam_h^n;
//   k_adj_vertex: lam_{F_v} = sum_x lam_F(x) delta, plus the kernel-gradient
//     terms sum_x (lam_U.u(x) + F_v.lam_F(x)) grad delta for lam_X;
//   k_adj_membrane: lam_X += (dF_v/dX) lam_{F_v} by forward-mode duals (the
//     force is minus an energy gradient, so its Jacobian is symmetric), and
//     dL/dk_j += sum_v lam_{F_v} . F_v^(j) / k_j per force term.
// The IBM kernel must be the 4-point phi4 (C^1); the linear hat has no
// derivative at the nodes.
#include <algorithm>

#include "common.h"
#include "lbm_dev.h"
#include "membrane_dev.h"
#include "stencil.h"

namespace hc {
namespace {

using lbm::cx;
using lbm::cy;
using lbm::cz;
using lbm::opp;
using lbm::wq;

// Lattice weight of direction j, exact in FP64.
__device__ __forceinline__ double wq64(int j) { return j == 0 ? 1.0 / 3 : (j < 7 ? 1.0 / 18 : 1.0 / 36); }

// The collision VJP in FP64 from FP32 inputs: the stored populations, force
// density, lam_u and the population cotangents, which are stored in FP32.
// Every contraction, f_eq and the d/d omega sum are formed in FP64 (an FP32
// f_eq would repeat the same rounding across a smooth flow and bias the sum
// over every site and step).  FP32 storage of the cotangents moves the
// full-size gradient by about 1% of its difference from the oracle's and
// takes the kernel from 416 to 264 bytes per site.
// LT: the lattice record by value (single-box kernel) or by reference to
// global memory (batched kernel), so that neither puts it in scratch.
template <class LT>
__device__ __forceinline__ void adj_collide_body(const float* __restrict__ lam1, float* __restrict__ lam0,
                                                 const float* __restrict__ h0, const float* __restrict__ F,
                                                 const float* __restrict__ lamu, float* __restrict__ lamF,
                                                 double* __restrict__ domega_part,
                                                 unsigned char* __restrict__ mask,
                                                 double* __restrict__ domega_in_part, LT L) {
  __shared__ double red[1 + kVisClasses][4];
  const int64_t N = L.np;   // slots of every (tile-major) lattice field
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dom = 0.0, dom_in = 0.0;
  int cls = -1;   // viscosity class of an interior site
  int x, y, z;
  if (s < N && node_of(L, s, x, y, z)) {
    // a site inside a cell relaxes with the interior rate (the marks of
    // this step's positions, cleared once read)
    double om = L.omega;
    bool inside = false;
    if (mask) {
      const unsigned b = mask[s];
      if (b) {
        cls = 31 - __clz(b);
        om = L.omega_in[cls];
        inside = true;
        mask[s] = 0;
      }
    }
    // pre-collision populations, pulled as in the forward step.  The
    // tile-major site index is separable (site = Sx(x) + Sy(y) + Sz(z)), so
    // the pull source x - e_q of each direction is a sum of one part per
    // axis; a source past a wall is the opposite population at the node.
    const int xm = x == 0 ? L.nx - 1 : x - 1, xp = x == L.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? L.ny - 1 : y - 1, yp = y == L.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? L.nz - 1 : z - 1, zp = z == L.nz - 1 ? 0 : z + 1;
    const unsigned py = (unsigned)L.tx << 9, pz = py * (unsigned)L.ty;
    const unsigned SX[3] = {(unsigned)(((xp >> 3) << 9) | (xp & 7)), (unsigned)(((x >> 3) << 9) | (x & 7)),
                            (unsigned)(((xm >> 3) << 9) | (xm & 7))};
    const unsigned SY[3] = {(unsigned)(yp >> 3) * py + (unsigned)((yp & 7) << 3),
                            (unsigned)(y >> 3) * py + (unsigned)((y & 7) << 3),
                            (unsigned)(ym >> 3) * py + (unsigned)((ym & 7) << 3)};
    const unsigned SZ[3] = {(unsigned)(zp >> 3) * pz + (unsigned)((zp & 7) << 6),
                            (unsigned)(z >> 3) * pz + (unsigned)((z & 7) << 6),
                            (unsigned)(zm >> 3) * pz + (unsigned)((zm & 7) << 6)};
    const unsigned hl = SX[1] + SY[1] + SZ[1];   // this node (== s)
    const int wa = L.wall_axis;
    const int wc = wa == 0 ? x : (wa == 1 ? y : z), wn = wa == 0 ? L.nx : (wa == 1 ? L.ny : L.nz);
    const bool wlo = wa >= 0 && wc == 0, whi = wa >= 0 && wc == wn - 1;
    // element offset of the value pulled into direction q
    auto source = [&](int q) -> int64_t {
      const int ex = cx[q], ey = cy[q], ez = cz[q];
      const int ew = wa == 0 ? ex : (wa == 1 ? ey : ez);
      if ((ew == 1 && wlo) || (ew == -1 && whi)) return (int64_t)opp[q] * N + hl;
      const unsigned sx = ex > 0 ? SX[2] : (ex < 0 ? SX[0] : SX[1]);
      const unsigned sy = ey > 0 ? SY[2] : (ey < 0 ? SY[0] : SY[1]);
      const unsigned sz = ez > 0 ? SZ[2] : (ez < 0 ? SZ[0] : SZ[1]);
      return (int64_t)q * N + (sx + sy + sz);
    };
    // Every sum over the directions of the VJP is a contraction of the
    // cotangents l_j with 1, e_j or e_j e_j (weighted by w_j), or with the
    // pulled populations g_j, so one pass over the directions accumulates
    // the moments of g (drho, j), the moments M0 = sum w l, M1 = sum w l e,
    // M2 = sum w l e e, and sum l g; no direction's values are kept.  A value
    // stored for a bounce-back carries the wall term c rho.
    const double fx = F[s], fy = F[N + s], fz = F[2 * N + s];
    double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    double M0 = 0.0, M1x = 0.0, M1y = 0.0, M1z = 0.0, Pg = 0.0, lrho = 0.0;
    double Mxx = 0.0, Myy = 0.0, Mzz = 0.0, Mxy = 0.0, Mxz = 0.0, Myz = 0.0;
#pragma unroll
    for (int j = 0; j < kQ; ++j) {
      const double gj = h0[source(j)];
      const double l = lam1[j * N + s];
      // (terms of zero directions are left out, not added as zeros)
      drho += gj;
      if (cx[j] != 0) jx += cx[j] * gj;
      if (cy[j] != 0) jy += cy[j] * gj;
      if (cz[j] != 0) jz += cz[j] * gj;
      lrho += (double)lbm::wall_coeff(L, j, x, y, z) * l;
      Pg += l * gj;
      const double wl = wq64(j) * l;
      M0 += wl;
      if (cx[j] != 0) M1x += cx[j] * wl;
      if (cy[j] != 0) M1y += cy[j] * wl;
      if (cz[j] != 0) M1z += cz[j] * wl;
      if (cx[j] != 0) Mxx += wl;
      if (cy[j] != 0) Myy += wl;
      if (cz[j] != 0) Mzz += wl;
      if (cx[j] * cy[j] != 0) Mxy += (cx[j] * cy[j]) * wl;
      if (cx[j] * cz[j] != 0) Mxz += (cx[j] * cz[j]) * wl;
      if (cy[j] * cz[j] != 0) Myz += (cy[j] * cz[j]) * wl;
    }
    const double rho = 1.0 + drho, inv = 1.0 / rho;
    const double ux = (jx + 0.5 * fx) * inv, uy = (jy + 0.5 * fy) * inv, uz = (jz + 0.5 * fz) * inv;
    const double src = 1.0 - 0.5 * om;
    const double uu = ux * ux + uy * uy + uz * uz, uF = ux * fx + uy * fy + uz * fz;
    const double M2ux = Mxx * ux + Mxy * uy + Mxz * uz, M2uy = Mxy * ux + Myy * uy + Myz * uz,
                 M2uz = Mxz * ux + Myz * uy + Mzz * uz;
    const double M2Fx = Mxx * fx + Mxy * fy + Mxz * fz, M2Fy = Mxy * fx + Myy * fy + Myz * fz,
                 M2Fz = Mxz * fx + Myz * fy + Mzz * fz;
    const double M1u = M1x * ux + M1y * uy + M1z * uz, M1F = M1x * fx + M1y * fy + M1z * fz;
    const double uMu = ux * M2ux + uy * M2uy + uz * M2uz, uMF = ux * M2Fx + uy * M2Fy + uz * M2Fz;
    const double orho = om * rho;
    // d f_eq / d rho at fixed u: sum w l phi, phi = 1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u
    double A = M0 * (1.0 - 1.5 * uu) + 3.0 * M1u + 4.5 * uMu;
    // omega d f_eq/du + (1 - omega/2) dS/du
    double Bx = orho * (3.0 * M1x + 9.0 * M2ux - 3.0 * ux * M0) + src * (9.0 * M2Fx - 3.0 * fx * M0);
    double By = orho * (3.0 * M1y + 9.0 * M2uy - 3.0 * uy * M0) + src * (9.0 * M2Fy - 3.0 * fy * M0);
    double Bz = orho * (3.0 * M1z + 9.0 * M2uz - 3.0 * uz * M0) + src * (9.0 * M2Fz - 3.0 * fz * M0);
    // (1 - omega/2) dS/dF at fixed u
    const double Gx = src * (3.0 * M1x - 3.0 * ux * M0 + 9.0 * M2ux);
    const double Gy = src * (3.0 * M1y - 3.0 * uy * M0 + 9.0 * M2uy);
    const double Gz = src * (3.0 * M1z - 3.0 * uz * M0 + 9.0 * M2uz);
    // d h / d omega = -(f - f_eq) - S / 2, summed against l:
    // sum l f_eq = drho M0 + rho (3 M1.u + 9/2 u.M2.u - 3/2 u.u M0),
    // sum l S = 3 M1.F - 3 u.F M0 + 9 u.M2.F
    const double lfeq = drho * M0 + rho * (3.0 * M1u + 4.5 * uMu - 1.5 * uu * M0);
    const double lS = 3.0 * M1F - 3.0 * uF * M0 + 9.0 * uMF;
    const double t = -(Pg - lfeq) - 0.5 * lS;
    if (inside) dom_in = t;
    else dom = t;
    A = om * A + lrho;
    Bx += lamu[s];
    By += lamu[N + s];
    Bz += lamu[2 * N + s];
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      lam0[source(i)] = (float)((1.0 - om) * (double)lam1[i * N + s] + A +
                                (Bx * (cx[i] - ux) + By * (cy[i] - uy) + Bz * (cz[i] - uz)) * inv);
    lamF[s] = (float)(Gx + 0.5 * Bx * inv);
    lamF[N + s] = (float)(Gy + 0.5 * By * inv);
    lamF[2 * N + s] = (float)(Gz + 0.5 * Bz * inv);
  }
  // per-block sums for the plasma sites and for each viscosity class, in a
  // fixed order (each block owns its slots across steps)
  for (int k = -1; k < kVisClasses; ++k) {
    double v = k < 0 ? dom : (cls == k ? dom_in : 0.0);
    for (int m = kWave / 2; m > 0; m >>= 1) v += __shfl_xor(v, m);
    if ((threadIdx.x & (kWave - 1)) == 0) red[k + 1][threadIdx.x / kWave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 1 + kVisClasses) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += red[threadIdx.x][w];
    if (threadIdx.x == 0)
      domega_part[blockIdx.x] += t;
    else
      domega_in_part[(int64_t)(threadIdx.x - 1) * gridDim.x + blockIdx.x] += t;
  }
}

__global__ __launch_bounds__(256) void k_adj_collide(const float* __restrict__ lam1,
                                                     float* __restrict__ lam0,
                                                     const float* __restrict__ h0,
                                                     const float* __restrict__ F,
                                                     const float* __restrict__ lamu,
                                                     float* __restrict__ lamF,
                                                     double* __restrict__ domega_part,
                                                     unsigned char* __restrict__ mask,
                                                     double* __restrict__ domega_in_part, Lattice L) {
  adj_collide_body<Lattice>(lam1, lam0, h0, F, lamu, lamF, domega_part, mask, domega_in_part, L);
}

// Batched form: box blockIdx.y (the grid's x extent is every box's own).
__global__ __launch_bounds__(256) void k_adj_collide_multi(const AdjCollideArgs* __restrict__ many) {
  const AdjCollideArgs& a = many[blockIdx.y];
  adj_collide_body<const Lattice&>(a.lam1, a.lam0, a.h0, a.F, a.lamu, a.lamF, a.domega_part, a.mask,
                                   a.domega_in_part, a.L);
}

__device__ __forceinline__ void adj_vertex_body(Cells C, Mesh M, Lattice L,
                                                const float* __restrict__ lamX1,
                                                const float4* __restrict__ macro,
                                                const float* __restrict__ lamF, float* __restrict__ lamFv,
                                                float* __restrict__ lamX0) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= (int64_t)C.n * M.nv) return;
  const int c = (int)(v / M.nv);
  const int64_t N = L.np;
  const int n3[3] = {L.nx, L.ny, L.nz};
  int base[3];
  float w[3][4], dw[3][4];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float x = C.off[v * 3 + d];
    const float fl = floorf(x);
    base[d] = C.origin[3 * c + d] + (int)fl - 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      w[d][k] = phi4(x - fl + 1.f - (float)k);
      dw[d][k] = dphi4(x - fl + 1.f - (float)k);
    }
  }
  const float lux = lamX1[3 * v], luy = lamX1[3 * v + 1], luz = lamX1[3 * v + 2];
  const float Fx = C.force[3 * v], Fy = C.force[3 * v + 1], Fz = C.force[3 * v + 2];
  float sFx = 0.f, sFy = 0.f, sFz = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
  for (int kz = 0; kz < 4; ++kz) {
    int pz = base[2] + kz, side = 0;
    if (L.bc[2] == 1) side |= pz < 0 ? 1 : (pz >= n3[2] ? 2 : 0); else pz = wrap(pz, n3[2]);
    for (int ky = 0; ky < 4; ++ky) {
      int py = base[1] + ky, sy = 0;
      if (L.bc[1] == 1) sy = py < 0 ? 1 : (py >= n3[1] ? 2 : 0); else py = wrap(py, n3[1]);
      for (int kx = 0; kx < 4; ++kx) {
        int px = base[0] + kx, sx = 0;
        if (L.bc[0] == 1) sx = px < 0 ? 1 : (px >= n3[0] ? 2 : 0); else px = wrap(px, n3[0]);
        const int sd = side | sy | sx;
        float ux, uy, uz, lFx = 0.f, lFy = 0.f, lFz = 0.f;
        if (sd == 1) {
          ux = L.ulo[0]; uy = L.ulo[1]; uz = L.ulo[2];
        } else if (sd == 2) {
          ux = L.uhi[0]; uy = L.uhi[1]; uz = L.uhi[2];
        } else {
          const int64_t s = site_of(L, px, py, pz);
          const float4 q = macro[s];
          ux = q.x; uy = q.y; uz = q.z;
          lFx = lamF[s]; lFy = lamF[N + s]; lFz = lamF[2 * N + s];
        }
        const float W = w[0][kx] * w[1][ky] * w[2][kz];
        sFx += W * lFx;
        sFy += W * lFy;
        sFz += W * lFz;
        const float a = lux * ux + luy * uy + luz * uz + Fx * lFx + Fy * lFy + Fz * lFz;
        gx += a * dw[0][kx] * w[1][ky] * w[2][kz];
        gy += a * w[0][kx] * dw[1][ky] * w[2][kz];
        gz += a * w[0][kx] * w[1][ky] * dw[2][kz];
      }
    }
  }
  lamFv[3 * v] = sFx;
  lamFv[3 * v + 1] = sFy;
  lamFv[3 * v + 2] = sFz;
  lamX0[3 * v] = lux + gx;
  lamX0[3 * v + 1] = luy + gy;
  lamX0[3 * v + 2] = luz + gz;
}

__global__ __launch_bounds__(256) void k_adj_vertex(Cells C, Mesh M, Lattice L,
                                                    const float* __restrict__ lamX1,
                                                    const float4* __restrict__ macro,
                                                    const float* __restrict__ lamF,
                                                    float* __restrict__ lamFv,
                                                    float* __restrict__ lamX0) {
  adj_vertex_body(C, M, L, lamX1, macro, lamF, lamFv, lamX0);
}

__global__ __launch_bounds__(256) void k_adj_vertex_multi(const AdjVertexArgs* __restrict__ many) {
  const AdjVertexArgs& a = many[blockIdx.y];
  adj_vertex_body(a.C, a.M, a.L, a.lamX1, a.macro, a.lamF, a.lamFv, a.lamX0);
}

__device__ inline V3<Dual> ldd(const float* p, const float* t, int i) {
  return {{p[3 * i], t[3 * i]}, {p[3 * i + 1], t[3 * i + 1]}, {p[3 * i + 2], t[3 * i + 2]}};
}
__device__ inline void add_tangent(long long* acc, int v, V3<Dual> f) {
  fix_add3(&acc[3 * v], &acc[3 * v + 1], &acc[3 * v + 2], f.x.d * kFixScaleF, f.y.d * kFixScaleF,
           f.z.d * kFixScaleF);
}
__device__ inline double dotv(V3<Dual> f, const float* lam, int v) {
  return (double)f.x.v * lam[3 * v] + (double)f.y.v * lam[3 * v + 1] + (double)f.z.v * lam[3 * v + 2];
}
__device__ inline double dotf(mem::f3 f, const float* lam, int v) {
  return (double)f.x * lam[3 * v] + (double)f.y * lam[3 * v + 1] + (double)f.z * lam[3 * v + 2];
}

// Sum of 4 doubles over the kAdjThreads threads of a work-group: within each
// wave by shuffles, then across waves in a fixed order (reproducible).
template <int kAdjThreads>
__device__ inline void block_sum4(double (&v)[4], double* red) {
  for (int m = kWave / 2; m > 0; m >>= 1)
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] += __shfl_xor(v[j], m);
  const int w = threadIdx.x / kWave, nw = kAdjThreads / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
    for (int j = 0; j < 4; ++j) red[j * nw + w] = v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    v[j] = 0.0;
    for (int q = 0; q < nw; ++q) v[j] += red[j * nw + q];
  }
}

// One work-group of kAdjThreads per cell (wider when the cells are few, as
// for the forward per-cell kernel).  LDS: positions, tangents
// (= lam_{F_v}), int64 accumulator of the Jacobian-vector product.
template <int kAdjThreads>
__device__ __forceinline__ void adj_membrane_body(Cells C, Mesh M, const float* __restrict__ lamFv,
                                                  float* __restrict__ lamX, double* __restrict__ dk) {
  extern __shared__ long long lds64[];
  __shared__ double red[4 * kAdjThreads / kWave];
  long long* acc = lds64;
  float* sp = reinterpret_cast<float*>(lds64 + 3 * M.nv);
  float* st = sp + 3 * M.nv;
  const int c = blockIdx.x, tid = threadIdx.x;
  const int64_t b3 = (int64_t)c * M.nv * 3;
  for (int i = tid; i < 3 * M.nv; i += kAdjThreads) {
    sp[i] = C.off[b3 + i];
    st[i] = lamFv[b3 + i];
    acc[i] = 0;
  }
  __syncthreads();
  // area and volume with their directional derivatives (float64)
  double A = 0, V = 0, dA = 0, dV = 0;
  for (int t = tid; t < M.nt; t += kAdjThreads) {
    const int a = M.tri[3 * t], b = M.tri[3 * t + 1], e = M.tri[3 * t + 2];
    double x[3][3], dx[3][3];
    for (int d = 0; d < 3; ++d) {
      x[0][d] = sp[3 * a + d]; x[1][d] = sp[3 * b + d]; x[2][d] = sp[3 * e + d];
      dx[0][d] = st[3 * a + d]; dx[1][d] = st[3 * b + d]; dx[2][d] = st[3 * e + d];
    }
    double u[3], w[3], du[3], dw2[3];
    for (int d = 0; d < 3; ++d) {
      u[d] = x[1][d] - x[0][d];
      w[d] = x[2][d] - x[0][d];
      du[d] = dx[1][d] - dx[0][d];
      dw2[d] = dx[2][d] - dx[0][d];
    }
    const double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    const double dn[3] = {du[1] * w[2] - du[2] * w[1] + u[1] * dw2[2] - u[2] * dw2[1],
                          du[2] * w[0] - du[0] * w[2] + u[2] * dw2[0] - u[0] * dw2[2],
                          du[0] * w[1] - du[1] * w[0] + u[0] * dw2[1] - u[1] * dw2[0]};
    const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    A += 0.5 * nn;
    dA += 0.5 * (n[0] * dn[0] + n[1] * dn[1] + n[2] * dn[2]) / nn;
    // V term: x0 . (x1 x x2) / 6 and its derivative
    auto trip = [](const double* p, const double* q, const double* r) {
      return p[0] * (q[1] * r[2] - q[2] * r[1]) + p[1] * (q[2] * r[0] - q[0] * r[2]) +
             p[2] * (q[0] * r[1] - q[1] * r[0]);
    };
    V += trip(x[0], x[1], x[2]) / 6.0;
    dV += (trip(dx[0], x[1], x[2]) + trip(x[0], dx[1], x[2]) + trip(x[0], x[1], dx[2])) / 6.0;
  }
  double av[4] = {A, V, dA, dV};
  block_sum4<kAdjThreads>(av, red);
  A = av[0];
  V = av[1];
  dA = av[2];
  dV = av[3];
  const float kl = C.k[4 * c], kb = C.k[4 * c + 1], ka = C.k[4 * c + 2], kv = C.k[4 * c + 3];
  const float a_rel = (float)((A - M.A0) / M.A0), v_rel = (float)((V - M.V0) / M.V0);
  const Dual ca = {-ka * a_rel, -ka * (float)(dA / M.A0)};
  const Dual cv = {-kv * v_rel / 6.f, -kv * (float)(dV / M.V0) / 6.f};
  double sl = 0, sb = 0, sa = 0, sv = 0;   // sum_v lam_{F_v} . F_v^(term) / k_term
  for (int t = tid; t < M.nt; t += kAdjThreads) {
    const int ia = M.tri[3 * t], ib = M.tri[3 * t + 1], ic = M.tri[3 * t + 2];
    V3<Dual> fa, fb, fc;
    mem::tri_forces<Dual>(ldd(sp, st, ia), ldd(sp, st, ib), ldd(sp, st, ic), ca, cv, fa, fb, fc);
    add_tangent(acc, ia, fa);
    add_tangent(acc, ib, fb);
    add_tangent(acc, ic, fc);
    mem::f3 pa, pb, pc;
    mem::tri_forces<float>(mem::ld3(sp, ia), mem::ld3(sp, ib), mem::ld3(sp, ic), -a_rel, 0.f, pa, pb, pc);
    sa += dotf(pa, st, ia) + dotf(pb, st, ib) + dotf(pc, st, ic);
    mem::tri_forces<float>(mem::ld3(sp, ia), mem::ld3(sp, ib), mem::ld3(sp, ic), 0.f, -v_rel / 6.f, pa,
                           pb, pc);
    sv += dotf(pa, st, ia) + dotf(pb, st, ib) + dotf(pc, st, ic);
  }
  for (int e = tid; e < M.ne; e += kAdjThreads) {
    const int i = M.edge[2 * e], j = M.edge[2 * e + 1];
    const V3<Dual> f = mem::link_force<Dual>(ldd(sp, st, i), ldd(sp, st, j), M.L0[e], kl);
    add_tangent(acc, i, f);
    add_tangent(acc, j, -1.f * f);
    sl += (dotv(f, st, i) - dotv(f, st, j)) / kl;
  }
  for (int h = tid; h < M.nh; h += kAdjThreads) {
    const int i = M.hinge_v[4 * h], j = M.hinge_v[4 * h + 1];
    const int k = M.hinge_v[4 * h + 2], l = M.hinge_v[4 * h + 3];
    V3<Dual> fi, fj, fk, fl;
    mem::hinge_forces<Dual>(ldd(sp, st, i), ldd(sp, st, j), ldd(sp, st, k), ldd(sp, st, l), M.theta0[h],
                            kb, fi, fj, fk, fl);
    add_tangent(acc, i, fi);
    add_tangent(acc, j, fj);
    add_tangent(acc, k, fk);
    add_tangent(acc, l, fl);
    sb += (dotv(fi, st, i) + dotv(fj, st, j) + dotv(fk, st, k) + dotv(fl, st, l)) / kb;
  }
  double sk[4] = {sl, sb, sa, sv};
  block_sum4<kAdjThreads>(sk, red);
  sl = sk[0];
  sb = sk[1];
  sa = sk[2];
  sv = sk[3];
  if (tid == 0) {
    dk[4 * c] += sl;
    dk[4 * c + 1] += sb;
    dk[4 * c + 2] += sa;
    dk[4 * c + 3] += sv;
  }
  __syncthreads();
  for (int i = tid; i < 3 * M.nv; i += kAdjThreads) lamX[b3 + i] += (float)((double)acc[i] * kFixInv);
}

template <int kAdjThreads>
__global__ __launch_bounds__(kAdjThreads) void k_adj_membrane(Cells C, Mesh M,
                                                              const float* __restrict__ lamFv,
                                                              float* __restrict__ lamX,
                                                              double* __restrict__ dk) {
  adj_membrane_body<kAdjThreads>(C, M, lamFv, lamX, dk);
}

template <int kAdjThreads>
__global__ __launch_bounds__(kAdjThreads) void k_adj_membrane_multi(const AdjMembraneArgs* __restrict__ many) {
  const AdjMembraneArgs& a = many[blockIdx.y];
  adj_membrane_body<kAdjThreads>(a.C, a.M, a.lamFv, a.lamX, a.dk);
}

// Loss (D_A - D_A*)^2 + (D_T - D_T*)^2 of every cell from its extents along
// x and y, and the seed cotangent lam_X = dL/dX (extreme vertices only;
// ties go to the lower vertex index).  One wave per cell.
__global__ __launch_bounds__(64) void k_loss_seed(Cells C, Mesh M, const double* __restrict__ targets,
                                                  double* __restrict__ loss, float* __restrict__ lamX) {
  const int c = blockIdx.x, tid = threadIdx.x;
  const int64_t b = (int64_t)c * M.nv;
  double mx[2] = {-1e300, -1e300}, mn[2] = {1e300, 1e300};
  int imx[2] = {0, 0}, imn[2] = {0, 0};
  for (int v = tid; v < M.nv; v += kWave) {
    for (int d = 0; d < 2; ++d) {
      const double x = (double)C.origin[3 * c + d] + (double)C.off[(b + v) * 3 + d];
      if (x > mx[d]) { mx[d] = x; imx[d] = v; }
      if (x < mn[d]) { mn[d] = x; imn[d] = v; }
    }
  }
  for (int m = kWave / 2; m > 0; m >>= 1) {
    for (int d = 0; d < 2; ++d) {
      const double omx = __shfl_xor(mx[d], m), omn = __shfl_xor(mn[d], m);
      const int oimx = __shfl_xor(imx[d], m), oimn = __shfl_xor(imn[d], m);
      if (omx > mx[d] || (omx == mx[d] && oimx < imx[d])) { mx[d] = omx; imx[d] = oimx; }
      if (omn < mn[d] || (omn == mn[d] && oimn < imn[d])) { mn[d] = omn; imn[d] = oimn; }
    }
  }
  for (int i = tid; i < 3 * M.nv; i += kWave) lamX[b * 3 + i] = 0.f;
  __syncthreads();
  if (tid == 0) {
    const double ea = (mx[0] - mn[0]) - targets[2 * c], et = (mx[1] - mn[1]) - targets[2 * c + 1];
    loss[c] = ea * ea + et * et;
    lamX[(b + imx[0]) * 3 + 0] += (float)(2.0 * ea);
    lamX[(b + imn[0]) * 3 + 0] -= (float)(2.0 * ea);
    lamX[(b + imx[1]) * 3 + 1] += (float)(2.0 * et);
    lamX[(b + imn[1]) * 3 + 1] -= (float)(2.0 * et);
  }
}

__global__ void k_sum_parts(const double* __restrict__ parts, int n, double* __restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += parts[i];   // fixed order
    *out = t;
  }
}

__global__ void k_fill_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Record blockIdx.y of a batch of copies, strided over the x blocks: in
// 16-byte words when both addresses and the size are multiples of 16, else
// in 4-byte words.
__global__ __launch_bounds__(256) void k_copy_many(const CopyRec* __restrict__ recs) {
  const CopyRec r = recs[blockIdx.y];
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, step = (int64_t)gridDim.x * blockDim.x;
  const bool wide = ((reinterpret_cast<uintptr_t>(r.dst) | reinterpret_cast<uintptr_t>(r.src) | r.bytes) & 15) == 0;
  if (wide) {
    using v4u = unsigned __attribute__((ext_vector_type(4)));
    const v4u* src = static_cast<const v4u*>(r.src);
    v4u* dst = static_cast<v4u*>(r.dst);
    for (int64_t i = t0, n = r.bytes >> 4; i < n; i += step) dst[i] = src[i];
  } else {
    const unsigned* src = static_cast<const unsigned*>(r.src);
    unsigned* dst = static_cast<unsigned*>(r.dst);
    for (int64_t i = t0, n = r.bytes >> 2; i < n; i += step) dst[i] = src[i];
  }
}

}  // namespace

hipError_t launch_adj_collide(const float* lam1, float* lam0, const float* g0, const float* F,
                              const float* lamu, float* lamF, double* domega_part, unsigned char* mask,
                              double* domega_in_part, const Lattice& L, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_collide, dim3((unsigned)((L.np + 255) / 256)), dim3(256), 0, s, lam1, lam0,
                     g0, F, lamu, lamF, domega_part, mask, domega_in_part, L);
  return hipGetLastError();
}

hipError_t launch_adj_vertex(const Cells& c, const Mesh& m, const Lattice& L, const float* lamX1,
                             const float4* macro, const float* lamF, float* lamFv, float* lamX0,
                             hipStream_t s) {
  const int64_t n = (int64_t)c.n * m.nv;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_vertex, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c, m, L, lamX1,
                     macro, lamF, lamFv, lamX0);
  return hipGetLastError();
}

hipError_t launch_adj_membrane(const Cells& c, const Mesh& m, const float* lamFv, float* lamX, double* dk,
                               hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  const size_t lds = (size_t)m.nv * 3 * (8 + 4 + 4);
  if (c.n <= 64)
    hipLaunchKernelGGL(k_adj_membrane<1024>, dim3(c.n), dim3(1024), lds, s, c, m, lamFv, lamX, dk);
  else if (c.n <= 1024)
    hipLaunchKernelGGL(k_adj_membrane<512>, dim3(c.n), dim3(512), lds, s, c, m, lamFv, lamX, dk);
  else
    hipLaunchKernelGGL(k_adj_membrane<256>, dim3(c.n), dim3(256), lds, s, c, m, lamFv, lamX, dk);
  return hipGetLastError();
}

hipError_t launch_adj_collide_multi(const AdjCollideArgs& a0, const AdjCollideArgs* dev, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_collide_multi, dim3((unsigned)((a0.L.np + 255) / 256), (unsigned)n), dim3(256), 0, s,
                     dev);
  return hipGetLastError();
}

hipError_t launch_adj_vertex_multi(const AdjVertexArgs& a0, const AdjVertexArgs* dev, int n, hipStream_t s) {
  const int64_t nv = (int64_t)a0.C.n * a0.M.nv;
  if (n == 0 || nv == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_vertex_multi, dim3((unsigned)((nv + 255) / 256), (unsigned)n), dim3(256), 0, s, dev);
  return hipGetLastError();
}

hipError_t launch_adj_membrane_multi(const AdjMembraneArgs& a0, const AdjMembraneArgs* dev, int n,
                                     hipStream_t s) {
  if (n == 0 || a0.C.n == 0) return hipSuccess;
  const size_t lds = (size_t)a0.M.nv * 3 * (8 + 4 + 4);
  const dim3 grid((unsigned)a0.C.n, (unsigned)n);
  if (a0.C.n <= 64)
    hipLaunchKernelGGL(k_adj_membrane_multi<1024>, grid, dim3(1024), lds, s, dev);
  else if (a0.C.n <= 1024)
    hipLaunchKernelGGL(k_adj_membrane_multi<512>, grid, dim3(512), lds, s, dev);
  else
    hipLaunchKernelGGL(k_adj_membrane_multi<256>, grid, dim3(256), lds, s, dev);
  return hipGetLastError();
}

hipError_t launch_loss_seed(const Cells& c, const Mesh& m, const double* targets, double* loss,
                            float* lamX, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_loss_seed, dim3(c.n), dim3(kWave), 0, s, c, m, targets, loss, lamX);
  return hipGetLastError();
}

hipError_t launch_sum_parts(const double* parts, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, parts, n, out);
  return hipGetLastError();
}

hipError_t launch_copy_many(const CopyRec* dev, int n, int64_t max_bytes, hipStream_t s) {
  if (n <= 0 || max_bytes <= 0) return hipSuccess;
  const int64_t per_block = 256 * 16 * 4;   // four 16-byte words per thread before the grid strides
  const unsigned bx = (unsigned)std::min<int64_t>((max_bytes + per_block - 1) / per_block, 1024);
  hipLaunchKernelGGL(k_copy_many, dim3(bx, (unsigned)n), dim3(256), 0, s, dev);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace hc
