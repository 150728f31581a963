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

// The collision VJP in FP64 from FP32 inputs (stored populations, force
// density, lam_u), with FP64 population cotangents.  The part of lam_f that
// d/d omega sees is its non-hydrodynamic (second-moment) part, which arises
// from differences between neighbouring sites' projections; an FP32 lam_f
// stores those projections to 7 digits and loses most of the differences in
// smooth regions, and an FP32 f_eq repeats the same rounding across a smooth
// flow, so both would bias the sum over every site and step.
__global__ __launch_bounds__(256) void k_adj_collide(const double* __restrict__ lam1,
                                                     double* __restrict__ lam0,
                                                     const float* __restrict__ h0,
                                                     const float* __restrict__ F,
                                                     const float* __restrict__ lamu,
                                                     float* __restrict__ lamF,
                                                     double* __restrict__ domega_part,
                                                     unsigned char* __restrict__ mask,
                                                     double* __restrict__ domega_in_part, Lattice L) {
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
    // cotangent of the post-collision values stored at this node; a value
    // stored for a bounce-back carries the wall term c rho
    double ls[kQ];
    double lrho = 0.0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      ls[i] = lam1[i * N + s];
      lrho += (double)lbm::wall_coeff(L, i, x, y, z) * ls[i];
    }
    // pre-collision populations, pulled as in the forward step
    float g[kQ];
    int64_t from[kQ];
    int qs[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      from[i] = lbm::pull_source(L, i, x, y, z, &qs[i]);
      g[i] = h0[qs[i] * N + from[i]];
    }
    const double fx = F[s], fy = F[N + s], fz = F[2 * N + s];
    double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      drho += g[i];
      jx += cx[i] * (double)g[i];
      jy += cy[i] * (double)g[i];
      jz += cz[i] * (double)g[i];
    }
    const double rho = 1.0 + drho, inv = 1.0 / rho;
    const double ux = (jx + 0.5 * fx) * inv, uy = (jy + 0.5 * fy) * inv, uz = (jz + 0.5 * fz) * inv;
    const double src = 1.0 - 0.5 * om;
    const double uu = ux * ux + uy * uy + uz * uz, uF = ux * fx + uy * fy + uz * fz;
    double A = 0.0, Bx = 0.0, By = 0.0, Bz = 0.0, Gx = 0.0, Gy = 0.0, Gz = 0.0, t = 0.0;
#pragma unroll
    for (int j = 0; j < kQ; ++j) {
      const double w = wq64(j);
      const double eu = cx[j] * ux + cy[j] * uy + cz[j] * uz;
      const double eF = cx[j] * fx + cy[j] * fy + cz[j] * fz;
      const double phi = 1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu;
      A += ls[j] * w * phi;                            // d f_eq / d rho at fixed u
      const double cu = om * w * rho, cs = src * w;
      // omega d f_eq/du + (1 - omega/2) dS/du
      Bx += ls[j] * (cu * (3.0 * cx[j] + 9.0 * eu * cx[j] - 3.0 * ux) + cs * (-3.0 * fx + 9.0 * eF * cx[j]));
      By += ls[j] * (cu * (3.0 * cy[j] + 9.0 * eu * cy[j] - 3.0 * uy) + cs * (-3.0 * fy + 9.0 * eF * cy[j]));
      Bz += ls[j] * (cu * (3.0 * cz[j] + 9.0 * eu * cz[j] - 3.0 * uz) + cs * (-3.0 * fz + 9.0 * eF * cz[j]));
      // (1 - omega/2) dS/dF at fixed u
      Gx += ls[j] * cs * (3.0 * (cx[j] - ux) + 9.0 * eu * cx[j]);
      Gy += ls[j] * cs * (3.0 * (cy[j] - uy) + 9.0 * eu * cy[j]);
      Gz += ls[j] * cs * (3.0 * (cz[j] - uz) + 9.0 * eu * cz[j]);
      // d h / d omega = -(f - f_eq) - S / 2
      const double geq = w * (drho + rho * (phi - 1.0));
      const double S = w * (3.0 * (eF - uF) + 9.0 * eu * eF);
      t += ls[j] * (-((double)g[j] - geq) - 0.5 * S);
    }
    if (inside) dom_in = t;
    else dom = t;
    A = om * A + lrho;
    Bx += lamu[s];
    By += lamu[N + s];
    Bz += lamu[2 * N + s];
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      lam0[qs[i] * N + from[i]] = (1.0 - om) * ls[i] + A +
                                 (Bx * (cx[i] - ux) + By * (cy[i] - uy) + Bz * (cz[i] - uz)) * inv;
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

__global__ __launch_bounds__(256) void k_adj_vertex(Cells C, Mesh M, Lattice L,
                                                    const float* __restrict__ lamX1,
                                                    const float4* __restrict__ macro,
                                                    const float* __restrict__ lamF,
                                                    float* __restrict__ lamFv,
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
__global__ __launch_bounds__(kAdjThreads) void k_adj_membrane(Cells C, Mesh M,
                                                              const float* __restrict__ lamFv,
                                                              float* __restrict__ lamX,
                                                              double* __restrict__ dk) {
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

}  // namespace

hipError_t launch_adj_collide(const double* lam1, double* lam0, const float* g0, const float* F,
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

hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace hc
