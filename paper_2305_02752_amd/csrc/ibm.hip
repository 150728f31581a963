// Immersed-boundary coupling (Sec. 2.3): spreading of vertex forces onto the
// lattice and interpolation of the lattice velocity back to the vertices,
// followed by explicit Euler advection (Sec. 2.6).
//
// Kernel: Peskin's 4-point function on nodes floor(X)-1 .. floor(X)+2 per
// axis (or the 2-point linear hat on floor(X), floor(X)+1); the 3-D weight
// is the product of the per-axis weights.  Periodic axes wrap; nodes past a
// wall receive no force and read the wall velocity.
//
// Spreading is gather-by-tile: one work-group per 8^3 tile walks the list of
// vertices whose stencil reaches the tile (built by the binning kernels) and
// accumulates their contributions in LDS as 2^-48 fixed-point int64 values.
// Integer addition is associative, so the result is bitwise independent of
// the order in which waves and lanes arrive -- no global atomics, no
// run-to-run drift.
#include "common.h"

namespace hc {
namespace {

__device__ inline float phi4(float r) {
  r = fabsf(r);
  if (r <= 1.f) return 0.125f * (3.f - 2.f * r + sqrtf(1.f + 4.f * r - 4.f * r * r));
  if (r < 2.f) return 0.125f * (5.f - 2.f * r - sqrtf(-7.f + 12.f * r - 4.f * r * r));
  return 0.f;
}

// Weight of stencil node k (0..K-1) for fractional position f in [0, 1).
__device__ inline float stencil_w(int K, float f, int k) {
  if (K == 4) return phi4(f + 1.f - (float)k);
  return k == 0 ? 1.f - f : f;
}

__device__ inline int wrap(int p, int n) {
  p %= n;
  return p < 0 ? p + n : p;
}

__global__ __launch_bounds__(256) void k_spread(Cells C, Mesh M, Lattice L, Bins B,
                                                float* __restrict__ F) {
  __shared__ long long acc[3][kTile * kTile * kTile];
  const int t = blockIdx.x;
  const int tx = t % L.tx, ty = (t / L.tx) % L.ty, tz = t / (L.tx * L.ty);
  const int x0 = tx * kTile, y0 = ty * kTile, z0 = tz * kTile;
  for (int i = threadIdx.x; i < kTile * kTile * kTile; i += blockDim.x) {
    acc[0][i] = 0;
    acc[1][i] = 0;
    acc[2][i] = 0;
  }
  __syncthreads();

  const int K = L.kernel;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;
  const int kx = K == 4 ? (lane & 3) : (lane & 1);
  const int ky = K == 4 ? ((lane >> 2) & 3) : ((lane >> 1) & 1);
  const int kz = K == 4 ? (lane >> 4) : (lane >> 2);
  const bool active = lane < K * K * K;
  const int b = K == 4 ? -1 : 0;
  const int e0 = B.touch_ptr[t], e1 = B.touch_ptr[t + 1];

  for (int e = e0 + wave; e < e1; e += nwaves) {
    const int v = __builtin_amdgcn_readfirstlane(B.touch[e]);
    const int c = v / M.nv;
    const float* o = C.off + (int64_t)v * 3;
    const float* fv = C.force + (int64_t)v * 3;
    const float ox = o[0], oy = o[1], oz = o[2];
    const float flx = floorf(ox), fly = floorf(oy), flz = floorf(oz);
    int px = C.origin[3 * c + 0] + (int)flx + b + kx;
    int py = C.origin[3 * c + 1] + (int)fly + b + ky;
    int pz = C.origin[3 * c + 2] + (int)flz + b + kz;
    bool ok = active;
    if (L.bc[0] == 1) ok = ok && px >= 0 && px < L.nx; else px = wrap(px, L.nx);
    if (L.bc[1] == 1) ok = ok && py >= 0 && py < L.ny; else py = wrap(py, L.ny);
    if (L.bc[2] == 1) ok = ok && pz >= 0 && pz < L.nz; else pz = wrap(pz, L.nz);
    ok = ok && px >= x0 && px < x0 + kTile && py >= y0 && py < y0 + kTile && pz >= z0 &&
         pz < z0 + kTile;
    if (ok) {
      const float w = stencil_w(K, ox - flx, kx) * stencil_w(K, oy - fly, ky) *
                      stencil_w(K, oz - flz, kz);
      const int li = ((pz - z0) * kTile + (py - y0)) * kTile + (px - x0);
      atomicAdd((unsigned long long*)&acc[0][li],
                (unsigned long long)__double2ll_rn((double)(w * fv[0]) * kFixScale));
      atomicAdd((unsigned long long*)&acc[1][li],
                (unsigned long long)__double2ll_rn((double)(w * fv[1]) * kFixScale));
      atomicAdd((unsigned long long*)&acc[2][li],
                (unsigned long long)__double2ll_rn((double)(w * fv[2]) * kFixScale));
    }
  }
  __syncthreads();

  const int64_t N = L.n;
  for (int i = threadIdx.x; i < kTile * kTile * kTile; i += blockDim.x) {
    const int lx = i % kTile, ly = (i / kTile) % kTile, lz = i / (kTile * kTile);
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    if (x >= L.nx || y >= L.ny || z >= L.nz) continue;
    const int64_t s = ((int64_t)z * L.ny + y) * L.nx + x;
    F[s] = L.g[0] + (float)((double)acc[0][i] * kFixInv);
    F[N + s] = L.g[1] + (float)((double)acc[1][i] * kFixInv);
    F[2 * N + s] = L.g[2] + (float)((double)acc[2][i] * kFixInv);
  }
}

__global__ __launch_bounds__(256) void k_interp_advect(Cells C, Mesh M, Lattice L,
                                                       const float* __restrict__ u,
                                                       int* __restrict__ flags) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= (int64_t)C.n * M.nv) return;
  const int c = (int)(v / M.nv);
  const int K = L.kernel;
  const int b = K == 4 ? -1 : 0;
  float* o = C.off + v * 3;
  const float ox = o[0], oy = o[1], oz = o[2];
  const float flx = floorf(ox), fly = floorf(oy), flz = floorf(oz);
  const float fx = ox - flx, fy = oy - fly, fz = oz - flz;
  const int bx = C.origin[3 * c + 0] + (int)flx + b;
  const int by = C.origin[3 * c + 1] + (int)fly + b;
  const int bz = C.origin[3 * c + 2] + (int)flz + b;
  float wx[4], wy[4], wz[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    wx[k] = k < K ? stencil_w(K, fx, k) : 0.f;
    wy[k] = k < K ? stencil_w(K, fy, k) : 0.f;
    wz[k] = k < K ? stencil_w(K, fz, k) : 0.f;
  }
  const int64_t N = L.n;
  float Ux = 0.f, Uy = 0.f, Uz = 0.f;
  for (int kz = 0; kz < K; ++kz) {
    int pz = bz + kz;
    int side_z = 0;
    if (L.bc[2] == 1) side_z = pz < 0 ? 1 : (pz >= L.nz ? 2 : 0); else pz = wrap(pz, L.nz);
    for (int ky = 0; ky < K; ++ky) {
      int py = by + ky;
      int side_y = 0;
      if (L.bc[1] == 1) side_y = py < 0 ? 1 : (py >= L.ny ? 2 : 0); else py = wrap(py, L.ny);
      for (int kx = 0; kx < K; ++kx) {
        int px = bx + kx;
        int side_x = 0;
        if (L.bc[0] == 1) side_x = px < 0 ? 1 : (px >= L.nx ? 2 : 0); else px = wrap(px, L.nx);
        const float w = wx[kx] * wy[ky] * wz[kz];
        const int side = side_x | side_y | side_z;
        float vx, vy, vz;
        if (side == 1) {
          vx = L.ulo[0]; vy = L.ulo[1]; vz = L.ulo[2];
        } else if (side == 2) {
          vx = L.uhi[0]; vy = L.uhi[1]; vz = L.uhi[2];
        } else {
          const int64_t s = ((int64_t)pz * L.ny + py) * L.nx + px;
          vx = u[s]; vy = u[N + s]; vz = u[2 * N + s];
        }
        Ux += w * vx;
        Uy += w * vy;
        Uz += w * vz;
      }
    }
  }
  const float nx = ox + Ux, ny = oy + Uy, nz = oz + Uz;
  if (!(isfinite(nx) && isfinite(ny) && isfinite(nz))) atomicOr(&flags[0], 1);
  float* vo = C.vel + v * 3;
  vo[0] = Ux;
  vo[1] = Uy;
  vo[2] = Uz;
  o[0] = nx;
  o[1] = ny;
  o[2] = nz;
}

}  // namespace

hipError_t launch_spread(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b, float* F,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_spread, dim3(L.ntiles), dim3(256), 0, s, c, m, L, b, F);
  return hipGetLastError();
}

hipError_t launch_interp_advect(const Cells& c, const Mesh& m, const Lattice& L, const float* u,
                                int* flags, hipStream_t s) {
  const int64_t n = (int64_t)c.n * m.nv;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_interp_advect, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c, m, L,
                     u, flags);
  return hipGetLastError();
}

}  // namespace hc
