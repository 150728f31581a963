// Immersed-boundary coupling (Sec. 2.3): spreading of vertex forces onto the
// lattice and interpolation of the lattice velocity back to the vertices,
// followed by explicit Euler advection (Sec. 2.6).
//
// Kernel: Peskin's 4-point function on nodes floor(X)-1 .. floor(X)+2 per
// axis (or the 2-point linear hat on floor(X), floor(X)+1); the 3-D weight
// is the product of the per-axis weights.  Periodic axes wrap; nodes past a
// wall receive no force and read the wall velocity.
//
// Spreading and interpolation are organised by tile: one work-group per 8^3
// tile walks the list of vertices whose stencil reaches the tile (built by
// the binning kernels).  Spreading accumulates in LDS as 2^-48 fixed-point
// int64 values; interpolation writes one partial sum per (vertex, tile) that
// a per-vertex pass adds up in a fixed order.
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

// Per-axis stencil of one vertex relative to a tile starting at t0: local
// node index inside the tile (-1 outside the tile or beyond a wall) and weight.
__device__ inline void axis_stencil(int base, float frac, int K, int n, int wall, int t0, int* l,
                                    float* w) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    l[k] = -1;
    w[k] = 0.f;
    if (k < K) {
      int p = base + k;
      bool in = true;
      if (wall) in = p >= 0 && p < n; else p = wrap(p, n);
      l[k] = (in && p >= t0 && p < t0 + kTile) ? p - t0 : -1;
      w[k] = stencil_w(K, frac, k);
    }
  }
}

// One work-group per tile; one thread per (vertex, tile) entry of the touch
// list: the thread evaluates its 3 x K axis weights once and adds the
// contributions of the stencil nodes inside the tile to the LDS accumulator.
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
  const int b = K == 4 ? -1 : 0;
  const int e0 = B.touch_ptr[t], e1 = B.touch_ptr[t + 1];
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int v = B.touch[e] >> 5;
    const int c = v / M.nv;
    const float* o = C.off + (int64_t)v * 3;
    const float* fv = C.force + (int64_t)v * 3;
    const float ox = o[0], oy = o[1], oz = o[2];
    const float fx = fv[0], fy = fv[1], fz = fv[2];
    const float flx = floorf(ox), fly = floorf(oy), flz = floorf(oz);
    int lx[4], ly[4], lz[4];
    float wx[4], wy[4], wz[4];
    axis_stencil(C.origin[3 * c + 0] + (int)flx + b, ox - flx, K, L.nx, L.bc[0] == 1, x0, lx, wx);
    axis_stencil(C.origin[3 * c + 1] + (int)fly + b, oy - fly, K, L.ny, L.bc[1] == 1, y0, ly, wy);
    axis_stencil(C.origin[3 * c + 2] + (int)flz + b, oz - flz, K, L.nz, L.bc[2] == 1, z0, lz, wz);
    for (int kz = 0; kz < K; ++kz) {
      if (lz[kz] < 0) continue;
      for (int ky = 0; ky < K; ++ky) {
        if (ly[ky] < 0) continue;
        const float wzy = wz[kz] * wy[ky];
        const int row = (lz[kz] * kTile + ly[ky]) * kTile;
        for (int kx = 0; kx < K; ++kx) {
          if (lx[kx] < 0) continue;
          const float w = wzy * wx[kx];
          const int li = row + lx[kx];
          atomicAdd((unsigned long long*)&acc[0][li],
                    (unsigned long long)__float2ll_rn(w * fx * (float)kFixScale));
          atomicAdd((unsigned long long*)&acc[1][li],
                    (unsigned long long)__float2ll_rn(w * fy * (float)kFixScale));
          atomicAdd((unsigned long long*)&acc[2][li],
                    (unsigned long long)__float2ll_rn(w * fz * (float)kFixScale));
        }
      }
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

// Interpolation, first half: one work-group per tile stages the tile's
// velocities in LDS; each (vertex, tile) entry sums w * u over its stencil
// nodes inside the tile and stores the partial sum in the vertex's slot.
__global__ __launch_bounds__(256) void k_interp_partials(Cells C, Mesh M, Lattice L, Bins B,
                                                         const float4* __restrict__ macro,
                                                         float4* __restrict__ partial) {
  __shared__ float4 su[kTile * kTile * kTile];
  const int t = blockIdx.x;
  const int tx = t % L.tx, ty = (t / L.tx) % L.ty, tz = t / (L.tx * L.ty);
  const int x0 = tx * kTile, y0 = ty * kTile, z0 = tz * kTile;
  const int e0 = B.touch_ptr[t], e1 = B.touch_ptr[t + 1];
  if (e0 == e1) return;
  for (int i = threadIdx.x; i < kTile * kTile * kTile; i += blockDim.x) {
    const int x = x0 + i % kTile, y = y0 + (i / kTile) % kTile, z = z0 + i / (kTile * kTile);
    su[i] = (x < L.nx && y < L.ny && z < L.nz) ? macro[((int64_t)z * L.ny + y) * L.nx + x]
                                                : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();
  const int K = L.kernel;
  const int b = K == 4 ? -1 : 0;
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int code = B.touch[e];
    const int v = code >> 5, j = code & 31;
    const int c = v / M.nv;
    const float* o = C.off + (int64_t)v * 3;
    const float ox = o[0], oy = o[1], oz = o[2];
    const float flx = floorf(ox), fly = floorf(oy), flz = floorf(oz);
    int lx[4], ly[4], lz[4];
    float wx[4], wy[4], wz[4];
    axis_stencil(C.origin[3 * c + 0] + (int)flx + b, ox - flx, K, L.nx, L.bc[0] == 1, x0, lx, wx);
    axis_stencil(C.origin[3 * c + 1] + (int)fly + b, oy - fly, K, L.ny, L.bc[1] == 1, y0, ly, wy);
    axis_stencil(C.origin[3 * c + 2] + (int)flz + b, oz - flz, K, L.nz, L.bc[2] == 1, z0, lz, wz);
    float ux = 0.f, uy = 0.f, uz = 0.f;
    for (int kz = 0; kz < K; ++kz) {
      if (lz[kz] < 0) continue;
      for (int ky = 0; ky < K; ++ky) {
        if (ly[ky] < 0) continue;
        const float wzy = wz[kz] * wy[ky];
        const int row = (lz[kz] * kTile + ly[ky]) * kTile;
        for (int kx = 0; kx < K; ++kx) {
          if (lx[kx] < 0) continue;
          const float w = wzy * wx[kx];
          const float4 q = su[row + lx[kx]];
          ux += w * q.x;
          uy += w * q.y;
          uz += w * q.z;
        }
      }
    }
    partial[(int64_t)v * L.max_touch + j] = make_float4(ux, uy, uz, 0.f);
  }
}

// Interpolation, second half, and explicit Euler advection: one thread per
// vertex sums its tile partials in slot order (fixed, so the result is
// reproducible), adds stencil nodes beyond a wall at the wall velocity, and
// moves the vertex.
__global__ __launch_bounds__(256) void k_advect(Cells C, Mesh M, Lattice L, Bins B,
                                                const float4* __restrict__ partial,
                                                int* __restrict__ flags) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= (int64_t)C.n * M.nv) return;
  float Ux = 0.f, Uy = 0.f, Uz = 0.f;
  for (int j = 0; j < L.max_touch; ++j) {
    if (B.touch_tile[v * L.max_touch + j] < 0) break;
    const float4 q = partial[v * L.max_touch + j];
    Ux += q.x;
    Uy += q.y;
    Uz += q.z;
  }
  float* o = C.off + v * 3;
  const float ox = o[0], oy = o[1], oz = o[2];
  if (L.wall_axis >= 0) {
    // the other two axes' weights sum to one, so a node layer beyond the
    // wall contributes its axis weight times the wall velocity
    const int d = L.wall_axis;
    const int c = (int)(v / M.nv);
    const int K = L.kernel;
    const float od = d == 0 ? ox : (d == 1 ? oy : oz);
    const float fl = floorf(od);
    const int n = d == 0 ? L.nx : (d == 1 ? L.ny : L.nz);
    const int base = C.origin[3 * c + d] + (int)fl + (K == 4 ? -1 : 0);
    float wlo = 0.f, whi = 0.f;
    for (int k = 0; k < K; ++k) {
      const int p = base + k;
      if (p < 0) wlo += stencil_w(K, od - fl, k);
      if (p >= n) whi += stencil_w(K, od - fl, k);
    }
    Ux += wlo * L.ulo[0] + whi * L.uhi[0];
    Uy += wlo * L.ulo[1] + whi * L.uhi[1];
    Uz += wlo * L.ulo[2] + whi * L.uhi[2];
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

hipError_t launch_interp_advect(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                                const float4* macro, float4* partial, int* flags, hipStream_t s) {
  const int64_t n = (int64_t)c.n * m.nv;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_interp_partials, dim3(L.ntiles), dim3(256), 0, s, c, m, L, b, macro,
                     partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_advect, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c, m, L, b,
                     partial, flags);
  return hipGetLastError();
}

}  // namespace hc
