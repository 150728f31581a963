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
// the binning kernels).  Spreading accumulates in LDS as 2^-40 fixed-point
// int64 values; interpolation writes one partial sum per (vertex, tile) that
// a per-vertex pass adds up in a fixed order.
// Integer addition is associative, so the result is bitwise independent of
// the order in which waves and lanes arrive -- no global atomics, no
// run-to-run drift.
#include "ibm_dev.h"
#include "lbm_dev.h"

namespace hc {
namespace {

// Per-axis stencil of one vertex relative to a tile starting at t0: local
// node index inside the tile (-1 outside the tile or beyond a wall) and
// weight; the first node is floor(X) - 1 (K = 4) or floor(X) (K = 2).
template <int K>
__device__ inline void axis_stencil(int origin, float x, int n, int wall, int t0, int (&l)[K],
                                    float (&w)[K]) {
  const float fl = floorf(x);
  const int base = origin + (int)fl - (K == 4 ? 1 : 0);
  const float f = x - fl;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int p = base + k;
    bool in = true;
    if (wall) in = p >= 0 && p < n; else p = wrap(p, n);
    l[k] = (in && p >= t0 && p < t0 + kTile) ? p - t0 : -1;
    w[k] = stencil_w<K>(f, k);
  }
}

// Sheared periodic images (Lees-Edwards, z gradient / x flow): the image
// index of each z stencil position (floor of its unwrapped index / nz), and
// the x stencils of the vertex as seen from the first and last of them
// (x - m Delta).  Consecutive positions cross at most one boundary, so two
// x stencils cover all K.
template <int K>
struct LeStencil {
  int m[K];
  int ma, mb;
  int lxa[K], lxb[K];
  float wxa[K], wxb[K];
};

template <int K>
__device__ inline void le_stencil(const Lattice& L, int ox, float x, int oz, float zoff, int t0,
                                  LeStencil<K>& S);

// Rotate a K-entry stencil by r so that lanes holding nearby vertices visit
// different nodes at the same time (fewer LDS same-address conflicts).
template <int K>
__device__ inline void rotate(int (&l)[K], float (&w)[K], int r) {
  int l2[K];
  float w2[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int src = (k + r) & (K - 1);
    l2[k] = l[0];
    w2[k] = w[0];
#pragma unroll
    for (int q = 1; q < K; ++q) {
      if (src == q) {
        l2[k] = l[q];
        w2[k] = w[q];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    l[k] = l2[k];
    w[k] = w2[k];
  }
}

template <int K>
__device__ inline void le_stencil(const Lattice& L, int ox, float x, int oz, float zoff, int t0,
                                  LeStencil<K>& S) {
  const int bz = oz + (int)floorf(zoff) - (K == 4 ? 1 : 0);
#pragma unroll
  for (int k = 0; k < K; ++k) S.m[k] = floor_div(bz + k, L.nz);
  S.ma = S.m[0];
  S.mb = S.m[K - 1];
  axis_stencil<K>(ox, x - (float)S.ma * L.le_delta, L.nx, 0, t0, S.lxa, S.wxa);
  axis_stencil<K>(ox, x - (float)S.mb * L.le_delta, L.nx, 0, t0, S.lxb, S.wxb);
}

__device__ inline void tile_origin(const Lattice& L, int t, int& x0, int& y0, int& z0) {
  x0 = (t % L.tx) * kTile;
  y0 = ((t / L.tx) % L.ty) * kTile;
  z0 = (t / (L.tx * L.ty)) * kTile;
}

// acc += trunc(q) for contributions of 2^31 or more (out of line, rare).
// Node contributions are converted to fixed point by truncation in both
// paths, so which path an entry takes never changes an integer.
__device__ __noinline__ void spread_add_wide(long long* a0, long long* a1, long long* a2, float x, float y,
                                             float z) {
  atomicAdd((unsigned long long*)a0, (unsigned long long)(long long)x);
  atomicAdd((unsigned long long*)a1, (unsigned long long)(long long)y);
  atomicAdd((unsigned long long*)a2, (unsigned long long)(long long)z);
}

// Spread phase of one tile: one thread per (vertex, tile) entry of the
// tile's list; the thread evaluates its 3 x K axis weights once and adds the
// contributions of the stencil nodes inside the tile to the LDS accumulator
// acc[3][512] (zeroed by the caller, synchronised after).
template <int K, bool LE = false>
__device__ inline void spread_tile(const Cells& C, const Mesh& M, const Lattice& L, const Bins& B,
                                   const float* __restrict__ vec, int t, int x0, int y0, int z0,
                                   long long (*acc)[kTile * kTile * kTile]) {
  const int64_t e0 = (int64_t)t * B.cap;
  const int64_t e1 = e0 + min(B.touch_cnt[t], B.cap);
  const int rot = threadIdx.x;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int v = B.touch[e] >> 5;
    const int c = v / M.nv;
    const float* o = C.off + (int64_t)v * 3;
    const float* fv = vec + (int64_t)v * 3;
    const float fx = fv[0] * kFixScaleF, fy = fv[1] * kFixScaleF, fz = fv[2] * kFixScaleF;
    int lx[K], ly[K], lz[K];
    float wx[K], wy[K], wz[K];
    LeStencil<K> S;
    if (LE) {
      le_stencil<K>(L, C.origin[3 * c + 0], o[0], C.origin[3 * c + 2], o[2], x0, S);
      rotate<K>(S.lxa, S.wxa, rot);
      rotate<K>(S.lxb, S.wxb, rot);
    } else {
      axis_stencil<K>(C.origin[3 * c + 0], o[0], L.nx, L.bc[0] == 1, x0, lx, wx);
      rotate<K>(lx, wx, rot);
    }
    axis_stencil<K>(C.origin[3 * c + 1], o[1], L.ny, L.bc[1] == 1, y0, ly, wy);
    axis_stencil<K>(C.origin[3 * c + 2], o[2], L.nz, L.bc[2] == 1, z0, lz, wz);
    rotate<K>(ly, wy, rot >> 2);
    // the x stencil of the image z position kz lies in (sheared images only)
    auto pick_x = [&](int kz) {
      if (!LE) return;
      const bool a = S.m[kz] == S.ma;
#pragma unroll
      for (int kx = 0; kx < K; ++kx) {
        lx[kx] = a ? S.lxa[kx] : S.lxb[kx];
        wx[kx] = a ? S.wxa[kx] : S.wxb[kx];
      }
    };
    // weights are at most 1, so one test per entry decides whether every
    // node contribution fits the 32-bit conversion
    if (fmaxf(fabsf(fx), fmaxf(fabsf(fy), fabsf(fz))) < kFix32Max) {
#pragma unroll
      for (int kz = 0; kz < K; ++kz) {
        if (lz[kz] < 0) continue;
        pick_x(kz);
        float gx[K], gy[K], gz[K];
#pragma unroll
        for (int kx = 0; kx < K; ++kx) {
          gx[kx] = wx[kx] * fx;
          gy[kx] = wx[kx] * fy;
          gz[kx] = wx[kx] * fz;
        }
#pragma unroll
        for (int ky = 0; ky < K; ++ky) {
          if (ly[ky] < 0) continue;
          const float wzy = wz[kz] * wy[ky];
          const int row = (lz[kz] * kTile + ly[ky]) * kTile;
#pragma unroll
          for (int kx = 0; kx < K; ++kx) {
            if (lx[kx] < 0) continue;
            const int li = row + lx[kx];
            atomicAdd((unsigned long long*)&acc[0][li], (unsigned long long)(long long)(int)(wzy * gx[kx]));
            atomicAdd((unsigned long long*)&acc[1][li], (unsigned long long)(long long)(int)(wzy * gy[kx]));
            atomicAdd((unsigned long long*)&acc[2][li], (unsigned long long)(long long)(int)(wzy * gz[kx]));
          }
        }
      }
    } else {
      for (int kz = 0; kz < K; ++kz) {
        if (lz[kz] < 0) continue;
        pick_x(kz);
        for (int ky = 0; ky < K; ++ky) {
          if (ly[ky] < 0) continue;
          const float wzy = wz[kz] * wy[ky];
          const int row = (lz[kz] * kTile + ly[ky]) * kTile;
          for (int kx = 0; kx < K; ++kx) {
            if (lx[kx] < 0) continue;
            const int li = row + lx[kx];
            // the same products as the 32-bit path: wzy * (wx * f)
            spread_add_wide(&acc[0][li], &acc[1][li], &acc[2][li], wzy * (wx[kx] * fx), wzy * (wx[kx] * fy),
                            wzy * (wx[kx] * fz));
          }
        }
      }
    }
  }
}

// Interpolation phase of one tile: one thread per (vertex, tile) entry sums
// w * u over its stencil nodes inside the tile (velocities staged in su) and
// stores the partial sum in the vertex's slot.  Partials are slot-major,
// [max_touch][cells x V]: entries of neighbouring vertices with the same
// slot, which one tile mostly holds together, share cache lines.
template <int K, bool LE = false>
__device__ inline void interp_tile(const Cells& C, const Mesh& M, const Lattice& L, const Bins& B,
                                   const float4* su, int t, int x0, int y0, int z0,
                                   float4* __restrict__ partial) {
  const int cnt = min(B.touch_cnt[t], B.cap);
  const int64_t e0 = (int64_t)t * B.cap, e1 = e0 + cnt;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int code = B.touch[e];
    const int v = code >> 5, j = code & 31;
    const int c = v / M.nv;
    const float* o = C.off + (int64_t)v * 3;
    int lx[K], ly[K], lz[K];
    float wx[K], wy[K], wz[K];
    LeStencil<K> S;
    if (LE)
      le_stencil<K>(L, C.origin[3 * c + 0], o[0], C.origin[3 * c + 2], o[2], x0, S);
    else
      axis_stencil<K>(C.origin[3 * c + 0], o[0], L.nx, L.bc[0] == 1, x0, lx, wx);
    axis_stencil<K>(C.origin[3 * c + 1], o[1], L.ny, L.bc[1] == 1, y0, ly, wy);
    axis_stencil<K>(C.origin[3 * c + 2], o[2], L.nz, L.bc[2] == 1, z0, lz, wz);
    float ux = 0.f, uy = 0.f, uz = 0.f;
#pragma unroll
    for (int kz = 0; kz < K; ++kz) {
      if (lz[kz] < 0) continue;
      float shift = 0.f;   // velocity of the image this z position lies in
      if (LE) {
        const bool a = S.m[kz] == S.ma;
#pragma unroll
        for (int kx = 0; kx < K; ++kx) {
          lx[kx] = a ? S.lxa[kx] : S.lxb[kx];
          wx[kx] = a ? S.wxa[kx] : S.wxb[kx];
        }
        shift = (float)S.m[kz] * L.le_u;
      }
#pragma unroll
      for (int ky = 0; ky < K; ++ky) {
        if (ly[ky] < 0) continue;
        const float wzy = wz[kz] * wy[ky];
        const int row = (lz[kz] * kTile + ly[ky]) * kTile;
#pragma unroll
        for (int kx = 0; kx < K; ++kx) {
          if (lx[kx] < 0) continue;
          const float w = wzy * wx[kx];
          const float4 q = su[row + lx[kx]];
          ux += w * (LE ? q.x + shift : q.x);
          uy += w * q.y;
          uz += w * q.z;
        }
      }
    }
    partial[(int64_t)j * C.n * M.nv + v] = make_float4(ux, uy, uz, 0.f);
  }
}

// Spreading of a vertex field alone (the reverse sweep spreads cotangents
// with it): writes body * g + the spread field, tile-major (padding slots
// receive body * g).
template <int K>
__global__ __launch_bounds__(256) void k_spread(Cells C, Mesh M, Lattice L, Bins B,
                                                const float* __restrict__ vec, float body,
                                                float* __restrict__ F) {
  __shared__ long long acc[3][kTile * kTile * kTile];
  const int t = blockIdx.x;
  int x0, y0, z0;
  tile_origin(L, t, x0, y0, z0);
  for (int i = threadIdx.x; i < kTile * kTile * kTile; i += blockDim.x) {
    acc[0][i] = 0;
    acc[1][i] = 0;
    acc[2][i] = 0;
  }
  __syncthreads();
  spread_tile<K>(C, M, L, B, vec, t, x0, y0, z0, acc);
  __syncthreads();
  if (threadIdx.x == 0) B.touch_cnt[t] = 0;   // consumed: zero for the next binning

  const int64_t NP = L.np, h0 = (int64_t)t * 512;
  for (int i = threadIdx.x; i < kTile * kTile * kTile; i += blockDim.x) {
    F[h0 + i] = body * L.g[0] + (float)((double)acc[0][i] * kFixInv);
    F[NP + h0 + i] = body * L.g[1] + (float)((double)acc[1][i] * kFixInv);
    F[2 * NP + h0 + i] = body * L.g[2] + (float)((double)acc[2][i] * kFixInv);
  }
}

// Which tile block b works on.  Work-groups go to the 8 XCDs round-robin by
// block id; each XCD gets one contiguous range of tiles, walked in order, so
// the neighbours a tile pulls boundary populations from were mostly just
// processed on the same XCD and sit in its L2.  -1 for padding blocks.
__device__ inline int tile_of_block(const Lattice& L, int b) {
  const int per = (L.ntiles + 7) >> 3;
  const int t = (b & 7) * per + (b >> 3);
  return t < L.ntiles ? t : -1;
}

__host__ __device__ inline int tile_grid(const Lattice& L) { return ((L.ntiles + 7) >> 3) * 8; }

// The fused lattice pass of one step, one work-group per tile:
//  1. spread the vertex forces of every entry reaching the tile into LDS;
//  2. pull-stream + collide the tile's nodes (force = body force + spread
//     field) and store their post-collision populations, keeping (u, rho)
//     in LDS (and writing the force and (u, rho) fields out when fields is
//     non-zero); a site whose byte in mask (when given) is non-zero lies
//     inside a cell and relaxes at L.omega_in of its highest set bit (the
//     most viscous class containing it), and its byte is cleared;
//  3. interpolate u to the tile's entries into their partial-sum slots.
// The force and velocity fields never leave the chip.
template <int K, bool LE>
__global__ __launch_bounds__(256) void k_tile_step(Cells C, Mesh M, Lattice L, Bins B,
                                                   const float* __restrict__ gin,
                                                   float* __restrict__ gout,
                                                   float* __restrict__ F,
                                                   float4* __restrict__ macro,
                                                   float4* __restrict__ partial, int fields,
                                                   unsigned char* __restrict__ mask) {
  __shared__ long long acc[3][kTile * kTile * kTile];
  __shared__ float4 su[kTile * kTile * kTile];
  const int t = tile_of_block(L, blockIdx.x);
  if (t < 0) return;
  int x0, y0, z0;
  tile_origin(L, t, x0, y0, z0);
  for (int i = threadIdx.x; i < kTile * kTile * kTile; i += blockDim.x) {
    acc[0][i] = 0;
    acc[1][i] = 0;
    acc[2][i] = 0;
  }
  __syncthreads();
  if (C.n > 0) spread_tile<K, LE>(C, M, L, B, C.force, t, x0, y0, z0, acc);
  __syncthreads();

  const int64_t NP = L.np, h0 = (int64_t)t * 512;
  for (int i = threadIdx.x; i < kTile * kTile * kTile; i += blockDim.x) {
    const int x = x0 + (i & 7), y = y0 + ((i >> 3) & 7), z = z0 + (i >> 6);
    if (x >= L.nx || y >= L.ny || z >= L.nz) {
      su[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      continue;
    }
    float g[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      if (LE && !L.le_raw && ((lbm::cz[q] > 0 && z == 0) || (lbm::cz[q] < 0 && z == L.nz - 1))) {
        g[q] = lbm::le_pull(L, gin, q, x, y);
      } else {
        int qs;
        const int64_t src = lbm::pull_source(L, q, x, y, z, &qs);
        g[q] = gin[qs * NP + src];
      }
    }
    const float fx = L.g[0] + (float)((double)acc[0][i] * kFixInv);
    const float fy = L.g[1] + (float)((double)acc[1][i] * kFixInv);
    const float fz = L.g[2] + (float)((double)acc[2][i] * kFixInv);
    float rho, ux, uy, uz;
    const int64_t h = h0 + i;
    float omega = L.omega;
    if (mask) {
      const unsigned b = mask[h];
      if (b) {   // inside a cell: the most viscous class containing the site
        omega = L.omega_in[31 - __clz(b)];
        mask[h] = 0;
      }
    }
    lbm::collide(g, fx, fy, fz, omega, rho, ux, uy, uz);
    const float4 m = make_float4(ux, uy, uz, rho);
    su[i] = m;
    if (fields) {
      macro[h] = m;
      F[h] = fx;
      F[NP + h] = fy;
      F[2 * NP + h] = fz;
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) gout[q * NP + h] = g[q] + lbm::wall_coeff(L, q, x, y, z) * rho;
  }
  if (C.n == 0) return;
  __syncthreads();
  interp_tile<K, LE>(C, M, L, B, su, t, x0, y0, z0, partial);
  __syncthreads();   // every thread has read the count: leave it zero for the next binning
  if (threadIdx.x == 0) B.touch_cnt[t] = 0;
}

template <int K>
__global__ __launch_bounds__(256) void k_advect(Cells C, Mesh M, Lattice L, Bins B,
                                                const float4* __restrict__ partial,
                                                int* __restrict__ flags, int ab2) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= (int64_t)C.n * M.nv) return;
  float nx[3];
  ibmd::advect_vertex<K>(C, M, L, B, partial, flags, v, nx, nullptr, ab2 != 0);
}

}  // namespace

hipError_t launch_spread_vec(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                             const float* vec, float body, float* F, hipStream_t s) {
  if (L.kernel == 4)
    hipLaunchKernelGGL(k_spread<4>, dim3(L.ntiles), dim3(256), 0, s, c, m, L, b, vec, body, F);
  else
    hipLaunchKernelGGL(k_spread<2>, dim3(L.ntiles), dim3(256), 0, s, c, m, L, b, vec, body, F);
  return hipGetLastError();
}

hipError_t launch_tile_step(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                            const float* gin, float* gout, float* F, float4* macro, float4* partial,
                            bool fields, unsigned char* mask, hipStream_t s) {
  const dim3 grid((unsigned)tile_grid(L));
  const int fl = fields ? 1 : 0;
  if (L.kernel == 4 && L.le)
    hipLaunchKernelGGL((k_tile_step<4, true>), grid, dim3(256), 0, s, c, m, L, b, gin, gout, F,
                       macro, partial, fl, mask);
  else if (L.kernel == 4)
    hipLaunchKernelGGL((k_tile_step<4, false>), grid, dim3(256), 0, s, c, m, L, b, gin, gout, F,
                       macro, partial, fl, mask);
  else if (L.le)
    hipLaunchKernelGGL((k_tile_step<2, true>), grid, dim3(256), 0, s, c, m, L, b, gin, gout, F,
                       macro, partial, fl, mask);
  else
    hipLaunchKernelGGL((k_tile_step<2, false>), grid, dim3(256), 0, s, c, m, L, b, gin, gout, F,
                       macro, partial, fl, mask);
  return hipGetLastError();
}

hipError_t launch_advect(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                         const float4* partial, int* flags, bool ab2, hipStream_t s) {
  const int64_t n = (int64_t)c.n * m.nv;
  if (n == 0) return hipSuccess;
  const dim3 gv((unsigned)((n + 255) / 256));
  const int a2 = ab2 ? 1 : 0;
  if (L.kernel == 4)
    hipLaunchKernelGGL(k_advect<4>, gv, dim3(256), 0, s, c, m, L, b, partial, flags, a2);
  else
    hipLaunchKernelGGL(k_advect<2>, gv, dim3(256), 0, s, c, m, L, b, partial, flags, a2);
  return hipGetLastError();
}

}  // namespace hc
