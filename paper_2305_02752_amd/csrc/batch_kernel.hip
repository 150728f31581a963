// Batched coupled steps: many independent single-cell boxes of uneven size
// and parameters advanced by ONE persistent kernel launch.
//
// Work split (static, decided on the host): every box owns a group of
// work-groups sized in proportion to its lattice; all members of a group
// sit on the same XCD (block ids congruent modulo 8), so their data shares
// one L2.  Per step, inside the group:
//   rank 0:      membrane forces of the box's cell (Sec. 2.3 force sum),
//                the node range its IBM stencil can reach and, with an
//                interior viscosity, the marks of the nodes inside the cell;
//   -- group barrier --
//   all ranks:   for each of their tiles (full x rows, ty x tz rows):
//                spread the vertex forces onto the tile in LDS (2^-40 fixed
//                point), BGK+Guo collide (the interior rate at marked
//                nodes, clearing the mark) and stream every node (Sec. 2.2),
//                and add the tile's share of every vertex velocity
//                (Sec. 2.3 interpolation) to a fixed-point accumulator;
//   -- group barrier --
//   rank 0:      Euler advection of the vertices (Sec. 2.6).
// Group barriers are counters in global memory with a bounded spin: a wait
// that exceeds the bound sets an abort flag that every work-group polls,
// so a misconfigured launch ends with an error instead of hanging.
// Each box carries its own step counter, which fixes the parity of its
// population buffers; the launch therefore replays unchanged from a graph.
#include "batch.h"
#include "interior_dev.h"
#include "lbm_dev.h"
#include "membrane_dev.h"
#include "stencil.h"

namespace hc {
namespace {

// Does the node range [lo, hi] (unwrapped) meet [a, a + h) on an axis of n nodes?
__device__ inline bool range_meets(int lo, int hi, int a, int h, int n, bool wall) {
  if (wall) {
    lo = max(lo, 0);
    hi = min(hi, n - 1);
    return lo <= hi && lo < a + h && hi >= a;
  }
  if (hi - lo + 1 >= n) return true;
  const int l = wrap(lo, n), r = l + (hi - lo);
  return (l < a + h && r >= a) || (l - n < a + h && r - n >= a) || (l + n < a + h && r + n >= a);
}

// Axis stencil relative to [t0, t0 + h): local index (-1 outside or beyond
// a wall) and weight.
template <int K>
__device__ inline void axis_local(int origin, float x, int n, bool wall, int t0, int h, int (&l)[K],
                                  float (&w)[K]) {
  const float fl = floorf(x);
  const int base = origin + (int)fl - (K == 4 ? 1 : 0);
  const float f = x - fl;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int p = base + k;
    bool in = true;
    if (wall) in = p >= 0 && p < n; else p = wrap(p, n);
    l[k] = (in && p >= t0 && p < t0 + h) ? p - t0 : -1;
    w[k] = stencil_w<K>(f, k);
  }
}

// The wait polls with relaxed loads and takes one acquire fence when it
// ends: an acquire on every poll would invalidate the XCD's L2 each time,
// which the other work-groups of the XCD, still streaming, pay for.
__device__ inline bool group_barrier(int* ctr, int members, int& epoch, int* abort_flag,
                                     int spin_limit, int* s_ok) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ++epoch;
    const int target = epoch * members;
    int ok = 1, spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          ++spins > spin_limit) {
        atomicOr(abort_flag, 1);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

// Stencil node range of the cell per axis (for the tile skip test).
__device__ inline void cell_reach(const Batch& V, int box, int K, const float* off, const int* o3,
                                  float* red, int tid, int nthr) {
  float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int v = tid; v < V.M.nv; v += nthr)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      mn[d] = fminf(mn[d], off[3 * v + d]);
      mx[d] = fmaxf(mx[d], off[3 * v + d]);
    }
#pragma unroll
  for (int d = 0; d < 3; ++d)
    for (int m = kWave / 2; m > 0; m >>= 1) {
      mn[d] = fminf(mn[d], __shfl_xor(mn[d], m));
      mx[d] = fmaxf(mx[d], __shfl_xor(mx[d], m));
    }
  const int nw = nthr / kWave, wv = tid / kWave;
  __syncthreads();
  if ((tid & (kWave - 1)) == 0)
    for (int d = 0; d < 3; ++d) {
      red[6 * wv + d] = mn[d];
      red[6 * wv + 3 + d] = mx[d];
    }
  __syncthreads();
  if (tid == 0) {
    for (int d = 0; d < 3; ++d) {
      float a = red[d], b = red[3 + d];
      for (int w = 1; w < nw; ++w) {
        a = fminf(a, red[6 * w + d]);
        b = fmaxf(b, red[6 * w + 3 + d]);
      }
      V.bbox[6 * box + 2 * d] = o3[d] + (int)floorf(a) - (K == 4 ? 1 : 0);
      V.bbox[6 * box + 2 * d + 1] = o3[d] + (int)floorf(b) + (K == 4 ? 2 : 1);
    }
  }
  __syncthreads();
}

// Marks the nodes inside the box's cell (positions staged in sp by the
// membrane phase) for the interior relaxation rate.
__device__ inline void box_mark(const Batch& V, const BoxDesc& B, float* sp, const int (&o3)[3],
                                inside::Lds& S, int tid, int nthr) {
  if (!V.interior || B.omega_in == B.omega) return;
  inside::Grid G;
  G.n[0] = B.nx;
  G.n[1] = B.ny;
  G.n[2] = B.nz;
  for (int d = 0; d < 3; ++d) G.bc[d] = B.bc[d];
  G.le = 0;
  G.le_delta = 0.f;
  const long long nx = B.nx, ny = B.ny;
  inside::mark_cell(nullptr, sp, V.M.nv, V.M.tri, V.M.nt, o3, G,
                    [=](int x, int y, int z) { return ((int64_t)z * ny + y) * nx + x; },
                    V.mask + B.site_off, (unsigned char)1, V.flags + 2, S, tid, nthr);
}

// Integer test: does the K-node stencil starting at node `base` meet rows [a, a + h)?
template <int K>
__device__ inline bool stencil_meets(int base, int a, int h, int n, bool wall) {
  return range_meets(base, base + K - 1, a, h, n, wall);
}

template <int K>
__device__ void box_tile(const Batch& V, const BoxDesc& B, int box, int t, const float* __restrict__ gin,
                         float* __restrict__ gout, const float* __restrict__ off,
                         const float* __restrict__ force, const int* o3, long long* facc, float4* su,
                         int tid, int nthr) {
  const int nv = V.M.nv;
  const int y0 = (t % B.nty) * B.ty, z0 = (t / B.nty) * B.tz;
  const int hy = min(B.ty, B.ny - y0), hz = min(B.tz, B.nz - z0);
  const int nsite = B.nx * hy * hz;
  const int* bb = V.bbox + 6 * box;
  const bool near = V.has_cells && range_meets(bb[2], bb[3], y0, hy, B.ny, B.bc[1] == 1) &&
                    range_meets(bb[4], bb[5], z0, hz, B.nz, B.bc[2] == 1);
  if (near) {
    for (int i = tid; i < 3 * nsite; i += nthr) facc[i] = 0;
    __syncthreads();
    for (int v = tid; v < nv; v += nthr) {
      const float py = off[3 * v + 1], pz = off[3 * v + 2];
      const int sh = K == 4 ? 1 : 0;
      if (!stencil_meets<K>(o3[1] + (int)floorf(py) - sh, y0, hy, B.ny, B.bc[1] == 1) ||
          !stencil_meets<K>(o3[2] + (int)floorf(pz) - sh, z0, hz, B.nz, B.bc[2] == 1))
        continue;
      int lx[K], ly[K], lz[K];
      float wx[K], wy[K], wz[K];
      axis_local<K>(o3[1], py, B.ny, B.bc[1] == 1, y0, hy, ly, wy);
      axis_local<K>(o3[2], pz, B.nz, B.bc[2] == 1, z0, hz, lz, wz);
      axis_local<K>(o3[0], off[3 * v], B.nx, B.bc[0] == 1, 0, B.nx, lx, wx);
      const float fx = force[3 * v] * kFixScaleF, fy = force[3 * v + 1] * kFixScaleF,
                  fz = force[3 * v + 2] * kFixScaleF;
#pragma unroll
      for (int kz = 0; kz < K; ++kz) {
        if (lz[kz] < 0) continue;
#pragma unroll
        for (int ky = 0; ky < K; ++ky) {
          if (ly[ky] < 0) continue;
          const float wzy = wz[kz] * wy[ky];
          const int row = (lz[kz] * hy + ly[ky]) * B.nx;
#pragma unroll
          for (int kx = 0; kx < K; ++kx) {
            if (lx[kx] < 0) continue;
            const float w = wzy * wx[kx];
            const int li = 3 * (row + lx[kx]);
            fix_add3(&facc[li], &facc[li + 1], &facc[li + 2], w * fx, w * fy, w * fz);
          }
        }
      }
    }
    __syncthreads();
  }
  const int64_t N = B.n;
  const float* gi = gin + B.pop_off;
  float* go = gout + B.pop_off;
  lbm::Walls W;
  W.axis = B.wall_axis;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    W.lo[d] = B.ulo[d];
    W.hi[d] = B.uhi[d];
  }
  for (int i = tid; i < nsite; i += nthr) {
    const int x = i % B.nx, r = i / B.nx;
    const int y = y0 + r % hy, z = z0 + r / hy;
    const int64_t s = ((int64_t)z * B.ny + y) * B.nx + x;
    float g[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) g[q] = gi[q * N + s];
    float fx = B.g[0], fy = B.g[1], fz = B.g[2];
    if (near) {
      fx += (float)((double)facc[3 * i] * kFixInv);
      fy += (float)((double)facc[3 * i + 1] * kFixInv);
      fz += (float)((double)facc[3 * i + 2] * kFixInv);
    }
    float om = B.omega;
    if (V.interior) {
      unsigned char* mk = V.mask + B.site_off + s;
      if (*mk) {
        om = B.omega_in;
        *mk = 0;
      }
    }
    float rho, ux, uy, uz;
    lbm::collide(g, fx, fy, fz, om, rho, ux, uy, uz);
    if (near) su[i] = make_float4(ux, uy, uz, rho);
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      int64_t dst;
      float dw;
      const int qd = lbm::stream_target(q, x, y, z, B.nx, B.ny, B.nz, W, rho, &dst, &dw);
      go[qd * N + dst] = g[q] + dw;
    }
  }
  if (near) {
    __syncthreads();
    long long* U = V.uacc + (int64_t)box * nv * 3;
    for (int v = tid; v < nv; v += nthr) {
      const float py = off[3 * v + 1], pz = off[3 * v + 2];
      const int sh = K == 4 ? 1 : 0;
      if (!stencil_meets<K>(o3[1] + (int)floorf(py) - sh, y0, hy, B.ny, B.bc[1] == 1) ||
          !stencil_meets<K>(o3[2] + (int)floorf(pz) - sh, z0, hz, B.nz, B.bc[2] == 1))
        continue;
      int lx[K], ly[K], lz[K];
      float wx[K], wy[K], wz[K];
      axis_local<K>(o3[1], py, B.ny, B.bc[1] == 1, y0, hy, ly, wy);
      axis_local<K>(o3[2], pz, B.nz, B.bc[2] == 1, z0, hz, lz, wz);
      axis_local<K>(o3[0], off[3 * v], B.nx, B.bc[0] == 1, 0, B.nx, lx, wx);
      // every node contribution is rounded to fixed point on its own, so the
      // vertex velocity does not depend on how nodes are grouped into tiles
      long long sx = 0, sy = 0, sz = 0;
#pragma unroll
      for (int kz = 0; kz < K; ++kz) {
        if (lz[kz] < 0) continue;
#pragma unroll
        for (int ky = 0; ky < K; ++ky) {
          if (ly[ky] < 0) continue;
          const float wzy = wz[kz] * wy[ky] * kFixScaleF;
          const int row = (lz[kz] * hy + ly[ky]) * B.nx;
#pragma unroll
          for (int kx = 0; kx < K; ++kx) {
            if (lx[kx] < 0) continue;
            const float w = wzy * wx[kx];
            const float4 q = su[row + lx[kx]];
            sx += __float2ll_rn(w * q.x);
            sy += __float2ll_rn(w * q.y);
            sz += __float2ll_rn(w * q.z);
          }
        }
      }
      atomicAdd((unsigned long long*)&U[3 * v], (unsigned long long)sx);
      atomicAdd((unsigned long long*)&U[3 * v + 1], (unsigned long long)sy);
      atomicAdd((unsigned long long*)&U[3 * v + 2], (unsigned long long)sz);
    }
    __syncthreads();
  }
}

// Vertex velocity = fixed-point sum of tile shares + wall layers; Euler move
// with the rounding carried in the low parts (move_compensated).
template <int K>
__device__ void box_advect(const Batch& V, const BoxDesc& B, int box, const int* o3, int tid,
                           int nthr) {
  const int nv = V.M.nv;
  long long* U = V.uacc + (int64_t)box * nv * 3;
  float* off = V.off + (int64_t)box * nv * 3;
  float* lo = V.lo + (int64_t)box * nv * 3;
  float* vel = V.vel + (int64_t)box * nv * 3;
  for (int v = tid; v < nv; v += nthr) {
    float u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      u[d] = (float)((double)U[3 * v + d] * kFixInv);
      U[3 * v + d] = 0;
    }
    if (B.wall_axis >= 0) {
      const int d = B.wall_axis;
      const int n = d == 0 ? B.nx : (d == 1 ? B.ny : B.nz);
      const float od = off[3 * v + d], fl = floorf(od);
      const int base = o3[d] + (int)fl - (K == 4 ? 1 : 0);
      float wlo = 0.f, whi = 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int p = base + k;
        if (p < 0) wlo += stencil_w<K>(od - fl, k);
        if (p >= n) whi += stencil_w<K>(od - fl, k);
      }
#pragma unroll
      for (int e = 0; e < 3; ++e) u[e] += wlo * B.ulo[e] + whi * B.uhi[e];
    }
    bool finite = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float x = off[3 * v + d], l = lo[3 * v + d];
      move_compensated(x, l, u[d]);
      finite = finite && isfinite(x);
      off[3 * v + d] = x;
      lo[3 * v + d] = l;
      vel[3 * v + d] = u[d];
    }
    if (!finite) atomicOr(&V.flags[0], 1);
  }
  __syncthreads();
}

template <int K>
__global__ void k_batch(Batch V, int nsteps) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int s_ok;
  __shared__ double red[2 * 16];
  __shared__ float fred[6 * 16];
  const int4 me = V.wg[blockIdx.x];
  const int box = me.x, rank = me.y, members = me.z;
  if (box < 0) return;
  const BoxDesc B = V.box[box];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nv = V.M.nv;
  const int o3[3] = {V.origin[3 * box], V.origin[3 * box + 1], V.origin[3 * box + 2]};
  float* off = V.off + (int64_t)box * nv * 3;
  float* force = V.force + (int64_t)box * nv * 3;
  // LDS: membrane phase {acc int64 [3nv], pos float [3nv]}; tile phase
  // {facc int64 [3 cap], su float4 [cap]} (the phases never overlap)
  long long* acc = reinterpret_cast<long long*>(lds);
  float* sp = reinterpret_cast<float*>(lds + (size_t)nv * 3 * 8);
  long long* facc = reinterpret_cast<long long*>(lds);
  float4* su = reinterpret_cast<float4*>(lds + (size_t)V.tile_cap * 24);
  // marking scratch: over acc (free once the forces are out) when it fits,
  // else after sp
  inside::Lds& ms = *reinterpret_cast<inside::Lds*>(
      lds + ((size_t)nv * 24 >= sizeof(inside::Lds) ? 0 : (size_t)nv * 36));
  int epoch = 0;
  const int parity0 = V.box_step[box] & 1;
  int* ctr = V.bar + box;

  if (rank == 0 && V.has_cells) {
    mem::membrane_cell(V.M, off, V.k + 4 * box, V.trac ? V.trac + 3 * box : nullptr, force,
                       V.area + box, V.volume + box, acc, sp, red, tid, nthr);
    cell_reach(V, box, K, off, o3, fred, tid, nthr);
    box_mark(V, B, sp, o3, ms, tid, nthr);
  }
  if (!group_barrier(ctr, members, epoch, V.flags + 1, V.spin_limit, &s_ok)) return;
  const int ntiles = B.nty * B.ntz;
  for (int s = 0; s < nsteps; ++s) {
    const bool odd = ((parity0 + s) & 1) != 0;
    const float* gin = odd ? V.pops1 : V.pops0;
    float* gout = odd ? V.pops0 : V.pops1;
    for (int t = rank; t < ntiles; t += members)
      box_tile<K>(V, B, box, t, gin, gout, off, force, o3, facc, su, tid, nthr);
    if (!group_barrier(ctr, members, epoch, V.flags + 1, V.spin_limit, &s_ok)) return;
    if (rank == 0 && V.has_cells) {
      box_advect<K>(V, B, box, o3, tid, nthr);
      if (s + 1 < nsteps) {
        mem::membrane_cell(V.M, off, V.k + 4 * box, V.trac ? V.trac + 3 * box : nullptr, force,
                           V.area + box, V.volume + box, acc, sp, red, tid, nthr);
        cell_reach(V, box, K, off, o3, fred, tid, nthr);
        box_mark(V, B, sp, o3, ms, tid, nthr);
      }
    }
    if (!group_barrier(ctr, members, epoch, V.flags + 1, V.spin_limit, &s_ok)) return;
  }
  if (rank == 0 && tid == 0) V.box_step[box] += nsteps;
}

}  // namespace

size_t batch_lds_bytes(int nv, int tile_cap) {
  size_t mem = (size_t)nv * 3 * (8 + 4);
  if ((size_t)nv * 24 < sizeof(inside::Lds)) mem += sizeof(inside::Lds);
  const size_t tile = (size_t)tile_cap * (24 + 16);
  return mem > tile ? mem : tile;
}

const void* batch_kernel(int K) {
  return K == 4 ? reinterpret_cast<const void*>(&k_batch<4>)
                : reinterpret_cast<const void*>(&k_batch<2>);
}

hipError_t launch_batch(const Batch& V, int K, int nsteps, int grid, int block, hipStream_t s) {
  const size_t lds = batch_lds_bytes(V.M.nv, V.tile_cap);
  if (K == 4)
    hipLaunchKernelGGL(k_batch<4>, dim3(grid), dim3(block), lds, s, V, nsteps);
  else
    hipLaunchKernelGGL(k_batch<2>, dim3(grid), dim3(block), lds, s, V, nsteps);
  return hipGetLastError();
}

}  // namespace hc
