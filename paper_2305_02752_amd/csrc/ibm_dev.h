// Device helpers of the immersed-boundary coupling (Sec. 2.3) shared by the
// tile kernels and the fused per-cell kernel: Peskin's 4-point function,
// stencil weights, and the per-vertex close of the interpolation with the
// explicit Euler move (Sec. 2.6).
#pragma once

#include "common.h"
#include "stencil.h"

namespace hc {
namespace ibmd {

// Vertex velocity = tile partials summed in slot order (fixed, so the result
// is reproducible) + stencil nodes beyond a wall at the wall velocity; then
// X += U (Euler) or X += 3/2 U - 1/2 U_prev (second-order Adams-Bashforth,
// U_prev = the velocity stored by the previous move), reading X from src
// when given (else in place) and writing C.off; the low parts C.lo are
// carried in place (move_compensated).  The new offset is also
// returned in nxyz, and U is stored in C.vel when keep_vel (for the next
// Adams-Bashforth move, and for the read-out after the closing move).  The
// other two axes' weights sum to one, so a node layer beyond the wall
// contributes its axis weight times the wall velocity.
// PRE: the first kPre slots are requested together with the slot count (a
// latency-bound caller: the per-cell kernel, a few vertices per thread);
// otherwise slot by slot up to the count (the vertex-parallel move, bound by
// bandwidth, which the unused slots would waste).
template <int K, bool PRE = false>
__device__ inline void advect_vertex(const Cells& C, const Mesh& M, const Lattice& L, const Bins& B,
                                     const float4* __restrict__ partial, int* __restrict__ flags,
                                     int64_t v, float (&nxyz)[3], const float* src = nullptr,
                                     bool ab2 = false, bool keep_vel = true) {
  float Ux = 0.f, Uy = 0.f, Uz = 0.f;
  // With PRE the first kPre slots (every slot of a lattice without sheared
  // images) are requested together with the slot count, in bounds whatever
  // the count, so that the vertex waits for one memory round trip rather
  // than one per slot; every slot is summed in slot order either way.
  constexpr int kPre = 8;
  const int64_t stride = (int64_t)C.n * M.nv;
  const int npre = PRE ? min(kPre, L.max_touch) : 0;
  float3 q[kPre];
  if (PRE) {
#pragma unroll
    for (int j = 0; j < kPre; ++j) {   // slot min(j, npre - 1): every read in bounds, none behind a branch
      const float4 p = partial[min(j, npre - 1) * stride + v];
      q[j] = make_float3(p.x, p.y, p.z);
    }
  }
  const int nt = B.ntouch[v];
#pragma unroll
  for (int j = 0; j < kPre; ++j)
    if (j < nt && j < npre) {
      Ux += q[j].x;
      Uy += q[j].y;
      Uz += q[j].z;
    }
  for (int j = npre; j < nt; ++j) {
    const float4 p = partial[j * stride + v];
    Ux += p.x;
    Uy += p.y;
    Uz += p.z;
  }
  float* o = C.off + v * 3;
  const float* oi = (src ? src : C.off) + v * 3;
  const float ox = oi[0], oy = oi[1], oz = oi[2];
  if (L.wall_axis >= 0) {
    const int d = L.wall_axis;
    const int c = (int)(v / M.nv);
    const float od = d == 0 ? ox : (d == 1 ? oy : oz);
    const float fl = floorf(od);
    const int n = d == 0 ? L.nx : (d == 1 ? L.ny : L.nz);
    const int base = C.origin[3 * c + d] + (int)fl - (K == 4 ? 1 : 0);
    float wlo = 0.f, whi = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int p = base + k;
      if (p < 0) wlo += hc::stencil_w<K>(od - fl, k);
      if (p >= n) whi += hc::stencil_w<K>(od - fl, k);
    }
    Ux += wlo * L.ulo[0] + whi * L.uhi[0];
    Uy += wlo * L.ulo[1] + whi * L.uhi[1];
    Uz += wlo * L.ulo[2] + whi * L.uhi[2];
  }
  float* vo = C.vel + v * 3;
  float dx = Ux, dy = Uy, dz = Uz;
  if (ab2) {
    dx = 1.5f * Ux - 0.5f * vo[0];
    dy = 1.5f * Uy - 0.5f * vo[1];
    dz = 1.5f * Uz - 0.5f * vo[2];
  }
  float* lo = C.lo + v * 3;
  float nx = ox, ny = oy, nz = oz, lx = lo[0], ly = lo[1], lz = lo[2];
  hc::move_compensated(nx, lx, dx);
  hc::move_compensated(ny, ly, dy);
  hc::move_compensated(nz, lz, dz);
  if (!(isfinite(nx) && isfinite(ny) && isfinite(nz))) atomicOr(&flags[0], 1);
  lo[0] = lx;
  lo[1] = ly;
  lo[2] = lz;
  if (keep_vel) {   // read by the next Adams-Bashforth move and by the read-out
    vo[0] = Ux;
    vo[1] = Uy;
    vo[2] = Uz;
  }
  o[0] = nx;
  o[1] = ny;
  o[2] = nz;
  nxyz[0] = nx;
  nxyz[1] = ny;
  nxyz[2] = nz;
}

}  // namespace ibmd
}  // namespace hc
