// Fused per-cell kernel of the single-lattice step: one work-group per cell
// (1) closes the previous step's interpolation and moves the vertices
//     (Sec. 2.6 explicit Euler), when one is pending;
// (2) computes the membrane forces of the new positions (Sec. 2.3 force
//     sum) when they are due (refresh); between refreshes the forces of
//     the last one are held (Sec. 2.6 time-scale separation);
// (3) bins the cell's vertices to the tiles their IBM stencils reach.
// After a move, a cell whose bounding-box centre lies more than kRecentre
// lattice units from its integer origin along an axis is re-centred: the
// origin takes the nearest integer of that centre and every offset gives it
// up (TwoSum into the low part, so origin + offset + low part is unchanged).
// Offsets then stay within the cell's own size however far it travels, and
// keep the resolution a float has there.
// All three read the same 642 positions, so the cell is loaded once and its
// latency-bound steps overlap across the resident work-groups.
#include <algorithm>

#include "binning_dev.h"
#include "ibm_dev.h"
#include "membrane_dev.h"

namespace hc {
namespace {

constexpr float kRecentre = 8.f;

template <int kThreads>
__device__ void recentre_cell(const Cells& C, const Mesh& M, int c, float* sp, float (*ext)[kThreads / kWave],
                              int tid) {
  float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int v = tid; v < M.nv; v += kThreads) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      mn[d] = fminf(mn[d], sp[3 * v + d]);
      mx[d] = fmaxf(mx[d], sp[3 * v + d]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    for (int m = kWave / 2; m > 0; m >>= 1) {
      mn[d] = fminf(mn[d], __shfl_xor(mn[d], m));
      mx[d] = fmaxf(mx[d], __shfl_xor(mx[d], m));
    }
  }
  if ((tid & (kWave - 1)) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      ext[d][tid / kWave] = mn[d];
      ext[3 + d][tid / kWave] = mx[d];
    }
  }
  __syncthreads();
  int sh[3];
  bool any = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float a = ext[d][0], b = ext[3 + d][0];
    for (int w = 1; w < kThreads / kWave; ++w) {
      a = fminf(a, ext[d][w]);
      b = fmaxf(b, ext[3 + d][w]);
    }
    const float mid = 0.5f * (a + b);
    sh[d] = fabsf(mid) > kRecentre ? (int)floorf(mid + 0.5f) : 0;
    any = any || sh[d] != 0;
  }
  if (!any) return;   // the same decision in every thread
  const int64_t b3 = (int64_t)c * M.nv * 3;
  for (int v = tid; v < M.nv; v += kThreads) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (sh[d] == 0) continue;
      float hi = sp[3 * v + d], lo = C.lo[b3 + 3 * v + d];
      move_compensated(hi, lo, (float)-sh[d]);
      sp[3 * v + d] = hi;
      C.off[b3 + 3 * v + d] = hi;
      C.lo[b3 + 3 * v + d] = lo;
    }
  }
  if (tid < 3) C.origin[3 * c + tid] += sh[tid];
  __syncthreads();
}

// Work-group size: 256 threads when the cells fill the chip; with fewer
// cells than a few per CU each cell's work-group is widened so that its
// latency-bound loops take fewer rounds.
template <int K, int kCellThreads, bool LE>
__device__ __forceinline__ void cell_step_body(Cells C, Mesh M, Lattice L, Bins B,
                                               const float4* __restrict__ partial, int* __restrict__ flags,
                                               int advect, const float* __restrict__ src, int refresh, int ab2,
                                               int recentre, int keep_vel) {
  extern __shared__ long long lds64[];
  __shared__ double red[2 * kCellThreads / kWave];
  __shared__ float ext[6][kCellThreads / kWave];
  __shared__ int keys[bin::kHash], count[bin::kHash], base[bin::kHash];
  // LDS: [membrane accumulator, later the binning's slot records][offsets]
  const int region = max(24, bin::slot_lds_per_vertex(L.max_touch)) * M.nv;   // bytes
  long long* acc = lds64;
  unsigned short* srank = reinterpret_cast<unsigned short*>(lds64);
  unsigned char* shash = reinterpret_cast<unsigned char*>(srank + (size_t)M.nv * L.max_touch);
  float* sp = reinterpret_cast<float*>(reinterpret_cast<char*>(lds64) + ((region + 7) & ~7));
  const int c = blockIdx.x, tid = threadIdx.x;
  const int64_t b3 = (int64_t)c * M.nv * 3;
  if (advect) {
    for (int vl = tid; vl < M.nv; vl += kCellThreads) {
      float nx[3];
      ibmd::advect_vertex<K, true>(C, M, L, B, partial, flags, (int64_t)c * M.nv + vl, nx, src, ab2 != 0,
                             keep_vel != 0);
      sp[3 * vl] = nx[0];
      sp[3 * vl + 1] = nx[1];
      sp[3 * vl + 2] = nx[2];
    }
    if (recentre) {
      __syncthreads();   // every moved offset in sp
      recentre_cell<kCellThreads>(C, M, c, sp, ext, tid);
    }
  } else {
    for (int i = tid; i < 3 * M.nv; i += kCellThreads) sp[i] = C.off[b3 + i];
  }
  if (refresh) {
    // offsets staged in sp (the call synchronises before reading them)
    mem::membrane_cell(M, nullptr, C.k + 4 * c, C.traction ? C.traction + 3 * c : nullptr,
                       C.force + b3, C.area + c, C.volume + c, acc, sp, red, tid, kCellThreads);
  } else {
    __syncthreads();   // forces held from the last refresh; sp complete for the binning
  }
  __syncthreads();   // the accumulator is free: its space takes the slot records
  bin::bin_cell<LE>(C, M, L, B, c, sp, keys, count, base, srank, shash, tid, kCellThreads);
}

template <int K, int kCellThreads, bool LE>
__global__ __launch_bounds__(kCellThreads) void k_cell_step(Cells C, Mesh M, Lattice L, Bins B,
                                                           const float4* __restrict__ partial,
                                                           int* __restrict__ flags, int advect,
                                                           const float* __restrict__ src,
                                                           int refresh, int ab2, int recentre, int keep_vel) {
  cell_step_body<K, kCellThreads, LE>(C, M, L, B, partial, flags, advect, src, refresh, ab2, recentre, keep_vel);
}

// Batched form: box blockIdx.y.
template <int K, int kCellThreads>
__global__ __launch_bounds__(kCellThreads) void k_cell_step_multi(const CellStepArgs* __restrict__ many) {
  const CellStepArgs& a = many[blockIdx.y];
  cell_step_body<K, kCellThreads, false>(a.C, a.M, a.L, a.B, a.partial, a.flags, a.advect, a.src, a.refresh,
                                         a.ab2, a.recentre, 0);
}

}  // namespace

// Tile-list counts must be zero on entry (see launch_bin_vertices).
hipError_t launch_cell_step(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                            const float4* partial, int* flags, bool advect, const float* src,
                            bool refresh, bool ab2, bool recentre, bool keep_vel, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  const int region = std::max(24, bin::slot_lds_per_vertex(L.max_touch)) * m.nv;
  const size_t lds = (size_t)((region + 7) & ~7) + (size_t)m.nv * 3 * sizeof(float);
  const int adv = advect ? 1 : 0, ref = refresh ? 1 : 0, a2 = ab2 ? 1 : 0, rc = recentre ? 1 : 0;
  const int kv = keep_vel ? 1 : 0;
  auto go = [&](auto kern, int threads) {
    hipLaunchKernelGGL(kern, dim3(c.n), dim3(threads), lds, s, c, m, L, b, partial, flags, adv, src, ref, a2,
                       rc, kv);
  };
  // sheared images: one 256-thread form
  if (L.le) {
    if (L.kernel == 4) go(k_cell_step<4, 256, true>, 256);
    else go(k_cell_step<2, 256, true>, 256);
  } else if (c.n <= 64) {
    if (L.kernel == 4) go(k_cell_step<4, 1024, false>, 1024);
    else go(k_cell_step<2, 1024, false>, 1024);
  } else if (c.n <= 1024) {
    if (L.kernel == 4) go(k_cell_step<4, 512, false>, 512);
    else go(k_cell_step<2, 512, false>, 512);
  } else {
    if (L.kernel == 4) go(k_cell_step<4, 256, false>, 256);
    else go(k_cell_step<2, 256, false>, 256);
  }
  return hipGetLastError();
}

// Boxes of one shape without sheared images; every box holds the same number
// of cells.
hipError_t launch_cell_step_multi(const CellStepArgs& a0, const CellStepArgs* dev, int n, hipStream_t s) {
  if (n == 0 || a0.C.n == 0) return hipSuccess;
  if (a0.L.le) return hipErrorInvalidValue;
  const int region = std::max(24, bin::slot_lds_per_vertex(a0.L.max_touch)) * a0.M.nv;
  const size_t lds = (size_t)((region + 7) & ~7) + (size_t)a0.M.nv * 3 * sizeof(float);
  const dim3 grid((unsigned)a0.C.n, (unsigned)n);
  auto go = [&](auto kern, int threads) { hipLaunchKernelGGL(kern, grid, dim3(threads), lds, s, dev); };
  if (a0.C.n <= 64) {
    if (a0.L.kernel == 4) go(k_cell_step_multi<4, 1024>, 1024);
    else go(k_cell_step_multi<2, 1024>, 1024);
  } else if (a0.C.n <= 1024) {
    if (a0.L.kernel == 4) go(k_cell_step_multi<4, 512>, 512);
    else go(k_cell_step_multi<2, 512>, 512);
  } else {
    if (a0.L.kernel == 4) go(k_cell_step_multi<4, 256>, 256);
    else go(k_cell_step_multi<2, 256>, 256);
  }
  return hipGetLastError();
}

}  // namespace hc
