// Integer binning of vertices and cells to 8^3 lattice tiles.
//
// The paper keeps track of which subdomain holds which cell and rebalances
// by redistribution (Sec. 2.6); on one device the same bookkeeping decides
// which tile work-group sees which vertex.  Rules (all integer, exact on the
// float32 offsets):
//  owner tile of a vertex: node origin + floor(offset), wrapped, >> 3;
//  touch lists: tiles reached by the vertex's IBM stencil nodes;
//  cell lists:  tiles met by [floor(min)-1, floor(max)+2] of the cell.
// Lists are filled through per-tile counters (atomic slot reservation), so
// their content is exact while the order inside a tile is arbitrary; the
// read-out path sorts each tile segment.
#include "common.h"

namespace hc {
namespace {

__device__ inline int wrap(int p, int n) {
  p %= n;
  return p < 0 ? p + n : p;
}

// Distinct tiles (<= 3) reached along one axis by K stencil nodes starting at p0.
__device__ inline int axis_tiles(int p0, int K, int n, int wall, int* out) {
  int cnt = 0;
  for (int k = 0; k < K; ++k) {
    int p = p0 + k;
    if (wall) {
      if (p < 0 || p >= n) continue;
    } else {
      p = wrap(p, n);
    }
    const int t = p / kTile;
    bool seen = false;
    for (int q = 0; q < cnt; ++q) seen = seen || out[q] == t;
    if (!seen && cnt < 3) out[cnt++] = t;
  }
  return cnt;
}

// Rank of this lane's element in the per-tile counter, with one atomic per
// distinct tile in the wave (lanes of one cell mostly share tiles).
__device__ inline int wave_counted_rank(int* cnt, int tile, bool active) {
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long pending = __ballot(active);
  int rank = 0;
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int t = __shfl(tile, leader);
    const unsigned long long mask = pending & __ballot(active && tile == t);
    int base = 0;
    if (lane == leader) base = atomicAdd(&cnt[t], __popcll(mask));
    base = __shfl(base, leader);
    if ((mask >> lane) & 1ull) rank = base + __popcll(mask & ((1ull << lane) - 1ull));
    pending &= ~mask;
  }
  return rank;
}

__global__ __launch_bounds__(256) void k_bin_vertices(Cells C, Mesh M, Lattice L, Bins B) {
  const int64_t v0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = v0 < (int64_t)C.n * M.nv;
  const int64_t v = live ? v0 : 0;
  const int c = (int)(v / M.nv);
  const float* o = C.off + v * 3;
  const int K = L.kernel;
  const int b = K == 4 ? -1 : 0;
  int p[3];
  int n[3] = {L.nx, L.ny, L.nz};
  int T[3][3], nT[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    p[d] = C.origin[3 * c + d] + (int)floorf(o[d]);
    nT[d] = axis_tiles(p[d] + b, K, n[d], L.bc[d] == 1, T[d]);
    int q = L.bc[d] == 1 ? min(max(p[d], 0), n[d] - 1) : wrap(p[d], n[d]);
    p[d] = q / kTile;
  }
  if (live) B.owner[v] = (p[2] * L.ty + p[1]) * L.tx + p[0];
  const int ntouch = live ? nT[0] * nT[1] * nT[2] : 0;
  if (live && ntouch > L.max_touch) atomicOr(&B.flags[1], 2);  // excluded by the bound set at create
  // all lanes walk the same slot sequence so the wave can aggregate atomics
  for (int j = 0; j < L.max_touch; ++j) {
    const bool act = j < ntouch;
    int tile = 0;
    if (act) {
      const int a = j / (nT[0] * nT[1]), r = j % (nT[0] * nT[1]);
      tile = (T[2][a] * L.ty + T[1][r / nT[0]]) * L.tx + T[0][r % nT[0]];
    }
    const int rank = wave_counted_rank(B.touch_cnt, tile, act);
    if (live) {
      B.touch_tile[v * L.max_touch + j] = act ? tile : -1;
      if (act) B.touch_rank[v * L.max_touch + j] = rank;
    }
  }
}

__global__ __launch_bounds__(256) void k_fill_touch(int64_t nvtot, int max_touch, Bins B) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvtot) return;
  for (int j = 0; j < max_touch; ++j) {
    const int t = B.touch_tile[v * max_touch + j];
    if (t < 0) break;
    B.touch[B.touch_ptr[t] + B.touch_rank[v * max_touch + j]] = (int)(v * 32 + j);
  }
}

// One wave per cell: stencil bounding box -> covered tiles, counted per tile.
__global__ __launch_bounds__(64) void k_cell_tiles(Cells C, Mesh M, Lattice L, int* cnt,
                                                   int* tiles, int* rank, int max_per_cell,
                                                   int* flags) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const float* o = C.off + (int64_t)c * M.nv * 3;
  float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int v = lane; v < M.nv; v += kWave) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      mn[d] = fminf(mn[d], o[3 * v + d]);
      mx[d] = fmaxf(mx[d], o[3 * v + d]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    for (int m = kWave / 2; m > 0; m >>= 1) {
      mn[d] = fminf(mn[d], __shfl_xor(mn[d], m));
      mx[d] = fmaxf(mx[d], __shfl_xor(mx[d], m));
    }
  }
  if (lane != 0) return;
  int n[3] = {L.nx, L.ny, L.nz};
  int T[3][64], nT[3];
  for (int d = 0; d < 3; ++d) {
    int lo = C.origin[3 * c + d] + (int)floorf(mn[d]) - 1;
    int hi = C.origin[3 * c + d] + (int)floorf(mx[d]) + 2;
    nT[d] = 0;
    if (L.bc[d] == 1) {
      lo = max(lo, 0);
      hi = min(hi, n[d] - 1);
      for (int t = lo / kTile; t <= hi / kTile && nT[d] < 64; ++t) T[d][nT[d]++] = t;
    } else {
      if (hi - lo + 1 > n[d]) hi = lo + n[d] - 1;
      for (int p = lo; p <= hi; ++p) {
        const int t = wrap(p, n[d]) / kTile;
        bool seen = false;
        for (int q = 0; q < nT[d]; ++q) seen = seen || T[d][q] == t;
        if (!seen && nT[d] < 64) T[d][nT[d]++] = t;
      }
    }
  }
  int j = 0;
  for (int a = 0; a < nT[2]; ++a)
    for (int b = 0; b < nT[1]; ++b)
      for (int cc = 0; cc < nT[0]; ++cc) {
        if (j >= max_per_cell) {
          atomicOr(&flags[1], 1);
          continue;
        }
        const int tile = (T[2][a] * L.ty + T[1][b]) * L.tx + T[0][cc];
        tiles[(int64_t)c * max_per_cell + j] = tile;
        rank[(int64_t)c * max_per_cell + j] = atomicAdd(&cnt[tile], 1);
        ++j;
      }
  for (; j < max_per_cell; ++j) tiles[(int64_t)c * max_per_cell + j] = -1;
}

__global__ void k_fill_cells(int ncells, int max_per_cell, const int* tiles, const int* rank,
                             const int* ptr, int* list) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)ncells * max_per_cell) return;
  const int t = tiles[i];
  if (t < 0) return;
  list[ptr[t] + rank[i]] = (int)(i / max_per_cell);
}

// Exclusive scan of n counts into ptr[0..n] with one work-group.
__global__ __launch_bounds__(1024) void k_scan(const int* __restrict__ cnt, int* __restrict__ ptr,
                                               int n) {
  __shared__ int part[1024];
  const int tid = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int a = min(n, tid * chunk), b = min(n, a + chunk);
  int sum = 0;
  for (int i = a; i < b; ++i) sum += cnt[i];
  part[tid] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - sum;
  for (int i = a; i < b; ++i) {
    ptr[i] = run;
    run += cnt[i];
  }
  if (tid == 1023) ptr[n] = part[1023];
}

// Sort every segment [ptr[s], ptr[s+1]) of distinct ints by rank counting.
__global__ __launch_bounds__(256) void k_sort_segments(const int* __restrict__ ptr, int* list,
                                                       int* tmp) {
  const int s = blockIdx.x;
  const int a = ptr[s], b = ptr[s + 1];
  for (int i = a + threadIdx.x; i < b; i += blockDim.x) {
    const int x = list[i];
    int r = 0;
    for (int j = a; j < b; ++j) r += list[j] < x;
    tmp[a + r] = x;
  }
  __syncthreads();
  for (int i = a + threadIdx.x; i < b; i += blockDim.x) list[i] = tmp[i];
}

__global__ void k_fill_i32(int* p, int v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_scan(const int* cnt, int* ptr, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, cnt, ptr, n);
  return hipGetLastError();
}

hipError_t launch_bin_vertices(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                               hipStream_t s) {
  hipError_t e = launch_fill_i32(b.touch_cnt, 0, L.ntiles + 1, s);
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)c.n * m.nv;
  if (n > 0) {
    hipLaunchKernelGGL(k_bin_vertices, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c, m, L,
                       b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_scan(b.touch_cnt, b.touch_ptr, L.ntiles, s)) != hipSuccess) return e;
  if (n > 0) {
    hipLaunchKernelGGL(k_fill_touch, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       L.max_touch, b);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_bin_cells(const Cells& c, const Mesh& m, const Lattice& L, int* cnt, int* ptr,
                            int* rank, int* tiles, int* list, int64_t cap, int max_per_cell,
                            int* flags, hipStream_t s) {
  (void)cap;
  hipError_t e = launch_fill_i32(cnt, 0, L.ntiles + 1, s);
  if (e != hipSuccess) return e;
  if (c.n > 0) {
    hipLaunchKernelGGL(k_cell_tiles, dim3(c.n), dim3(64), 0, s, c, m, L, cnt, tiles, rank,
                       max_per_cell, flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_scan(cnt, ptr, L.ntiles, s)) != hipSuccess) return e;
  const int64_t n = (int64_t)c.n * max_per_cell;
  if (n > 0) {
    hipLaunchKernelGGL(k_fill_cells, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c.n,
                       max_per_cell, tiles, rank, ptr, list);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_sort_segments(const int* ptr, int* list, int* tmp, int nseg, hipStream_t s) {
  if (nseg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_segments, dim3(nseg), dim3(256), 0, s, ptr, list, tmp);
  return hipGetLastError();
}

}  // namespace hc
