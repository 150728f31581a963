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
#include "binning_dev.h"

namespace hc {
namespace {

template <bool LE>
__device__ __forceinline__ void bin_vertices_body(Cells C, Mesh M, Lattice L, Bins B) {
  extern __shared__ unsigned short slots[];
  __shared__ int keys[bin::kHash], count[bin::kHash], base[bin::kHash];
  const int c = blockIdx.x;
  unsigned short* srank = slots;
  unsigned char* shash = reinterpret_cast<unsigned char*>(slots + (size_t)M.nv * L.max_touch);
  bin::bin_cell<LE>(C, M, L, B, c, C.off + (int64_t)c * M.nv * 3, keys, count, base, srank, shash,
                    threadIdx.x, blockDim.x);
}

template <bool LE, int kThreads>
__global__ __launch_bounds__(kThreads) void k_bin_vertices(Cells C, Mesh M, Lattice L, Bins B) {
  bin_vertices_body<LE>(C, M, L, B);
}

// Batched form: box blockIdx.y.
template <int kThreads>
__global__ __launch_bounds__(kThreads) void k_bin_vertices_multi(const BinArgs* __restrict__ many) {
  const BinArgs& a = many[blockIdx.y];
  bin_vertices_body<false>(a.C, a.M, a.L, a.B);
}

// Copy the fixed-capacity tile lists into CSR form (read-out path).
__global__ __launch_bounds__(256) void k_compact_touch(Bins B, const int* __restrict__ ptr,
                                                       int* __restrict__ out) {
  const int t = blockIdx.x;
  const int n = ptr[t + 1] - ptr[t];
  for (int i = threadIdx.x; i < n; i += blockDim.x) out[ptr[t] + i] = B.touch[(int64_t)t * B.cap + i];
}

__global__ void k_clamp_counts(const int* __restrict__ cnt, int* __restrict__ out, int cap, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = min(cnt[i], cap);
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

// Exclusive scan of n counts into ptr[0..n]: per-block scan of 4096
// entries (coalesced), a one-block scan of the block sums, then the offsets.
constexpr int kScanBlock = 1024, kScanItems = 4;

__device__ inline int block_exclusive_scan(int x, int* part, int* total) {
  const int tid = threadIdx.x;
  part[tid] = x;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const int y = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += y;
    __syncthreads();
  }
  const int incl = part[tid];
  *total = part[kScanBlock - 1];
  __syncthreads();
  return incl - x;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_blocks(const int* __restrict__ cnt,
                                                            int* __restrict__ ptr,
                                                            int* __restrict__ sums, int n) {
  __shared__ int part[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanItems;
  int x[kScanItems], s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    x[k] = i < n ? cnt[i] : 0;
    s += x[k];
  }
  int total;
  int run = block_exclusive_scan(s, part, &total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    if (i < n) ptr[i] = run;
    run += x[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(int* __restrict__ sums, int nb,
                                                          int* __restrict__ ptr, int n) {
  __shared__ int part[kScanBlock];
  int carry = 0;
  for (int a = 0; a < nb; a += kScanBlock) {
    const int i = a + threadIdx.x;
    const int x = i < nb ? sums[i] : 0;
    int total;
    const int ex = block_exclusive_scan(x, part, &total);
    if (i < nb) sums[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) ptr[n] = carry;
}

__global__ __launch_bounds__(256) void k_scan_add(int* __restrict__ ptr, const int* __restrict__ sums,
                                                  int n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ptr[i] += sums[i / (kScanBlock * kScanItems)];
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

hipError_t launch_scan(const int* cnt, int* ptr, int* sums, int n, hipStream_t s) {
  const int nb = (n + kScanBlock * kScanItems - 1) / (kScanBlock * kScanItems);
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(kScanBlock), 0, s, cnt, ptr, sums, n);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, s, sums, nb, ptr, n);
  hipLaunchKernelGGL(k_scan_add, dim3((n + 255) / 256), dim3(256), 0, s, ptr, sums, n);
  return hipGetLastError();
}

// The tile-list counts must be zero on entry: every kernel that consumes
// the lists (the lattice pass, the vector spread) zeroes its tile's count
// when done, and the API zeroes them at bind time and after a read-out.
hipError_t launch_bin_vertices(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                               hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  const size_t lds = (size_t)m.nv * bin::slot_lds_per_vertex(L.max_touch);
  // wider work-groups when the cells are few (one work-group per cell)
  if (L.le)
    hipLaunchKernelGGL((k_bin_vertices<true, 256>), dim3(c.n), dim3(256), lds, s, c, m, L, b);
  else if (c.n <= 64)
    hipLaunchKernelGGL((k_bin_vertices<false, 1024>), dim3(c.n), dim3(1024), lds, s, c, m, L, b);
  else
    hipLaunchKernelGGL((k_bin_vertices<false, 256>), dim3(c.n), dim3(256), lds, s, c, m, L, b);
  return hipGetLastError();
}

hipError_t launch_bin_vertices_multi(const BinArgs& a0, const BinArgs* dev, int n, hipStream_t s) {
  if (n == 0 || a0.C.n == 0) return hipSuccess;
  if (a0.L.le) return hipErrorInvalidValue;
  const size_t lds = (size_t)a0.M.nv * bin::slot_lds_per_vertex(a0.L.max_touch);
  const dim3 grid((unsigned)a0.C.n, (unsigned)n);
  if (a0.C.n <= 64)
    hipLaunchKernelGGL((k_bin_vertices_multi<1024>), grid, dim3(1024), lds, s, dev);
  else
    hipLaunchKernelGGL((k_bin_vertices_multi<256>), grid, dim3(256), lds, s, dev);
  return hipGetLastError();
}

hipError_t launch_touch_csr(const Lattice& L, const Bins& b, int* cnt_tmp, int* ptr, int* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_clamp_counts, dim3((L.ntiles + 255) / 256), dim3(256), 0, s, b.touch_cnt,
                     cnt_tmp, b.cap, L.ntiles);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_scan(cnt_tmp, ptr, b.scan_tmp, L.ntiles, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_compact_touch, dim3(L.ntiles), dim3(256), 0, s, b, ptr, out);
  return hipGetLastError();
}

hipError_t launch_bin_cells(const Cells& c, const Mesh& m, const Lattice& L, int* cnt, int* ptr,
                            int* rank, int* tiles, int* list, int64_t cap, int max_per_cell,
                            int* flags, int* scan_tmp, hipStream_t s) {
  (void)cap;
  hipError_t e = launch_fill_i32(cnt, 0, L.ntiles + 1, s);
  if (e != hipSuccess) return e;
  if (c.n > 0) {
    hipLaunchKernelGGL(k_cell_tiles, dim3(c.n), dim3(64), 0, s, c, m, L, cnt, tiles, rank,
                       max_per_cell, flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_scan(cnt, ptr, scan_tmp, L.ntiles, s)) != hipSuccess) return e;
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
