// Device helpers of the vertex/cell binning to 8^3 tiles, shared by the
// binning kernels and the fused per-cell kernel.
#pragma once

#include <climits>

#include "stencil.h"

namespace hc {
namespace bin {

// Distinct tiles reached along one axis by K stencil nodes starting at p0,
// appended to out[cnt, cap) (already listed tiles are skipped), in stencil
// order.  Positions that stay inside the lattice (no wrap) are consecutive
// and meet at most two tiles (interior tiles are 8 wide): those take the
// first and last position's tiles directly.
__device__ inline int axis_tiles(int p0, int K, int n, int wall, int* out, int cnt = 0,
                                 int cap = 3) {
  if (cnt == 0 && cap >= 2) {
    const int q0 = wall ? max(p0, 0) : wrap(p0, n);
    const int q1 = wall ? min(p0 + K - 1, n - 1) : q0 + K - 1;
    if (wall || q1 < n) {
      if (q1 < q0) return 0;   // every position past a wall
      out[0] = q0 / kTile;
      const int t1 = q1 / kTile;
      if (t1 == out[0]) return 1;
      out[1] = t1;
      return 2;
    }
  }
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
    if (!seen && cnt < cap) out[cnt++] = t;
  }
  return cnt;
}

// Tiles reached by the stencil of a vertex of cell c at offset o, per axis,
// and its owner tile.  The reached tiles are the products T[2] x T[1] x T[0].
// With sheared periodic images the z stencil may reach two images, and each
// image's nodes sit at the vertex's x displaced by that image's shift; the
// reached tiles are then the (z tile, x tile) pairs of each image's own
// nodes times the y tiles.  Those pairs (at most 4: one z tile per image
// when the stencil crosses the boundary, with at most 2 x tiles each) are
// stored as T[2][p], T[0][p] with nT[0] = pairs and nT[2] = 1.
// LE = false compiles the enumeration without the sheared-image branch (its
// dynamically indexed arrays would otherwise move the arrays of every
// lattice into scratch memory); such a caller must not be given images.
template <bool LE = true>
__device__ inline int vertex_tiles(const Cells& C, const Lattice& L, int c, const float* o,
                                   int (&T)[3][4], int (&nT)[3]) {
  const int K = L.kernel;
  const int b = K == 4 ? -1 : 0;
  const int n[3] = {L.nx, L.ny, L.nz};
  int own[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int p = C.origin[3 * c + d] + (int)floorf(o[d]);
    nT[d] = axis_tiles(p + b, K, n[d], L.bc[d] == 1, T[d]);
    own[d] = (L.bc[d] == 1 ? min(max(p, 0), n[d] - 1) : wrap(p, n[d])) / kTile;
  }
  if (LE && L.le) {
    const int pz = C.origin[3 * c + 2] + (int)floorf(o[2]);
    const int ma = floor_div(pz + b, L.nz);
    int xt[2][4], nxt[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      // one rounding, as the lattice pass forms the same displaced x
      const float xi = fmaf(-(float)(ma + i), L.le_delta, o[0]);
      nxt[i] = axis_tiles(C.origin[3 * c] + (int)floorf(xi) + b, K, L.nx, 0, xt[i], 0, 4);
    }
    int np = 0;
    for (int k = 0; k < K; ++k) {
      const int p = pz + b + k;
      const int i = floor_div(p, L.nz) - ma;   // 0 or 1: the image of this z node
      const int zt = wrap(p, L.nz) / kTile;
      for (int q = 0; q < nxt[i]; ++q) {
        bool seen = false;
        for (int r = 0; r < np; ++r) seen = seen || (T[2][r] == zt && T[0][r] == xt[i][q]);
        if (!seen && np < 4) {
          T[0][np] = xt[i][q];
          T[2][np] = zt;
          ++np;
        }
      }
    }
    nT[0] = np;
    nT[2] = 1;
    const float xo = o[0] - (float)floor_div(pz, L.nz) * L.le_delta;
    own[0] = wrap(C.origin[3 * c] + (int)floorf(xo), L.nx) / kTile;
  }
  return (own[2] * L.ty + own[1]) * L.tx + own[0];
}

// Tile of slot j of a vertex: j runs over x fastest, then y, then z (over
// the (z, x) pairs, then y, with sheared images).
template <bool LE = true>
__device__ inline int slot_tile(const Lattice& L, const int (&T)[3][4], const int (&nT)[3], int j) {
  if (LE && L.le) {
    const int p = j % nT[0], r = j / nT[0];
    return (T[2][p] * L.ty + T[1][r]) * L.tx + T[0][p];
  }
  const int a = j / (nT[0] * nT[1]), r = j % (nT[0] * nT[1]);
  return (T[2][a] * L.ty + T[1][r / nT[0]]) * L.tx + T[0][r % nT[0]];
}

constexpr int kHash = 256;   // distinct tiles one cell may reach

// LDS bytes per vertex that bin_cell needs for its slot records.
__host__ __device__ inline int slot_lds_per_vertex(int max_touch) { return 3 * max_touch; }

// One work-group per cell.  Every (vertex, reached tile) pair gets a local
// rank in an LDS table keyed by tile; then one global atomic per distinct
// tile reserves a contiguous block of that tile's list, and the pairs are
// written at block base + local rank.  Tile lists have a fixed capacity of
// B.cap entries; an overflow raises flags[1] bit 4.
// The table is indexed directly on plain lattices: the tiles a cell reaches
// form a cyclic box of at most kSpan tiles per axis (from the cell's extent
// in stencil positions), and a pair's slot is its tile's offset in that
// box.  Larger cells, and lattices with sheared images, use an LDS hash
// with linear probing instead.
// pos: the cell's vertex offsets [nv][3] (global or LDS); keys, count and
// base: LDS arrays of kHash ints; srank / shash: LDS [nv * max_touch]
// records of each pair's rank and table slot (rank 0xffff: no slot).
constexpr int kSpan = 6;   // tiles per axis of the direct table (kSpan^3 <= kHash)
static_assert(kSpan * kSpan * kSpan <= kHash, "direct table exceeds the LDS table");

__device__ inline int wave_min_i(int v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = min(v, __shfl_xor(v, d));
  return v;
}

template <bool LE = true>
__device__ inline void bin_cell(const Cells& C, const Mesh& M, const Lattice& L, const Bins& B, int c,
                                const float* pos, int* keys, int* count, int* base,
                                unsigned short* srank, unsigned char* shash, int tid, int nthr) {
  const bool plain = !(LE && L.le);
  const int K = L.kernel, b0 = K == 4 ? -1 : 0;
  const int n[3] = {L.nx, L.ny, L.nz}, T[3] = {L.tx, L.ty, L.tz};
  // the cell's extent in floor(offset) per axis: -min in keys[250..252], max in keys[253..255]
  if (plain && tid < 6) keys[250 + tid] = INT_MIN;
  __syncthreads();
  if (plain) {
    int e[6] = {INT_MIN, INT_MIN, INT_MIN, INT_MIN, INT_MIN, INT_MIN};
    for (int vl = tid; vl < M.nv; vl += nthr)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int f = (int)floorf(pos[3 * vl + d]);
        e[d] = max(e[d], -f);
        e[3 + d] = max(e[3 + d], f);
      }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int w = -wave_min_i(-e[q]);
      if ((tid & (kWave - 1)) == 0) atomicMax(&keys[250 + q], w);
    }
  }
  __syncthreads();
  // first tile and span of the cyclic box of reached tiles per axis
  bool direct = plain;
  int t_lo[3] = {0, 0, 0};
  if (plain) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int lo = C.origin[3 * c + d] - keys[250 + d] + b0;
      const int hi = C.origin[3 * c + d] + keys[253 + d] + b0 + K - 1;
      int span;
      if (L.bc[d] == 1) {
        const int a = max(lo, 0), z = min(hi, n[d] - 1);
        t_lo[d] = a / kTile;
        span = z >= a ? z / kTile - t_lo[d] + 1 : 1;
      } else if (hi - lo + 1 >= n[d]) {
        t_lo[d] = 0;
        span = T[d];
      } else {
        t_lo[d] = wrap(lo, n[d]) / kTile;
        const int t_hi = wrap(hi, n[d]) / kTile;
        span = (t_hi - t_lo[d] + T[d]) % T[d] + 1;
      }
      direct = direct && span <= kSpan;
    }
  }
  __syncthreads();   // every thread has read the extent
  for (int i = tid; i < kHash; i += nthr) {
    keys[i] = -1;
    count[i] = 0;
  }
  __syncthreads();
  for (int vl = tid; vl < M.nv; vl += nthr) {
    const int64_t v = (int64_t)c * M.nv + vl;
    int Tt[3][4], nT[3];
    B.owner[v] = vertex_tiles<LE>(C, L, c, pos + 3 * vl, Tt, nT);
    int ntouch = nT[0] * nT[1] * nT[2];
    if (ntouch > L.max_touch) {  // excluded by the per-axis bound set at create
      atomicOr(&B.flags[1], 2);
      ntouch = L.max_touch;
    }
    B.ntouch[v] = ntouch;
    // the hash table: slot of a tile, or kHash when the table is full
    auto hash_slot = [&](int tile) {
      int h = (int)(((unsigned)tile * 2654435761u) >> 24);
      for (int probe = 0; probe < kHash; ++probe) {
        // nearly every lookup finds a key already present: read before CAS
        const int cur = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
        if (cur == tile) return h;
        if (cur == -1) {
          const int prev = atomicCAS(&keys[h], -1, tile);
          if (prev == -1 || prev == tile) return h;
        }
        h = (h + 1) & (kHash - 1);
      }
      return kHash;
    };
    auto record = [&](int j, int h) {
      const int s = vl * L.max_touch + j;
      if (h == kHash) {
        atomicOr(&B.flags[1], 8);
        srank[s] = 0xffff;
        return;
      }
      srank[s] = (unsigned short)atomicAdd(&count[h], 1);
      shash[s] = (unsigned char)h;
    };
    if (!plain) {
      for (int j = 0; j < ntouch; ++j) record(j, hash_slot(slot_tile<LE>(L, Tt, nT, j)));
      continue;
    }
    // plain lattices: slot j runs over the per-axis tiles, x fastest (as slot_tile)
    int j = 0;
#pragma unroll
    for (int iz = 0; iz < 3; ++iz) {
      if (iz >= nT[2]) break;
#pragma unroll
      for (int iy = 0; iy < 3; ++iy) {
        if (iy >= nT[1]) break;
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) {
          if (ix >= nT[0] || j >= ntouch) break;
          const int tile = (Tt[2][iz] * L.ty + Tt[1][iy]) * L.tx + Tt[0][ix];
          int h;
          if (direct) {   // the tile's offset in the cell's box, per axis
            int rx = Tt[0][ix] - t_lo[0], ry = Tt[1][iy] - t_lo[1], rz = Tt[2][iz] - t_lo[2];
            rx += rx < 0 ? T[0] : 0;
            ry += ry < 0 ? T[1] : 0;
            rz += rz < 0 ? T[2] : 0;
            h = (rz * kSpan + ry) * kSpan + rx;
            if (keys[h] != tile) keys[h] = tile;   // every writer stores the same tile
          } else {
            h = hash_slot(tile);
          }
          record(j, h);
          ++j;
        }
      }
    }
  }
  __syncthreads();
  for (int h = tid; h < kHash; h += nthr) {
    if (keys[h] < 0) continue;
    base[h] = atomicAdd(&B.touch_cnt[keys[h]], count[h]);
    if (base[h] + count[h] > B.cap) atomicOr(&B.flags[1], 4);
  }
  __syncthreads();
  for (int vl = tid; vl < M.nv; vl += nthr) {
    const int64_t v = (int64_t)c * M.nv + vl;
    const int ntouch = B.ntouch[v];
    for (int j = 0; j < ntouch; ++j) {
      const int s = vl * L.max_touch + j;
      if (srank[s] == 0xffff) continue;
      const int h = shash[s];
      const int p = base[h] + srank[s];
      if (p < B.cap) B.touch[(int64_t)keys[h] * B.cap + p] = (int)(v * 32 + j);
    }
  }
}

}  // namespace bin
}  // namespace hc
