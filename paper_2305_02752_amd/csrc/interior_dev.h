// Lattice sites inside one cell (interior viscosity: Sec. 1, the cytosol is
// five times more viscous than plasma; Sec. 3.4, stiffened cells change the
// internal viscosity ratio), shared by the single-lattice marking kernel and
// the batched persistent kernel.  A site is inside by ray parity along z:
// the vertical line through it crosses the closed membrane at heights
// z_1 < z_2 < ..., and the site is inside when it lies strictly between
// z_(2k-1) and z_(2k).
//
// One work-group per cell.  The cell's (x, y) node columns within its
// bounding box form a small grid, held in LDS in chunks of whole rows of at
// most kMaxCols columns (one chunk for an undeformed cell); every triangle
// adds its crossing height to each column its projection covers (edge
// points are kept by exactly one of the two triangles sharing the edge:
// after orienting the triangle counter-clockwise in projection, edge P -> Q
// keeps them when Q.y > P.y, or Q.y == P.y and Q.x < P.x); each column then
// sorts its crossings and marks the nodes between pairs.
#pragma once

#include "common.h"
#include "stencil.h"

namespace hc {
namespace inside {

constexpr int kMaxCols = 320;        // (x, y) columns held in LDS at once (whole rows)
constexpr int kMaxCross = 8;         // crossings per column
constexpr int kMaxWaves = 16;        // wavefronts per work-group (up to 1024 threads)
constexpr float kMaxSpan = 1024.f;   // bounding-box side beyond which a cell is refused
constexpr float kMaxOff = 16777216.f;   // offsets from the cell origin beyond which it is refused

// LDS scratch of one marking work-group.
struct Lds {
  int cnt[kMaxCols];
  float zc[kMaxCols][kMaxCross];
  float bb[kMaxWaves][6];
  int box[6];   // lo_x, lo_y, ncx, ncy, lo_z, hi_z (cell-local nodes)
  float xr[2];  // the cell's x extent (cell-local)
};

// The lattice the marks go to.
struct Grid {
  int n[3];
  int bc[3];
  int le;           // sheared periodic images across z (flow along x)
  float le_delta;   // their displacement at this step
};

// The edge tests and crossing heights are evaluated without contraction to
// fused multiply-adds, so every decision is the one plain float32
// arithmetic (each product and sum rounded) takes.
__device__ inline bool edge_in(float px, float py, float qx, float qy, float x, float y) {
#pragma clang fp contract(off)
  const float w = (qx - px) * (y - py) - (qy - py) * (x - px);
  const bool keep = qy > py || (qy == py && qx < px);
  return w > 0.f || (w == 0.f && keep);
}

// Writes `bit` to mask[site(x, y, z)] for every lattice site inside the
// cell whose vertex offsets (from its integer origin o) are in sp [nv][3]
// in LDS; with src non-null they are first copied there from src (global),
// in the same pass that finds the cell's extent.  All nthr threads of the work-group call it (nthr a
// multiple of 64, at most 1024); it synchronises the work-group.  A cell
// too large for the column grid raises bit 4 of *err; more than kMaxCross
// crossings on a column raise bit 5.
template <class Site>
__device__ void mark_cell(const float* __restrict__ src, float* sp, int nv, const int* __restrict__ tri,
                          int nt, const int (&o)[3],
                          const Grid& G, Site site, unsigned char* __restrict__ mask, unsigned char bit,
                          int* err, Lds& S, int tid, int nthr) {
#pragma clang fp contract(off)
  float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
  for (int v = tid; v < nv; v += nthr) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float p;
      if (src) {
        p = src[3 * v + d];
        sp[3 * v + d] = p;
      } else {
        p = sp[3 * v + d];
      }
      lo[d] = fminf(lo[d], p);
      hi[d] = fmaxf(hi[d], p);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d)
    for (int m = kWave / 2; m > 0; m >>= 1) {
      lo[d] = fminf(lo[d], __shfl_xor(lo[d], m));
      hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], m));
    }
  if ((tid & (kWave - 1)) == 0)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      S.bb[tid / kWave][d] = lo[d];
      S.bb[tid / kWave][3 + d] = hi[d];
    }
  __syncthreads();
  if (tid == 0) {
    float l[3] = {S.bb[0][0], S.bb[0][1], S.bb[0][2]}, h[3] = {S.bb[0][3], S.bb[0][4], S.bb[0][5]};
    for (int w = 1; w < nthr / kWave; ++w)
      for (int d = 0; d < 3; ++d) {
        l[d] = fminf(l[d], S.bb[w][d]);
        h[d] = fmaxf(h[d], S.bb[w][3 + d]);
      }
    const float sx = h[0] - l[0], sy = h[1] - l[1], sz = h[2] - l[2];
    bool near = true;   // offsets small enough for exact integer conversion
    for (int d = 0; d < 3; ++d) near = near && fabsf(l[d]) < kMaxOff && fabsf(h[d]) < kMaxOff;
    if (near && sx < kMaxSpan && sy < kMaxSpan && sz < kMaxSpan) {
      S.box[0] = (int)ceilf(l[0]);
      S.box[1] = (int)ceilf(l[1]);
      S.box[2] = (int)floorf(h[0]) - S.box[0] + 1;
      S.box[3] = (int)floorf(h[1]) - S.box[1] + 1;
      S.box[4] = (int)ceilf(l[2]);
      S.box[5] = (int)floorf(h[2]);
      S.xr[0] = l[0];
      S.xr[1] = h[0];
    } else {   // non-finite positions (reported by the vertex move) or a cell far too large
      S.box[2] = S.box[3] = 0;
      if (sx >= kMaxSpan || sy >= kMaxSpan || sz >= kMaxSpan || !near) atomicOr(err, 16);
    }
  }
  __syncthreads();
  const int ly = S.box[1], ncy = S.box[3];
  if (ncy <= 0 || (!G.le && S.box[2] <= 0)) return;
  const int ox = o[0], oy = o[1], oz = o[2];
  // Sheared periodic images (gradient z, flow x): the nodes of image m,
  // m = floor(unwrapped z / nz), are inside when the cell's copy displaced
  // by -m Delta along x contains them, so their columns sit at cell-frame
  // x + m Delta.  Without images there is one pass, m = 0, with integer
  // columns.
  int m_lo = 0, m_hi = 0;
  if (G.le) {
    m_lo = floor_div(oz + S.box[4], G.n[2]);
    m_hi = floor_div(oz + S.box[5], G.n[2]);
  }
  for (int m = m_lo; m <= m_hi; ++m) {
    const float shift = G.le ? (float)m * G.le_delta : 0.f;
    // with a shift the column range is widened by one: columns outside the
    // cell's projection cross nothing
    const int lx = G.le ? (int)floorf(S.xr[0] - shift) : S.box[0];
    const int ncx = G.le ? (int)floorf(S.xr[1] - shift) - lx + 2 : S.box[2];
    if (ncx > kMaxCols) {   // a cell wider than the column grid along x
      if (tid == 0) atomicOr(err, 16);
      return;
    }
    // the columns in chunks of whole rows that fit the LDS grid (one chunk for
    // an undeformed cell)
    const int rows = kMaxCols / ncx;
    for (int r0 = 0; r0 < ncy; r0 += rows) {
      const int nr = min(rows, ncy - r0);
      for (int i = tid; i < nr * ncx; i += nthr) S.cnt[i] = 0;
      __syncthreads();
      for (int t = tid; t < nt; t += nthr) {
        const int ia = tri[3 * t], ib = tri[3 * t + 1], ic = tri[3 * t + 2];
        float ax = sp[3 * ia], ay = sp[3 * ia + 1], az = sp[3 * ia + 2];
        float bx = sp[3 * ib], by = sp[3 * ib + 1], bz = sp[3 * ib + 2];
        float cx = sp[3 * ic], cy = sp[3 * ic + 1], cz = sp[3 * ic + 2];
        const float area2 = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
        if (area2 == 0.f) continue;
        if (area2 < 0.f) {   // orient counter-clockwise in projection
          float tx = bx, ty = by, tz = bz;
          bx = cx, by = cy, bz = cz;
          cx = tx, cy = ty, cz = tz;
        }
        const float A = fabsf(area2);
        const float tx0 = fminf(ax, fminf(bx, cx)), tx1 = fmaxf(ax, fmaxf(bx, cx));
        const int x0 = max(G.le ? (int)floorf(tx0 - shift) : (int)ceilf(tx0), lx);
        const int x1 = min(G.le ? (int)floorf(tx1 - shift) + 1 : (int)floorf(tx1), lx + ncx - 1);
        const int y0 = max((int)ceilf(fminf(ay, fminf(by, cy))), ly + r0);
        const int y1 = min((int)floorf(fmaxf(ay, fmaxf(by, cy))), ly + r0 + nr - 1);
        for (int iy = y0; iy <= y1; ++iy)
          for (int ix = x0; ix <= x1; ++ix) {
            const float x = (float)ix + shift, y = (float)iy;
            if (!(edge_in(ax, ay, bx, by, x, y) && edge_in(bx, by, cx, cy, x, y) &&
                  edge_in(cx, cy, ax, ay, x, y)))
              continue;
            const float wa = (bx - x) * (cy - y) - (by - y) * (cx - x);
            const float wb = (cx - x) * (ay - y) - (cy - y) * (ax - x);
            const float wc = (ax - x) * (by - y) - (ay - y) * (bx - x);
            const float z = (wa * az + wb * bz + wc * cz) / A;
            const int col = (iy - ly - r0) * ncx + (ix - lx);
            const int slot = atomicAdd(&S.cnt[col], 1);
            if (slot < kMaxCross) S.zc[col][slot] = z;
            else atomicOr(err, 32);
          }
      }
      __syncthreads();
      for (int col = tid; col < nr * ncx; col += nthr) {
        const int n = min(S.cnt[col], kMaxCross);
        if (n < 2) continue;
        float z[kMaxCross];
        for (int k = 0; k < kMaxCross; ++k) z[k] = k < n ? S.zc[col][k] : 3e38f;
        for (int i = 1; i < kMaxCross; ++i)   // insertion sort, fixed trip counts
          for (int j = i; j > 0; --j)
            if (z[j] < z[j - 1]) {
              const float s = z[j];
              z[j] = z[j - 1];
              z[j - 1] = s;
            }
        int xs = ox + lx + col % ncx, ys = oy + ly + r0 + col / ncx;
        if (G.bc[0] == 1) {
          if (xs < 0 || xs >= G.n[0]) continue;
        } else {
          xs = wrap(xs, G.n[0]);
        }
        if (G.bc[1] == 1) {
          if (ys < 0 || ys >= G.n[1]) continue;
        } else {
          ys = wrap(ys, G.n[1]);
        }
        for (int k = 0; k + 1 < n; k += 2) {
          // the heights lie within the cell's bounded z extent
          const int z0 = (int)floorf(z[k]) + 1, z1 = (int)ceilf(z[k + 1]) - 1;
          for (int iz = z0; iz <= z1; ++iz) {
            int zs = oz + iz;
            if (G.le && floor_div(zs, G.n[2]) != m) continue;   // a node of another image
            if (G.bc[2] == 1) {
              if (zs < 0 || zs >= G.n[2]) continue;
            } else {
              zs = wrap(zs, G.n[2]);
            }
            const int64_t h = site(xs, ys, zs);
            mask[h] = bit;
          }
        }
      }
      __syncthreads();   // the grid is reused by the next chunk
    }
  }
}

}  // namespace inside
}  // namespace hc
