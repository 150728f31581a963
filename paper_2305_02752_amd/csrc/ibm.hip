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
__device__ __forceinline__ void spread_body(Cells C, Mesh M, Lattice L, Bins B,
                                            const float* __restrict__ vec, float body, float* __restrict__ F) {
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

template <int K>
__global__ __launch_bounds__(256) void k_spread(Cells C, Mesh M, Lattice L, Bins B,
                                                const float* __restrict__ vec, float body,
                                                float* __restrict__ F) {
  spread_body<K>(C, M, L, B, vec, body, F);
}

template <int K>
__global__ __launch_bounds__(256) void k_spread_multi(const SpreadArgs* __restrict__ many) {
  const SpreadArgs& a = many[blockIdx.y];
  spread_body<K>(a.C, a.M, a.L, a.B, a.vec, a.body, a.F);
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

// ---------------------------------------------------------------------------
// Sorted-entry form of the two immersed-boundary phases (plain lattices).
//
// The (vertex, tile) entries of a tile are staged in LDS as compact records:
// per axis the tile-local nodes of the stencil positions that fall inside
// the tile, in stencil order, with their stencil index; the fractional
// position; the vertex force.  The records are ordered by the shape of
// their in-tile box (nodes per axis), so the lanes of a wave share their
// loop bounds, and each lane walks only its entry's in-tile nodes with
// statically indexed registers.  All four stencil weights of an axis come
// from one square root: with s = sqrt(1 + 4f(1 - f)), the weights of the
// nodes floor(X) - 1 .. floor(X) + 2 are (3 - 2f - s)/8, (3 - 2f + s)/8,
// (1 + 2f + s)/8 and (1 + 2f - s)/8 (Peskin's 4-point function at
// distances 1 + f, f, 1 - f, 2 - f).
//
// Spreading accumulates in LDS as int32 fixed point (node contributions
// truncated) at a power-of-two scale chosen per tile from a bound
// on every node sum: the sum over the tile's entries of their largest force
// component times the largest weight one entry puts on one node.  The bound
// is summed in integers (each term rounded up on a 2^-bexp grid of the tile's
// largest component), so it does not depend on the order of the entries;
// integer node sums do not either, so the result is bitwise reproducible
// although the order of the records is not.
namespace srt {

constexpr int kStage = 512;   // records staged at once (two per thread)
constexpr int kKeys = 64;     // box shapes: 1..4 in-tile nodes on each axis

struct Smem {
  int acc[3][512];          // spread accumulator; then the velocity (float bits)
  int4 geo[kStage];         // axis words x, y, z; entry code (vertex * 32 + slot)
  float4 fr[kStage];        // fractions x, y, z; force x
  float2 fyz[kStage];       // force y, z
  int cnt[kKeys];           // records per box shape, then the first record of each shape
  unsigned fmax;            // largest force component magnitude (float bits)
  int fsum;                 // sum of the entries' largest components, in units of fmax 2^-bexp
};

// In-tile stencil list along one axis: of the K positions base + k (wrapped
// on a periodic axis, dropped past a wall), those in [t0, t0 + 8) in
// stencil order; slot s holds (node - t0) | k << 3 at bits 5s..5s+4, the
// count sits at bits 20..22.  A stencil that does not run over the end of
// the lattice meets the tile in one contiguous run of positions.
template <int K>
__device__ __forceinline__ unsigned axis_word(int base, int n, int wall, int t0) {
  const int p0 = wall ? base : wrap(base, n);
  if (wall || p0 + K <= n) {
    const int lo = max(max(p0, t0), 0), hi = min(min(p0 + K, t0 + kTile), n);
    const int c = max(hi - lo, 0);
    const unsigned first = (unsigned)((lo - t0) | ((lo - p0) << 3));
    unsigned w = 0;
#pragma unroll
    for (int s = 0; s < K; ++s)   // slot s: node and stencil index both one past slot s - 1
      if (s < c) w |= (first + (unsigned)(s | (s << 3))) << (5 * s);
    return w | ((unsigned)c << 20);
  }
  unsigned w = 0;
  int c = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int q = p0 + k;
    q = q >= n ? q - n : q;   // q < n + K <= 2n (sides are at least 4)
    if (q >= t0 && q < t0 + kTile) {
      w |= (unsigned)((q - t0) | (k << 3)) << (5 * c);
      ++c;
    }
  }
  return w | ((unsigned)c << 20);
}

template <int K>
__device__ __forceinline__ void weights(float f, float (&W)[4]) {
  if (K == 4) {
    const float s = __builtin_amdgcn_sqrtf(fmaf(4.f * f, 1.f - f, 1.f));
    const float a = 3.f - 2.f * f, b = 1.f + 2.f * f;
    W[0] = 0.125f * (a - s);
    W[1] = 0.125f * (a + s);
    W[2] = 0.125f * (b + s);
    W[3] = 0.125f * (b - s);
  } else {
    W[0] = 1.f - f;
    W[1] = f;
    W[2] = 0.f;
    W[3] = 0.f;
  }
}

struct Axis {
  int n;
  int l[4];
  float w[4];
};

template <int K>
__device__ __forceinline__ void decode(unsigned word, float f, Axis& A) {
  float W[4];
  weights<K>(f, W);
  A.n = (int)((word >> 20) & 7u);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const unsigned q = (word >> (5 * s)) & 31u;
    const unsigned k = q >> 3;
    A.l[s] = (int)(q & 7u);
    const float lo = (k & 1u) ? W[1] : W[0], hi = (k & 1u) ? W[3] : W[2];
    A.w[s] = (k & 2u) ? hi : lo;
  }
}

// Largest weight one entry can put on one node: the product over the axes
// of the largest per-axis weight, 1/2 for the 4-point function and 1 for
// the hat (lattice sides of at least 4 keep the K positions of an axis on
// distinct nodes).
__device__ __forceinline__ float max_node_weight(const Lattice& L) { return L.kernel == 4 ? 0.125f : 1.f; }

// Units of fmax 2^-bexp that bound an entry's largest force component fm
// from above (fm <= fmax, rfmax a reciprocal of fmax within a few ulp: the
// product is within 0.2 units, so truncating and adding one unit bounds it);
// the grid is set by the list capacity (cap 2^bexp <= 2^30), so a full
// tile list's units sum to below 2^31.
__device__ __forceinline__ int bound_units(float fm, float fmax, float rfmax, int bexp) {
  return fmax > 0.f ? (int)(fm * rfmax * ldexpf(1.f, bexp)) + 1 : 1;
}

// Exponent k of the fixed-point scale 2^k: with the entries' largest force
// components summing to at most fsum units of fmax 2^-bexp, every node sum
// stays below 2^30 (half the int32 range, which also covers the rounding of
// the weights and of the contributions).
__device__ __forceinline__ int fix_exponent(int fsum, float fmax, float wmax, int bexp) {
  const float x = (float)fsum * ldexpf(fmax, -bexp) * wmax;
  if (!(x > 0.f)) return 30;     // no force (or NaN): any scale
  if (!(x < 3.0e38f)) return 0;  // infinite force: the move's non-finite check reports it
  int e;
  frexpf(x, &e);                 // x = m 2^e, m in [0.5, 1)
  return min(max(30 - e, -100), 100);
}

// Wave-wide max / sum with DPP lane swaps inside each row of 16 lanes (xor
// 1, xor 2, then the mirrored half-row and row), and the four row results
// combined in scalar registers; every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_swap(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ float wave_max(float v) {
  unsigned u = __float_as_uint(v);   // non-negative floats order as their bits
  u = max(u, (unsigned)dpp_swap<0xB1>((int)u));    // quad_perm [1,0,3,2]
  u = max(u, (unsigned)dpp_swap<0x4E>((int)u));    // quad_perm [2,3,0,1]
  u = max(u, (unsigned)dpp_swap<0x141>((int)u));   // row_half_mirror
  u = max(u, (unsigned)dpp_swap<0x140>((int)u));   // row_mirror
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)u, 0), b = (unsigned)__builtin_amdgcn_readlane((int)u, 16);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)u, 32), d = (unsigned)__builtin_amdgcn_readlane((int)u, 48);
  return __uint_as_float(max(max(a, b), max(c, d)));
}

__device__ __forceinline__ int wave_sum(int v) {
  v += dpp_swap<0xB1>(v);
  v += dpp_swap<0x4E>(v);
  v += dpp_swap<0x141>(v);
  v += dpp_swap<0x140>(v);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
         __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

__device__ __forceinline__ float entry_fmax(const Cells& C, const Bins& B, int t, int i) {
  const int v = B.touch[(int64_t)t * B.cap + i] >> 5;
  const float* fv = C.force + (int64_t)v * 3;
  return fmaxf(fabsf(fv[0]), fmaxf(fabsf(fv[1]), fabsf(fv[2])));
}

// Largest force component over entries [0, ne) of tile t into S.fmax, then
// the bound sum into S.fsum (both zeroed and synchronised by the caller).
// Each entry's largest component is gathered once and kept in the record
// space (free until the staging) when the list fits it, else gathered
// again for the sum.  Ends synchronised.
constexpr int kBoundKeep = (int)(sizeof(float4) * kStage / sizeof(float));
__device__ __forceinline__ void force_bound(const Cells& C, const Bins& B, int t, int ne, Smem& S) {
  float* kept = reinterpret_cast<float*>(S.fr);
  const bool keep = ne <= kBoundKeep;
  float m = 0.f;
  for (int i = threadIdx.x; i < ne; i += blockDim.x) {
    const float f = entry_fmax(C, B, t, i);
    if (keep) kept[i] = f;
    m = fmaxf(m, f);
  }
  m = wave_max(m);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(&S.fmax, __float_as_uint(m));
  __syncthreads();
  const float fmx = __uint_as_float(S.fmax), rf = __builtin_amdgcn_rcpf(fmx);
  int u = 0;
  for (int i = threadIdx.x; i < ne; i += blockDim.x)
    u += bound_units(keep ? kept[i] : entry_fmax(C, B, t, i), fmx, rf, B.bexp);
  u = wave_sum(u);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&S.fsum, u);
  __syncthreads();
}

// Chunks of a list longer than kStage: a first one of 1..kStage entries,
// then full ones, so that the last chunk staged for the spread is a full
// one, and it is still staged when the interpolation starts.
__device__ __forceinline__ int first_chunk(int ne) { return ne - (ne - 1) / kStage * kStage; }

// Stage entries [e0, e0 + m) of tile t (m <= kStage, two per thread) as
// records ordered by box shape; with_force also stages the forces, and with
// bound as well the force bound of these entries (S.fmax, S.fsum: the whole
// tile's when they are all staged at once).  Ends synchronised.
template <int K>
__device__ __forceinline__ void stage(const Cells& C, const Mesh& M, const Lattice& L, const Bins& B, int t,
                             int x0, int y0, int z0, int e0, int m, bool with_force, bool bound,
                             Smem& S) {
  for (int i = threadIdx.x; i < kKeys; i += blockDim.x) S.cnt[i] = 0;
  __syncthreads();
  int4 g[2];
  float4 fr[2];
  float2 fyz[2];
  int key[2], rank[2];
  float fm[2] = {0.f, 0.f};
  const int b = K == 4 ? -1 : 0;
  const float rnv = __builtin_amdgcn_rcpf((float)M.nv);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = (int)threadIdx.x + h * (int)blockDim.x;
    key[h] = -1;
    rank[h] = 0;
    g[h] = make_int4(0, 0, 0, 0);
    fr[h] = make_float4(0.f, 0.f, 0.f, 0.f);
    fyz[h] = make_float2(0.f, 0.f);
    if (i < m) {
      const int code = B.touch[(int64_t)t * B.cap + e0 + i];
      const int v = code >> 5, c = div_small(v, M.nv, rnv);
      const float* o = C.off + (int64_t)v * 3;
      const float ox = o[0], oy = o[1], oz = o[2];
      const float fx = floorf(ox), fy = floorf(oy), fz = floorf(oz);
      const unsigned wx = axis_word<K>(C.origin[3 * c] + (int)fx + b, L.nx, L.bc[0] == 1, x0);
      const unsigned wy = axis_word<K>(C.origin[3 * c + 1] + (int)fy + b, L.ny, L.bc[1] == 1, y0);
      const unsigned wz = axis_word<K>(C.origin[3 * c + 2] + (int)fz + b, L.nz, L.bc[2] == 1, z0);
      g[h] = make_int4((int)wx, (int)wy, (int)wz, code);
      fr[h] = make_float4(ox - fx, oy - fy, oz - fz, 0.f);
      if (with_force) {
        const float* fv = C.force + (int64_t)v * 3;
        fr[h].w = fv[0];
        fyz[h] = make_float2(fv[1], fv[2]);
        fm[h] = fmaxf(fabsf(fv[0]), fmaxf(fabsf(fv[1]), fabsf(fv[2])));
      }
      const int nx = (int)((wx >> 20) & 7u), ny = (int)((wy >> 20) & 7u), nz = (int)((wz >> 20) & 7u);
      key[h] = ((max(nz, 1) - 1) * 4 + (max(ny, 1) - 1)) * 4 + (max(nx, 1) - 1);
      rank[h] = atomicAdd(&S.cnt[key[h]], 1);
    }
  }
  if (bound) {
    const float w = wave_max(fmaxf(fm[0], fm[1]));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(&S.fmax, __float_as_uint(w));
  }
  __syncthreads();
  if (bound) {   // S.fmax is complete: the bound sum (read after the final barrier)
    const float fmx = __uint_as_float(S.fmax), rf = __builtin_amdgcn_rcpf(fmx);
    int u = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (key[h] >= 0) u += bound_units(fm[h], fmx, rf, B.bexp);
    u = wave_sum(u);
    if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&S.fsum, u);
  }
  if (threadIdx.x < kKeys) {   // first record of each shape: exclusive scan in the first wave
    const int own = S.cnt[threadIdx.x];
    int v = own;
#pragma unroll
    for (int d = 1; d < kKeys; d <<= 1) {
      const int u = __shfl_up(v, d);
      if ((int)threadIdx.x >= d) v += u;
    }
    S.cnt[threadIdx.x] = v - own;
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (key[h] < 0) continue;
    const int p = S.cnt[key[h]] + rank[h];
    S.geo[p] = g[h];
    S.fr[p] = fr[h];
    S.fyz[p] = fyz[h];
  }
  __syncthreads();
}

// Spread the m staged records into S.acc at the scale 2^kexp.  Node
// contributions are truncated (RN false) or rounded to nearest (RN true).
// A node sum's error is then at most one unit per contribution, or about
// the square root of the contributions times half a unit; the unit grows
// with the tile's force bound, i.e. with its entries, so crowded tiles
// (more than kRoundAbove entries) round.
constexpr int kRoundAbove = 1024;
template <int K, bool RN>
__device__ __forceinline__ void spread(int m, float scale, Smem& S) {
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const int4 g = S.geo[i];
    const float4 fr = S.fr[i];
    const float2 fyz = S.fyz[i];
    Axis X, Y, Z;
    decode<K>((unsigned)g.x, fr.x, X);
    decode<K>((unsigned)g.y, fr.y, Y);
    decode<K>((unsigned)g.z, fr.z, Z);
    const float fx = fr.w * scale, fy = fyz.x * scale, fz = fyz.y * scale;
    float gx[K], gy[K], gz[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
      gx[s] = X.w[s] * fx;
      gy[s] = X.w[s] * fy;
      gz[s] = X.w[s] * fz;
    }
#pragma unroll
    for (int iz = 0; iz < K; ++iz) {
      if (iz >= Z.n) continue;
#pragma unroll
      for (int iy = 0; iy < K; ++iy) {
        if (iy >= Y.n) continue;
        const float wzy = Z.w[iz] * Y.w[iy];
        const int row = Z.l[iz] * (kTile * kTile) + Y.l[iy] * kTile;
#pragma unroll
        for (int ix = 0; ix < K; ++ix) {
          if (ix >= X.n) continue;
          const int li = row + X.l[ix];
          if (RN) {
            atomicAdd(&S.acc[0][li], __float2int_rn(wzy * gx[ix]));
            atomicAdd(&S.acc[1][li], __float2int_rn(wzy * gy[ix]));
            atomicAdd(&S.acc[2][li], __float2int_rn(wzy * gz[ix]));
          } else {
            atomicAdd(&S.acc[0][li], (int)(wzy * gx[ix]));
            atomicAdd(&S.acc[1][li], (int)(wzy * gy[ix]));
            atomicAdd(&S.acc[2][li], (int)(wzy * gz[ix]));
          }
        }
      }
    }
  }
}

// Interpolation partial sums of the m staged records from the velocity
// held in S.acc (float bits), summed over the in-tile nodes in stencil
// order, into the records' partial-sum slots.
template <int K>
__device__ __forceinline__ void interp(int m, const Smem& S, int64_t stride, float4* __restrict__ partial) {
  const float* ux = reinterpret_cast<const float*>(S.acc[0]);
  const float* uy = reinterpret_cast<const float*>(S.acc[1]);
  const float* uz = reinterpret_cast<const float*>(S.acc[2]);
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const int4 g = S.geo[i];
    const float4 fr = S.fr[i];
    Axis X, Y, Z;
    decode<K>((unsigned)g.x, fr.x, X);
    decode<K>((unsigned)g.y, fr.y, Y);
    decode<K>((unsigned)g.z, fr.z, Z);
    // x slots past the entry's count read its first node with weight zero,
    // so a row's reads carry no branch and issue together
    float wx[K];
    int lx[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
      wx[s] = s < X.n ? X.w[s] : 0.f;
      lx[s] = s < X.n ? X.l[s] : X.l[0];
    }
    float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
    for (int iz = 0; iz < K; ++iz) {
      if (iz >= Z.n) continue;
#pragma unroll
      for (int iy = 0; iy < K; ++iy) {
        if (iy >= Y.n) continue;
        const float wzy = Z.w[iz] * Y.w[iy];
        const int row = Z.l[iz] * (kTile * kTile) + Y.l[iy] * kTile;
        float rx = 0.f, ry = 0.f, rz = 0.f;
#pragma unroll
        for (int ix = 0; ix < K; ++ix) {
          const int li = row + lx[ix];
          rx += wx[ix] * ux[li];
          ry += wx[ix] * uy[li];
          rz += wx[ix] * uz[li];
        }
        sx += wzy * rx;
        sy += wzy * ry;
        sz += wzy * rz;
      }
    }
    const int v = g.w >> 5, j = g.w & 31;
    partial[(int64_t)j * stride + v] = make_float4(sx, sy, sz, 0.f);
  }
}

}  // namespace srt

// The fused lattice pass of a plain lattice (no sheared images), one
// work-group per tile, with the sorted-entry IBM phases:
//  1. stage the tile's entries (records ordered by in-tile box shape) and
//     spread their forces into LDS (int32 fixed point at the tile's scale);
//  2. pull-stream + collide the tile's nodes (force = body force + spread
//     field), store their post-collision populations and keep (u, rho) in
//     LDS (writing the force and (u, rho) fields out when fields is
//     non-zero); interior sites as in k_tile_step;
//  3. interpolate u to the staged entries into their partial-sum slots.
// Tiles with more entries than the LDS stages at once take them in chunks
// (the scale then comes from a first pass over all their forces, and the
// interpolation stages again every chunk but the last).
// The struct arguments come by value from the single-box kernel (its own
// parameters) and by reference to global memory from the batched one: a
// reference to a kernel's by-value parameter, or a by-value copy of a record
// in global memory, would put the lattice record in scratch.
template <int K, bool W, class CT, class MT, class LT, class BT>
__device__ __forceinline__ void tile_step_sorted_body(CT C, MT M, LT L, BT B,
                                                      const float* __restrict__ gin,
                                                      float* __restrict__ gout, float* __restrict__ F,
                                                      float4* __restrict__ macro,
                                                      float4* __restrict__ partial, int fields,
                                                      unsigned char* __restrict__ mask) {
  __shared__ srt::Smem S;
  const int t = tile_of_block(L, blockIdx.x);
  if (t < 0) return;
  int x0, y0, z0;
  tile_origin(L, t, x0, y0, z0);
  for (int i = threadIdx.x; i < kTile * kTile * kTile; i += blockDim.x) {
    S.acc[0][i] = 0;
    S.acc[1][i] = 0;
    S.acc[2][i] = 0;
  }
  if (threadIdx.x == 0) {
    S.fmax = 0u;
    S.fsum = 0;
  }
  const int ne = C.n > 0 ? min(B.touch_cnt[t], B.cap) : 0;
  __syncthreads();
  int kexp = 0;
  if (ne > 0) {
    const bool one = ne <= srt::kStage;
    if (!one) srt::force_bound(C, B, t, ne, S);   // the scale must cover every chunk
    for (int e0 = 0, m = srt::first_chunk(ne); e0 < ne; e0 += m, m = srt::kStage) {
      srt::stage<K>(C, M, L, B, t, x0, y0, z0, e0, m, true, one, S);
      if (e0 == 0) kexp = srt::fix_exponent(S.fsum, __uint_as_float(S.fmax), srt::max_node_weight(L), B.bexp);
      if (ne > srt::kRoundAbove) srt::spread<K, true>(m, ldexpf(1.f, kexp), S);
      else srt::spread<K, false>(m, ldexpf(1.f, kexp), S);
      __syncthreads();
    }
  }

  const int64_t NP = L.np, h0 = (int64_t)t * 512;
  float* su0 = reinterpret_cast<float*>(S.acc[0]);
  float* su1 = reinterpret_cast<float*>(S.acc[1]);
  float* su2 = reinterpret_cast<float*>(S.acc[2]);
  // The tile-major site index is separable, site = Sx(x) + Sy(y) + Sz(z), so
  // the pull source x - e_q of every direction is two additions of the
  // parts of the node and its neighbours (wrapped) along each axis.  Site
  // indices stay below 2^30, so they serve as 32-bit element offsets.
  const unsigned py = (unsigned)L.tx << 9, pz = py * (unsigned)L.ty;
  for (int i = threadIdx.x; i < kTile * kTile * kTile; i += blockDim.x) {
    const int x = x0 + (i & 7), y = y0 + ((i >> 3) & 7), z = z0 + (i >> 6);
    if (x >= L.nx || y >= L.ny || z >= L.nz) {
      su0[i] = 0.f;
      su1[i] = 0.f;
      su2[i] = 0.f;
      continue;
    }
    const int xm = x == 0 ? L.nx - 1 : x - 1, xp = x == L.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? L.ny - 1 : y - 1, yp = y == L.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? L.nz - 1 : z - 1, zp = z == L.nz - 1 ? 0 : z + 1;
    // parts of the source coordinate x - e for e = -1, 0, +1
    const unsigned SX[3] = {(unsigned)(((xp >> 3) << 9) | (xp & 7)), (unsigned)(((x >> 3) << 9) | (x & 7)),
                            (unsigned)(((xm >> 3) << 9) | (xm & 7))};
    const unsigned SY[3] = {(unsigned)(yp >> 3) * py + (unsigned)((yp & 7) << 3),
                            (unsigned)(y >> 3) * py + (unsigned)((y & 7) << 3),
                            (unsigned)(ym >> 3) * py + (unsigned)((ym & 7) << 3)};
    const unsigned SZ[3] = {(unsigned)(zp >> 3) * pz + (unsigned)((zp & 7) << 6),
                            (unsigned)(z >> 3) * pz + (unsigned)((z & 7) << 6),
                            (unsigned)(zm >> 3) * pz + (unsigned)((zm & 7) << 6)};
    const unsigned hl = SX[1] + SY[1] + SZ[1];   // this node's site
    // wall layers: a source past the wall is the opposite population at the node itself
    bool lo = false, hi = false;
    if (W) {
      const int c = L.wall_axis == 0 ? x : (L.wall_axis == 1 ? y : z);
      const int n = L.wall_axis == 0 ? L.nx : (L.wall_axis == 1 ? L.ny : L.nz);
      lo = c == 0;
      hi = c == n - 1;
    }
    float g[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const unsigned src = SX[lbm::cx[q] + 1] + SY[lbm::cy[q] + 1] + SZ[lbm::cz[q] + 1];
      if (W) {
        const int ew = L.wall_axis == 0 ? lbm::cx[q] : (L.wall_axis == 1 ? lbm::cy[q] : lbm::cz[q]);
        const bool past = (ew == 1 && lo) || (ew == -1 && hi);
        g[q] = past ? gin[(int64_t)lbm::opp[q] * NP + hl] : gin[(int64_t)q * NP + src];
      } else {
        g[q] = (gin + (int64_t)q * NP)[src];
      }
    }
    // each thread reads and then overwrites only its own nodes' slots
    const float fx = L.g[0] + ldexpf((float)S.acc[0][i], -kexp);
    const float fy = L.g[1] + ldexpf((float)S.acc[1][i], -kexp);
    const float fz = L.g[2] + ldexpf((float)S.acc[2][i], -kexp);
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
    su0[i] = ux;
    su1[i] = uy;
    su2[i] = uz;
    if (fields) {
      macro[h] = make_float4(ux, uy, uz, rho);
      F[h] = fx;
      F[NP + h] = fy;
      F[2 * NP + h] = fz;
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      float v = g[q];
      if (W) {   // the value heading into a moving wall carries Ladd's term
        const int ew = L.wall_axis == 0 ? lbm::cx[q] : (L.wall_axis == 1 ? lbm::cy[q] : lbm::cz[q]);
        if (ew == -1 && lo) v += L.wc_lo[q] * rho;
        if (ew == 1 && hi) v += L.wc_hi[q] * rho;
      }
      // streamed out past the caches: the next step reads these values
      // back only after every tile has written (measured 2.875 -> 2.823 ms)
      __builtin_nontemporal_store(v, (gout + (int64_t)q * NP) + h);
    }
  }
  if (ne == 0) return;
  __syncthreads();
  const int64_t stride = (int64_t)C.n * M.nv;
  if (ne <= srt::kStage) {
    srt::interp<K>(ne, S, stride, partial);
  } else {
    // the last chunk of the spread is still staged; the others stage again
    srt::interp<K>(srt::kStage, S, stride, partial);
    __syncthreads();
    for (int e0 = 0, m = srt::first_chunk(ne); e0 < ne - srt::kStage; e0 += m, m = srt::kStage) {
      srt::stage<K>(C, M, L, B, t, x0, y0, z0, e0, m, false, false, S);
      srt::interp<K>(m, S, stride, partial);
      __syncthreads();
    }
  }
  __syncthreads();   // every thread has read the count: leave it zero for the next binning
  if (threadIdx.x == 0) B.touch_cnt[t] = 0;
}

template <int K, bool W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_tile_step_sorted(
    Cells C, Mesh M, Lattice L, Bins B,
                                                          const float* __restrict__ gin,
                                                          float* __restrict__ gout,
                                                          float* __restrict__ F,
                                                          float4* __restrict__ macro,
                                                          float4* __restrict__ partial, int fields,
                                                          unsigned char* __restrict__ mask) {
  tile_step_sorted_body<K, W, Cells, Mesh, Lattice, Bins>(C, M, L, B, gin, gout, F, macro, partial, fields, mask);
}

// Batched form: box blockIdx.y.
template <int K, bool W>
__global__ __launch_bounds__(256) void k_tile_step_sorted_multi(const TileStepArgs* __restrict__ many) {
  const TileStepArgs& a = many[blockIdx.y];
  tile_step_sorted_body<K, W, const Cells&, const Mesh&, const Lattice&, const Bins&>(
      a.C, a.M, a.L, a.B, a.gin, a.gout, a.F, a.macro, a.partial, a.fields, a.mask);
}

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

hipError_t launch_spread_vec_multi(const SpreadArgs& a0, const SpreadArgs* dev, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)a0.L.ntiles, (unsigned)n);
  if (a0.L.kernel == 4)
    hipLaunchKernelGGL(k_spread_multi<4>, grid, dim3(256), 0, s, dev);
  else
    hipLaunchKernelGGL(k_spread_multi<2>, grid, dim3(256), 0, s, dev);
  return hipGetLastError();
}

// Boxes of one shape and one kind of boundary (walled or not), without
// sheared images.
hipError_t launch_tile_step_multi(const TileStepArgs& a0, const TileStepArgs* dev, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (a0.L.le) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tile_grid(a0.L), (unsigned)n);
  const bool w = a0.L.wall_axis >= 0;
  if (a0.L.kernel == 4) {
    if (w) hipLaunchKernelGGL((k_tile_step_sorted_multi<4, true>), grid, dim3(256), 0, s, dev);
    else hipLaunchKernelGGL((k_tile_step_sorted_multi<4, false>), grid, dim3(256), 0, s, dev);
  } else {
    if (w) hipLaunchKernelGGL((k_tile_step_sorted_multi<2, true>), grid, dim3(256), 0, s, dev);
    else hipLaunchKernelGGL((k_tile_step_sorted_multi<2, false>), grid, dim3(256), 0, s, dev);
  }
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
  else if (L.kernel == 4 && L.wall_axis >= 0)
    hipLaunchKernelGGL((k_tile_step_sorted<4, true>), grid, dim3(256), 0, s, c, m, L, b, gin, gout, F,
                       macro, partial, fl, mask);
  else if (L.kernel == 4)
    hipLaunchKernelGGL((k_tile_step_sorted<4, false>), grid, dim3(256), 0, s, c, m, L, b, gin, gout, F,
                       macro, partial, fl, mask);
  else if (L.le)
    hipLaunchKernelGGL((k_tile_step<2, true>), grid, dim3(256), 0, s, c, m, L, b, gin, gout, F,
                       macro, partial, fl, mask);
  else if (L.wall_axis >= 0)
    hipLaunchKernelGGL((k_tile_step_sorted<2, true>), grid, dim3(256), 0, s, c, m, L, b, gin, gout, F,
                       macro, partial, fl, mask);
  else
    hipLaunchKernelGGL((k_tile_step_sorted<2, false>), grid, dim3(256), 0, s, c, m, L, b, gin, gout, F,
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
