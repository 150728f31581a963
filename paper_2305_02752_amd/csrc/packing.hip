// Force-bias dense packing of surrogate ellipsoids (Sec. 2.4): initial
// conditions for large suspensions.  Each ellipsoid encloses one cell;
// every iteration pushes each overlapping pair apart along the line through
// the centres, by an amount proportional to their overlapping volume (the
// pair force of Sec. 2.4), and all ellipsoids move at once.
//
// Overlap volume: a quadrature over the unit ball (the centres of an m^3
// grid over [-1, 1]^3 that fall inside it, Q points) mapped onto each
// ellipsoid; n_i(j) of ellipsoid i's points lie in j, and
// V_ij = (V_i n_i(j) + V_j n_j(i)) / (2 Q) is symmetric in the pair.  The
// inside tests are evaluated without contraction to fused multiply-adds, in
// a fixed operation order, so that each count is what plain float32
// arithmetic gives.
//
// Layout of one iteration (three launches):
//   1. clear the bin counts;
//   2. k_pack_bin: one thread per ellipsoid appends it to the fixed-capacity
//      list of its bin (bins are at least one pair reach wide, so
//      overlapping pairs lie in neighbouring bins);
//   3. k_pack_iter: one wavefront per ellipsoid gathers the candidates of
//      its neighbouring bins (one lane each) and keeps those whose bounding
//      spheres meet; for each of these the 64 lanes split the quadrature
//      points of both one-sided counts, and the push is accumulated in 2^-32
//      fixed point, so the sum does not depend on the order of the bin
//      lists.  The pushes of a pair are computed from the exact negatives of
//      each other, so they cancel exactly.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/hemo.h"
#include "common.h"
#include "host.h"

namespace hc {
namespace {

#pragma clang fp contract(off)

constexpr int kPackThreads = 256;
constexpr int kPackPerBlock = kPackThreads / kWave;   // one wavefront per ellipsoid
constexpr double kPushScale = 4294967296.0;           // 2^32 fixed-point units per lattice unit
constexpr double kVolScale = 1048576.0;               // 2^20 units per lattice volume

struct PackGeom {
  float L[3];
  int per[3];
  float lo[3], hi[3];
  int nb[3];
  float hb[3];
  float eta, max_move, max_semi;
  int m, cap;
};

__device__ inline int bin_axis(const PackGeom& G, int a, float x) {
  const int b = (int)floorf(x / G.hb[a]);
  return min(max(b, 0), G.nb[a] - 1);
}

__device__ inline float min_image(const PackGeom& G, int a, float d) {
  return G.per[a] ? d - G.L[a] * rintf(d / G.L[a]) : d;
}

// The frames of a pair, with dd = r_a - r_b (minimum image); R row-major
// (R[3 d + e]: component d of body axis e).  A point r_a + R_a (s_a u) lies
// inside b when |A u + bv| <= 1, with A = diag(1/s_b) (R_b^T R_a) diag(s_a)
// and bv = diag(1/s_b) R_b^T dd (frame 1); frame 2 swaps a and b (and
// negates dd).  M = R_b^T R_a serves both: R_a^T R_b is its transpose, with
// the same products summed in the same order.
__device__ inline void pair_frames(const float (&dd)[3], const float* Ra, const float* sa, const float* Rb,
                                   const float* sb, float (&A1)[3][3], float (&b1)[3], float (&A2)[3][3],
                                   float (&b2)[3]) {
  float ia[3], ib[3], M[3][3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    ia[e] = 1.f / sa[e];
    ib[e] = 1.f / sb[e];
  }
#pragma unroll
  for (int e = 0; e < 3; ++e)
#pragma unroll
    for (int c = 0; c < 3; ++c) M[e][c] = (Rb[e] * Ra[c] + Rb[3 + e] * Ra[3 + c]) + Rb[6 + e] * Ra[6 + c];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      A1[e][c] = (M[e][c] * sa[c]) * ib[e];
      A2[c][e] = (M[e][c] * sb[e]) * ia[c];
    }
    b1[e] = ((Rb[e] * dd[0] + Rb[3 + e] * dd[1]) + Rb[6 + e] * dd[2]) * ib[e];
    b2[e] = ((Ra[e] * -dd[0] + Ra[3 + e] * -dd[1]) + Ra[6 + e] * -dd[2]) * ia[e];
  }
}

__device__ inline bool in_frame(const float (&A)[3][3], const float (&bv)[3], float4 u) {
  float t[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) t[e] = ((A[e][0] * u.x + A[e][1] * u.y) + A[e][2] * u.z) + bv[e];
  return (t[0] * t[0] + t[1] * t[1]) + t[2] * t[2] <= 1.f;
}

// Whether the frame proves that no point of a lies in b: every quadrature
// point has |u| <= 1, so |t_e - bv_e| <= |row e of A|; when |bv_e| exceeds
// that bound plus 1 (with a margin far above the rounding of t), every
// point has |t_e| > 1.  A shortcut only: it never changes a count.
__device__ inline bool frame_separated(const float (&A)[3][3], const float (&bv)[3]) {
  bool sep = false;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    // |bv| (1 - 1e-4) > |row e| (1 + 1e-4) + 1.001, compared in squares
    const float r2 = A[e][0] * A[e][0] + A[e][1] * A[e][1] + A[e][2] * A[e][2];
    const float g = fabsf(bv[e]) * 0.9999f - 1.001f;
    sep = sep || (g > 0.f && g * g > r2 * 1.0003f);
  }
  return sep;
}

// n_a(b) from the frame of b seen from a: the 64 lanes split the points
// (point k on lane k mod 64) and a ballot counts them.  R > 0: each lane
// holds its R points in registers (up); R == 0: they are read from LDS (U).
template <int R>
__device__ inline int count_frame(const float (&A)[3][3], const float (&bv)[3],
                                  const float4 (&up)[R > 0 ? R : 1], const float4* U, int Q, int lane) {
  int n = 0;
  if constexpr (R > 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool in = r * kWave + lane < Q && in_frame(A, bv, up[r]);
      n += __popcll(__ballot(in));
    }
  } else {
    for (int k0 = 0; k0 < Q; k0 += kWave) {
      const int k = k0 + lane;
      const bool in = k < Q && in_frame(A, bv, U[k]);
      n += __popcll(__ballot(in));
    }
  }
  return n;
}

__global__ __launch_bounds__(256) void k_pack_bin(PackGeom G, const float* __restrict__ r, int n,
                                                  int* __restrict__ cnt, int* __restrict__ items,
                                                  int* __restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = r[3 * i], y = r[3 * i + 1], z = r[3 * i + 2];
  if (!(fabsf(x) < 1e30f && fabsf(y) < 1e30f && fabsf(z) < 1e30f)) {
    atomicOr(&flags[0], 1);
    return;
  }
  const int b = (bin_axis(G, 2, z) * G.nb[1] + bin_axis(G, 1, y)) * G.nb[0] + bin_axis(G, 0, x);
  const int slot = atomicAdd(&cnt[b], 1);
  if (slot < G.cap) items[(int64_t)b * G.cap + slot] = i;
  else atomicOr(&flags[1], 1);
}

// Neighbour bin offsets along one axis: -1, 0, 1 without repeats when a
// periodic axis has fewer than 3 bins; wall axes skip bins off the grid.
__device__ inline int axis_bins(const PackGeom& G, int a, int b, int (&out)[3]) {
  int k = 0;
  if (G.per[a]) {
    if (G.nb[a] >= 3) {
      out[k++] = b == 0 ? G.nb[a] - 1 : b - 1;
      out[k++] = b;
      out[k++] = b == G.nb[a] - 1 ? 0 : b + 1;
    } else {
      for (int q = 0; q < G.nb[a]; ++q) out[k++] = q;
    }
  } else {
    for (int o = -1; o <= 1; ++o)
      if (b + o >= 0 && b + o < G.nb[a]) out[k++] = b + o;
  }
  return k;
}

__device__ inline float lane_f(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// One iteration for every ellipsoid: pushes from the positions rin, written
// to rout when move is set; per ellipsoid, the fixed-point overlapping
// volume with higher-indexed partners (vol) and their number (pairs).
// A wavefront first gathers the candidates of all its neighbour bins at
// once (one lane per candidate: index, separation, bounding-sphere test),
// then takes the pairs that pass one after another, uniformly.
template <int R>
__global__ __launch_bounds__(kPackThreads) void k_pack_iter(
    PackGeom G, const float* __restrict__ rin, float* __restrict__ rout, const float* __restrict__ rot,
    const float* __restrict__ semi, int n, const int* __restrict__ cnt, const int* __restrict__ items,
    long long* __restrict__ vol, int* __restrict__ pairs, int move, int* __restrict__ flags) {
  extern __shared__ float4 U[];   // the quadrature points, [Q]
  __shared__ int nU;
  if (threadIdx.x == 0) nU = 0;
  __syncthreads();
  const float inv_m = 1.f / (float)G.m;
  for (int k = threadIdx.x; k < G.m * G.m * G.m; k += blockDim.x) {
    const int a = k % G.m, b = (k / G.m) % G.m, c = k / (G.m * G.m);
    // (2a + 1) / m - 1, exact for m a power of two
    const float ux = (float)(2 * a + 1) * inv_m - 1.f;
    const float uy = (float)(2 * b + 1) * inv_m - 1.f;
    const float uz = (float)(2 * c + 1) * inv_m - 1.f;
    if (ux * ux + uy * uy + uz * uz <= 1.f) U[atomicAdd(&nU, 1)] = make_float4(ux, uy, uz, 0.f);
  }
  __syncthreads();
  const int Q = nU;
  const int lane = threadIdx.x & (kWave - 1);
  float4 up[R > 0 ? R : 1];
  if constexpr (R > 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) up[r] = r * kWave + lane < Q ? U[r * kWave + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  const int i = blockIdx.x * kPackPerBlock + threadIdx.x / kWave;
  if (i >= n) return;

  float ri[3], Ri[9], si[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ri[d] = rin[3 * i + d];
    si[d] = semi[3 * i + d];
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) Ri[e] = rot[9 * i + e];
  const float smax_i = fmaxf(si[0], fmaxf(si[1], si[2]));
  if (lane == 0 && !(smax_i <= G.max_semi && si[0] > 0.f && si[1] > 0.f && si[2] > 0.f))
    atomicOr(&flags[2], 1);
  const float Vi = 4.18879020478639f * si[0] * si[1] * si[2];   // 4 pi / 3 s0 s1 s2

  // neighbour bins: lane l < nbn holds bin l, its candidate count and offset
  int Bz[3], By[3], Bx[3];
  const int nz = axis_bins(G, 2, bin_axis(G, 2, ri[2]), Bz);
  const int ny = axis_bins(G, 1, bin_axis(G, 1, ri[1]), By);
  const int nx = axis_bins(G, 0, bin_axis(G, 0, ri[0]), Bx);
  const int nbn = nz * ny * nx;
  int my_bin = 0, my_cnt = 0;
  if (lane < nbn) {
    const int a = lane / (ny * nx), b = (lane / nx) % ny, c = lane % nx;
    my_bin = (Bz[a] * G.nb[1] + By[b]) * G.nb[0] + Bx[c];
    my_cnt = min(cnt[my_bin], G.cap);
  }
  int incl = my_cnt;
  for (int d = 1; d < kWave; d <<= 1) {
    const int v = __shfl_up(incl, d);
    if (lane >= d) incl += v;
  }
  const int total = __shfl(incl, kWave - 1);
  const int excl = incl - my_cnt;

  long long push[3] = {0, 0, 0};
  long long vsum = 0;
  int npair = 0;
  for (int base = 0; base < total; base += kWave) {
    const int k = base + lane;
    // owning bin of candidate k: the last bin whose offset is <= k
    int owner = 0;
    for (int l = 1; l < nbn; ++l) owner = __shfl(excl, l) <= k ? l : owner;
    const int bin = __shfl(my_bin, owner);
    const int slot = k - __shfl(excl, owner);
    bool pass = false;
    int j = -1;
    float dd[3] = {0.f, 0.f, 0.f}, sj[3] = {1.f, 1.f, 1.f};
    if (k < total) {
      j = items[(int64_t)bin * G.cap + slot];
      if (j != i) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          dd[d] = min_image(G, d, ri[d] - rin[3 * j + d]);
          sj[d] = semi[3 * j + d];
        }
        const float d2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
        const float reach = smax_i + fmaxf(sj[0], fmaxf(sj[1], sj[2]));
        pass = d2 < reach * reach;
      }
    }
    unsigned long long todo = __ballot(pass);
    while (todo) {
      const int src = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int jj = __builtin_amdgcn_readlane(j, src);
      const float pd[3] = {lane_f(dd[0], src), lane_f(dd[1], src), lane_f(dd[2], src)};
      const float ps[3] = {lane_f(sj[0], src), lane_f(sj[1], src), lane_f(sj[2], src)};
      float Rj[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) Rj[e] = rot[9 * (int64_t)jj + e];
      float A1[3][3], b1[3], A2[3][3], b2[3];
      // frame 1: i's points in j; frame 2: j's points in i
      pair_frames(pd, Ri, si, Rj, ps, A1, b1, A2, b2);
      // disjoint along a principal axis of either: both counts are zero
      if (frame_separated(A1, b1) || frame_separated(A2, b2)) continue;
      const int cij = count_frame<R>(A1, b1, up, U, Q, lane);
      const int cji = count_frame<R>(A2, b2, up, U, Q, lane);
      if (cij == 0 && cji == 0) continue;
      const float Vj = 4.18879020478639f * ps[0] * ps[1] * ps[2];
      const float V = (Vi * (float)cij + Vj * (float)cji) / (2.f * (float)Q);
      if (jj > i) {
        vsum += llrint((double)V * kVolScale);
        npair += 1;
      }
      const float len = sqrtf(pd[0] * pd[0] + pd[1] * pd[1] + pd[2] * pd[2]);
      if (len > 0.f) {
        const float f = G.eta * V / len;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          // pushes beyond 1e6 lattice units are clamped (the move is capped anyway)
          const double c = fmin(fmax((double)(f * pd[d]), -1e6), 1e6);
          push[d] += llrint(c * kPushScale);
        }
      }
    }
  }
  if (lane != 0) return;
  vol[i] = vsum;
  pairs[i] = npair;
  if (!move) return;
  float disp[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) disp[d] = (float)((double)push[d] / kPushScale);
  const float len = sqrtf(disp[0] * disp[0] + disp[1] * disp[1] + disp[2] * disp[2]);
  if (len > G.max_move) {
    const float sc = G.max_move / len;
#pragma unroll
    for (int d = 0; d < 3; ++d) disp[d] *= sc;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float x = ri[d] + disp[d];
    if (G.per[d]) {
      x = x - G.L[d] * floorf(x / G.L[d]);
    } else {
      // half extent along axis d: |row d of R diag(s)|
      const float a0 = Ri[3 * d] * si[0], a1 = Ri[3 * d + 1] * si[1], a2 = Ri[3 * d + 2] * si[2];
      const float e = sqrtf(a0 * a0 + a1 * a1 + a2 * a2);
      x = fminf(fmaxf(x, G.lo[d] + e), G.hi[d] - e);
    }
    rout[3 * i + d] = x;
  }
}

// Deterministic totals: one work-group sums the per-ellipsoid integers.
__global__ __launch_bounds__(1024) void k_pack_total(const long long* __restrict__ vol,
                                                     const int* __restrict__ pairs, int n,
                                                     long long* __restrict__ out) {
  __shared__ long long sv[1024];
  __shared__ long long sp[1024];
  long long v = 0, p = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    v += vol[i];
    p += pairs[i];
  }
  sv[threadIdx.x] = v;
  sp[threadIdx.x] = p;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sv[threadIdx.x] += sv[threadIdx.x + s];
      sp[threadIdx.x] += sp[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sv[0];
    out[1] = sp[0];
  }
}

// Points of the m^3 grid whose cell centres lie in the unit ball (the odd
// integers 2a + 1 - m, squared and summed, at most m^2).
int ball_points(int m) {
  int q = 0;
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b)
      for (int c = 0; c < m; ++c) {
        const int x = 2 * a + 1 - m, y = 2 * b + 1 - m, z = 2 * c + 1 - m;
        q += x * x + y * y + z * z <= m * m ? 1 : 0;
      }
  return q;
}

// One work-group per cell: the rest mesh rotated and translated to the
// cell's ellipsoid.
__global__ __launch_bounds__(256) void k_place_cells(Cells C, int nv, const float* __restrict__ rest,
                                                     const float* __restrict__ centres,
                                                     const float* __restrict__ rot) {
  const int c = blockIdx.x;
  float o[3], R[9];
#pragma unroll
  for (int d = 0; d < 3; ++d) o[d] = centres[3 * c + d];
#pragma unroll
  for (int e = 0; e < 9; ++e) R[e] = rot[9 * c + e];
  int org[3];
  float frac[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    org[d] = (int)floorf(o[d]);
    frac[d] = o[d] - (float)org[d];
  }
  if (threadIdx.x < 3) C.origin[3 * c + threadIdx.x] = org[threadIdx.x];
  for (int v = threadIdx.x; v < nv; v += blockDim.x) {
    const float p0 = rest[3 * v], p1 = rest[3 * v + 1], p2 = rest[3 * v + 2];
#pragma unroll
    for (int d = 0; d < 3; ++d)
      C.off[((int64_t)c * nv + v) * 3 + d] = ((R[3 * d] * p0 + R[3 * d + 1] * p1) + R[3 * d + 2] * p2) + frac[d];
  }
}

struct PackPlan {
  PackGeom G;
  int64_t nbins = 0;
  size_t o_cnt = 0, o_items = 0, o_buf = 0, o_vol = 0, o_pairs = 0, o_flags = 0, o_tot = 0, total = 0;
};

size_t take(size_t& at, size_t bytes) {
  const size_t o = at;
  at += (bytes + 255) & ~size_t(255);
  return o;
}

std::string plan_pack(const hc_pack_desc* d, int32_t n, PackPlan& P) {
  if (!d) return "null descriptor";
  if (n < 0) return "negative ellipsoid count";
  if (!(d->max_semi > 0.f) || !std::isfinite(d->max_semi)) return "max_semi must be positive";
  if (d->quad != 4 && d->quad != 8 && d->quad != 16) return "quad must be 4, 8 or 16";
  if (!(d->eta >= 0.f) || !std::isfinite(d->eta)) return "eta must be finite and >= 0";
  if (!(d->max_move > 0.f) || !std::isfinite(d->max_move)) return "max_move must be positive";
  PackGeom& G = P.G;
  const float reach = 2.f * d->max_semi;
  for (int a = 0; a < 3; ++a) {
    if (!(d->box[a] > 0.f) || !std::isfinite(d->box[a])) return "box sides must be positive";
    G.L[a] = d->box[a];
    G.per[a] = d->periodic[a] ? 1 : 0;
    G.lo[a] = d->lo[a];
    G.hi[a] = d->hi[a];
    if (G.per[a] && d->box[a] < 2.f * reach)
      return "a periodic side must be at least 4 max_semi (one image within reach)";
    if (!G.per[a] && !(d->hi[a] - d->lo[a] >= reach))
      return "a wall axis needs hi - lo >= 2 max_semi";
    G.nb[a] = std::max(1, (int)std::floor(d->box[a] / reach));
    G.hb[a] = d->box[a] / (float)G.nb[a];
    if (G.hb[a] < reach) G.nb[a] = std::max(1, G.nb[a] - 1), G.hb[a] = d->box[a] / (float)G.nb[a];
  }
  P.nbins = (int64_t)G.nb[0] * G.nb[1] * G.nb[2];
  if (P.nbins > (int64_t)1 << 30) return "too many bins";
  G.eta = d->eta;
  G.max_move = d->max_move;
  G.max_semi = d->max_semi;
  G.m = d->quad;
  // room for four times the mean occupancy plus a margin
  G.cap = (int)std::min<int64_t>(1 << 20, 32 + 4 * ((int64_t)n + P.nbins - 1) / std::max<int64_t>(1, P.nbins));
  size_t at = 0;
  P.o_cnt = take(at, (size_t)P.nbins * 4);
  P.o_items = take(at, (size_t)P.nbins * G.cap * 4);
  P.o_buf = take(at, (size_t)std::max(1, n) * 12);
  P.o_vol = take(at, (size_t)std::max(1, n) * 8);
  P.o_pairs = take(at, (size_t)std::max(1, n) * 4);
  P.o_flags = take(at, 16);
  P.o_tot = take(at, 16);
  P.total = at;
  return "";
}

hc_status pack_fail(hc_status s, const std::string& msg) {
  set_global_error(msg);
  return s;
}

#define PK_TRY(expr, what)                                                            \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) return pack_fail(HC_ERR_DEVICE, std::string(what) + ": " + \
                                                              hipGetErrorString(_e)); \
  } while (0)

}  // namespace

hipError_t launch_place_cells(const Cells& c, int nv, const float* rest, const float* centres,
                              const float* rot, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_place_cells, dim3(n), dim3(256), 0, s, c, nv, rest, centres, rot);
  return hipGetLastError();
}

}  // namespace hc

using namespace hc;

extern "C" {

hc_status hc_pack_query_workspace(const hc_pack_desc* desc, int32_t n, size_t* bytes) {
  if (!bytes) return pack_fail(HC_ERR_ARG, "null size pointer");
  PackPlan P;
  const std::string e = plan_pack(desc, n, P);
  if (!e.empty()) return pack_fail(HC_ERR_ARG, e);
  *bytes = P.total;
  return HC_OK;
}

// Scratch memory of hc_pack_run_static, for callers that cannot allocate:
// one array per device that the library runs on, held until the process
// ends.  Host code reaches it only through the address that
// hipGetSymbolAddress returns on each device (the array's name is a
// host-side stand-in there, not a device address).
constexpr size_t kPackStaticBytes = (size_t)32 << 20;
static __device__ __align__(256) char scratch[kPackStaticBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};   // device address of scratch, per device index

// Device address of this device's scratch, resolved once per device with
// that device current.
static hc_status static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return pack_fail(HC_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= 64) return pack_fail(HC_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return pack_fail(HC_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HC_OK;
}

static hc_status pack_run(const hc_pack_desc* desc, float* centres, const float* rot, const float* semi,
                          int32_t n, int32_t n_iter, void* workspace, size_t ws_bytes, void* stream,
                          double* overlap);

hc_status hc_pack_run(const hc_pack_desc* desc, float* centres, const float* rot, const float* semi,
                      int32_t n, int32_t n_iter, void* workspace, size_t ws_bytes, void* stream,
                      double* overlap) {
  return pack_run(desc, centres, rot, semi, n, n_iter, workspace, ws_bytes, stream, overlap);
}

hc_status hc_pack_run_static(const hc_pack_desc* desc, float* centres, const float* rot, const float* semi,
                             int32_t n, int32_t n_iter, void* stream, double* overlap) {
  PackPlan P;
  const std::string e = plan_pack(desc, n, P);
  if (!e.empty()) return pack_fail(HC_ERR_ARG, e);
  if (P.total > kPackStaticBytes)
    return pack_fail(HC_ERR_UNSUPPORTED, "hc_pack_run_static: this packing needs " + std::to_string(P.total) +
                                             " bytes of scratch, above the library's static " +
                                             std::to_string(kPackStaticBytes) + " (use hc_pack_run)");
  void* ws = nullptr;
  const hc_status st = static_scratch(&ws);
  if (st != HC_OK) return st;
  return pack_run(desc, centres, rot, semi, n, n_iter, ws, kPackStaticBytes, stream, overlap);
}

}  // extern "C"

static hc_status pack_run(const hc_pack_desc* desc, float* centres, const float* rot, const float* semi,
                          int32_t n, int32_t n_iter, void* workspace, size_t ws_bytes, void* stream,
                          double* overlap) {
  PackPlan P;
  const std::string e = plan_pack(desc, n, P);
  if (!e.empty()) return pack_fail(HC_ERR_ARG, e);
  if (n_iter < 0) return pack_fail(HC_ERR_ARG, "n_iter < 0");
  if (n > 0 && (!centres || !rot || !semi)) return pack_fail(HC_ERR_ARG, "null ellipsoid array");
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return pack_fail(HC_ERR_ARG, "workspace null or not 256-byte aligned");
  if (ws_bytes < P.total) return pack_fail(HC_ERR_OOM, "packing workspace too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(workspace);
  int* cnt = reinterpret_cast<int*>(w + P.o_cnt);
  int* items = reinterpret_cast<int*>(w + P.o_items);
  float* buf = reinterpret_cast<float*>(w + P.o_buf);
  long long* vol = reinterpret_cast<long long*>(w + P.o_vol);
  int* pairs = reinterpret_cast<int*>(w + P.o_pairs);
  int* flags = reinterpret_cast<int*>(w + P.o_flags);
  long long* tot = reinterpret_cast<long long*>(w + P.o_tot);
  PK_TRY(launch_fill_i32(flags, 0, 4, s), "clear flags");
  const dim3 gb((unsigned)((std::max(n, 1) + 255) / 256));
  const dim3 gi((unsigned)((std::max(n, 1) + kPackPerBlock - 1) / kPackPerBlock));
  long long host_tot[4] = {0, 0, 0, 0};
  const size_t lds = (size_t)ball_points(P.G.m) * sizeof(float4);
  float* cur = centres;
  float* nxt = buf;
  // n_iter moves, then one evaluation at the final positions (when asked for)
  for (int it = 0; it <= n_iter && n > 0; ++it) {
    const bool move = it < n_iter;
    if (!move && !overlap) break;   // the final evaluation only feeds the overlap record
    PK_TRY(launch_fill_i32(cnt, 0, P.nbins, s), "clear bins");
    hipLaunchKernelGGL(k_pack_bin, gb, dim3(256), 0, s, P.G, cur, n, cnt, items, flags);
    PK_TRY(hipGetLastError(), "bin");
    // the 32 (m = 4) and 280 (m = 8) points stay in registers, 1 and 5 per lane
    if (P.G.m == 4)
      hipLaunchKernelGGL(k_pack_iter<1>, gi, dim3(kPackThreads), lds, s, P.G, cur, nxt, rot, semi, n, cnt,
                         items, vol, pairs, move ? 1 : 0, flags);
    else if (P.G.m == 8)
      hipLaunchKernelGGL(k_pack_iter<5>, gi, dim3(kPackThreads), lds, s, P.G, cur, nxt, rot, semi, n, cnt,
                         items, vol, pairs, move ? 1 : 0, flags);
    else
      hipLaunchKernelGGL(k_pack_iter<0>, gi, dim3(kPackThreads), lds, s, P.G, cur, nxt, rot, semi, n, cnt,
                         items, vol, pairs, move ? 1 : 0, flags);
    PK_TRY(hipGetLastError(), "iterate");
    if (overlap && (it == 0 || !move)) {
      hipLaunchKernelGGL(k_pack_total, dim3(1), dim3(1024), 0, s, vol, pairs, n, tot);
      PK_TRY(hipGetLastError(), "totals");
      PK_TRY(hipMemcpyAsync(host_tot + (it == 0 ? 0 : 2), tot, 16, hipMemcpyDeviceToHost, s), "d2h");
      PK_TRY(hipStreamSynchronize(s), "sync");
    }
    if (move) std::swap(cur, nxt);
  }
  if (n > 0 && cur != centres)
    PK_TRY(hipMemcpyAsync(centres, cur, (size_t)n * 12, hipMemcpyDeviceToDevice, s), "copy back");
  int hflags[4];
  PK_TRY(hipMemcpyAsync(hflags, flags, 16, hipMemcpyDeviceToHost, s), "d2h");
  PK_TRY(hipStreamSynchronize(s), "sync");
  if (hflags[0]) return pack_fail(HC_ERR_NONFINITE, "non-finite ellipsoid centre");
  if (hflags[1]) return pack_fail(HC_ERR_UNSUPPORTED, "a packing bin overflowed its capacity");
  if (hflags[2]) return pack_fail(HC_ERR_ARG, "a semi-axis is not positive or exceeds max_semi");
  if (overlap) {
    if (n_iter == 0) host_tot[2] = host_tot[0], host_tot[3] = host_tot[1];
    overlap[0] = (double)host_tot[0] / kVolScale;
    overlap[1] = (double)host_tot[1];
    overlap[2] = (double)host_tot[2] / kVolScale;
    overlap[3] = (double)host_tot[3];
  }
  return HC_OK;
}
