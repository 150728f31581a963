// Internal declarations shared by the HIP kernels and the C ABI layer of
// libhemo.  Device views are plain structs of pointers passed by value to
// the kernels; no torch or host-library types appear here.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

// D3Q19 weights and odd coefficients k = 3 w as FP32 constants whose
// mass and momentum identities hold exactly (the collision explains the choice).
#define HC_W0 0x1.555558p-2f
#define HC_W1 0x1.c71c7p-5f
#define HC_W2 0x1.c71c7p-6f
#define HC_K1 0x1.555554p-3f
#define HC_K2 0x1.555556p-4f

namespace hc {

constexpr int kQ = 19;          // D3Q19
constexpr int kTile = 8;        // binning tile side (lattice nodes)
constexpr int kMaxTouch = 27;   // tiles reached by one stencil: <= 3 per axis (a periodic
                                // axis whose last tile is 1-2 nodes wide), else 2
constexpr int kWave = 64;       // gfx950 wavefront width
// Fixed-point scale of the deterministic force accumulation: 2^40 units per
// lattice force unit (resolution 9.1e-13, accumulator range +-8.4e6).
constexpr double kFixScale = 1099511627776.0;
constexpr float kFixScaleF = 1099511627776.0f;
constexpr double kFixInv = 1.0 / 1099511627776.0;

// Largest float below 2^31: scaled contributions under it take the native
// 32-bit conversion; larger ones the 64-bit one.  Both give the same integer
// (round to nearest even of the same float), so the choice never changes a
// result.
constexpr float kFix32Max = 2147483520.0f;

// Distinct interior viscosity ratios (classes) one lattice may hold at once.
constexpr int kVisClasses = 8;

[[maybe_unused]] static __device__ __noinline__ void fix_add3_wide(long long* a0, long long* a1,
                                                                   long long* a2, float x, float y,
                                                                   float z) {
  atomicAdd((unsigned long long*)a0, (unsigned long long)__float2ll_rn(x));
  atomicAdd((unsigned long long*)a1, (unsigned long long)__float2ll_rn(y));
  atomicAdd((unsigned long long*)a2, (unsigned long long)__float2ll_rn(z));
}

// acc[k] += round(q_k) for three scaled components; the wide path is a real
// branch, taken only by lanes holding a contribution of 2^31 or more.
__device__ inline void fix_add3(long long* a0, long long* a1, long long* a2, float x, float y,
                                float z) {
  if (fmaxf(fabsf(x), fmaxf(fabsf(y), fabsf(z))) < kFix32Max) {
    atomicAdd((unsigned long long*)a0, (unsigned long long)(long long)__float2int_rn(x));
    atomicAdd((unsigned long long*)a1, (unsigned long long)(long long)__float2int_rn(y));
    atomicAdd((unsigned long long*)a2, (unsigned long long)(long long)__float2int_rn(z));
  } else {
    fix_add3_wide(a0, a1, a2, x, y, z);
  }
}

struct Lattice {
  int nx, ny, nz;
  int bc[3];
  int wall_axis;            // -1 when fully periodic
  float tau, omega;
  float g[3];               // body force density
  float ulo[3], uhi[3];     // wall velocities (wall axis only)
  float wc_lo[kQ], wc_hi[kQ];   // Ladd's moving-wall coefficients -6 w_q (e_q . u_wall) of the
                                // lower and upper wall (0 without a wall)
  int kernel;               // 4 or 2
  int le;                   // Lees-Edwards images across z (flow along x)
  float le_u;               // image velocity U
  float le_delta;           // displacement U t mod nx at this step (IBM stencils)
  float le_pull_delta;      // displacement of the previous step, whose streaming the pull completes
  int le_raw;               // the stored state is a plain permutation of the pre-collision
                            // populations (fresh from a write or init): pull periodically
  float omega_in[kVisClasses];   // relaxation rates inside the cells, per viscosity class
                                 // (classes in increasing viscosity ratio)
  int64_t n;                // nx * ny * nz
  int64_t np;               // ntiles * 512: site slots of every lattice field
  int tx, ty, tz, ntiles;   // tile grid
  int max_touch;            // touch-list slots per vertex (product over axes)
};

// Site order of every lattice field on the device (populations, force,
// velocity and their cotangents): 8^3 tiles in (tz, ty, tx) order, the 512
// sites of a tile in (z, y, x) order.  A work-group that owns a tile reads
// and writes each population as one contiguous 2 KiB block.  Sides that are
// not multiples of 8 leave padding slots, which are never read.
static_assert(kTile == 8, "site_of assumes 8^3 tiles");
__host__ __device__ inline int64_t site_of(const Lattice& L, int x, int y, int z) {
  const int t = ((z >> 3) * L.ty + (y >> 3)) * L.tx + (x >> 3);
  return (int64_t)t * 512 + (((z & 7) << 6) | ((y & 7) << 3) | (x & 7));
}

// floor(a / b) for b > 0.
__host__ __device__ inline int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Node of slot h, or false for a padding slot.
__host__ __device__ inline bool node_of(const Lattice& L, int64_t h, int& x, int& y, int& z) {
  const int t = (int)(h >> 9), i = (int)(h & 511);
  x = (t % L.tx) * kTile + (i & 7);
  y = ((t / L.tx) % L.ty) * kTile + ((i >> 3) & 7);
  z = (t / (L.tx * L.ty)) * kTile + (i >> 6);
  return x < L.nx && y < L.ny && z < L.nz;
}

// Mesh tables shared by every cell (built on the host from the rest shape).
struct Mesh {
  int nv, nt, ne, nh;
  const int* tri;           // [nt][3]
  const int* edge;          // [ne][2] (i < j)
  const float* L0;          // [ne] rest length
  const int* hinge_v;       // [nh][4] (i, j, k, l): i->j in (i, j, k), j->i in (j, i, l)
  const float* theta0;      // [nh]
  const int* hinge_own;     // [nh] bit 0: evaluates triangle (i, j, k), bit 1: (j, i, l)
  const float* pole;        // [nv] +1 / -1 / 0: pole traction sign
  float inv_npole;          // 1 / |P+|
  double A0, V0;
};

struct Cells {
  int n;
  int* origin;              // [n][3]
  float* off;               // [n][nv][3]
  float* lo;                // [n][nv][3] low parts of the positions (see move_compensated)
  float* force;             // [n][nv][3]
  float* vel;               // [n][nv][3] interpolated velocity of the last step
  const float* k;           // [n][4]
  const float* traction;    // [n][3] or nullptr
  double* area;             // [n]
  double* volume;           // [n]
};

struct Bins {
  int* owner;               // [n*nv]
  int* ntouch;              // [n*nv] tiles reached by the vertex's stencil
  int* slot;                // [n*nv][max_touch] hash slot << 16 | rank (binning scratch)
  int* touch_cnt;           // [ntiles] entries in each tile list
  int* touch;               // [ntiles][cap] vertex * 32 + j (its j-th reached tile)
  int cap;                  // fixed capacity of one tile list
  int bexp;                 // force-bound grid 2^-bexp of the tile's largest component (cap * 2^bexp <= 2^30)
  int* flags;               // [4]: 0 non-finite, 1 list overflow
  int* scan_tmp;            // block sums of the tile scan
};

// Launchers (one per kernel family); all enqueue on `s`.
hipError_t launch_membrane(const Cells& c, const Mesh& m, hipStream_t s);
hipError_t launch_bin_vertices(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                               hipStream_t s);
hipError_t launch_bin_cells(const Cells& c, const Mesh& m, const Lattice& L, int* cnt, int* ptr,
                            int* rank, int* tiles, int* list, int64_t cap, int max_per_cell,
                            int* flags, int* scan_tmp, hipStream_t s);
hipError_t launch_touch_csr(const Lattice& L, const Bins& b, int* cnt_tmp, int* ptr, int* out,
                            hipStream_t s);
hipError_t launch_sort_segments(const int* ptr, int* list, int* tmp, int nseg, hipStream_t s);
hipError_t launch_scan(const int* cnt, int* ptr, int* sums, int n, hipStream_t s);
hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t s);
// spread an arbitrary per-vertex vector field (vec [n*nv][3]) plus body * g
hipError_t launch_spread_vec(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                             const float* vec, float body, float* F, hipStream_t s);
// adjoint kernels
hipError_t launch_adj_collide(const float* lam1, float* lam0, const float* g0, const float* F,
                              const float* lamu, float* lamF, double* domega_part, unsigned char* mask,
                              double* domega_in_part, const Lattice& L, hipStream_t s);
hipError_t launch_adj_vertex(const Cells& c, const Mesh& m, const Lattice& L, const float* lamX1,
                             const float4* macro, const float* lamF, float* lamFv, float* lamX0,
                             hipStream_t s);
hipError_t launch_adj_membrane(const Cells& c, const Mesh& m, const float* lamFv, float* lamX,
                               double* dk, hipStream_t s);
hipError_t launch_loss_seed(const Cells& c, const Mesh& m, const double* targets, double* loss,
                            float* lamX, hipStream_t s);
hipError_t launch_sum_parts(const double* parts, int n, double* out, hipStream_t s);
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s);
// interpolation close (tile partials summed per vertex) + Euler or AB2 move
hipError_t launch_advect(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                         const float4* partial, int* flags, bool ab2, hipStream_t s);
// fused lattice pass: spread + collide/stream + interpolation partials;
// with fields set it also writes the force field F and (u, rho) to macro
hipError_t launch_tile_step(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                            const float* gin, float* gout, float* F, float4* macro, float4* partial,
                            bool fields, unsigned char* mask, hipStream_t s);
// Mark the sites inside the cells in the site-ordered mask, which must hold
// zeros on entry: a site inside a cell of viscosity class k (cls[c], or 0
// for every cell when cls is null) gets the byte 1 << k.  With several
// classes the marking runs once per class in increasing order (only_class),
// so a site inside cells of different classes ends with the highest class,
// whatever the order of the cells.  The lattice pass reads and clears the
// mask.
hipError_t launch_mark_interior(const Cells& c, const Mesh& m, const Lattice& L, unsigned char* mask,
                                const unsigned char* cls, int only_class, int* flags, hipStream_t s);
// fused per-cell kernel: [advect of the pending step] + membrane + binning
// (src: offsets to move from, or null to move in place; refresh: compute
// the membrane forces, else hold the stored ones; ab2: Adams-Bashforth move)
hipError_t launch_cell_step(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                            const float4* partial, int* flags, bool advect, const float* src,
                            bool refresh, bool ab2, bool recentre, bool keep_vel, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// Device-to-device copies of n records in one launch (bytes a multiple of 4;
// records with 16-byte aligned ends move in 16-byte words).  max_bytes: the
// largest record, which sets the grid.
struct CopyRec {
  void* dst;
  const void* src;
  int64_t bytes;
};
hipError_t launch_copy_many(const CopyRec* dev, int n, int64_t max_bytes, hipStream_t s);

// Batched forms of the per-step kernels for several boxes of one shape (one
// launch covers every box: work-group (x, y) does work-group x of box y with
// box y's arguments, read from the device array `dev` of n records; `a0` is
// box 0's record on the host, which fixes the grid and the kernel variant).
struct CellStepArgs {
  Cells C; Mesh M; Lattice L; Bins B;
  const float4* partial; int* flags; int advect; const float* src; int refresh; int ab2; int recentre;
};
struct TileStepArgs {
  Cells C; Mesh M; Lattice L; Bins B;
  const float* gin; float* gout; float* F; float4* macro; float4* partial; int fields; unsigned char* mask;
};
struct BinArgs { Cells C; Mesh M; Lattice L; Bins B; };
struct SpreadArgs { Cells C; Mesh M; Lattice L; Bins B; const float* vec; float body; float* F; };
struct AdjCollideArgs {
  const float* lam1; float* lam0; const float* h0; const float* F; const float* lamu; float* lamF;
  double* domega_part; unsigned char* mask; double* domega_in_part; Lattice L;
};
struct AdjVertexArgs {
  Cells C; Mesh M; Lattice L;
  const float* lamX1; const float4* macro; const float* lamF; float* lamFv; float* lamX0;
};
struct AdjMembraneArgs { Cells C; Mesh M; const float* lamFv; float* lamX; double* dk; };
hipError_t launch_cell_step_multi(const CellStepArgs& a0, const CellStepArgs* dev, int n, hipStream_t s);
hipError_t launch_tile_step_multi(const TileStepArgs& a0, const TileStepArgs* dev, int n, hipStream_t s);
hipError_t launch_bin_vertices_multi(const BinArgs& a0, const BinArgs* dev, int n, hipStream_t s);
hipError_t launch_spread_vec_multi(const SpreadArgs& a0, const SpreadArgs* dev, int n, hipStream_t s);
hipError_t launch_adj_collide_multi(const AdjCollideArgs& a0, const AdjCollideArgs* dev, int n, hipStream_t s);
hipError_t launch_adj_vertex_multi(const AdjVertexArgs& a0, const AdjVertexArgs* dev, int n, hipStream_t s);
hipError_t launch_adj_membrane_multi(const AdjMembraneArgs& a0, const AdjMembraneArgs* dev, int n,
                                     hipStream_t s);

// stored (pull-form) state of a uniform equilibrium on the tile-major lattice
hipError_t launch_init_equilibrium(float* g, float rho0, float ux, float uy, float uz,
                                   const Lattice& L, hipStream_t s);
// uniform equilibrium on n sites in any order (fully periodic boxes)
hipError_t launch_init_uniform(float* g, float rho0, float ux, float uy, float uz, int64_t n,
                               hipStream_t s);
// natural <-> device site order: to_natural writes g[19][n] (pre-collision
// populations, x fastest) from the stored state h; from_natural the inverse;
// field_to_natural copies `comps` float components of a [comps][np] field
// (or, with comps == 4, a float4 [np] field into [4][n])
hipError_t launch_to_natural(const float* h, float* g, const Lattice& L, hipStream_t s);
hipError_t launch_from_natural(const float* g, float* h, const Lattice& L, hipStream_t s);
hipError_t launch_field_to_natural(const float* f, float* out, int comps, const Lattice& L,
                                   hipStream_t s);

}  // namespace hc
