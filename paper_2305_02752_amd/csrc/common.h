// Internal declarations shared by the HIP kernels and the C ABI layer of
// libhemo.  Device views are plain structs of pointers passed by value to
// the kernels; no torch or host-library types appear here.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hc {

constexpr int kQ = 19;          // D3Q19
constexpr int kTile = 8;        // binning tile side (lattice nodes)
constexpr int kMaxTouch = 27;   // tiles reached by one stencil: <= 3 per axis (a periodic
                                // axis whose last tile is 1-2 nodes wide), else 2
constexpr int kWave = 64;       // gfx950 wavefront width
// Fixed-point scale of the deterministic force accumulation: 2^48 units per
// lattice force unit (resolution 3.6e-15, range +-32768).
constexpr double kFixScale = 281474976710656.0;
constexpr double kFixInv = 1.0 / 281474976710656.0;

struct Lattice {
  int nx, ny, nz;
  int bc[3];
  int wall_axis;            // -1 when fully periodic
  float tau, omega;
  float g[3];               // body force density
  float ulo[3], uhi[3];     // wall velocities (wall axis only)
  int kernel;               // 4 or 2
  int64_t n;                // nx * ny * nz
  int tx, ty, tz, ntiles;   // tile grid
  int max_touch;            // touch-list slots per vertex (product over axes)
};

// Mesh tables shared by every cell (built on the host from the rest shape).
struct Mesh {
  int nv, nt, nh;
  const int* tri;           // [nt][3]
  const int* vlink_ptr;     // [nv+1]  per-vertex neighbour list
  const int* vlink_j;
  const float* vlink_L0;    // rest length of that link
  const int* vtri_ptr;      // [nv+1]  per-vertex incident triangles
  const int* vtri;          // [.][3]  (t, j, k): t = (v, j, k) counter-clockwise
  const int* vhinge_ptr;    // [nv+1]  per-vertex hinge roles
  const int* vhinge;        // h * 4 + role, role 0..3 = i, j, k, l
  const int* hinge_v;       // [nh][4] (i, j, k, l)
  const int* hinge_t;       // [nh][2] triangles (i, j, k) and (j, i, l)
  const float* theta0;      // [nh]
  const float* pole;        // [nv] +1 / -1 / 0: pole traction sign
  float inv_npole;          // 1 / |P+|
  double A0, V0;
};

struct Cells {
  int n;
  int* origin;              // [n][3]
  float* off;               // [n][nv][3]
  float* force;             // [n][nv][3]
  float* vel;               // [n][nv][3] interpolated velocity of the last step
  const float* k;           // [n][4]
  const float* traction;    // [n][3] or nullptr
  double* area;             // [n]
  double* volume;           // [n]
};

struct Bins {
  int* owner;               // [n*nv]
  int* touch_tile;          // [n*nv][8] tile ids reached (-1 unused)
  int* touch_rank;          // [n*nv][8] slot within the tile list
  int* touch_cnt;           // [ntiles+1]
  int* touch_ptr;           // [ntiles+1]
  int* touch;               // [capacity] vertex * 32 + slot (slot j of touch_tile)
  int64_t touch_cap;
  int* flags;               // [4]: 0 non-finite, 1 list overflow
};

// Launchers (one per kernel family); all enqueue on `s`.
hipError_t launch_membrane(const Cells& c, const Mesh& m, hipStream_t s);
hipError_t launch_bin_vertices(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                               hipStream_t s);
hipError_t launch_bin_cells(const Cells& c, const Mesh& m, const Lattice& L, int* cnt, int* ptr,
                            int* rank, int* tiles, int* list, int64_t cap, int max_per_cell,
                            int* flags, hipStream_t s);
hipError_t launch_sort_segments(const int* ptr, int* list, int* tmp, int nseg, hipStream_t s);
hipError_t launch_scan(const int* cnt, int* ptr, int n, hipStream_t s);
hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t s);
hipError_t launch_spread(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                         float* F, hipStream_t s);
hipError_t launch_collide_stream(const float* gin, float* gout, const float* F, float4* macro,
                                 const Lattice& L, hipStream_t s);
hipError_t launch_interp_advect(const Cells& c, const Mesh& m, const Lattice& L, const Bins& b,
                                const float4* macro, float4* partial, int* flags, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_init_equilibrium(float* g, float rho0, float ux, float uy, float uz,
                                   const Lattice& L, hipStream_t s);

}  // namespace hc
