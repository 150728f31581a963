// Device views of the batched single-cell boxes (persistent kernel).
#pragma once

#include "common.h"

namespace hc {

struct BoxDesc {
  int nx, ny, nz, wall_axis;
  int bc[3];
  int ty, tz, nty, ntz;     // tile = all x, ty rows in y, tz rows in z
  float omega;
  float omega_in;           // relaxation rate inside the cell (omega when the ratio is 1)
  float g[3], ulo[3], uhi[3];
  long long pop_off;        // float offset of the box in a population buffer
  long long site_off;       // offset of the box's first node among all boxes' nodes
  long long n;              // nodes
};

struct Batch {
  int nbox;
  int has_cells;
  const BoxDesc* box;
  float* pops0;
  float* pops1;
  Mesh M;
  int* origin;              // [nbox][3]
  float* off;               // [nbox][nv][3]
  float* lo;                // [nbox][nv][3] low parts of the positions (see move_compensated)
  float* force;             // [nbox][nv][3]
  float* vel;               // [nbox][nv][3]
  const float* k;           // [nbox][4]
  const float* trac;        // [nbox][3] or nullptr
  double* area;             // [nbox]
  double* volume;           // [nbox]
  long long* uacc;          // [nbox][nv][3] fixed-point vertex velocity
  int* bbox;                // [nbox][6] stencil node range per axis
  const int4* wg;           // per work-group: box (-1 idle), rank, members
  int* bar;                 // [nbox] barrier counters, zeroed before a launch
  int* box_step;            // [nbox] steps taken
  unsigned char* mask;      // [all nodes] 1 inside the box's cell (set and cleared each step)
  int interior;             // some box has omega_in != omega
  int* flags;               // [0] non-finite position, [1] barrier abort, [2] marking limits
  int spin_limit;
  int tile_cap;             // largest tile in nodes
};

size_t batch_lds_bytes(int nv, int tile_cap);
const void* batch_kernel(int K);
hipError_t launch_batch(const Batch& V, int K, int nsteps, int grid, int block, hipStream_t s);

}  // namespace hc
