// Host-side helpers shared by the single-lattice and batched C ABI layers.
#pragma once

#include <string>
#include <vector>

#include "../../include/hemo.h"
#include "common.h"

namespace hc {

constexpr int kNPole = 32;   // vertices per traction pole

struct HostMesh {
  int nv = 0, nt = 0, ne = 0, nh = 0;
  std::vector<int> tri, edge, hinge_v, hinge_own;
  std::vector<float> L0, theta0, pole;
  double A0 = 0, V0 = 0;
};

// Validate a closed, consistently oriented mesh and derive the rest state
// (edge lengths, dihedral angles, area, volume, traction poles) in float64.
// Returns an empty string on success, else the reason.
std::string build_mesh(const hc_mesh_desc* d, HostMesh& m);

// Message returned by hc_last_error(NULL): errors of calls without a context.
void set_global_error(const std::string& msg);

// Place the rest mesh (rest [nv][3]) at every centre with every rotation
// (device arrays centres [n][3], rot [n][9] row-major, columns = body axes):
// origin = floor(centre), offsets = R rest + (centre - origin), into C.
hipError_t launch_place_cells(const Cells& c, int nv, const float* rest, const float* centres,
                              const float* rot, int n, hipStream_t s);

}  // namespace hc
