// Marking of the lattice sites inside the cells for the interior viscosity
// (Sec. 1, Sec. 3.4): one work-group per cell runs inside::mark_cell, which
// states the ray-parity rule.  The marks are bytes in the site-ordered
// mask: 1 << k for a cell of viscosity class k (cells of different
// stiffness may carry different interior viscosities, Sec. 3.4), which the
// lattice pass reads (and clears) to pick the relaxation time.
#include "interior_dev.h"

namespace hc {
namespace {

constexpr int kMarkThreads = 256;

__global__ __launch_bounds__(kMarkThreads) void k_mark_interior(Cells C, Mesh M, Lattice L,
                                                                unsigned char* __restrict__ mask,
                                                                const unsigned char* __restrict__ cls,
                                                                int only_class, int* __restrict__ flags) {
  extern __shared__ float sp[];   // [nv][3] offsets
  __shared__ inside::Lds S;
  const int c = blockIdx.x, tid = threadIdx.x;
  if (only_class >= 0 && cls[c] != only_class) return;   // another class's pass
  const int64_t b3 = (int64_t)c * M.nv * 3;
  const int o[3] = {C.origin[3 * c], C.origin[3 * c + 1], C.origin[3 * c + 2]};
  inside::Grid G;
  for (int d = 0; d < 3; ++d) G.bc[d] = L.bc[d];
  G.n[0] = L.nx;
  G.n[1] = L.ny;
  G.n[2] = L.nz;
  G.le = L.le;
  G.le_delta = L.le_delta;
  const unsigned char bit = (unsigned char)(1u << (cls ? cls[c] : 0));
  inside::mark_cell(C.off + b3, sp, M.nv, M.tri, M.nt, o, G, [&](int x, int y, int z) { return site_of(L, x, y, z); },
                    mask, bit, flags + 1, S, tid, kMarkThreads);
}

}  // namespace

hipError_t launch_mark_interior(const Cells& c, const Mesh& m, const Lattice& L, unsigned char* mask,
                                const unsigned char* cls, int only_class, int* flags, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  const size_t lds = (size_t)m.nv * 3 * sizeof(float);
  hipLaunchKernelGGL(k_mark_interior, dim3(c.n), dim3(kMarkThreads), lds, s, c, m, L, mask, cls, only_class,
                     flags);
  return hipGetLastError();
}

}  // namespace hc
