// Membrane forces of every cell: one work-group of kCellThreads threads
// per cell (the element loops are split across its waves; the area and
// volume sums are reduced in a fixed order).
#include "membrane_dev.h"

namespace hc {
namespace {

constexpr int kCellThreads = 256;

__global__ __launch_bounds__(kCellThreads) void k_membrane(Cells C, Mesh M) {
  extern __shared__ long long lds64[];
  __shared__ double red[2 * kCellThreads / kWave];
  long long* acc = lds64;                                   // [nv][3] fixed-point forces
  float* sp = reinterpret_cast<float*>(lds64 + 3 * M.nv);   // [nv][3] positions
  const int c = blockIdx.x;
  const int64_t base = (int64_t)c * M.nv * 3;
  mem::membrane_cell(M, C.off + base, C.k + 4 * c, C.traction ? C.traction + 3 * c : nullptr,
                     C.force + base, C.area + c, C.volume + c, acc, sp, red, threadIdx.x,
                     kCellThreads);
}

}  // namespace

hipError_t launch_membrane(const Cells& c, const Mesh& m, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  const size_t lds = (size_t)m.nv * 3 * (sizeof(long long) + sizeof(float));
  hipLaunchKernelGGL(k_membrane, dim3(c.n), dim3(kCellThreads), lds, s, c, m);
  return hipGetLastError();
}

}  // namespace hc
