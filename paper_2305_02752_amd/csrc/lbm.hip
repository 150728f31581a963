// Lattice initialisation and the streaming copy kernel used as the
// measured bandwidth reference.  (The collide + stream update itself runs
// inside the fused per-tile lattice pass; its per-node arithmetic is in the
// shared lattice header.)
#include "lbm_dev.h"

namespace hc {
namespace {

using lbm::cx;
using lbm::cy;
using lbm::cz;
using lbm::wq;

__device__ inline float feq_shifted(int q, float rho0, float ux, float uy, float uz) {
  const float uu = ux * ux + uy * uy + uz * uz;
  const float eu = cx[q] * ux + cy[q] * uy + cz[q] * uz;
  return wq[q] * ((rho0 - 1.f) + rho0 * (3.f * eu + 4.5f * eu * eu - 1.5f * uu));
}

// Stored (pull-form) state whose next pre-collision populations are the
// uniform equilibrium (Sec. 2.2, shifted g = f - w): every slot holds
// f_eq_q, except that a population leaving through a wall holds the value
// its bounce-back delivers, f_eq of the opposite direction.  Padding slots
// are zeroed.
__global__ void k_init_equilibrium(float* __restrict__ g, float rho0, float ux, float uy, float uz,
                                   Lattice L) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= L.np) return;
  int x, y, z;
  const bool live = node_of(L, h, x, y, z);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    float v = 0.f;
    if (live) v = feq_shifted(lbm::wall_crossed(L, q, x, y, z) ? lbm::opp[q] : q, rho0, ux, uy, uz);
    g[q * L.np + h] = v;
  }
}

__global__ void k_init_uniform(float* __restrict__ g, float rho0, float ux, float uy, float uz,
                               int64_t n) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
#pragma unroll
  for (int q = 0; q < kQ; ++q) g[q * n + s] = feq_shifted(q, rho0, ux, uy, uz);
}

// Pre-collision populations in natural order (x fastest): g_q(x) is what
// the next collision at x would pull.
__global__ void k_to_natural(const float* __restrict__ h, float* __restrict__ g, Lattice L) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= L.n) return;
  const int x = (int)(s % L.nx), y = (int)((s / L.nx) % L.ny), z = (int)(s / ((int64_t)L.nx * L.ny));
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    if (L.le && !L.le_raw && ((cz[q] > 0 && z == 0) || (cz[q] < 0 && z == L.nz - 1))) {
      g[q * L.n + s] = lbm::le_pull(L, h, q, x, y);   // crossing the sheared boundary
      continue;
    }
    int qs;
    const int64_t src = lbm::pull_source(L, q, x, y, z, &qs);
    g[q * L.n + s] = h[qs * L.np + src];
  }
}

// Inverse of k_to_natural for a plain state (periodic or walled pull): every
// stored slot is the pull source of exactly one (population, node) pair, so
// the scatter writes each slot once.  The result is a raw state.
__global__ void k_from_natural(const float* __restrict__ g, float* __restrict__ h, Lattice L) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= L.n) return;
  const int x = (int)(s % L.nx), y = (int)((s / L.nx) % L.ny), z = (int)(s / ((int64_t)L.nx * L.ny));
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    int qs;
    const int64_t src = lbm::pull_source(L, q, x, y, z, &qs);
    h[qs * L.np + src] = g[q * L.n + s];
  }
}

// comps components of a [comps][np] field (comps == 4: a float4 [np] field)
// to [comps][n] in natural order.
__global__ void k_field_to_natural(const float* __restrict__ f, float* __restrict__ out, int comps,
                                   Lattice L) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= L.n) return;
  const int x = (int)(s % L.nx), y = (int)((s / L.nx) % L.ny), z = (int)(s / ((int64_t)L.nx * L.ny));
  const int64_t h = site_of(L, x, y, z);
  for (int c = 0; c < comps; ++c)
    out[c * L.n + s] = comps == 4 ? f[4 * h + c] : f[c * L.np + h];
}

// Streaming copy used as the measured bandwidth reference: each thread
// keeps four 16-byte loads in flight and the data bypasses the caches
// (nontemporal loads and stores), one pass over the buffer.  Measured on a
// 4 GiB buffer, this form moves about 6.1 TB/s (read + write); a grid-stride
// loop of single 16-byte copies about 4.9 TB/s and hipMemcpyAsync about
// 4.5 TB/s.
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 4;

__global__ __launch_bounds__(256) void k_copy16(v4f* __restrict__ dst, const v4f* __restrict__ src,
                                                int64_t n16) {
  const int64_t base = (int64_t)blockIdx.x * 256 * kCopyUnroll + threadIdx.x;
  v4f v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const int64_t i = base + (int64_t)u * 256;
    if (i < n16) v[u] = __builtin_nontemporal_load(src + i);
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const int64_t i = base + (int64_t)u * 256;
    if (i < n16) __builtin_nontemporal_store(v[u], dst + i);
  }
}

}  // namespace

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return hipSuccess;
  const int64_t blocks = (n16 + 256 * kCopyUnroll - 1) / (256 * kCopyUnroll);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (v4f*)dst, (const v4f*)src, n16);
  return hipGetLastError();
}

hipError_t launch_init_equilibrium(float* g, float rho0, float ux, float uy, float uz,
                                   const Lattice& L, hipStream_t s) {
  hipLaunchKernelGGL(k_init_equilibrium, dim3((unsigned)((L.np + 255) / 256)), dim3(256), 0, s, g,
                     rho0, ux, uy, uz, L);
  return hipGetLastError();
}

hipError_t launch_init_uniform(float* g, float rho0, float ux, float uy, float uz, int64_t n,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_init_uniform, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, rho0, ux,
                     uy, uz, n);
  return hipGetLastError();
}

hipError_t launch_to_natural(const float* h, float* g, const Lattice& L, hipStream_t s) {
  hipLaunchKernelGGL(k_to_natural, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, s, h, g, L);
  return hipGetLastError();
}

hipError_t launch_from_natural(const float* g, float* h, const Lattice& L, hipStream_t s) {
  hipLaunchKernelGGL(k_from_natural, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, s, g, h, L);
  return hipGetLastError();
}

hipError_t launch_field_to_natural(const float* f, float* out, int comps, const Lattice& L,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_field_to_natural, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, s, f, out,
                     comps, L);
  return hipGetLastError();
}

}  // namespace hc
