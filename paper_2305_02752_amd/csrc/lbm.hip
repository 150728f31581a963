// D3Q19 BGK collide + stream with external force, one pass over SoA
// populations (Sec. 2.2 LBGK update, moments, second-order equilibrium).
//
// Populations are stored shifted, g_i = f_i - w_i, so that the O(1e-3)
// deviations carrying the flow keep full float32 resolution.  Forcing
// follows Guo, Zheng & Shi (2002): the velocity includes half the force and
// the source (1 - omega/2) w_i [3 (e_i - u) + 9 (e_i.u) e_i].F is added
// after relaxation.  Streaming pushes each post-collision value to
// x + e_i; periodic axes wrap, the (single) wall axis reflects with
// half-way bounce-back plus Ladd's moving-wall term -6 w_i rho (e_i.u_w).
#include "common.h"

namespace hc {
namespace {

// Direction set (order documented in hemo.h) and weights.
__device__ constexpr int cx[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int cy[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int cz[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__device__ constexpr float wq[kQ] = {1.f / 3,  1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18,
                                     1.f / 18, 1.f / 18, 1.f / 36, 1.f / 36, 1.f / 36,
                                     1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36,
                                     1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
__device__ constexpr int opp[kQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

__global__ __launch_bounds__(256) void k_collide_stream(const float* __restrict__ gin,
                                                        float* __restrict__ gout,
                                                        const float* __restrict__ F,
                                                        float4* __restrict__ macro,
                                                        Lattice L) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = L.n;
  if (s >= N) return;
  const int x = (int)(s % L.nx);
  const int64_t r = s / L.nx;
  const int y = (int)(r % L.ny);
  const int z = (int)(r / L.ny);

  float g[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) g[i] = gin[i * N + s];

  float fx = L.g[0], fy = L.g[1], fz = L.g[2];
  if (F) {
    fx = F[s];
    fy = F[N + s];
    fz = F[2 * N + s];
  }
  float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    drho += g[i];
    jx += cx[i] * g[i];
    jy += cy[i] * g[i];
    jz += cz[i] * g[i];
  }
  const float rho = 1.f + drho;
  const float inv = 1.f / rho;
  const float ux = (jx + 0.5f * fx) * inv;
  const float uy = (jy + 0.5f * fy) * inv;
  const float uz = (jz + 0.5f * fz) * inv;
  if (macro) macro[s] = make_float4(ux, uy, uz, rho);

  const float om = L.omega;
  const float src = 1.f - 0.5f * om;
  const float uu = ux * ux + uy * uy + uz * uz;
  const float uF = ux * fx + uy * fy + uz * fz;

#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const float eu = cx[i] * ux + cy[i] * uy + cz[i] * uz;
    const float eF = cx[i] * fx + cy[i] * fy + cz[i] * fz;
    const float geq = wq[i] * (drho + rho * (3.f * eu + 4.5f * eu * eu - 1.5f * uu));
    const float post = g[i] - om * (g[i] - geq) + src * wq[i] * (3.f * (eF - uF) + 9.f * eu * eF);
    int xt = x + cx[i], yt = y + cy[i], zt = z + cz[i];
    // a population leaving through the wall axis bounces back; lo selects the wall
    int crossed = 0;  // 0: none, 1: lower wall, 2: upper wall
    if (L.wall_axis == 0 && cx[i] != 0) crossed = xt < 0 ? 1 : (xt >= L.nx ? 2 : 0);
    if (L.wall_axis == 1 && cy[i] != 0) crossed = yt < 0 ? 1 : (yt >= L.ny ? 2 : 0);
    if (L.wall_axis == 2 && cz[i] != 0) crossed = zt < 0 ? 1 : (zt >= L.nz ? 2 : 0);
    const bool bounce = crossed != 0;
    const float uw = crossed == 1 ? cx[i] * L.ulo[0] + cy[i] * L.ulo[1] + cz[i] * L.ulo[2]
                                  : cx[i] * L.uhi[0] + cy[i] * L.uhi[1] + cz[i] * L.uhi[2];
    if (bounce) {
      gout[opp[i] * N + s] = post - 6.f * wq[i] * rho * uw;
    } else {
      xt = xt < 0 ? xt + L.nx : (xt >= L.nx ? xt - L.nx : xt);
      yt = yt < 0 ? yt + L.ny : (yt >= L.ny ? yt - L.ny : yt);
      zt = zt < 0 ? zt + L.nz : (zt >= L.nz ? zt - L.nz : zt);
      const int64_t st = ((int64_t)zt * L.ny + yt) * L.nx + xt;
      gout[i * N + st] = post;
    }
  }
}

__global__ void k_init_equilibrium(float* __restrict__ g, float rho0, float ux, float uy, float uz,
                                   int64_t N) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  const float uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const float eu = cx[i] * ux + cy[i] * uy + cz[i] * uz;
    g[i * N + s] = wq[i] * ((rho0 - 1.f) + rho0 * (3.f * eu + 4.5f * eu * eu - 1.5f * uu));
  }
}

// Streaming copy used as the measured bandwidth reference.
__global__ __launch_bounds__(256) void k_copy16(float4* __restrict__ dst,
                                                const float4* __restrict__ src, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
}

}  // namespace

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return hipSuccess;
  int64_t blocks = (n16 + 255) / 256;
  if (blocks > 256 * 64) blocks = 256 * 64;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (float4*)dst,
                     (const float4*)src, n16);
  return hipGetLastError();
}

hipError_t launch_collide_stream(const float* gin, float* gout, const float* F, float4* macro,
                                 const Lattice& L, hipStream_t s) {
  const int64_t blocks = (L.n + 255) / 256;
  hipLaunchKernelGGL(k_collide_stream, dim3((unsigned)blocks), dim3(256), 0, s, gin, gout, F, macro,
                     L);
  return hipGetLastError();
}

hipError_t launch_init_equilibrium(float* g, float rho0, float ux, float uy, float uz,
                                   const Lattice& L, hipStream_t s) {
  const int64_t blocks = (L.n + 255) / 256;
  hipLaunchKernelGGL(k_init_equilibrium, dim3((unsigned)blocks), dim3(256), 0, s, g, rho0, ux, uy,
                     uz, L.n);
  return hipGetLastError();
}

}  // namespace hc
