// C ABI of the batched form: many independent single-cell boxes run by one
// persistent kernel launch (see batch_kernel.hip), replayed from a captured
// hipGraph, with a tile-shape autotuner.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "batch.h"
#include "host.h"

using namespace hc;

namespace {

thread_local std::string g_batch_error;
constexpr int kXcd = 8;          // MI355X: 8 XCDs, work-groups dealt round-robin
constexpr int kMaxGrid = 8192;   // upper bound on resident work-groups
constexpr int kSpinLimit = 1 << 22;

struct Lay {
  size_t total = 0;
  size_t add(size_t b) {
    const size_t a = total;
    total += (b + 255) & ~size_t(255);
    return a;
  }
};

}  // namespace

struct hc_batch {
  int nbox = 0, K = 4;
  std::vector<hc_lattice_desc> lat;
  HostMesh hm;
  std::vector<BoxDesc> box;
  int64_t sites = 0;
  int ty = 4, tz = 4, block = 256;
  int grid = 0;
  std::vector<int4> wg;
  Batch V{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_steps = -1;
  int64_t launches = 0;
  char* ws = nullptr;
  bool have_cells = false;
  std::string err;
  size_t o_pop0, o_pop1, o_snap_pop, o_box, o_tri, o_edge, o_L0, o_hv, o_th0, o_pole, o_own, o_origin,
      o_off, o_lo, o_force, o_vel, o_snap_off, o_snap_lo, o_k, o_trac, o_area, o_vol, o_uacc, o_bbox, o_wg, o_bar,
      o_step, o_snap_step, o_flags, o_mask;
};

namespace {

hc_status bfail(hc_batch* b, hc_status s, const std::string& m) {
  if (b) b->err = m; else g_batch_error = m;
  return s;
}
hc_status bcheck(hc_batch* b, hipError_t e, const char* what) {
  if (e == hipSuccess) return HC_OK;
  return bfail(b, HC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HB_TRY(expr)            \
  do {                          \
    hc_status _s = (expr);      \
    if (_s != HC_OK) return _s; \
  } while (0)

template <class T>
T* bat(hc_batch* b, size_t off) {
  return reinterpret_cast<T*>(b->ws + off);
}

void plan(hc_batch* b, Lay& L) {
  const int64_t P = 19 * b->sites;
  const int64_t B = b->nbox, nv = b->hm.nv;
  const HostMesh& m = b->hm;
  b->o_pop0 = L.add(P * 4);
  b->o_pop1 = L.add(P * 4);
  b->o_snap_pop = L.add(P * 4);
  b->o_box = L.add(B * sizeof(BoxDesc));
  b->o_tri = L.add(m.tri.size() * 4);
  b->o_edge = L.add(m.edge.size() * 4);
  b->o_L0 = L.add(m.L0.size() * 4);
  b->o_hv = L.add(m.hinge_v.size() * 4);
  b->o_th0 = L.add(m.theta0.size() * 4);
  b->o_pole = L.add(m.pole.size() * 4);
  b->o_own = L.add(m.hinge_own.size() * 4);
  b->o_origin = L.add(B * 12);
  b->o_off = L.add(B * nv * 12);
  b->o_lo = L.add(B * nv * 12);
  b->o_force = L.add(B * nv * 12);
  b->o_vel = L.add(B * nv * 12);
  b->o_snap_off = L.add(B * nv * 12);
  b->o_snap_lo = L.add(B * nv * 12);
  b->o_k = L.add(B * 16);
  b->o_trac = L.add(B * 12);
  b->o_area = L.add(B * 8);
  b->o_vol = L.add(B * 8);
  b->o_uacc = L.add(B * nv * 24);
  b->o_bbox = L.add(B * 24);
  b->o_wg = L.add((size_t)kMaxGrid * sizeof(int4));
  b->o_bar = L.add(B * 4);
  b->o_step = L.add(B * 4);
  b->o_snap_step = L.add(B * 4);
  b->o_flags = L.add(16);
  b->o_mask = L.add(b->sites);
}

hc_status bsync(hc_batch* b) { return bcheck(b, hipStreamSynchronize(b->stream), "sync"); }

hc_status h2d(hc_batch* b, void* d, const void* h, size_t n) {
  if (!n) return HC_OK;
  return bcheck(b, hipMemcpyAsync(d, h, n, hipMemcpyHostToDevice, b->stream), "h2d");
}
hc_status d2h(hc_batch* b, void* h, const void* d, size_t n) {
  if (!n) return HC_OK;
  return bcheck(b, hipMemcpyAsync(h, d, n, hipMemcpyDeviceToHost, b->stream), "d2h");
}
hc_status d2d(hc_batch* b, void* d, const void* s, size_t n) {
  if (!n) return HC_OK;
  return bcheck(b, hipMemcpyAsync(d, s, n, hipMemcpyDeviceToDevice, b->stream), "d2d");
}

void drop_graph(hc_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_steps = -1;
}

// Tile shape, work-group size and the static box -> work-group assignment.
hc_status apply_tiling(hc_batch* b, int ty, int tz, int block) {
  if (ty < 1 || tz < 1 || (block != 256 && block != 512 && block != 1024))
    return bfail(b, HC_ERR_ARG, "tiling: ty, tz >= 1 and block in {256, 512, 1024}");
  int cap = 0;
  for (auto& B : b->box) {
    B.ty = std::min(ty, B.ny);
    B.tz = std::min(tz, B.nz);
    B.nty = (B.ny + B.ty - 1) / B.ty;
    B.ntz = (B.nz + B.tz - 1) / B.tz;
    cap = std::max(cap, B.nx * B.ty * B.tz);
  }
  const size_t lds = batch_lds_bytes(b->hm.nv, cap);
  if (lds > 160 * 1024) return bfail(b, HC_ERR_UNSUPPORTED, "tiling: tile too large for LDS");
  HB_TRY(bcheck(b, hipFuncSetAttribute(batch_kernel(b->K), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds),
                "lds attribute"));
  int per_cu = 0;
  HB_TRY(bcheck(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel(b->K), block, lds),
                "occupancy"));
  int dev = 0, cus = 0;
  HB_TRY(bcheck(b, hipGetDevice(&dev), "device"));
  HB_TRY(bcheck(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "cus"));
  const int resident = std::min(per_cu * cus, kMaxGrid);
  const int per_xcd = resident / kXcd;
  if (per_xcd < 1) return bfail(b, HC_ERR_UNSUPPORTED, "tiling: no resident work-group");
  if (b->nbox > per_xcd * kXcd)
    return bfail(b, HC_ERR_UNSUPPORTED, "more boxes than resident work-groups");
  // members per box in proportion to its nodes, at least one
  const int total = per_xcd * kXcd;
  std::vector<int> w(b->nbox);
  for (int i = 0; i < b->nbox; ++i)
    w[i] = std::max(1, (int)std::floor((double)b->box[i].n / (double)b->sites * total));
  std::vector<int> order(b->nbox);
  for (int i = 0; i < b->nbox; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b->box[a].n > b->box[c].n; });
  std::vector<int> used(kXcd, 0);
  std::vector<double> load(kXcd, 0.0);
  std::vector<int4> wg(total, int4{-1, 0, 0, 0});
  for (int r = 0; r < b->nbox; ++r) {
    const int i = order[r];
    // boxes still to place need one slot each
    int x = -1;
    for (int c = 0; c < kXcd; ++c)
      if (used[c] < per_xcd && (x < 0 || load[c] < load[x])) x = c;
    if (x < 0) return bfail(b, HC_ERR_UNSUPPORTED, "no slot left for a box");
    int free_total = 0;
    for (int c = 0; c < kXcd; ++c) free_total += per_xcd - used[c];
    const int reserve = b->nbox - r - 1;
    const int m = std::max(1, std::min({w[i], per_xcd - used[x], free_total - reserve}));
    for (int k = 0; k < m; ++k) wg[x + kXcd * (used[x] + k)] = int4{i, k, m, 0};
    used[x] += m;
    load[x] += (double)b->box[i].n;
  }
  int maxu = 0;
  for (int c = 0; c < kXcd; ++c) maxu = std::max(maxu, used[c]);
  b->grid = maxu * kXcd;
  wg.resize(b->grid);
  b->wg = wg;
  b->ty = ty;
  b->tz = tz;
  b->block = block;
  b->V.tile_cap = cap;
  if (b->ws) {
    HB_TRY(h2d(b, bat<void>(b, b->o_box), b->box.data(), b->box.size() * sizeof(BoxDesc)));
    HB_TRY(h2d(b, bat<void>(b, b->o_wg), b->wg.data(), b->wg.size() * sizeof(int4)));
    HB_TRY(bsync(b));
  }
  drop_graph(b);
  return HC_OK;
}

hc_status launch_steps(hc_batch* b, int n, hipStream_t s) {
  HB_TRY(bcheck(b, launch_fill_i32(b->V.bar, 0, b->nbox, s), "barrier reset"));
  HB_TRY(bcheck(b, launch_batch(b->V, b->K, n, b->grid, b->block, s), "batch kernel"));
  return HC_OK;
}

hc_status snapshot(hc_batch* b, bool save) {
  const size_t P = (size_t)19 * b->sites * 4;
  const size_t X = (size_t)b->nbox * b->hm.nv * 12;
  // every box has taken the same number of steps, so all share one parity
  int step0 = 0;
  HB_TRY(d2h(b, &step0, b->V.box_step, 4));
  HB_TRY(bsync(b));
  float* cur = (step0 & 1) ? b->V.pops1 : b->V.pops0;
  if (save) {
    HB_TRY(d2d(b, bat<void>(b, b->o_snap_pop), cur, P));
    HB_TRY(d2d(b, bat<void>(b, b->o_snap_off), b->V.off, X));
    HB_TRY(d2d(b, bat<void>(b, b->o_snap_lo), b->V.lo, X));
    HB_TRY(d2d(b, bat<void>(b, b->o_snap_step), b->V.box_step, (size_t)b->nbox * 4));
  } else {
    int snap_step = 0;
    HB_TRY(d2h(b, &snap_step, bat<void>(b, b->o_snap_step), 4));
    HB_TRY(bsync(b));
    float* dst = (snap_step & 1) ? b->V.pops1 : b->V.pops0;
    HB_TRY(d2d(b, dst, bat<void>(b, b->o_snap_pop), P));
    HB_TRY(d2d(b, b->V.off, bat<void>(b, b->o_snap_off), X));
    HB_TRY(d2d(b, b->V.lo, bat<void>(b, b->o_snap_lo), X));
    HB_TRY(d2d(b, b->V.box_step, bat<void>(b, b->o_snap_step), (size_t)b->nbox * 4));
  }
  return bsync(b);
}

std::string cache_key(hc_batch* b) {
  hipDeviceProp_t p;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&p, dev);
  int maxside = 0;
  for (auto& B : b->box) maxside = std::max({maxside, B.nx, B.ny, B.nz});
  std::ostringstream k;
  std::string arch = p.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  k << arch << "|K" << b->K << "|boxes" << b->nbox << "|sites" << b->sites << "|max" << maxside;
  return k.str();
}

}  // namespace

extern "C" {

hc_status hc_batch_create(int32_t n_boxes, const hc_lattice_desc* boxes, const hc_mesh_desc* mesh,
                          hc_batch** out) {
  if (!out || !boxes || n_boxes <= 0) return bfail(nullptr, HC_ERR_ARG, "batch: bad arguments");
  *out = nullptr;
  hc_batch* b = new hc_batch();
  std::string e = build_mesh(mesh, b->hm);
  if (!e.empty()) {
    delete b;
    return bfail(nullptr, HC_ERR_ARG, e);
  }
  b->nbox = n_boxes;
  b->K = boxes[0].ibm_kernel;
  for (int i = 0; i < n_boxes; ++i) {
    const hc_lattice_desc& d = boxes[i];
    std::string why;
    if (d.nx < 4 || d.ny < 4 || d.nz < 4) why = "box sides must be >= 4";
    if (!(d.tau > 0.5f)) why = "tau must exceed 1/2";
    if (d.ibm_kernel != b->K || (d.ibm_kernel != HC_PHI4 && d.ibm_kernel != HC_PHI2))
      why = "all boxes need the same ibm_kernel (HC_PHI4 or HC_PHI2)";
    int walls = 0, wall_axis = -1;
    for (int a = 0; a < 3; ++a)
      if (d.bc[a] == HC_WALL) {
        ++walls;
        wall_axis = a;
      } else if (d.bc[a] != HC_PERIODIC) {
        why = "bc must be HC_PERIODIC or HC_WALL";
      }
    if (walls > 1) why = "at most one wall axis per box";
    if (wall_axis >= 0 && (d.wall_u_lo[wall_axis] != 0.f || d.wall_u_hi[wall_axis] != 0.f))
      why = "wall velocities must be tangential";
    if (d.lees_edwards_u != 0.f) why = "Lees-Edwards images are not available to the batched form";
    if (!why.empty()) {
      delete b;
      return bfail(nullptr, HC_ERR_ARG, "box " + std::to_string(i) + ": " + why);
    }
    BoxDesc B{};
    B.nx = d.nx;
    B.ny = d.ny;
    B.nz = d.nz;
    B.wall_axis = wall_axis;
    for (int a = 0; a < 3; ++a) {
      B.bc[a] = d.bc[a];
      B.g[a] = d.body_force[a];
      B.ulo[a] = d.wall_u_lo[a];
      B.uhi[a] = d.wall_u_hi[a];
    }
    B.omega = 1.0f / d.tau;
    B.omega_in = B.omega;
    B.n = (int64_t)d.nx * d.ny * d.nz;
    B.pop_off = 19 * b->sites;
    B.site_off = b->sites;
    b->sites += B.n;
    b->box.push_back(B);
    b->lat.push_back(d);
  }
  *out = b;
  return HC_OK;
}

void hc_batch_destroy(hc_batch* b) {
  if (!b) return;
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}

const char* hc_batch_last_error(const hc_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

hc_status hc_batch_set_stream(hc_batch* b, void* s) {
  if (!b) return HC_ERR_ARG;
  b->stream = reinterpret_cast<hipStream_t>(s);
  return HC_OK;
}

hc_status hc_batch_query_workspace(const hc_batch* b, size_t* bytes) {
  if (!b || !bytes) return HC_ERR_ARG;
  Lay L;
  plan(const_cast<hc_batch*>(b), L);
  *bytes = L.total;
  return HC_OK;
}

hc_status hc_batch_bind_workspace(hc_batch* b, void* dev, size_t bytes) {
  if (!b || !dev) return bfail(b, HC_ERR_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(dev) & 255) return bfail(b, HC_ERR_ARG, "workspace not 256-aligned");
  Lay L;
  plan(b, L);
  if (bytes < L.total) return bfail(b, HC_ERR_OOM, "workspace smaller than hc_batch_query_workspace");
  b->ws = static_cast<char*>(dev);
  const HostMesh& m = b->hm;
  Batch& V = b->V;
  V.nbox = b->nbox;
  V.has_cells = 0;
  V.box = bat<BoxDesc>(b, b->o_box);
  V.pops0 = bat<float>(b, b->o_pop0);
  V.pops1 = bat<float>(b, b->o_pop1);
  V.M.nv = m.nv;
  V.M.nt = m.nt;
  V.M.ne = m.ne;
  V.M.nh = m.nh;
  V.M.tri = bat<int>(b, b->o_tri);
  V.M.edge = bat<int>(b, b->o_edge);
  V.M.L0 = bat<float>(b, b->o_L0);
  V.M.hinge_v = bat<int>(b, b->o_hv);
  V.M.theta0 = bat<float>(b, b->o_th0);
  V.M.pole = bat<float>(b, b->o_pole);
  V.M.hinge_own = bat<int>(b, b->o_own);
  V.M.inv_npole = 1.0f / kNPole;
  V.M.A0 = m.A0;
  V.M.V0 = m.V0;
  V.origin = bat<int>(b, b->o_origin);
  V.off = bat<float>(b, b->o_off);
  V.lo = bat<float>(b, b->o_lo);
  V.force = bat<float>(b, b->o_force);
  V.vel = bat<float>(b, b->o_vel);
  V.k = bat<float>(b, b->o_k);
  V.trac = nullptr;
  V.area = bat<double>(b, b->o_area);
  V.volume = bat<double>(b, b->o_vol);
  V.uacc = bat<long long>(b, b->o_uacc);
  V.bbox = bat<int>(b, b->o_bbox);
  V.wg = bat<int4>(b, b->o_wg);
  V.bar = bat<int>(b, b->o_bar);
  V.box_step = bat<int>(b, b->o_step);
  V.flags = bat<int>(b, b->o_flags);
  V.mask = bat<unsigned char>(b, b->o_mask);
  V.interior = 0;
  for (auto& B : b->box) V.interior |= B.omega_in != B.omega;
  V.spin_limit = kSpinLimit;
  HB_TRY(h2d(b, (void*)V.M.tri, m.tri.data(), m.tri.size() * 4));
  HB_TRY(h2d(b, (void*)V.M.edge, m.edge.data(), m.edge.size() * 4));
  HB_TRY(h2d(b, (void*)V.M.L0, m.L0.data(), m.L0.size() * 4));
  HB_TRY(h2d(b, (void*)V.M.hinge_v, m.hinge_v.data(), m.hinge_v.size() * 4));
  HB_TRY(h2d(b, (void*)V.M.theta0, m.theta0.data(), m.theta0.size() * 4));
  HB_TRY(h2d(b, (void*)V.M.pole, m.pole.data(), m.pole.size() * 4));
  HB_TRY(h2d(b, (void*)V.M.hinge_own, m.hinge_own.data(), m.hinge_own.size() * 4));
  HB_TRY(bcheck(b, launch_fill_i32(V.box_step, 0, b->nbox, b->stream), "clear"));
  HB_TRY(bcheck(b, launch_fill_i32(V.flags, 0, 4, b->stream), "clear"));
  HB_TRY(bcheck(b, launch_fill_i32(reinterpret_cast<int*>(V.mask), 0, (b->sites + 3) / 4, b->stream),
                "clear"));
  HB_TRY(bcheck(b, launch_fill_i32(reinterpret_cast<int*>(V.uacc), 0,
                                   (int64_t)b->nbox * m.nv * 6, b->stream),
                "clear"));
  for (auto& B : b->box)
    HB_TRY(bcheck(b, launch_init_uniform(V.pops0 + B.pop_off, 1.f, 0.f, 0.f, 0.f, B.n, b->stream),
                  "init"));
  if (!b->cap_stream) HB_TRY(bcheck(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "stream"));
  HB_TRY(apply_tiling(b, b->ty, b->tz, b->block));
  return bsync(b);
}

hc_status hc_batch_set_cells(hc_batch* b, const int32_t* origin, const float* offsets, const float* k,
                             const float* traction) {
  if (!b || !b->ws) return bfail(b, HC_ERR_STATE, "no workspace bound");
  if (!origin || !offsets || !k) return bfail(b, HC_ERR_ARG, "null cell array");
  const size_t nv = b->hm.nv, B = b->nbox;
  HB_TRY(h2d(b, b->V.origin, origin, B * 12));
  HB_TRY(h2d(b, b->V.off, offsets, B * nv * 12));
  HB_TRY(bcheck(b, launch_fill_i32(reinterpret_cast<int*>(b->V.lo), 0, (int64_t)(B * nv * 3), b->stream),
                "clear position low parts"));
  HB_TRY(h2d(b, (void*)b->V.k, k, B * 16));
  if (traction) {
    HB_TRY(h2d(b, bat<void>(b, b->o_trac), traction, B * 12));
    b->V.trac = bat<float>(b, b->o_trac);
  } else {
    b->V.trac = nullptr;
  }
  b->V.has_cells = 1;
  drop_graph(b);
  return bsync(b);
}

hc_status hc_batch_set_interior_viscosity(hc_batch* b, const float* ratio) {
  if (!b || !b->ws) return bfail(b, HC_ERR_STATE, "no workspace bound");
  if (!ratio) return bfail(b, HC_ERR_ARG, "null ratio array");
  for (int i = 0; i < b->nbox; ++i)
    if (!(ratio[i] > 0.f) || !std::isfinite(ratio[i]))
      return bfail(b, HC_ERR_ARG, "box " + std::to_string(i) + ": ratio must be finite and > 0");
  int any = 0;
  for (int i = 0; i < b->nbox; ++i) {
    BoxDesc& B = b->box[i];
    const double tau = b->lat[i].tau;
    B.omega_in = (float)(1.0 / (0.5 + (double)ratio[i] * (tau - 0.5)));
    any |= B.omega_in != B.omega;
  }
  b->V.interior = any;
  HB_TRY(h2d(b, bat<void>(b, b->o_box), b->box.data(), b->box.size() * sizeof(BoxDesc)));
  drop_graph(b);
  return bsync(b);
}

hc_status hc_batch_set_tiling(hc_batch* b, int32_t ty, int32_t tz, int32_t block) {
  if (!b || !b->ws) return bfail(b, HC_ERR_STATE, "no workspace bound");
  return apply_tiling(b, ty, tz, block);
}

hc_status hc_batch_get_tiling(const hc_batch* b, int32_t* ty, int32_t* tz, int32_t* block,
                              int32_t* grid) {
  if (!b) return HC_ERR_ARG;
  if (ty) *ty = b->ty;
  if (tz) *tz = b->tz;
  if (block) *block = b->block;
  if (grid) *grid = b->grid;
  return HC_OK;
}

hc_status hc_batch_run(hc_batch* b, int32_t n) {
  if (!b || !b->ws) return bfail(b, HC_ERR_STATE, "no workspace bound");
  if (n <= 0) return n == 0 ? HC_OK : bfail(b, HC_ERR_ARG, "n_steps < 0");
  if (!b->exec || b->graph_steps != n) {
    drop_graph(b);
    HB_TRY(bcheck(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed), "capture"));
    hc_status s = launch_steps(b, n, b->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (s != HC_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    HB_TRY(bcheck(b, e, "end capture"));
    b->graph = g;
    HB_TRY(bcheck(b, hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "instantiate"));
    b->graph_steps = n;
  }
  HB_TRY(bcheck(b, hipGraphLaunch(b->exec, b->stream), "graph launch"));
  b->launches += 1;
  return HC_OK;
}

hc_status hc_batch_sync(hc_batch* b) {
  if (!b || !b->ws) return bfail(b, HC_ERR_STATE, "no workspace bound");
  HB_TRY(bsync(b));
  int f[4];
  HB_TRY(d2h(b, f, b->V.flags, 16));
  HB_TRY(bsync(b));
  if (f[0] || f[1] || f[2]) {
    HB_TRY(bcheck(b, launch_fill_i32(b->V.flags, 0, 4, b->stream), "clear"));
    HB_TRY(bsync(b));
    if (f[1]) return bfail(b, HC_ERR_DEVICE, "group barrier timed out (work-groups not co-resident)");
    if (f[2] & 16)
      return bfail(b, HC_ERR_UNSUPPORTED, "interior marking: a cell wider than 320 columns or 1024 nodes");
    if (f[2] & 32)
      return bfail(b, HC_ERR_UNSUPPORTED, "interior marking: more than 8 membrane crossings on a column");
    return bfail(b, HC_ERR_NONFINITE, "non-finite vertex position");
  }
  return HC_OK;
}

hc_status hc_batch_autotune(hc_batch* b, const char* cache_path, int32_t trial_steps, int32_t* ty,
                            int32_t* tz, int32_t* block) {
  if (!b || !b->ws) return bfail(b, HC_ERR_STATE, "no workspace bound");
  const std::string key = cache_key(b);
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      int a, c, d;
      if ((ls >> k >> a >> c >> d) && k == key) {
        HB_TRY(apply_tiling(b, a, c, d));
        if (ty) *ty = a;
        if (tz) *tz = c;
        if (block) *block = d;
        return HC_OK;
      }
    }
  }
  if (trial_steps < 1) trial_steps = 10;
  const int shapes[][2] = {{1, 1}, {1, 2}, {2, 2}, {2, 4}, {4, 4}, {4, 8}, {8, 8}};
  const int blocks[] = {256, 512};
  hipEvent_t e0, e1;
  HB_TRY(bcheck(b, hipEventCreate(&e0), "event"));
  HB_TRY(bcheck(b, hipEventCreate(&e1), "event"));
  HB_TRY(snapshot(b, true));
  float best = 1e30f;
  int bt = b->ty, bz = b->tz, bb = b->block;
  for (auto& sh : shapes)
    for (int bl : blocks) {
      if (apply_tiling(b, sh[0], sh[1], bl) != HC_OK) continue;
      HB_TRY(launch_steps(b, 1, b->stream));   // warm-up
      HB_TRY(bcheck(b, hipEventRecord(e0, b->stream), "event"));
      HB_TRY(launch_steps(b, trial_steps, b->stream));
      HB_TRY(bcheck(b, hipEventRecord(e1, b->stream), "event"));
      HB_TRY(bsync(b));
      float ms = 0.f;
      HB_TRY(bcheck(b, hipEventElapsedTime(&ms, e0, e1), "event"));
      int f[4];
      HB_TRY(d2h(b, f, b->V.flags, 16));
      HB_TRY(bsync(b));
      HB_TRY(snapshot(b, false));
      if (f[1]) {   // a timed-out configuration is discarded
        HB_TRY(bcheck(b, launch_fill_i32(b->V.flags, 0, 4, b->stream), "clear"));
        continue;
      }
      if (ms < best) {
        best = ms;
        bt = sh[0];
        bz = sh[1];
        bb = bl;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HB_TRY(apply_tiling(b, bt, bz, bb));
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    out << key << " " << bt << " " << bz << " " << bb << "\n";
  }
  if (ty) *ty = bt;
  if (tz) *tz = bz;
  if (block) *block = bb;
  return HC_OK;
}

hc_status hc_batch_box_steps(hc_batch* b, int32_t box, int64_t* steps) {
  if (!b || !b->ws || box < 0 || box >= b->nbox || !steps) return bfail(b, HC_ERR_ARG, "bad box");
  int s = 0;
  HB_TRY(d2h(b, &s, b->V.box_step + box, 4));
  HB_TRY(bsync(b));
  *steps = s;
  return HC_OK;
}

hc_status hc_batch_read_populations(hc_batch* b, int32_t box, float* host, int64_t count) {
  int64_t st = 0;
  HB_TRY(hc_batch_box_steps(b, box, &st));
  const BoxDesc& B = b->box[box];
  if (!host || count != 19 * B.n) return bfail(b, HC_ERR_ARG, "population count mismatch");
  const float* src = ((st & 1) ? b->V.pops1 : b->V.pops0) + B.pop_off;
  HB_TRY(d2h(b, host, src, (size_t)count * 4));
  return bsync(b);
}

hc_status hc_batch_write_populations(hc_batch* b, int32_t box, const float* host, int64_t count) {
  int64_t st = 0;
  HB_TRY(hc_batch_box_steps(b, box, &st));
  const BoxDesc& B = b->box[box];
  if (!host || count != 19 * B.n) return bfail(b, HC_ERR_ARG, "population count mismatch");
  float* dst = ((st & 1) ? b->V.pops1 : b->V.pops0) + B.pop_off;
  HB_TRY(h2d(b, dst, host, (size_t)count * 4));
  return bsync(b);
}

hc_status hc_batch_read_vertices(hc_batch* b, int32_t box, int32_t* origin, float* offsets,
                                 float* force, float* vel) {
  if (!b || !b->ws || box < 0 || box >= b->nbox) return bfail(b, HC_ERR_ARG, "bad box");
  const size_t nv = b->hm.nv;
  if (origin) HB_TRY(d2h(b, origin, b->V.origin + 3 * box, 12));
  if (offsets) HB_TRY(d2h(b, offsets, b->V.off + nv * 3 * box, nv * 12));
  if (force) HB_TRY(d2h(b, force, b->V.force + nv * 3 * box, nv * 12));
  if (vel) HB_TRY(d2h(b, vel, b->V.vel + nv * 3 * box, nv * 12));
  return bsync(b);
}

hc_status hc_batch_launches(const hc_batch* b, int64_t* graph_launches) {
  if (!b || !graph_launches) return HC_ERR_ARG;
  *graph_launches = b->launches;
  return HC_OK;
}

}  // extern "C"
