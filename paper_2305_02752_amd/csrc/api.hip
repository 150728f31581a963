// C ABI of libhemo (declared in include/hemo.h): context set-up, workspace
// carving, mesh-table construction and the per-step launch sequence.
//
// A coupled step enqueues, in order (Sec. 2.3 coupling, Sec. 2.6 Euler):
//   membrane forces (one wave per cell) -> vertex binning to tiles ->
//   LDS spread per tile -> collide + stream -> interpolation + advection.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/hemo.h"
#include "common.h"
#include "host.h"

using namespace hc;

namespace {

constexpr int kMaxCellTiles = 512;   // cell cover read-out: 8 tiles per axis per cell
thread_local std::string g_create_error;

struct Layout {
  size_t total = 0;
  size_t add(size_t bytes) {
    const size_t at = total;
    total += (bytes + 255) & ~size_t(255);
    return at;
  }
};

}  // namespace

struct hc_ctx {
  Lattice L{};
  HostMesh hm;
  Mesh M{};
  Cells C{};
  Bins B{};
  int max_cells = 0;
  int list_cap = 0;            // entries per tile list
  int* touch_ptr = nullptr;    // CSR form of the tile lists (read-out only)
  int* touch_csr = nullptr;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  float* pops[2] = {nullptr, nullptr};
  int cur = 0;
  float* F = nullptr;
  float4* macro = nullptr;     // (ux, uy, uz, rho) per site of the last step
  float4* partial = nullptr;   // interpolation partial sums [touch slot][cells x V]
  int *cell_cnt = nullptr, *cell_ptr = nullptr, *cell_tiles = nullptr, *cell_rank = nullptr,
      *cell_list = nullptr;
  int64_t step = 0;
  bool have_cells = false;
  // the last step's vertex move is still to be applied (it runs fused into
  // the next step's per-cell kernel, or in flush() before the state is seen)
  bool advect_pending = false;
  bool fields = true;          // write the force and (u, rho) fields each step
  // cell integration (Sec. 2.6): membrane forces every force_every steps,
  // Euler or Adams-Bashforth moves; have_prev: C.vel holds the previous U
  int force_every = 1;
  int scheme = HC_EULER;
  bool have_prev = false;
  // offsets re-centred after moves; off while the adjoint records a forward
  // run (its segment replay keeps one origin per cell)
  bool recentre = true;
  // interior viscosity (Sec. 1, Sec. 3.4): sites inside the cells relax with
  // ratio times the plasma viscosity.  One ratio for every cell
  // (uniform_ratio; 1 switches the marking off) or one per cell, as up to
  // kVisClasses distinct ratios (class_ratio, increasing) and a class per cell
  float uniform_ratio = 1.f;
  int n_vclass = 1;
  float class_ratio[kVisClasses] = {1.f};
  bool per_cell_ratio = false;
  unsigned char* mask = nullptr;   // [np] site-ordered inside marks, zero between steps
  unsigned char* cell_class = nullptr;   // [max_cells] viscosity class of each cell
  // optional per-kernel timing with events on the context stream
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_pairs[HC_NUM_KERNELS];
  size_t ev_next = 0;
  std::string err;
  // reverse mode: checkpoints, one recomputed segment, cotangents
  char* adj_ws = nullptr;
  int adj_n = 0, adj_ck = 0, adj_nseg = 0;
  bool adj_ready = false;
  float *ck_pops = nullptr, *ck_off = nullptr, *ck_lo = nullptr, *sg_lo = nullptr;
  float *sg_pops = nullptr, *sg_off = nullptr, *sg_F = nullptr, *sg_Fv = nullptr;
  float4* sg_macro = nullptr;
  float* lam_f[2] = {nullptr, nullptr};   // population cotangents (FP32 storage, FP64 arithmetic)
  float* lam_X[2] = {nullptr, nullptr};
  float *lam_Fv = nullptr, *lam_u = nullptr, *lam_F = nullptr, *vel_scratch = nullptr;
  double *dom_part = nullptr, *dk = nullptr, *loss = nullptr, *targets = nullptr, *scal = nullptr;
  double* dom_in_part = nullptr;   // d/d omega_in partial sums (sites inside cells)
  // workspace offsets
  size_t o_pops[2], o_F, o_macro, o_partial, o_origin, o_off, o_lo, o_force, o_vel, o_k, o_trac, o_area, o_vol;
  size_t o_tri, o_edge, o_L0, o_hv, o_th0, o_pole, o_own;
  size_t o_owner, o_ntouch, o_scan, o_slot, o_tcnt, o_tptr, o_touch, o_csr, o_flags;
  size_t o_ccnt, o_cptr, o_ctiles, o_crank, o_clist, o_mask, o_cclass, o_rest;
  std::vector<float> rest;   // the rest mesh [nv][3], copied at create
};

namespace {

hc_status fail(hc_ctx* c, hc_status s, const std::string& msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return s;
}

hc_status check(hc_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return HC_OK;
  return fail(c, HC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HC_TRY(expr)                        \
  do {                                      \
    hc_status _s = (expr);                  \
    if (_s != HC_OK) return _s;             \
  } while (0)

template <class T>
T* at(hc_ctx* c, size_t off) {
  return reinterpret_cast<T*>(c->ws + off);
}

void plan(hc_ctx* c, Layout& lay) {
  const int64_t N = c->L.np;   // lattice fields are stored tile-major with padding
  const int64_t C = c->max_cells, nv = c->hm.nv;
  const int64_t NT = c->L.ntiles;
  c->o_pops[0] = lay.add(19 * N * 4);
  c->o_pops[1] = lay.add(19 * N * 4);
  c->o_F = lay.add(3 * N * 4);
  c->o_macro = lay.add(N * 16);
  c->o_origin = lay.add(C * 3 * 4);
  c->o_off = lay.add(C * nv * 3 * 4);
  c->o_lo = lay.add(C * nv * 3 * 4);
  c->o_force = lay.add(C * nv * 3 * 4);
  c->o_vel = lay.add(C * nv * 3 * 4);
  c->o_k = lay.add(C * 4 * 4);
  c->o_trac = lay.add(C * 3 * 4);
  c->o_area = lay.add(C * 8);
  c->o_vol = lay.add(C * 8);
  const HostMesh& m = c->hm;
  c->o_tri = lay.add(m.tri.size() * 4);
  c->o_edge = lay.add(m.edge.size() * 4);
  c->o_L0 = lay.add(m.L0.size() * 4);
  c->o_hv = lay.add(m.hinge_v.size() * 4);
  c->o_th0 = lay.add(m.theta0.size() * 4);
  c->o_pole = lay.add(m.pole.size() * 4);
  c->o_own = lay.add(m.hinge_own.size() * 4);
  c->o_owner = lay.add(C * nv * 4);
  c->o_ntouch = lay.add(C * nv * 4);
  c->o_scan = lay.add(((NT + 4095) / 4096 + 1) * 4);
  c->o_slot = lay.add(std::max<int64_t>(1, C * nv * c->L.max_touch) * 4);
  c->o_tcnt = lay.add((NT + 1) * 4);
  c->o_tptr = lay.add((NT + 1) * 4);
  c->o_touch = lay.add(NT * (int64_t)c->list_cap * 4);
  c->o_csr = lay.add(std::max<int64_t>(1, C * nv * c->L.max_touch) * 4);
  c->o_partial = lay.add(std::max<int64_t>(1, C * nv * c->L.max_touch) * 16);
  c->o_flags = lay.add(16);
  c->o_ccnt = lay.add((NT + 1) * 4);
  c->o_cptr = lay.add((NT + 1) * 4);
  c->o_ctiles = lay.add(std::max<int64_t>(1, C * kMaxCellTiles) * 4);
  c->o_crank = lay.add(std::max<int64_t>(1, C * kMaxCellTiles) * 4);
  c->o_clist = lay.add(std::max<int64_t>(1, C * kMaxCellTiles) * 4);
  c->o_mask = lay.add(N);
  c->o_cclass = lay.add(std::max<int64_t>(1, C));
  c->o_rest = lay.add(nv * 3 * 4);
}

hc_status need_ws(hc_ctx* c) {
  if (!c) return HC_ERR_ARG;
  if (!c->ws) return fail(c, HC_ERR_STATE, "no workspace bound (hc_bind_workspace)");
  return HC_OK;
}

hc_status sync(hc_ctx* c, const char* what) { return check(c, hipStreamSynchronize(c->stream), what); }

hc_status copy_d2h(hc_ctx* c, void* dst, const void* src, size_t bytes) {
  if (!bytes) return HC_OK;
  return check(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream), "d2h copy");
}
hc_status copy_h2d(hc_ctx* c, void* dst, const void* src, size_t bytes) {
  if (!bytes) return HC_OK;
  return check(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream), "h2d copy");
}

int ev_take(hc_ctx* c) {
  if (c->ev_next == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    c->ev_pool.push_back(e);
  }
  return (int)c->ev_next++;
}

// Launch `fn` bracketed by timing events when profiling is on.
template <class Fn>
hc_status timed(hc_ctx* c, int kernel, const char* what, Fn fn) {
  if (!c->prof) return check(c, fn(), what);
  const int a = ev_take(c), b = ev_take(c);
  if (a < 0 || b < 0) return fail(c, HC_ERR_DEVICE, "event creation failed");
  HC_TRY(check(c, hipEventRecord(c->ev_pool[a], c->stream), "event record"));
  HC_TRY(check(c, fn(), what));
  HC_TRY(check(c, hipEventRecord(c->ev_pool[b], c->stream), "event record"));
  c->ev_pairs[kernel].push_back({a, b});
  return HC_OK;
}

hc_status copy_d2d(hc_ctx* c, void* dst, const void* src, size_t bytes) {
  if (!bytes) return HC_OK;
  return check(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream), "d2d copy");
}

// Lees-Edwards image displacements U t mod nx (in double: t grows) for the
// step about to run (IBM stencils) and for the step before it, whose
// streaming the next pull completes.
bool interior_on(const hc_ctx* c) { return c->n_vclass > 1 || c->class_ratio[0] != 1.f; }

// Relaxation rates inside the cells: tau_in - 1/2 = ratio (tau - 1/2).
void interior_update(hc_ctx* c) {
  for (int k = 0; k < kVisClasses; ++k) {
    const double r = k < c->n_vclass ? c->class_ratio[k] : 1.0;
    c->L.omega_in[k] = (float)(1.0 / (0.5 + r * ((double)c->L.tau - 0.5)));
  }
}

void interior_uniform(hc_ctx* c) {
  c->per_cell_ratio = false;
  c->n_vclass = 1;
  c->class_ratio[0] = c->uniform_ratio;
  interior_update(c);
}

// One marking pass, or one per viscosity class in increasing order, so that
// a site inside cells of several classes keeps the most viscous one.
hipError_t mark_interior(hc_ctx* c, const Cells& C) {
  if (c->n_vclass <= 1)
    return launch_mark_interior(C, c->M, c->L, c->mask, nullptr, -1, c->B.flags, c->stream);
  for (int k = 0; k < c->n_vclass; ++k) {
    const hipError_t e =
        launch_mark_interior(C, c->M, c->L, c->mask, c->cell_class, k, c->B.flags, c->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void le_update(hc_ctx* c) {
  if (!c->L.le) return;
  auto shift = [&](int64_t t) {
    const double n = c->L.nx;
    return (float)std::fmod(std::fmod((double)c->L.le_u * (double)t, n) + n, n);
  };
  c->L.le_delta = shift(c->step);
  c->L.le_pull_delta = shift(c->step - 1);
}

// One coupled step.  The vertex move that closes the step (interpolated
// velocity, Euler or Adams-Bashforth) is left pending: the next step's
// per-cell kernel applies it before the membrane forces, or flush() applies
// it on its own.  The membrane forces are recomputed every force_every
// steps and held in between.
hc_status one_step(hc_ctx* c) {
  le_update(c);
  Cells C = c->C;
  C.n = c->have_cells ? c->C.n : 0;
  const bool adv = c->advect_pending;
  const bool ab2 = adv && c->scheme == HC_AB2 && c->have_prev;
  const bool refresh = c->step % c->force_every == 0;
  HC_TRY(timed(c, HC_K_CELL, "cell step", [&] {
    return launch_cell_step(C, c->M, c->L, c->B, c->partial, c->B.flags, adv, nullptr, refresh, ab2,
                            c->recentre, c->scheme == HC_AB2, c->stream);
  }));
  if (adv) c->have_prev = true;
  unsigned char* mask = nullptr;
  if (interior_on(c) && C.n > 0) {
    mask = c->mask;
    HC_TRY(timed(c, HC_K_INTERIOR, "interior marking", [&] { return mark_interior(c, C); }));
  }
  HC_TRY(timed(c, HC_K_LATTICE, "lattice pass", [&] {
    return launch_tile_step(C, c->M, c->L, c->B, c->pops[c->cur], c->pops[c->cur ^ 1], c->F,
                            c->macro, c->partial, c->fields, mask, c->stream);
  }));
  c->advect_pending = C.n > 0;
  c->cur ^= 1;
  c->step += 1;
  c->L.le_raw = 0;   // the new state holds post-collision values
  return HC_OK;
}

// Apply a pending vertex move, so that positions and velocities are current.
hc_status flush(hc_ctx* c) {
  if (!c->advect_pending) return HC_OK;
  c->advect_pending = false;
  const bool ab2 = c->scheme == HC_AB2 && c->have_prev;
  c->have_prev = true;
  return timed(c, HC_K_ADVECT, "advect", [&] {
    return launch_advect(c->C, c->M, c->L, c->B, c->partial, c->B.flags, ab2, c->stream);
  });
}

hc_status run_steps(hc_ctx* c, int n) {
  for (int i = 0; i < n; ++i) HC_TRY(one_step(c));
  return flush(c);
}

struct AdjPlan {
  size_t total = 0;
  size_t ck_pops, ck_off, ck_lo, sg_lo, sg_pops, sg_off, sg_F, sg_macro, sg_Fv, lf0, lf1, lx0, lx1, lfv, lu, lF, vel,
      dom, dom_in, dk, loss, tg, scal;
};

AdjPlan adj_plan(const hc_ctx* c, int n, int ck) {
  AdjPlan p;
  Layout L;
  const int64_t N = c->L.np, P = 19 * N, X = (int64_t)c->max_cells * c->hm.nv * 3;
  const int64_t nck = (n + ck - 1) / ck, C = c->max_cells;
  p.ck_pops = L.add(nck * P * 4);
  p.ck_off = L.add(nck * X * 4);
  p.ck_lo = L.add(nck * X * 4);
  p.sg_lo = L.add(X * 4);
  p.sg_pops = L.add((ck + 1) * P * 4);
  p.sg_off = L.add((ck + 1) * X * 4);
  p.sg_F = L.add(ck * 3 * N * 4);
  p.sg_macro = L.add(ck * N * 16);
  p.sg_Fv = L.add(ck * X * 4);
  p.lf0 = L.add(P * 4);
  p.lf1 = L.add(P * 4);
  p.lx0 = L.add(X * 4);
  p.lx1 = L.add(X * 4);
  p.lfv = L.add(X * 4);
  p.lu = L.add(3 * N * 4);
  p.lF = L.add(3 * N * 4);
  p.vel = L.add(X * 4);
  p.dom = L.add(((N + 255) / 256) * 8);
  p.dom_in = L.add(kVisClasses * ((N + 255) / 256) * 8);
  p.dk = L.add(C * 4 * 8);
  p.loss = L.add(C * 8);
  p.tg = L.add(C * 2 * 8);
  p.scal = L.add(128);   // d/d omega sums (plasma + 8 classes) and scalars
  p.total = L.total;
  return p;
}

// One forward step of the recomputed segment at slot i, keeping everything
// the reverse sweep reads.  It runs the forward step's kernels (field output
// on), so a recomputed state equals the forward one bit for bit.  The move
// that produces slot i's positions from slot i - 1 runs inside slot i's
// per-cell kernel, as in the forward step.
hc_status adj_forward_into(hc_ctx* c, int i) {
  const int64_t N = c->L.np, P = 19 * N, X = (int64_t)c->C.n * c->hm.nv * 3;
  Cells Ci = c->C;
  Ci.off = c->sg_off + i * X;
  Ci.lo = c->sg_lo;   // carried in place through the segment, from its checkpoint
  Ci.force = c->sg_Fv + i * X;
  Ci.vel = c->vel_scratch;
  float* Fi = c->sg_F + i * 3 * N;
  float4* Mi = c->sg_macro + i * N;
  const float* prev = i > 0 ? c->sg_off + (i - 1) * X : nullptr;
  HC_TRY(check(c, launch_cell_step(Ci, c->M, c->L, c->B, c->partial, c->B.flags, i > 0, prev, true,
                                   false, false, false, c->stream),
               "cell step"));
  unsigned char* mask = nullptr;
  if (interior_on(c)) {   // the forward step's marks, from slot i's positions
    mask = c->mask;
    HC_TRY(check(c, mark_interior(c, Ci), "interior marking"));
  }
  HC_TRY(check(c, launch_tile_step(Ci, c->M, c->L, c->B, c->sg_pops + i * P, c->sg_pops + (i + 1) * P,
                                   Fi, Mi, c->partial, true, mask, c->stream),
               "lattice pass"));
  return HC_OK;
}

// Reverse of step i of the segment: (lam_f, lam_X)^{i+1} -> (lam_f, lam_X)^i.
hc_status adj_reverse_step(hc_ctx* c, int i, int a) {
  const int64_t N = c->L.np, P = 19 * N, X = (int64_t)c->C.n * c->hm.nv * 3;
  Cells Ci = c->C;
  Ci.off = c->sg_off + i * X;
  Ci.lo = c->sg_lo;   // carried in place through the segment, from its checkpoint
  Ci.force = c->sg_Fv + i * X;
  Ci.vel = c->vel_scratch;
  float* lf1 = c->lam_f[a];
  float* lf0 = c->lam_f[a ^ 1];
  float* lx1 = c->lam_X[a];
  float* lx0 = c->lam_X[a ^ 1];
  HC_TRY(check(c, launch_bin_vertices(Ci, c->M, c->L, c->B, c->stream), "binning"));
  HC_TRY(check(c, launch_spread_vec(Ci, c->M, c->L, c->B, lx1, 0.f, c->lam_u, c->stream), "spread"));
  unsigned char* mask = nullptr;
  if (interior_on(c)) {   // the marks step i relaxed with (read and cleared by the collide VJP)
    mask = c->mask;
    HC_TRY(check(c, mark_interior(c, Ci), "interior marking"));
  }
  HC_TRY(check(c, launch_adj_collide(lf1, lf0, c->sg_pops + i * P, c->sg_F + i * 3 * N, c->lam_u,
                                     c->lam_F, c->dom_part, mask, c->dom_in_part, c->L, c->stream),
               "adjoint collide"));
  HC_TRY(check(c, launch_adj_vertex(Ci, c->M, c->L, lx1, c->sg_macro + i * N, c->lam_F, c->lam_Fv, lx0,
                                    c->stream),
               "adjoint ibm"));
  HC_TRY(check(c, launch_adj_membrane(Ci, c->M, c->lam_Fv, lx0, c->dk, c->stream), "adjoint membrane"));
  return HC_OK;
}

}  // namespace

extern "C" {

hc_status hc_create(const hc_lattice_desc* lat, const hc_mesh_desc* mesh, int32_t max_cells,
                    hc_ctx** out) {
  if (!out || !lat) return fail(nullptr, HC_ERR_ARG, "hc_create: null argument");
  *out = nullptr;
  if (lat->nx < 4 || lat->ny < 4 || lat->nz < 4)
    return fail(nullptr, HC_ERR_ARG, "lattice sides must be >= 4");
  if ((int64_t)lat->nx * lat->ny * lat->nz > (int64_t)1 << 31)
    return fail(nullptr, HC_ERR_UNSUPPORTED, "lattice above 2^31 nodes");
  if (!(lat->tau > 0.5f)) return fail(nullptr, HC_ERR_ARG, "tau must exceed 1/2");
  if (lat->ibm_kernel != HC_PHI4 && lat->ibm_kernel != HC_PHI2)
    return fail(nullptr, HC_ERR_ARG, "ibm_kernel must be HC_PHI4 or HC_PHI2");
  if (max_cells < 0) return fail(nullptr, HC_ERR_ARG, "max_cells < 0");
  if (max_cells >= (1 << 20)) return fail(nullptr, HC_ERR_UNSUPPORTED, "2^20 cells or more");
  if (mesh && (int64_t)max_cells * mesh->n_vert >= ((int64_t)1 << 26))
    return fail(nullptr, HC_ERR_UNSUPPORTED, "more than 2^26 vertices");
  int walls = 0, wall_axis = -1;
  for (int d = 0; d < 3; ++d) {
    if (lat->bc[d] != HC_PERIODIC && lat->bc[d] != HC_WALL)
      return fail(nullptr, HC_ERR_ARG, "bc must be HC_PERIODIC or HC_WALL");
    if (lat->bc[d] == HC_WALL) {
      ++walls;
      wall_axis = d;
    }
  }
  if (walls > 1) return fail(nullptr, HC_ERR_UNSUPPORTED, "at most one wall axis");
  const bool le = lat->lees_edwards_u != 0.f;
  if (le && (walls > 0 || lat->nx % kTile != 0 || lat->nz % kTile != 0))
    return fail(nullptr, HC_ERR_UNSUPPORTED,
                "Lees-Edwards images need every axis periodic and nx, nz multiples of 8");
  if (!std::isfinite(lat->lees_edwards_u)) return fail(nullptr, HC_ERR_ARG, "lees_edwards_u not finite");
  if (wall_axis >= 0 && (lat->wall_u_lo[wall_axis] != 0.f || lat->wall_u_hi[wall_axis] != 0.f))
    return fail(nullptr, HC_ERR_ARG, "wall velocities must be tangential");
  hc_ctx* c = new hc_ctx();
  std::string e = build_mesh(mesh, c->hm);
  if (!e.empty()) {
    delete c;
    return fail(nullptr, HC_ERR_ARG, e);
  }
  c->rest.assign(mesh->rest_pos, mesh->rest_pos + 3 * (size_t)mesh->n_vert);
  Lattice& L = c->L;
  L.nx = lat->nx;
  L.ny = lat->ny;
  L.nz = lat->nz;
  for (int d = 0; d < 3; ++d) {
    L.bc[d] = lat->bc[d];
    L.g[d] = lat->body_force[d];
    L.ulo[d] = lat->wall_u_lo[d];
    L.uhi[d] = lat->wall_u_hi[d];
  }
  L.wall_axis = wall_axis;
  {
    static const int ex[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static const int ey[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static const int ez[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    for (int q = 0; q < kQ; ++q) {
      // -6 w = -2 k with the collision's FP32 odd coefficients k
      const double k = q == 0 ? 0.0 : (q < 7 ? (double)HC_K1 : (double)HC_K2);
      const bool on = wall_axis >= 0;
      L.wc_lo[q] = on ? (float)(-2.0 * k * (ex[q] * L.ulo[0] + ey[q] * L.ulo[1] + ez[q] * L.ulo[2])) : 0.f;
      L.wc_hi[q] = on ? (float)(-2.0 * k * (ex[q] * L.uhi[0] + ey[q] * L.uhi[1] + ez[q] * L.uhi[2])) : 0.f;
    }
  }
  L.tau = lat->tau;
  L.omega = 1.0f / lat->tau;
  L.kernel = lat->ibm_kernel;
  L.le = le ? 1 : 0;
  L.le_u = lat->lees_edwards_u;
  L.le_delta = 0.f;
  L.le_pull_delta = 0.f;
  L.le_raw = 1;
  L.n = (int64_t)L.nx * L.ny * L.nz;
  L.tx = (L.nx + kTile - 1) / kTile;
  L.ty = (L.ny + kTile - 1) / kTile;
  L.tz = (L.nz + kTile - 1) / kTile;
  L.ntiles = L.tx * L.ty * L.tz;
  L.np = (int64_t)L.ntiles * kTile * kTile * kTile;
  // a K-node stencil window meets 3 tiles along a periodic axis only when the
  // last tile is at most K-2 nodes wide; otherwise 2 (1 for a 1-tile axis)
  const int sides[3] = {L.nx, L.ny, L.nz};
  int reach[3];
  for (int d = 0; d < 3; ++d) {
    const int last = sides[d] - (sides[d] - 1) / kTile * kTile;
    int per_axis = sides[d] <= kTile ? 1 : 2;
    if (L.bc[d] == HC_PERIODIC && sides[d] > kTile && last <= L.kernel - 2) per_axis = 3;
    reach[d] = std::min(per_axis, (sides[d] + kTile - 1) / kTile);
  }
  L.max_touch = reach[0] * reach[1] * reach[2];
  // with sheared images the (z tile, x tile) pairs: one z tile per image
  // when the stencil crosses the boundary (sides are multiples of 8), each
  // with the x tiles of its own displaced copy; at most 4
  if (le) L.max_touch = reach[1] * std::min(4, std::max(reach[2], 2) * reach[0]);
  c->max_cells = max_cells;
  // tile-list capacity: 4 entries per tile node (about 4x the densest
  // suspension's mean), capped by what all vertices could ever need
  c->list_cap = (int)std::max<int64_t>(
      1, std::min<int64_t>((int64_t)4 * kTile * kTile * kTile,
                           (int64_t)max_cells * c->hm.nv * L.max_touch));
  *out = c;
  return HC_OK;
}

void hc_destroy(hc_ctx* ctx) {
  if (!ctx) return;
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
}

hc_status hc_profile(hc_ctx* c, int32_t enable) {
  if (!c) return HC_ERR_ARG;
  HC_TRY(sync(c, "profile"));
  c->prof = enable != 0;
  c->ev_next = 0;
  for (auto& v : c->ev_pairs) v.clear();
  return HC_OK;
}

hc_status hc_profile_read(hc_ctx* c, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return HC_ERR_ARG;
  HC_TRY(sync(c, "profile read"));
  for (int k = 0; k < HC_NUM_KERNELS; ++k) {
    double sum = 0.0;
    for (auto& pr : c->ev_pairs[k]) {
      float ms = 0.f;
      HC_TRY(check(c, hipEventElapsedTime(&ms, c->ev_pool[pr.first], c->ev_pool[pr.second]),
                   "event time"));
      sum += ms;
    }
    total_ms[k] = sum;
    launches[k] = (int64_t)c->ev_pairs[k].size();
  }
  return HC_OK;
}

}  // extern "C"

namespace hc {
void set_global_error(const std::string& msg) { g_create_error = msg; }
}  // namespace hc

extern "C" {

const char* hc_last_error(const hc_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

hc_status hc_set_stream(hc_ctx* c, void* s) {
  if (!c) return HC_ERR_ARG;
  c->stream = reinterpret_cast<hipStream_t>(s);
  return HC_OK;
}

static hc_status densest_tile(hc_ctx* c, int32_t* out);

hc_status hc_set_list_capacity(hc_ctx* c, int32_t entries) {
  if (!c) return HC_ERR_ARG;
  if (c->ws) return fail(c, HC_ERR_STATE, "set the list capacity before binding the workspace");
  if (entries < 64 || entries > (1 << 14)) return fail(c, HC_ERR_ARG, "list capacity outside [64, 16384]");
  c->list_cap = entries;
  return HC_OK;
}

hc_status hc_densest_tile(hc_ctx* c, int32_t* entries, int32_t* capacity) {
  HC_TRY(need_ws(c));
  if (!entries) return fail(c, HC_ERR_ARG, "null pointer");
  HC_TRY(flush(c));
  HC_TRY(densest_tile(c, entries));
  if (capacity) *capacity = c->list_cap;
  return HC_OK;
}

hc_status hc_query_workspace(const hc_ctx* c, size_t* bytes) {
  if (!c || !bytes) return HC_ERR_ARG;
  Layout lay;
  plan(const_cast<hc_ctx*>(c), lay);
  *bytes = lay.total;
  return HC_OK;
}

hc_status hc_bind_workspace(hc_ctx* c, void* dev, size_t bytes) {
  if (!c || !dev) return fail(c, HC_ERR_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(dev) & 255) return fail(c, HC_ERR_ARG, "workspace not 256-aligned");
  Layout lay;
  plan(c, lay);
  if (bytes < lay.total) return fail(c, HC_ERR_OOM, "workspace smaller than hc_query_workspace");
  c->ws = static_cast<char*>(dev);
  c->ws_bytes = bytes;
  c->pops[0] = at<float>(c, c->o_pops[0]);
  c->pops[1] = at<float>(c, c->o_pops[1]);
  c->cur = 0;
  c->F = at<float>(c, c->o_F);
  c->macro = at<float4>(c, c->o_macro);
  c->partial = at<float4>(c, c->o_partial);
  const HostMesh& m = c->hm;
  Mesh& M = c->M;
  M.nv = m.nv;
  M.nt = m.nt;
  M.ne = m.ne;
  M.nh = m.nh;
  M.tri = at<int>(c, c->o_tri);
  M.edge = at<int>(c, c->o_edge);
  M.L0 = at<float>(c, c->o_L0);
  M.hinge_v = at<int>(c, c->o_hv);
  M.theta0 = at<float>(c, c->o_th0);
  M.pole = at<float>(c, c->o_pole);
  M.hinge_own = at<int>(c, c->o_own);
  M.inv_npole = 1.0f / kNPole;
  M.A0 = m.A0;
  M.V0 = m.V0;
  Cells& C = c->C;
  C.n = 0;
  C.origin = at<int>(c, c->o_origin);
  C.off = at<float>(c, c->o_off);
  C.lo = at<float>(c, c->o_lo);
  C.force = at<float>(c, c->o_force);
  C.vel = at<float>(c, c->o_vel);
  C.k = at<float>(c, c->o_k);
  C.traction = nullptr;
  C.area = at<double>(c, c->o_area);
  C.volume = at<double>(c, c->o_vol);
  Bins& B = c->B;
  B.owner = at<int>(c, c->o_owner);
  B.ntouch = at<int>(c, c->o_ntouch);
  B.scan_tmp = at<int>(c, c->o_scan);
  B.slot = at<int>(c, c->o_slot);
  B.touch_cnt = at<int>(c, c->o_tcnt);
  B.touch = at<int>(c, c->o_touch);
  B.cap = c->list_cap;
  B.bexp = 30;
  while ((int64_t)B.cap << B.bexp > ((int64_t)1 << 30)) --B.bexp;   // cap 2^bexp <= 2^30
  c->touch_ptr = at<int>(c, c->o_tptr);
  c->touch_csr = at<int>(c, c->o_csr);
  B.flags = at<int>(c, c->o_flags);
  c->cell_cnt = at<int>(c, c->o_ccnt);
  c->cell_ptr = at<int>(c, c->o_cptr);
  c->cell_tiles = at<int>(c, c->o_ctiles);
  c->cell_rank = at<int>(c, c->o_crank);
  c->cell_list = at<int>(c, c->o_clist);
  c->mask = at<unsigned char>(c, c->o_mask);
  c->cell_class = at<unsigned char>(c, c->o_cclass);
  interior_update(c);
  HC_TRY(copy_h2d(c, (void*)M.tri, m.tri.data(), m.tri.size() * 4));
  HC_TRY(copy_h2d(c, (void*)M.edge, m.edge.data(), m.edge.size() * 4));
  HC_TRY(copy_h2d(c, (void*)M.L0, m.L0.data(), m.L0.size() * 4));
  HC_TRY(copy_h2d(c, (void*)M.hinge_v, m.hinge_v.data(), m.hinge_v.size() * 4));
  HC_TRY(copy_h2d(c, (void*)M.theta0, m.theta0.data(), m.theta0.size() * 4));
  HC_TRY(copy_h2d(c, (void*)M.pole, m.pole.data(), m.pole.size() * 4));
  HC_TRY(copy_h2d(c, (void*)M.hinge_own, m.hinge_own.data(), m.hinge_own.size() * 4));
  HC_TRY(copy_h2d(c, at<float>(c, c->o_rest), c->rest.data(), c->rest.size() * 4));
  HC_TRY(check(c, launch_fill_i32(B.flags, 0, 4, c->stream), "clear flags"));
  HC_TRY(check(c, launch_fill_i32(B.touch_cnt, 0, c->L.ntiles, c->stream), "clear tile lists"));
  HC_TRY(check(c, launch_fill_i32(reinterpret_cast<int*>(c->mask), 0, c->L.np / 4, c->stream),
               "clear interior marks"));
  HC_TRY(check(c, launch_init_equilibrium(c->pops[0], 1.f, 0.f, 0.f, 0.f, c->L, c->stream), "init"));
  return sync(c, "bind");
}

// Entries of the fullest tile list for the current positions (a binning
// pass counts every (vertex, tile) pair, also past the capacity); leaves the
// lists and the overflow flag clear.
static hc_status densest_tile(hc_ctx* c, int32_t* out) {
  *out = 0;
  if (!c->have_cells) return HC_OK;
  const int NT = c->L.ntiles;
  HC_TRY(check(c, launch_fill_i32(c->B.touch_cnt, 0, NT, c->stream), "clear tile lists"));
  HC_TRY(check(c, launch_bin_vertices(c->C, c->M, c->L, c->B, c->stream), "binning"));
  std::vector<int> cnt(NT);
  HC_TRY(copy_d2h(c, cnt.data(), c->B.touch_cnt, (size_t)NT * 4));
  HC_TRY(check(c, launch_fill_i32(c->B.touch_cnt, 0, NT, c->stream), "clear tile lists"));
  HC_TRY(check(c, launch_fill_i32(c->B.flags, 0, 4, c->stream), "clear flags"));
  HC_TRY(sync(c, "densest tile"));
  for (int t = 0; t < NT; ++t) *out = std::max(*out, cnt[t]);
  return HC_OK;
}

// Shared by the two ways of setting cells: stiffnesses, traction and the
// reset of everything that belonged to the previous cells.
static hc_status cells_changed(hc_ctx* c, int32_t n, const float* k, const float* traction) {
  HC_TRY(copy_h2d(c, (void*)c->C.k, k, (size_t)n * 4 * 4));
  if (traction) {
    HC_TRY(copy_h2d(c, at<float>(c, c->o_trac), traction, (size_t)n * 3 * 4));
    c->C.traction = at<float>(c, c->o_trac);
  } else {
    c->C.traction = nullptr;
  }
  c->C.n = n;
  c->have_cells = n > 0;
  HC_TRY(check(c, launch_fill_i32(reinterpret_cast<int*>(c->C.lo), 0, (int64_t)n * c->hm.nv * 3, c->stream),
               "clear position low parts"));
  c->advect_pending = false;
  c->have_prev = false;
  c->adj_ready = false;   // a reverse sweep would recompute with the new cells
  if (c->per_cell_ratio) interior_uniform(c);   // per-cell ratios belong to the old cells
  HC_TRY(check(c, launch_fill_i32(c->B.touch_cnt, 0, c->L.ntiles, c->stream), "clear tile lists"));
  c->step = 0;
  HC_TRY(sync(c, "set_cells"));
  // a tile list that would overflow at the first step is refused here, with
  // the capacity it needs (lists only fill past their capacity when cells
  // crowd; later overflows are reported by hc_sync)
  int32_t dense = 0;
  HC_TRY(densest_tile(c, &dense));
  if (dense > c->list_cap) {
    char msg[200];
    std::snprintf(msg, sizeof(msg),
                  "the fullest tile list needs %d entries, capacity %d: create the context with "
                  "hc_set_list_capacity >= %d before binding its workspace",
                  dense, c->list_cap, dense);
    return fail(c, HC_ERR_UNSUPPORTED, msg);
  }
  return HC_OK;
}

hc_status hc_set_cells(hc_ctx* c, int32_t n, const int32_t* origin, const float* offsets,
                       const float* k, const float* traction) {
  HC_TRY(need_ws(c));
  if (n < 0 || n > c->max_cells) return fail(c, HC_ERR_ARG, "cell count outside [0, max_cells]");
  if (n > 0 && (!origin || !offsets || !k)) return fail(c, HC_ERR_ARG, "null cell array");
  const int64_t nv = c->hm.nv;
  HC_TRY(copy_h2d(c, c->C.origin, origin, (size_t)n * 3 * 4));
  HC_TRY(copy_h2d(c, c->C.off, offsets, (size_t)n * nv * 3 * 4));
  return cells_changed(c, n, k, traction);
}

hc_status hc_place_cells(hc_ctx* c, int32_t n, const float* centres, const float* rot, const float* k,
                         const float* traction) {
  HC_TRY(need_ws(c));
  if (n < 0 || n > c->max_cells) return fail(c, HC_ERR_ARG, "cell count outside [0, max_cells]");
  if (n > 0 && (!centres || !rot || !k)) return fail(c, HC_ERR_ARG, "null cell array");
  HC_TRY(check(c, launch_place_cells(c->C, c->hm.nv, at<float>(c, c->o_rest), centres, rot, n, c->stream),
               "place cells"));
  return cells_changed(c, n, k, traction);
}

hc_status hc_init_equilibrium(hc_ctx* c, float rho0, const float u0[3]) {
  HC_TRY(need_ws(c));
  const float z[3] = {0.f, 0.f, 0.f};
  const float* u = u0 ? u0 : z;
  HC_TRY(check(c, launch_init_equilibrium(c->pops[c->cur], rho0, u[0], u[1], u[2], c->L, c->stream),
               "init"));
  c->L.le_raw = 1;
  return HC_OK;
}

hc_status hc_step(hc_ctx* c, int32_t n) {
  HC_TRY(need_ws(c));
  if (n < 0) return fail(c, HC_ERR_ARG, "n_steps < 0");
  return run_steps(c, n);
}

hc_status hc_sync(hc_ctx* c) {
  HC_TRY(need_ws(c));
  HC_TRY(sync(c, "sync"));
  int flags[4];
  HC_TRY(copy_d2h(c, flags, c->B.flags, sizeof(flags)));
  HC_TRY(sync(c, "sync flags"));
  if (flags[0] || flags[1]) {
    HC_TRY(check(c, launch_fill_i32(c->B.flags, 0, 4, c->stream), "clear flags"));
    HC_TRY(sync(c, "sync"));
    if (flags[0]) return fail(c, HC_ERR_NONFINITE, "non-finite vertex position");
    if (flags[1] & 2) return fail(c, HC_ERR_DEVICE, "touch slots overflow");
    if (flags[1] & 4) return fail(c, HC_ERR_UNSUPPORTED, "a tile list exceeded its capacity");
    if (flags[1] & 8) return fail(c, HC_ERR_UNSUPPORTED, "a cell reaches more than 256 tiles");
    if (flags[1] & 16)
      return fail(c, HC_ERR_UNSUPPORTED,
                  "a cell is too wide for the interior marking (over 320 columns along x)");
    if (flags[1] & 32)
      return fail(c, HC_ERR_UNSUPPORTED, "a node column crosses a membrane more than 8 times");
    return fail(c, HC_ERR_UNSUPPORTED, "a cell covers more than 216 tiles");
  }
  return HC_OK;
}

// The idle population buffer (overwritten by the next step) stages the
// natural-order copies of the read-out and write-in calls.
hc_status hc_read_populations(hc_ctx* c, float* host, int64_t count) {
  HC_TRY(need_ws(c));
  if (!host || count != 19 * c->L.n) return fail(c, HC_ERR_ARG, "population count mismatch");
  float* tmp = c->pops[c->cur ^ 1];
  le_update(c);
  HC_TRY(check(c, launch_to_natural(c->pops[c->cur], tmp, c->L, c->stream), "to natural"));
  HC_TRY(copy_d2h(c, host, tmp, (size_t)count * 4));
  return sync(c, "read populations");
}

hc_status hc_write_populations(hc_ctx* c, const float* host, int64_t count) {
  HC_TRY(need_ws(c));
  if (!host || count != 19 * c->L.n) return fail(c, HC_ERR_ARG, "population count mismatch");
  float* tmp = c->pops[c->cur ^ 1];
  HC_TRY(copy_h2d(c, tmp, host, (size_t)count * 4));
  HC_TRY(check(c, launch_from_natural(tmp, c->pops[c->cur], c->L, c->stream), "from natural"));
  c->L.le_raw = 1;
  return sync(c, "write populations");
}

hc_status hc_set_field_output(hc_ctx* c, int32_t enable) {
  if (!c) return HC_ERR_ARG;
  c->fields = enable != 0;
  return HC_OK;
}

hc_status hc_read_macro(hc_ctx* c, float* rho, float* u, int64_t n_sites) {
  HC_TRY(need_ws(c));
  if (!c->fields) return fail(c, HC_ERR_STATE, "field output is switched off");
  if (n_sites != c->L.n) return fail(c, HC_ERR_ARG, "site count mismatch");
  float* tmp = c->pops[c->cur ^ 1];   // [4][n]: ux, uy, uz, rho
  HC_TRY(check(c, launch_field_to_natural(reinterpret_cast<const float*>(c->macro), tmp, 4, c->L,
                                          c->stream),
               "to natural"));
  if (u) HC_TRY(copy_d2h(c, u, tmp, (size_t)n_sites * 12));
  if (rho) HC_TRY(copy_d2h(c, rho, tmp + 3 * n_sites, (size_t)n_sites * 4));
  return sync(c, "read macro");
}

hc_status hc_read_force_field(hc_ctx* c, float* f, int64_t n_sites) {
  HC_TRY(need_ws(c));
  if (!c->fields) return fail(c, HC_ERR_STATE, "field output is switched off");
  if (!f || n_sites != c->L.n) return fail(c, HC_ERR_ARG, "site count mismatch");
  float* tmp = c->pops[c->cur ^ 1];
  HC_TRY(check(c, launch_field_to_natural(c->F, tmp, 3, c->L, c->stream), "to natural"));
  HC_TRY(copy_d2h(c, f, tmp, (size_t)n_sites * 12));
  return sync(c, "read force field");
}

hc_status hc_read_vertices(hc_ctx* c, int32_t* origin, float* offsets, float* force,
                           int64_t n_cells) {
  HC_TRY(need_ws(c));
  if (n_cells != c->C.n) return fail(c, HC_ERR_ARG, "cell count mismatch");
  const size_t nv = c->hm.nv;
  if (origin) HC_TRY(copy_d2h(c, origin, c->C.origin, (size_t)n_cells * 12));
  if (offsets) HC_TRY(copy_d2h(c, offsets, c->C.off, (size_t)n_cells * nv * 12));
  if (force) HC_TRY(copy_d2h(c, force, c->C.force, (size_t)n_cells * nv * 12));
  return sync(c, "read vertices");
}

hc_status hc_read_vertex_velocity(hc_ctx* c, float* vel, int64_t n_cells) {
  HC_TRY(need_ws(c));
  if (!vel || n_cells != c->C.n) return fail(c, HC_ERR_ARG, "cell count mismatch");
  HC_TRY(copy_d2h(c, vel, c->C.vel, (size_t)n_cells * c->hm.nv * 12));
  return sync(c, "read vertex velocity");
}

hc_status hc_write_vertices(hc_ctx* c, const int32_t* origin, const float* offsets,
                            int64_t n_cells) {
  HC_TRY(need_ws(c));
  if (n_cells != c->C.n || !origin || !offsets) return fail(c, HC_ERR_ARG, "cell count mismatch");
  HC_TRY(copy_h2d(c, c->C.origin, origin, (size_t)n_cells * 12));
  HC_TRY(copy_h2d(c, c->C.off, offsets, (size_t)n_cells * c->hm.nv * 12));
  HC_TRY(check(c, launch_fill_i32(reinterpret_cast<int*>(c->C.lo), 0, n_cells * c->hm.nv * 3, c->stream),
               "clear position low parts"));
  c->have_prev = false;   // new positions: an Adams-Bashforth run restarts with Euler
  return sync(c, "write vertices");
}

hc_status hc_compute_forces(hc_ctx* c, double* area, double* volume, int64_t n_cells) {
  HC_TRY(need_ws(c));
  if (n_cells != c->C.n) return fail(c, HC_ERR_ARG, "cell count mismatch");
  HC_TRY(check(c, launch_membrane(c->C, c->M, c->stream), "membrane"));
  if (area) HC_TRY(copy_d2h(c, area, c->C.area, (size_t)n_cells * 8));
  if (volume) HC_TRY(copy_d2h(c, volume, c->C.volume, (size_t)n_cells * 8));
  return sync(c, "compute forces");
}

hc_status hc_num_tiles(const hc_ctx* c, int32_t* n) {
  if (!c || !n) return HC_ERR_ARG;
  *n = c->L.ntiles;
  return HC_OK;
}

hc_status hc_read_bins(hc_ctx* c, int32_t* owner, int32_t* touch_ptr, int32_t* touch,
                       int64_t cap_touch, int32_t* cell_ptr, int32_t* cells, int64_t cap_cells) {
  HC_TRY(need_ws(c));
  if (!touch_ptr || !cell_ptr) return fail(c, HC_ERR_ARG, "null pointer array");
  const int NT = c->L.ntiles;
  HC_TRY(check(c, launch_fill_i32(c->B.touch_cnt, 0, NT, c->stream), "clear tile lists"));
  HC_TRY(check(c, launch_bin_vertices(c->C, c->M, c->L, c->B, c->stream), "binning"));
  HC_TRY(check(c, launch_touch_csr(c->L, c->B, c->cell_cnt, c->touch_ptr, c->touch_csr, c->stream),
               "tile lists"));
  // the lists are copied out: leave zero counts for the next step's binning
  HC_TRY(check(c, launch_fill_i32(c->B.touch_cnt, 0, NT, c->stream), "clear tile lists"));
  HC_TRY(check(c, launch_sort_segments(c->touch_ptr, c->touch_csr, c->B.slot, NT, c->stream),
               "sort"));
  HC_TRY(check(c, launch_bin_cells(c->C, c->M, c->L, c->cell_cnt, c->cell_ptr, c->cell_rank,
                                   c->cell_tiles, c->cell_list,
                                   (int64_t)c->max_cells * kMaxCellTiles, kMaxCellTiles,
                                   c->B.flags, c->B.scan_tmp, c->stream),
               "cell binning"));
  HC_TRY(check(c, launch_sort_segments(c->cell_ptr, c->cell_list, c->cell_rank, NT, c->stream),
               "sort"));
  HC_TRY(copy_d2h(c, touch_ptr, c->touch_ptr, (size_t)(NT + 1) * 4));
  HC_TRY(copy_d2h(c, cell_ptr, c->cell_ptr, (size_t)(NT + 1) * 4));
  HC_TRY(sync(c, "read bins"));
  int flags[4];
  HC_TRY(copy_d2h(c, flags, c->B.flags, sizeof(flags)));
  HC_TRY(sync(c, "read bins"));
  if (flags[1]) return fail(c, HC_ERR_UNSUPPORTED, "tile-list or cell-cover capacity exceeded");
  if (touch_ptr[NT] > cap_touch || cell_ptr[NT] > cap_cells)
    return fail(c, HC_ERR_ARG, "bin capacity too small");
  if (owner) HC_TRY(copy_d2h(c, owner, c->B.owner, (size_t)c->C.n * c->hm.nv * 4));
  if (touch) HC_TRY(copy_d2h(c, touch, c->touch_csr, (size_t)touch_ptr[NT] * 4));
  if (cells) HC_TRY(copy_d2h(c, cells, c->cell_list, (size_t)cell_ptr[NT] * 4));
  HC_TRY(sync(c, "read bins"));
  if (touch)
    for (int64_t i = 0; i < touch_ptr[NT]; ++i) touch[i] >>= 5;  // drop the slot index
  return HC_OK;
}

// Checkpoint layout: header {step, cells, have_prev, force_every, scheme,
// raw state flag} (int64 x 2, int32 x 4), then the stored populations, origins, offsets,
// vertex velocities and held vertex forces.
constexpr size_t kCkHeader = 32;

hc_status hc_checkpoint_size(const hc_ctx* c, size_t* bytes) {
  if (!c || !bytes) return HC_ERR_ARG;
  const size_t X = (size_t)c->C.n * c->hm.nv * 12;
  *bytes = kCkHeader + (size_t)19 * c->L.np * 4 + (size_t)c->C.n * 12 + 4 * X;
  return HC_OK;
}

hc_status hc_checkpoint_save(hc_ctx* c, void* host, size_t bytes) {
  HC_TRY(need_ws(c));
  size_t need;
  hc_checkpoint_size(c, &need);
  if (!host || bytes < need) return fail(c, HC_ERR_ARG, "checkpoint buffer too small");
  HC_TRY(flush(c));
  char* p = static_cast<char*>(host);
  const int64_t h64[2] = {c->step, c->C.n};
  const int32_t h32[4] = {c->have_prev ? 1 : 0, c->force_every, c->scheme, c->L.le_raw};
  std::memcpy(p, h64, 16);
  std::memcpy(p + 16, h32, 16);
  p += kCkHeader;
  const size_t X = (size_t)c->C.n * c->hm.nv * 12;
  HC_TRY(copy_d2h(c, p, c->pops[c->cur], (size_t)19 * c->L.np * 4));
  p += (size_t)19 * c->L.np * 4;
  HC_TRY(copy_d2h(c, p, c->C.origin, (size_t)c->C.n * 12));
  p += (size_t)c->C.n * 12;
  HC_TRY(copy_d2h(c, p, c->C.off, X));
  p += X;
  HC_TRY(copy_d2h(c, p, c->C.lo, X));
  p += X;
  HC_TRY(copy_d2h(c, p, c->C.vel, X));
  p += X;
  HC_TRY(copy_d2h(c, p, c->C.force, X));
  return sync(c, "checkpoint save");
}

hc_status hc_checkpoint_restore(hc_ctx* c, const void* host, size_t bytes) {
  HC_TRY(need_ws(c));
  size_t need;
  hc_checkpoint_size(c, &need);
  if (!host || bytes < need) return fail(c, HC_ERR_ARG, "checkpoint buffer too small");
  const char* p = static_cast<const char*>(host);
  int64_t h64[2];
  int32_t h32[4];
  std::memcpy(h64, p, 16);
  std::memcpy(h32, p + 16, 16);
  if (h64[1] != c->C.n) return fail(c, HC_ERR_ARG, "checkpoint cell count differs");
  if (h32[1] < 1 || (h32[2] != HC_EULER && h32[2] != HC_AB2))
    return fail(c, HC_ERR_ARG, "checkpoint header is not valid");
  p += kCkHeader;
  const size_t X = (size_t)c->C.n * c->hm.nv * 12;
  HC_TRY(copy_h2d(c, c->pops[c->cur], p, (size_t)19 * c->L.np * 4));
  p += (size_t)19 * c->L.np * 4;
  HC_TRY(copy_h2d(c, c->C.origin, p, (size_t)c->C.n * 12));
  p += (size_t)c->C.n * 12;
  HC_TRY(copy_h2d(c, c->C.off, p, X));
  p += X;
  HC_TRY(copy_h2d(c, c->C.lo, p, X));
  p += X;
  HC_TRY(copy_h2d(c, c->C.vel, p, X));
  p += X;
  HC_TRY(copy_h2d(c, c->C.force, p, X));
  c->step = h64[0];
  c->adj_ready = false;   // a reverse sweep belongs to the state its forward ran from
  c->have_prev = h32[0] != 0;
  c->force_every = h32[1];
  c->scheme = h32[2];
  c->L.le_raw = h32[3];
  c->advect_pending = false;
  return sync(c, "checkpoint restore");
}

hc_status hc_set_integration(hc_ctx* c, int32_t force_every, int32_t scheme) {
  if (!c) return HC_ERR_ARG;
  if (force_every < 1) return fail(c, HC_ERR_ARG, "force_every must be >= 1");
  if (scheme != HC_EULER && scheme != HC_AB2) return fail(c, HC_ERR_ARG, "scheme must be HC_EULER or HC_AB2");
  HC_TRY(flush(c));
  if (force_every != c->force_every || scheme != c->scheme) c->adj_ready = false;
  c->force_every = force_every;
  c->scheme = scheme;
  return HC_OK;
}

hc_status hc_set_interior_viscosity(hc_ctx* c, float ratio) {
  if (!c) return HC_ERR_ARG;
  if (!std::isfinite(ratio) || !(ratio > 0.f)) return fail(c, HC_ERR_ARG, "ratio must be positive");
  if (c->adj_ready && (ratio != c->uniform_ratio || c->per_cell_ratio))
    return fail(c, HC_ERR_STATE, "the interior viscosity cannot change between hc_adj_forward and "
                                 "hc_adj_backward (bind the adjoint workspace again)");
  c->uniform_ratio = ratio;
  interior_uniform(c);
  return HC_OK;
}

hc_status hc_set_cell_viscosity(hc_ctx* c, const float* ratio, int64_t n_cells) {
  HC_TRY(need_ws(c));
  if (!ratio || n_cells != c->C.n) return fail(c, HC_ERR_ARG, "one ratio per current cell");
  std::vector<float> cls;
  for (int64_t i = 0; i < n_cells; ++i) {
    if (!std::isfinite(ratio[i]) || !(ratio[i] > 0.f)) return fail(c, HC_ERR_ARG, "ratios must be positive");
    cls.push_back(ratio[i]);
  }
  std::sort(cls.begin(), cls.end());
  cls.erase(std::unique(cls.begin(), cls.end()), cls.end());
  if ((int)cls.size() > kVisClasses)
    return fail(c, HC_ERR_UNSUPPORTED, "more than 8 distinct interior viscosity ratios");
  const bool on = cls.size() > 1 || (!cls.empty() && cls[0] != 1.f);
  if (c->adj_ready)
    return fail(c, HC_ERR_STATE, "the interior viscosity cannot change between hc_adj_forward and "
                                 "hc_adj_backward (bind the adjoint workspace again)");
  std::vector<uint8_t> k((size_t)n_cells);
  for (int64_t i = 0; i < n_cells; ++i)
    k[i] = (uint8_t)(std::lower_bound(cls.begin(), cls.end(), ratio[i]) - cls.begin());
  HC_TRY(copy_h2d(c, c->cell_class, k.data(), (size_t)n_cells));
  HC_TRY(sync(c, "set cell viscosity"));
  c->per_cell_ratio = true;
  c->n_vclass = std::max<int>(1, (int)cls.size());
  for (int i = 0; i < kVisClasses; ++i) c->class_ratio[i] = i < (int)cls.size() ? cls[i] : 1.f;
  interior_update(c);
  return HC_OK;
}

hc_status hc_read_interior(hc_ctx* c, uint8_t* host, int64_t n_sites) {
  HC_TRY(need_ws(c));
  if (!host || n_sites != c->L.n) return fail(c, HC_ERR_ARG, "site count mismatch");
  HC_TRY(flush(c));
  le_update(c);   // the image shift of the step about to run
  Cells C = c->C;
  C.n = c->have_cells ? c->C.n : 0;
  const Lattice& L = c->L;
  HC_TRY(check(c, mark_interior(c, C), "interior marking"));
  std::vector<uint8_t> m((size_t)L.np);
  HC_TRY(copy_d2h(c, m.data(), c->mask, (size_t)L.np));
  HC_TRY(check(c, launch_fill_i32(reinterpret_cast<int*>(c->mask), 0, L.np / 4, c->stream),
               "clear interior marks"));
  HC_TRY(hc_sync(c));
  for (int z = 0; z < L.nz; ++z)
    for (int y = 0; y < L.ny; ++y)
      for (int x = 0; x < L.nx; ++x)
        host[((int64_t)z * L.ny + y) * L.nx + x] = m[(size_t)site_of(L, x, y, z)];
  return HC_OK;
}

hc_status hc_device_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15) ||
      (bytes & 15))
    return fail(nullptr, HC_ERR_ARG, "copy: null or misaligned pointer / size");
  hipError_t e = launch_copy(dst, src, bytes, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(nullptr, HC_ERR_DEVICE, hipGetErrorString(e));
  return HC_OK;
}

hc_status hc_set_params(hc_ctx* c, const float* k, float tau) {
  HC_TRY(need_ws(c));
  if (!(tau > 0.5f)) return fail(c, HC_ERR_ARG, "tau must exceed 1/2");
  if (k) HC_TRY(copy_h2d(c, (void*)c->C.k, k, (size_t)c->C.n * 16));
  c->adj_ready = false;   // the forward's checkpoints were taken under the old parameters
  c->L.tau = tau;
  c->L.omega = 1.0f / tau;
  interior_update(c);
  return sync(c, "set params");
}

hc_status hc_adj_query_workspace(const hc_ctx* c, int32_t n_steps, int32_t ckpt_every, size_t* bytes) {
  if (!c || !bytes || n_steps < 1 || ckpt_every < 1) return HC_ERR_ARG;
  *bytes = adj_plan(c, n_steps, std::min(ckpt_every, n_steps)).total;
  return HC_OK;
}

hc_status hc_adj_bind_workspace(hc_ctx* c, void* dev, size_t bytes, int32_t n_steps,
                                int32_t ckpt_every) {
  HC_TRY(need_ws(c));
  if (!dev || n_steps < 1 || ckpt_every < 1) return fail(c, HC_ERR_ARG, "adjoint: bad arguments");
  if (reinterpret_cast<uintptr_t>(dev) & 255) return fail(c, HC_ERR_ARG, "workspace not 256-aligned");
  if (c->L.kernel != HC_PHI4)
    return fail(c, HC_ERR_UNSUPPORTED, "adjoint needs the differentiable 4-point kernel");
  if (c->L.le) return fail(c, HC_ERR_UNSUPPORTED, "adjoint does not cover Lees-Edwards images");
  if (c->force_every != 1 || c->scheme != HC_EULER)
    return fail(c, HC_ERR_UNSUPPORTED, "adjoint differentiates the Euler step with forces every step");
  const int ck = std::min(ckpt_every, n_steps);
  const AdjPlan p = adj_plan(c, n_steps, ck);
  if (bytes < p.total) return fail(c, HC_ERR_OOM, "adjoint workspace too small");
  char* w = static_cast<char*>(dev);
  c->adj_ws = w;
  c->adj_n = n_steps;
  c->adj_ck = ck;
  c->adj_nseg = (n_steps + ck - 1) / ck;
  c->ck_pops = reinterpret_cast<float*>(w + p.ck_pops);
  c->ck_off = reinterpret_cast<float*>(w + p.ck_off);
  c->ck_lo = reinterpret_cast<float*>(w + p.ck_lo);
  c->sg_lo = reinterpret_cast<float*>(w + p.sg_lo);
  c->sg_pops = reinterpret_cast<float*>(w + p.sg_pops);
  c->sg_off = reinterpret_cast<float*>(w + p.sg_off);
  c->sg_F = reinterpret_cast<float*>(w + p.sg_F);
  c->sg_macro = reinterpret_cast<float4*>(w + p.sg_macro);
  c->sg_Fv = reinterpret_cast<float*>(w + p.sg_Fv);
  c->lam_f[0] = reinterpret_cast<float*>(w + p.lf0);
  c->lam_f[1] = reinterpret_cast<float*>(w + p.lf1);
  c->lam_X[0] = reinterpret_cast<float*>(w + p.lx0);
  c->lam_X[1] = reinterpret_cast<float*>(w + p.lx1);
  c->lam_Fv = reinterpret_cast<float*>(w + p.lfv);
  c->lam_u = reinterpret_cast<float*>(w + p.lu);
  c->lam_F = reinterpret_cast<float*>(w + p.lF);
  c->vel_scratch = reinterpret_cast<float*>(w + p.vel);
  c->dom_part = reinterpret_cast<double*>(w + p.dom);
  c->dom_in_part = reinterpret_cast<double*>(w + p.dom_in);
  c->dk = reinterpret_cast<double*>(w + p.dk);
  c->loss = reinterpret_cast<double*>(w + p.loss);
  c->targets = reinterpret_cast<double*>(w + p.tg);
  c->scal = reinterpret_cast<double*>(w + p.scal);
  c->adj_ready = false;
  return HC_OK;
}

hc_status hc_adj_forward(hc_ctx* c, const double* targets, double* loss) {
  HC_TRY(need_ws(c));
  if (!c->adj_ws) return fail(c, HC_ERR_STATE, "no adjoint workspace bound");
  if (!c->have_cells || !targets || !loss) return fail(c, HC_ERR_STATE, "adjoint: no cells or targets");
  if (c->force_every != 1 || c->scheme != HC_EULER)
    return fail(c, HC_ERR_UNSUPPORTED, "adjoint differentiates the Euler step with forces every step");
  const int64_t P = 19 * c->L.np, X = (int64_t)c->C.n * c->hm.nv * 3;
  HC_TRY(copy_h2d(c, c->targets, targets, (size_t)c->C.n * 16));
  // no re-centring while recording; the force and (u, rho) fields (when
  // field output is on) only at the last step: the loss needs neither, and
  // the reverse sweep's recomputation writes its own
  c->recentre = false;
  struct Restore {
    hc_ctx* c;
    bool fields;
    ~Restore() {
      c->recentre = true;
      c->fields = fields;
    }
  } restore{c, c->fields};
  for (int s = 0; s < c->adj_n; ++s) {
    c->fields = restore.fields && s + 1 == c->adj_n;
    if (s % c->adj_ck == 0) {
      const int k = s / c->adj_ck;
      HC_TRY(copy_d2d(c, c->ck_pops + k * P, c->pops[c->cur], (size_t)P * 4));
      HC_TRY(copy_d2d(c, c->ck_off + k * X, c->C.off, (size_t)X * 4));
      HC_TRY(copy_d2d(c, c->ck_lo + k * X, c->C.lo, (size_t)X * 4));
    }
    HC_TRY(one_step(c));
    if ((s + 1) % c->adj_ck == 0 || s + 1 == c->adj_n) HC_TRY(flush(c));
  }
  HC_TRY(check(c, launch_loss_seed(c->C, c->M, c->targets, c->loss, c->lam_X[0], c->stream), "loss"));
  HC_TRY(copy_d2h(c, loss, c->loss, (size_t)c->C.n * 8));
  HC_TRY(sync(c, "adjoint forward"));
  c->adj_ready = true;
  return HC_OK;
}

hc_status hc_adj_backward(hc_ctx* c, double* grad) {
  HC_TRY(need_ws(c));
  if (!c->adj_ready || !grad) return fail(c, HC_ERR_STATE, "hc_adj_forward must run first");
  const int64_t N = c->L.np, P = 19 * N, X = (int64_t)c->C.n * c->hm.nv * 3;
  const int nblk = (int)((N + 255) / 256);
  HC_TRY(check(c, launch_fill_i32(reinterpret_cast<int*>(c->lam_f[0]), 0, P, c->stream), "zero"));   // +0.0f
  HC_TRY(check(c, launch_zero_f64(c->dk, (int64_t)c->C.n * 4, c->stream), "zero"));
  HC_TRY(check(c, launch_zero_f64(c->dom_part, nblk, c->stream), "zero"));
  HC_TRY(check(c, launch_zero_f64(c->dom_in_part, (int64_t)kVisClasses * nblk, c->stream), "zero"));
  int a = 0;   // lam_f[a], lam_X[a] hold the cotangents of the later state
  for (int seg = c->adj_nseg - 1; seg >= 0; --seg) {
    const int s0 = seg * c->adj_ck, len = std::min(c->adj_ck, c->adj_n - s0);
    HC_TRY(copy_d2d(c, c->sg_pops, c->ck_pops + seg * P, (size_t)P * 4));
    HC_TRY(copy_d2d(c, c->sg_off, c->ck_off + seg * X, (size_t)X * 4));
    HC_TRY(copy_d2d(c, c->sg_lo, c->ck_lo + seg * X, (size_t)X * 4));
    for (int i = 0; i < len; ++i) HC_TRY(adj_forward_into(c, i));
    for (int i = len - 1; i >= 0; --i) {
      HC_TRY(adj_reverse_step(c, i, a));
      a ^= 1;
    }
  }
  HC_TRY(check(c, launch_sum_parts(c->dom_part, nblk, c->scal, c->stream), "sum"));
  for (int k = 0; k < kVisClasses; ++k)
    HC_TRY(check(c, launch_sum_parts(c->dom_in_part + (int64_t)k * nblk, nblk, c->scal + 1 + k, c->stream),
                 "sum"));
  std::vector<double> dk((size_t)c->C.n * 4);
  double dom[1 + kVisClasses] = {};
  HC_TRY(copy_d2h(c, dk.data(), c->dk, dk.size() * 8));
  HC_TRY(copy_d2h(c, dom, c->scal, sizeof(dom)));
  HC_TRY(sync(c, "adjoint backward"));
  // tau = 1/omega outside the cells; inside a cell of class k,
  // tau_k = 1/2 + ratio_k (tau - 1/2)
  const double om = c->L.omega;
  double dtau = -om * om * dom[0];
  for (int k = 0; k < c->n_vclass; ++k) {
    const double ok = c->L.omega_in[k];
    dtau -= (double)c->class_ratio[k] * ok * ok * dom[1 + k];
  }
  for (int i = 0; i < c->C.n; ++i) {
    for (int j = 0; j < 4; ++j) grad[5 * i + j] = dk[4 * i + j];
    grad[5 * i + 4] = dtau;
  }
  return HC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The adjoint over several boxes of one shape: every per-step kernel runs as
// one batched launch over all boxes (work-group (x, y) = work-group x of box
// y), on the first context's stream, so the boxes share the chip instead of
// taking turns.  The arithmetic per box is that of hc_adj_forward /
// hc_adj_backward, so each box's loss and gradient equal its single-box ones.

namespace {

// Device copy of per-box argument records, laid out [record set][box].
template <class T>
struct DevTable {
  T* dev = nullptr;
  std::vector<T> host;
  int n = 0;   // boxes per record set
  ~DevTable() {
    if (dev) (void)hipFree(dev);
  }
  T& at(int set, int box) { return host[(size_t)set * n + box]; }
  const T* set(int k) const { return dev + (size_t)k * n; }
  const T& first(int k) const { return host[(size_t)k * n]; }
  hipError_t upload(hipStream_t s) {
    hipError_t e = hipMalloc(&dev, host.size() * sizeof(T));
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(dev, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);   // the host records may go once the copy is done
  }
};

hc_status multi_check(hc_ctx* const* cs, int n, bool need_ready) {
  if (!cs || n < 1) return HC_ERR_ARG;
  for (int b = 0; b < n; ++b) {
    hc_ctx* c = cs[b];
    if (!c || !c->ws) return fail(cs[0], HC_ERR_STATE, "batched adjoint: a box has no workspace bound");
    if (!c->adj_ws) return fail(cs[0], HC_ERR_STATE, "no adjoint workspace bound");
    if (!c->have_cells) return fail(cs[0], HC_ERR_STATE, "adjoint: no cells");
    if (c->force_every != 1 || c->scheme != HC_EULER || c->L.le || interior_on(c) || c->L.kernel != HC_PHI4)
      return fail(cs[0], HC_ERR_UNSUPPORTED,
                  "batched adjoint: Euler steps with forces every step, 4-point kernel, no sheared images, "
                  "no interior viscosity");
    if (need_ready && !c->adj_ready) return fail(cs[0], HC_ERR_STATE, "hc_adj_multi_forward must run first");
    if (!need_ready && c->advect_pending) return fail(cs[0], HC_ERR_STATE, "a vertex move is pending");
    const hc_ctx* a = cs[0];
    if (c->L.nx != a->L.nx || c->L.ny != a->L.ny || c->L.nz != a->L.nz || c->L.wall_axis != a->L.wall_axis ||
        c->L.bc[0] != a->L.bc[0] || c->L.bc[1] != a->L.bc[1] || c->L.bc[2] != a->L.bc[2] ||
        c->hm.nv != a->hm.nv || c->C.n != a->C.n || c->adj_n != a->adj_n || c->adj_ck != a->adj_ck ||
        c->L.max_touch != a->L.max_touch || c->B.cap != a->B.cap)
      return fail(cs[0], HC_ERR_ARG, "batched adjoint: boxes differ in shape, boundaries, cells or run length");
  }
  for (int b = 0; b < n; ++b)
    for (int e = b + 1; e < n; ++e)
      if (cs[b] == cs[e]) return fail(cs[0], HC_ERR_ARG, "batched adjoint: a context appears twice");
  for (int b = 0; b < n; ++b) HC_TRY(sync(cs[b], "batched adjoint"));   // earlier work on every stream
  return HC_OK;
}

hc_status mcheck(hc_ctx* c, hipError_t e, const char* what) { return check(c, e, what); }

hc_status mcopy(hc_ctx* c, void* dst, const void* src, size_t bytes, hipMemcpyKind k, hipStream_t s) {
  if (!bytes) return HC_OK;
  return check(c, hipMemcpyAsync(dst, src, bytes, k, s), "batched adjoint copy");
}

}  // namespace

extern "C" {

hc_status hc_adj_multi_forward(hc_ctx* const* cs, int32_t n, const double* targets, double* loss) {
  HC_TRY(multi_check(cs, n, false));
  if (!targets || !loss) return fail(cs[0], HC_ERR_ARG, "null targets or loss");
  hc_ctx* c0 = cs[0];
  hipStream_t s = c0->stream;
  const int C = c0->C.n, ns = c0->adj_n, ck = c0->adj_ck;
  const int64_t P = 19 * c0->L.np, X = (int64_t)C * c0->hm.nv * 3;
  // record sets: [parity q][advect] for the per-cell kernel; [fields][parity
  // q] for the lattice pass, which writes the force and (u, rho) fields (when
  // the context has field output on) at the last step only: the loss needs
  // neither, and the reverse sweep's recomputation writes its own
  DevTable<CellStepArgs> cell;
  DevTable<TileStepArgs> tile;
  cell.n = tile.n = n;
  cell.host.resize((size_t)4 * n);
  tile.host.resize((size_t)4 * n);
  for (int b = 0; b < n; ++b) {
    hc_ctx* c = cs[b];
    for (int q = 0; q < 2; ++q) {
      const int in = c->cur ^ q;
      for (int adv = 0; adv < 2; ++adv)
        cell.at(2 * q + adv, b) = CellStepArgs{c->C, c->M, c->L, c->B, c->partial, c->B.flags, adv, nullptr, 1, 0, 0};
      for (int fl = 0; fl < 2; ++fl)
        tile.at(2 * fl + q, b) = TileStepArgs{c->C, c->M, c->L, c->B, c->pops[in], c->pops[in ^ 1], c->F, c->macro,
                                              c->partial, fl && c->fields ? 1 : 0, nullptr};
    }
    HC_TRY(mcopy(c0, c->targets, targets + (size_t)b * C * 2, (size_t)C * 16, hipMemcpyHostToDevice, s));
  }
  // checkpoint k (at step k ck): every box's populations, offsets and low
  // parts, copied in one launch
  DevTable<CopyRec> save;
  const int nck = (ns + ck - 1) / ck;
  save.n = 3 * n;
  save.host.resize((size_t)nck * 3 * n);
  for (int k = 0; k < nck; ++k)
    for (int b = 0; b < n; ++b) {
      hc_ctx* c = cs[b];
      const int q = (k * ck) & 1;
      save.at(k, 3 * b) = CopyRec{c->ck_pops + k * P, c->pops[c->cur ^ q], (int64_t)P * 4};
      save.at(k, 3 * b + 1) = CopyRec{c->ck_off + k * X, c->C.off, (int64_t)X * 4};
      save.at(k, 3 * b + 2) = CopyRec{c->ck_lo + k * X, c->C.lo, (int64_t)X * 4};
    }
  HC_TRY(mcheck(c0, cell.upload(s), "batched adjoint tables"));
  HC_TRY(mcheck(c0, tile.upload(s), "batched adjoint tables"));
  HC_TRY(mcheck(c0, save.upload(s), "batched adjoint tables"));
  for (int st = 0; st < ns; ++st) {
    const int q = st & 1;
    if (st % ck == 0)
      HC_TRY(mcheck(c0, launch_copy_many(save.set(st / ck), 3 * n, (int64_t)P * 4, s), "checkpoint"));
    const int adv = st % ck != 0 ? 1 : 0;   // each segment ends with its move applied
    HC_TRY(mcheck(c0, launch_cell_step_multi(cell.first(2 * q + adv), cell.set(2 * q + adv), n, s), "cell step"));
    const int tset = (st + 1 == ns ? 2 : 0) + q;
    HC_TRY(mcheck(c0, launch_tile_step_multi(tile.first(tset), tile.set(tset), n, s), "lattice pass"));
    if ((st + 1) % ck == 0 || st + 1 == ns)
      for (int b = 0; b < n; ++b) {
        hc_ctx* c = cs[b];
        HC_TRY(mcheck(c0, launch_advect(c->C, c->M, c->L, c->B, c->partial, c->B.flags, false, s), "advect"));
      }
  }
  for (int b = 0; b < n; ++b) {
    hc_ctx* c = cs[b];
    HC_TRY(mcheck(c0, launch_loss_seed(c->C, c->M, c->targets, c->loss, c->lam_X[0], s), "loss"));
    HC_TRY(mcopy(c0, loss + (size_t)b * C, c->loss, (size_t)C * 8, hipMemcpyDeviceToHost, s));
  }
  HC_TRY(mcheck(c0, hipStreamSynchronize(s), "batched adjoint forward"));
  for (int b = 0; b < n; ++b) {
    hc_ctx* c = cs[b];
    c->cur ^= ns & 1;
    c->step += ns;
    c->advect_pending = false;
    c->have_prev = true;
    c->L.le_raw = 0;
    c->adj_ready = true;
  }
  return HC_OK;
}

hc_status hc_adj_multi_backward(hc_ctx* const* cs, int32_t n, double* grad) {
  HC_TRY(multi_check(cs, n, true));
  if (!grad) return fail(cs[0], HC_ERR_ARG, "null gradient");
  hc_ctx* c0 = cs[0];
  hipStream_t s = c0->stream;
  const int C = c0->C.n, ck = c0->adj_ck;
  const int64_t N = c0->L.np, P = 19 * N, X = (int64_t)C * c0->hm.nv * 3;
  const int nblk = (int)((N + 255) / 256);
  DevTable<CellStepArgs> cell;
  DevTable<TileStepArgs> tile;
  DevTable<BinArgs> bins;
  DevTable<SpreadArgs> spread;
  DevTable<AdjCollideArgs> coll;
  DevTable<AdjVertexArgs> vert;
  DevTable<AdjMembraneArgs> memb;
  cell.n = tile.n = bins.n = spread.n = coll.n = vert.n = memb.n = n;
  cell.host.resize((size_t)ck * n);
  tile.host.resize((size_t)ck * n);
  bins.host.resize((size_t)ck * n);
  spread.host.resize((size_t)2 * ck * n);
  coll.host.resize((size_t)2 * ck * n);
  vert.host.resize((size_t)2 * ck * n);
  memb.host.resize((size_t)2 * ck * n);
  for (int b = 0; b < n; ++b) {
    hc_ctx* c = cs[b];
    for (int i = 0; i < ck; ++i) {
      Cells Ci = c->C;
      Ci.off = c->sg_off + i * X;
      Ci.lo = c->sg_lo;
      Ci.force = c->sg_Fv + i * X;
      Ci.vel = c->vel_scratch;
      const float* prev = i > 0 ? c->sg_off + (i - 1) * X : nullptr;
      cell.at(i, b) = CellStepArgs{Ci, c->M, c->L, c->B, c->partial, c->B.flags, i > 0 ? 1 : 0, prev, 1, 0, 0};
      tile.at(i, b) = TileStepArgs{Ci, c->M, c->L, c->B, c->sg_pops + i * P, c->sg_pops + (i + 1) * P,
                                   c->sg_F + i * 3 * N, c->sg_macro + i * N, c->partial, 1, nullptr};
      bins.at(i, b) = BinArgs{Ci, c->M, c->L, c->B};
      for (int a = 0; a < 2; ++a) {
        const int k = 2 * i + a;
        spread.at(k, b) = SpreadArgs{Ci, c->M, c->L, c->B, c->lam_X[a], 0.f, c->lam_u};
        coll.at(k, b) = AdjCollideArgs{c->lam_f[a], c->lam_f[a ^ 1], c->sg_pops + i * P, c->sg_F + i * 3 * N,
                                       c->lam_u, c->lam_F, c->dom_part, nullptr, c->dom_in_part, c->L};
        vert.at(k, b) = AdjVertexArgs{Ci, c->M, c->L, c->lam_X[a], c->sg_macro + i * N, c->lam_F, c->lam_Fv,
                                      c->lam_X[a ^ 1]};
        memb.at(k, b) = AdjMembraneArgs{Ci, c->M, c->lam_Fv, c->lam_X[a ^ 1], c->dk};
      }
    }
    HC_TRY(mcheck(c0, launch_fill_i32(reinterpret_cast<int*>(c->lam_f[0]), 0, P, s), "zero"));   // +0.0f
    HC_TRY(mcheck(c0, launch_zero_f64(c->dk, (int64_t)C * 4, s), "zero"));
    HC_TRY(mcheck(c0, launch_zero_f64(c->dom_part, nblk, s), "zero"));
    HC_TRY(mcheck(c0, launch_zero_f64(c->dom_in_part, (int64_t)kVisClasses * nblk, s), "zero"));
  }
  HC_TRY(mcheck(c0, cell.upload(s), "batched adjoint tables"));
  HC_TRY(mcheck(c0, tile.upload(s), "batched adjoint tables"));
  HC_TRY(mcheck(c0, bins.upload(s), "batched adjoint tables"));
  HC_TRY(mcheck(c0, spread.upload(s), "batched adjoint tables"));
  HC_TRY(mcheck(c0, coll.upload(s), "batched adjoint tables"));
  HC_TRY(mcheck(c0, vert.upload(s), "batched adjoint tables"));
  HC_TRY(mcheck(c0, memb.upload(s), "batched adjoint tables"));
  // segment seg starts from checkpoint seg: every box's copies in one launch
  DevTable<CopyRec> restore;
  restore.n = 3 * n;
  restore.host.resize((size_t)c0->adj_nseg * 3 * n);
  for (int seg = 0; seg < c0->adj_nseg; ++seg)
    for (int b = 0; b < n; ++b) {
      hc_ctx* c = cs[b];
      restore.at(seg, 3 * b) = CopyRec{c->sg_pops, c->ck_pops + seg * P, (int64_t)P * 4};
      restore.at(seg, 3 * b + 1) = CopyRec{c->sg_off, c->ck_off + seg * X, (int64_t)X * 4};
      restore.at(seg, 3 * b + 2) = CopyRec{c->sg_lo, c->ck_lo + seg * X, (int64_t)X * 4};
    }
  HC_TRY(mcheck(c0, restore.upload(s), "batched adjoint tables"));
  int a = 0;   // lam_f[a], lam_X[a] hold the cotangents of the later state
  for (int seg = c0->adj_nseg - 1; seg >= 0; --seg) {
    const int len = std::min(ck, c0->adj_n - seg * ck);
    HC_TRY(mcheck(c0, launch_copy_many(restore.set(seg), 3 * n, (int64_t)P * 4, s), "checkpoint restore"));
    for (int i = 0; i < len; ++i) {
      HC_TRY(mcheck(c0, launch_cell_step_multi(cell.first(i), cell.set(i), n, s), "cell step"));
      HC_TRY(mcheck(c0, launch_tile_step_multi(tile.first(i), tile.set(i), n, s), "lattice pass"));
    }
    for (int i = len - 1; i >= 0; --i) {
      const int k = 2 * i + a;
      HC_TRY(mcheck(c0, launch_bin_vertices_multi(bins.first(i), bins.set(i), n, s), "binning"));
      HC_TRY(mcheck(c0, launch_spread_vec_multi(spread.first(k), spread.set(k), n, s), "spread"));
      HC_TRY(mcheck(c0, launch_adj_collide_multi(coll.first(k), coll.set(k), n, s), "adjoint collide"));
      HC_TRY(mcheck(c0, launch_adj_vertex_multi(vert.first(k), vert.set(k), n, s), "adjoint ibm"));
      HC_TRY(mcheck(c0, launch_adj_membrane_multi(memb.first(k), memb.set(k), n, s), "adjoint membrane"));
      a ^= 1;
    }
  }
  std::vector<double> dk((size_t)n * C * 4), dom((size_t)n * (1 + kVisClasses));
  for (int b = 0; b < n; ++b) {
    hc_ctx* c = cs[b];
    HC_TRY(mcheck(c0, launch_sum_parts(c->dom_part, nblk, c->scal, s), "sum"));
    HC_TRY(mcopy(c0, dk.data() + (size_t)b * C * 4, c->dk, (size_t)C * 32, hipMemcpyDeviceToHost, s));
    HC_TRY(mcopy(c0, dom.data() + (size_t)b * (1 + kVisClasses), c->scal, 8, hipMemcpyDeviceToHost, s));
  }
  HC_TRY(mcheck(c0, hipStreamSynchronize(s), "batched adjoint backward"));
  for (int b = 0; b < n; ++b) {
    const double om = cs[b]->L.omega;
    const double dtau = -om * om * dom[(size_t)b * (1 + kVisClasses)];
    for (int i = 0; i < C; ++i) {
      for (int j = 0; j < 4; ++j) grad[((size_t)b * C + i) * 5 + j] = dk[((size_t)b * C + i) * 4 + j];
      grad[((size_t)b * C + i) * 5 + 4] = dtau;
    }
  }
  return HC_OK;
}

hc_status hc_get_step(const hc_ctx* c, int64_t* step) {
  if (!c || !step) return HC_ERR_ARG;
  *step = c->step;
  return HC_OK;
}

}  // extern "C"
