/*
 * hemo.h -- C ABI of the MI355X coupled fluid-cell step library (libhemo.so).
 *
 * One coupled time step (HemoCell model, arXiv 2305.02752):
 *   1. membrane forces on triangulated cells: F = F_link + F_bend + F_area
 *      + F_volume (+ pole traction)                       -- Sec. 2.3, force sum
 *   2. immersed-boundary spreading of vertex forces onto the lattice as an
 *      external force density (Peskin kernel)              -- Sec. 2.3
 *   3. D3Q19 BGK collide and stream with the force term     -- Sec. 2.2, LBGK update
 *   4. interpolation of the lattice velocity to the vertices -- Sec. 2.3
 *   5. explicit Euler advection of the vertices             -- Sec. 2.6
 *
 * Conventions
 *  - Every call returns hc_status; hc_last_error() gives a message.  No C++
 *    exception crosses this boundary.
 *  - A context is single-stream and not thread-safe.  All device work is
 *    enqueued on the stream given by hc_set_stream (default: the null
 *    stream).  Device errors that happen asynchronously (including the
 *    non-finite flag raised by the kernels) surface at hc_sync or at the next
 *    read.
 *  - Device memory is owned by the caller: hc_query_workspace reports the
 *    bytes the context needs and hc_bind_workspace hands over one device
 *    buffer of at least that size (256-byte aligned).  The library never
 *    frees it and allocates no device memory of its own, except the
 *    argument tables of hc_adj_multi_forward / hc_adj_multi_backward (one
 *    record per box and step kind, tens of MB at most), which each call
 *    allocates and frees before it returns.
 *  - Host read/write calls take caller-owned host arrays with an explicit
 *    element count; a mismatch returns HC_ERR_ARG.  They synchronise the
 *    stream before returning.
 *  - Layouts: populations [19][nz][ny][nx] float32, x fastest, direction
 *    order 0:(0,0,0) 1:(1,0,0) 2:(-1,0,0) 3:(0,1,0) 4:(0,-1,0) 5:(0,0,1)
 *    6:(0,0,-1) 7:(1,1,0) 8:(-1,-1,0) 9:(1,-1,0) 10:(-1,1,0) 11:(1,0,1)
 *    12:(-1,0,-1) 13:(1,0,-1) 14:(-1,0,1) 15:(0,1,1) 16:(0,-1,-1)
 *    17:(0,1,-1) 18:(0,-1,1); populations are exchanged SHIFTED,
 *    g_i = f_i - w_i (w: 1/3, 1/18 x6, 1/36 x12).  Vector fields [3][nz][ny][nx].
 *    Cells: origin int32 [C][3], offsets float32 [C][V][3] (absolute
 *    position = origin + offset), stiffness float32 [C][4] = link, bend,
 *    area, volume, traction float32 [C][3].
 */
#ifndef HEMO_H
#define HEMO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HC_OK = 0,
  HC_ERR_ARG = 1,          /* invalid argument or size mismatch               */
  HC_ERR_STATE = 2,        /* call out of order (no workspace, no cells, ...)  */
  HC_ERR_DEVICE = 3,       /* HIP runtime error                                */
  HC_ERR_OOM = 4,          /* workspace too small                              */
  HC_ERR_NONFINITE = 5,    /* a kernel saw a non-finite vertex position        */
  HC_ERR_UNSUPPORTED = 6   /* configuration outside what the library handles   */
} hc_status;

enum { HC_PERIODIC = 0, HC_WALL = 1 };
enum { HC_PHI2 = 2, HC_PHI4 = 4 };

typedef struct hc_ctx hc_ctx;

/* Lattice description (Sec. 2.2 and Sec. 2.5).
 *  nx, ny, nz   lattice nodes per axis (node i sits at coordinate i), >= 4.
 *  bc[3]        HC_PERIODIC or HC_WALL per axis (x, y, z); at most one wall
 *               axis.  A wall lies half a spacing outside the first and last
 *               node (half-way bounce-back); no-slip, Sec. 2.5.
 *  tau          BGK relaxation time (> 0.5); nu = (tau - 1/2)/3 (Sec. 2.2).
 *  body_force   uniform force density added to every node (lattice units).
 *  wall_u_lo/hi velocity of the lower / upper wall of the wall axis
 *               (moving walls impose shear, Sec. 2.5); must be tangential.
 *  ibm_kernel   HC_PHI4 (Peskin 4-point, default) or HC_PHI2 (linear hat,
 *               the "linear interpolation" of Sec. 2.3).
 *  lees_edwards_u  0, or the velocity U of Lees-Edwards sheared periodic
 *               images (Sec. 2.5: boundary-free uniform shear): z is the
 *               gradient axis, x the flow axis; the image above the box is
 *               displaced by +U t along x and moves with +U, the one below
 *               by -U t and -U.  Populations crossing the z boundary are
 *               interpolated along the displaced image row and changed by
 *               the Galilean equilibrium term; IBM stencil nodes in an image
 *               use the vertex's displaced image.  Requires every axis
 *               periodic and nx, nz multiples of 8; not available to the
 *               batched form or the adjoint.                                 */
typedef struct {
  int32_t nx, ny, nz;
  int32_t bc[3];
  float tau;
  float body_force[3];
  float wall_u_lo[3];
  float wall_u_hi[3];
  int32_t ibm_kernel;
  float lees_edwards_u;
} hc_lattice_desc;

/* Cell surface mesh shared by all cells (Sec. 2.3: triangulated membrane).
 *  tri       host int32 [n_tri][3], counter-clockwise seen from outside,
 *            closed 2-manifold, vertex valence <= 8.
 *  rest_pos  host float32 [n_vert][3]: the stress-free shape; rest edge
 *            lengths, dihedral angles, area and volume are taken from it.
 *            The 32 vertices with the largest / smallest rest x receive the
 *            pole traction.  Copied at hc_create.                           */
typedef struct {
  int32_t n_vert, n_tri;
  const int32_t* tri;
  const float* rest_pos;
} hc_mesh_desc;

/* Create a context for one lattice with room for max_cells cells. */
hc_status hc_create(const hc_lattice_desc* lat, const hc_mesh_desc* mesh, int32_t max_cells,
                    hc_ctx** out);
void hc_destroy(hc_ctx* ctx);
const char* hc_last_error(const hc_ctx* ctx);

/* hip_stream: a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream). */
hc_status hc_set_stream(hc_ctx* ctx, void* hip_stream);

/* Entries per tile list (Sec. 2.6 domain bookkeeping: which tile holds
 * which vertex stencils).  Each 8^3 tile keeps one list of the (vertex,
 * tile) pairs that reach it, of fixed capacity: 2048 by default (4 per
 * node, about 4x the mean of a 44% haematocrit suspension).  entries in
 * [64, 16384]; only before hc_bind_workspace (HC_ERR_STATE after), since
 * the lists live in the workspace.  hc_set_cells refuses cells whose
 * fullest list would exceed the capacity (HC_ERR_UNSUPPORTED, with the
 * capacity needed); a list that overflows later, as cells crowd, loses
 * entries of that step and is reported by hc_sync (HC_ERR_UNSUPPORTED).
 * A checkpoint holds no list state, so such a run continues from its last
 * checkpoint (hc_checkpoint_restore) in a context created with a larger
 * capacity and the same cells (hc_set_cells). */
hc_status hc_set_list_capacity(hc_ctx* ctx, int32_t entries);
/* Entries the fullest tile list holds for the current positions (after
 * applying a pending move), and the capacity (may be NULL). */
hc_status hc_densest_tile(hc_ctx* ctx, int32_t* entries, int32_t* capacity);

/* Device bytes the context needs (populations x2, fields, cells, bins). */
hc_status hc_query_workspace(const hc_ctx* ctx, size_t* bytes);
/* dev_ptr: device buffer of >= the queried bytes, 256-byte aligned, owned by
 * the caller and kept alive until hc_destroy. */
hc_status hc_bind_workspace(hc_ctx* ctx, void* dev_ptr, size_t bytes);

/* Upload n <= max_cells cells (host arrays; traction may be NULL = none). */
hc_status hc_set_cells(hc_ctx* ctx, int32_t n, const int32_t* origin, const float* offsets,
                       const float* k, const float* traction);

/* Populations at equilibrium f_i = f_eq(rho0, u0) (Sec. 2.2 equilibrium). */
hc_status hc_init_equilibrium(hc_ctx* ctx, float rho0, const float u0[3]);

/* Enqueue n_steps coupled steps (steps 1-5 above). */
hc_status hc_step(hc_ctx* ctx, int32_t n_steps);

/* Wait for the stream; HC_ERR_NONFINITE if a kernel flagged a non-finite
 * position since the last sync (the flag is then cleared). */
hc_status hc_sync(hc_ctx* ctx);

/* Shifted populations g = f - w, count = 19 * nx * ny * nz. */
hc_status hc_read_populations(hc_ctx* ctx, float* host, int64_t count);
hc_status hc_write_populations(hc_ctx* ctx, const float* host, int64_t count);

/* Density [N] and velocity [3][N] of the last step's moments (velocity
 * includes half the force density, Guo forcing); N = nx * ny * nz.
 * Either pointer may be NULL.  HC_ERR_STATE when the field output is off. */
hc_status hc_read_macro(hc_ctx* ctx, float* rho, float* u, int64_t n_sites);

/* Whether each step writes its force field and (u, rho) field to device
 * memory for hc_read_force_field / hc_read_macro (default on).  The step
 * keeps both on chip, so turning the output off saves 28 bytes per site
 * per step of HBM writes. */
hc_status hc_set_field_output(hc_ctx* ctx, int32_t enable);

/* Force density [3][N] (body force + spread membrane forces) of the last step. */
hc_status hc_read_force_field(hc_ctx* ctx, float* f, int64_t n_sites);

/* Current cells; vertex_force = membrane forces of the last evaluation
 * (may be NULL).  Counts: origin 3C, offsets and force 3CV.  Each offset
 * coordinate is kept as a float plus a float low part that carries the
 * rounding of every move (so that a slowly moving vertex does not drift by
 * up to half an ulp per step); the offsets read here are the high parts, and
 * hc_write_vertices, hc_set_cells and hc_place_cells clear the low parts. */
hc_status hc_read_vertices(hc_ctx* ctx, int32_t* origin, float* offsets, float* vertex_force,
                           int64_t n_cells);
hc_status hc_write_vertices(hc_ctx* ctx, const int32_t* origin, const float* offsets,
                            int64_t n_cells);
/* Vertex velocity U_v interpolated in the last step (Sec. 2.3), float32
 * [C][V][3]; the last step moved each vertex by U_v (Sec. 2.6, Euler). */
hc_status hc_read_vertex_velocity(hc_ctx* ctx, float* vel, int64_t n_cells);

/* Evaluate membrane forces of the current positions only (steps 1 of the
 * step); area and volume per cell (float64, may be NULL) are returned. */
hc_status hc_compute_forces(hc_ctx* ctx, double* area, double* volume, int64_t n_cells);

/* Bin the current positions to 8^3 tiles (Tx = ceil(nx/8), ...; tile id
 * (tz*Ty + ty)*Tx + tx) and read the lists back:
 *  owner [C*V]        tile of node origin + floor(offset) per vertex
 *  touch_ptr [NT+1], touch [touch_ptr[NT]]
 *                     per tile, the vertices whose IBM stencil reaches it,
 *                     sorted by vertex index
 *  cell_ptr [NT+1], cells [cell_ptr[NT]]
 *                     per tile, the cells whose stencil bounding box
 *                     [floor(min)-1, floor(max)+2] meets it, sorted
 * cap_touch / cap_cells give the capacities of touch / cells; if too small
 * HC_ERR_ARG is returned and the needed sizes are in touch_ptr[NT] and
 * cell_ptr[NT]. */
hc_status hc_read_bins(hc_ctx* ctx, int32_t* owner, int32_t* touch_ptr, int32_t* touch,
                       int64_t cap_touch, int32_t* cell_ptr, int32_t* cells, int64_t cap_cells);
hc_status hc_num_tiles(const hc_ctx* ctx, int32_t* n_tiles);

/* Checkpoint (Sec. 2.6: pause, save, continue): the step counter and
 * integration settings, the stored lattice state (the library's own
 * layout), cell origins and offsets (with their low parts), the last vertex velocities and the
 * held vertex forces -- everything a resumed run needs to continue bit for
 * bit, also in the middle of a force-refresh interval.  The buffer is
 * opaque to the caller; restore checks the cell count. */
hc_status hc_checkpoint_size(const hc_ctx* ctx, size_t* bytes);
hc_status hc_checkpoint_save(hc_ctx* ctx, void* host, size_t bytes);
hc_status hc_checkpoint_restore(hc_ctx* ctx, const void* host, size_t bytes);

/* Cell integration with separated time scales (Sec. 2.6: cells move by
 * Euler or Adams-Bashforth, and the constitutive model is evaluated less
 * often than the fluid is advanced).  force_every >= 1: the membrane forces
 * (with the pole traction) are recomputed at every force_every-th step,
 * counted from hc_set_cells, and held in between.  scheme: HC_EULER
 * (X += U) or HC_AB2 (X += 3/2 U^n - 1/2 U^{n-1}; the first move after
 * hc_set_cells or hc_write_vertices is an Euler move).  Defaults: 1,
 * HC_EULER.  The adjoint calls require the defaults. */
enum { HC_EULER = 0, HC_AB2 = 1 };
hc_status hc_set_integration(hc_ctx* ctx, int32_t force_every, int32_t scheme);

/* Interior viscosity (Sec. 1: the cytosol is more viscous than plasma;
 * Sec. 3.4: stiffened cells raise the internal viscosity ratio).  Sites
 * inside a cell relax with tau_in = 1/2 + ratio (tau - 1/2); the others
 * with tau.  A site is inside by ray parity along z: the vertical line
 * through it crosses the membrane at z_1 < z_2 < ..., and the site lies
 * strictly between z_(2k-1) and z_(2k); a point on a projected triangle
 * edge is counted by exactly one of the two triangles sharing the edge.
 * The marks are recomputed every step from the positions the step spreads
 * from.  ratio > 0; 1 (the default) switches the marking off.  Limits per
 * cell: at most 320 node columns along x, bounding-box sides under 1024,
 * and 8 membrane crossings per column (hc_sync reports HC_ERR_UNSUPPORTED
 * beyond).  With Lees-Edwards images, a node in the image above or below
 * is inside when the cell's copy displaced by -/+ the image shift contains
 * it (the reading the IBM stencils follow).  The adjoint calls include the
 * interior sites in d/d tau through tau_in; the ratios may not change
 * between hc_adj_forward and hc_adj_backward (HC_ERR_STATE). */
hc_status hc_set_interior_viscosity(hc_ctx* ctx, float ratio);

/* One interior viscosity ratio per current cell, ratio [n_cells] (mixtures
 * of healthy and stiffened cells, Sec. 3.4), at most 8 distinct values
 * (HC_ERR_UNSUPPORTED beyond).  A site inside several cells (overlap) takes
 * the largest of their ratios.  Replaces the single ratio until the next
 * hc_set_cells or hc_set_interior_viscosity call, either of which returns
 * to the single ratio of the last hc_set_interior_viscosity (1 if none).
 * Same refusals as hc_set_interior_viscosity; n_cells must equal the
 * current cell count. */
hc_status hc_set_cell_viscosity(hc_ctx* ctx, const float* ratio, int64_t n_cells);

/* The inside marks of the current positions (after applying a pending
 * vertex move), uint8 [N] in natural site order (x fastest): 1 << k for a
 * site inside a cell of viscosity class k, the highest such k where cells
 * of several classes overlap (classes are the distinct ratios in
 * increasing order; a single ratio is class 0), 0 outside every cell.  Synchronous; reports marking overflows as hc_sync
 * does. */
hc_status hc_read_interior(hc_ctx* ctx, uint8_t* inside, int64_t n_sites);

/* Per-kernel timing.  hc_profile(ctx, 1) clears the record and brackets
 * every subsequent launch of the step with events on the context stream;
 * hc_profile_read waits for the stream and returns, per kernel family
 * (index HC_K_*), the summed device time in milliseconds and the number of
 * launches since the last hc_profile call.  Arrays hold HC_NUM_KERNELS. */
enum {
  HC_K_CELL = 0,     /* per cell: pending vertex move, membrane forces, binning */
  HC_K_LATTICE = 1,  /* per tile: IBM spread, collide + stream, IBM interpolation */
  HC_K_ADVECT = 2,   /* vertex move closing the last step of an hc_step call */
  HC_K_INTERIOR = 3, /* per cell: marking of the sites inside it (interior viscosity) */
  HC_NUM_KERNELS = 4
};
hc_status hc_profile(hc_ctx* ctx, int32_t enable);
hc_status hc_profile_read(hc_ctx* ctx, double* total_ms, int64_t* launches);

/* Device-to-device copy of `bytes` with the library's own streaming copy
 * kernel (16-byte nontemporal vector loads and stores, four in flight per
 * thread, one pass), enqueued on hip_stream.  Used as
 * the measured bandwidth reference beside the roofline.  dst and src must
 * not overlap and must be 16-byte aligned. */
hc_status hc_device_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Force-bias packing of surrogate ellipsoids (Sec. 2.4: random positions and
 * orientations, then iterations that push every overlapping pair apart
 * along the line through the centres in proportion to their overlapping
 * volume).  Stateless; errors are reported by hc_last_error(NULL).
 *
 * Ellipsoid i: centre r_i, rotation R_i (row-major 3x3, columns = body axes
 * in the world frame), semi-axes s_i along those axes.  Overlap volume:
 * the unit ball is sampled at the centres of the quad^3 grid cells over
 * [-1, 1]^3 that lie inside it (Q points) and mapped onto each ellipsoid;
 * with n_i(j) of i's points inside j, V_ij = (V_i n_i(j) + V_j n_j(i)) / 2Q.
 * One iteration moves every ellipsoid at once by
 *   eta * sum_j V_ij (r_i - r_j) / |r_i - r_j|
 * (minimum image on periodic axes; a pair with coincident centres exerts
 * nothing), shortened to max_move when longer; periodic axes then wrap the
 * centre into [0, box), wall axes clamp it so that the ellipsoid's extent
 * along the axis stays within [lo, hi].  Orientations stay fixed.  The
 * pushes are summed in fixed point, so a run is bitwise reproducible.
 * ------------------------------------------------------------------------- */
typedef struct {
  float box[3];          /* domain sides */
  int32_t periodic[3];   /* per axis: 1 periodic (side >= 4 max_semi), 0 walls */
  float lo[3], hi[3];    /* wall axes: allowed extent, hi - lo >= 2 max_semi */
  float max_semi;        /* bound on every semi-axis; sets the neighbour bins */
  float eta;             /* displacement per unit overlapping volume (>= 0) */
  float max_move;        /* longest move per iteration (> 0) */
  int32_t quad;          /* quadrature grid per axis: 4, 8 or 16 */
} hc_pack_desc;

/* Device workspace bytes for n ellipsoids (256-byte aligned buffer). */
hc_status hc_pack_query_workspace(const hc_pack_desc* desc, int32_t n, size_t* bytes);

/* n_iter iterations on device arrays: centres [n][3] (in/out), rot [n][9],
 * semi [n][3], all float32, enqueued on hip_stream.  overlap (host, may be
 * NULL): double [4], {total overlapping volume sum_{i<j} V_ij, overlapping pairs}
 * before the first move, then the same at the returned centres; when given,
 * the call synchronises.  The call always ends by reading device flags
 * (synchronous): HC_ERR_NONFINITE for a non-finite centre, HC_ERR_ARG for a
 * semi-axis outside (0, max_semi], HC_ERR_UNSUPPORTED when a neighbour bin
 * overflows its capacity. */
hc_status hc_pack_run(const hc_pack_desc* desc, float* centres, const float* rot, const float* semi,
                      int32_t n, int32_t n_iter, void* workspace, size_t ws_bytes, void* hip_stream,
                      double* overlap);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * iterations as hc_pack_run, with the packing's scratch (bin lists, counters,
 * the second centre buffer, overlap sums) in a static array of the library,
 * 32 MiB per device, held until the process ends; nothing is allocated.
 * Sizes needing more scratch than that (about 200,000 ellipsoids at the
 * density of the RBC surrogate suspension) return HC_ERR_UNSUPPORTED, as
 * hc_pack_query_workspace reports the need.  Every call on one device shares
 * that device's array and leaves its contents behind (the call clears what
 * must start at zero): calls that overlap on one device race.  Results are
 * those of hc_pack_run, bit for bit. */
hc_status hc_pack_run_static(const hc_pack_desc* desc, float* centres, const float* rot, const float* semi,
                             int32_t n, int32_t n_iter, void* hip_stream, double* overlap);

/* Cells from packed ellipsoids without a host round trip (Sec. 2.4: each
 * ellipsoid encloses one cell): the context's rest mesh, rotated by rot
 * (device [n][9], as for hc_pack_run) and translated to centres (device
 * [n][3]), becomes cell c with origin floor(centre) and offsets
 * R rest + (centre - origin), computed in float32.  k (host [n][4]) and
 * traction (host [n][3] or NULL) as for hc_set_cells, whose resets this
 * call shares. */
hc_status hc_place_cells(hc_ctx* ctx, int32_t n, const float* centres, const float* rot, const float* k,
                         const float* traction);

/* Steps taken since hc_set_cells / restore. */
hc_status hc_get_step(const hc_ctx* ctx, int64_t* step);

/* Replace the stiffnesses k [C][4] (NULL: keep) and the relaxation time. */
hc_status hc_set_params(hc_ctx* ctx, const float* k, float tau);

/* ---------------------------------------------------------------------------
 * Adjoint form.  The membrane parameters are fitted to single-cell
 * stretching and shearing measurements (Sec. 2.3); these calls give the
 * exact gradient of a cell-shape loss with respect to the stiffnesses and
 * the relaxation time by a hand-written reverse sweep of the coupled step.
 *
 * Loss per cell c after n steps: (D_A - D_A*)^2 + (D_T - D_T*)^2 with
 * D_A = max x - min x and D_T = max y - min y over its vertices.
 * hc_adj_forward runs n steps from the current state (checkpointing every
 * ckpt_every steps) and returns the loss; the context then holds the final
 * state, as after hc_step(n) (with field output on, the force and (u, rho)
 * fields of the last step: earlier steps do not write them).
 * hc_adj_backward recomputes one segment at a
 * time from its checkpoint, keeping every state, and sweeps it backwards.
 * grad [C][5] = dL_c/d(k_link, k_bend, k_area, k_volume) of cell c, and in
 * column 4 dL/dtau, where L is the sum of all cells' losses (tau is shared
 * by the lattice; with an interior viscosity it includes the interior
 * sites through tau_in = 1/2 + ratio (tau - 1/2)).  Needs the 4-point
 * kernel, Euler moves with forces every step and no Lees-Edwards images
 * (HC_ERR_UNSUPPORTED otherwise).  hc_adj_backward refers to the last
 * hc_adj_forward: hc_set_params, hc_set_cells, hc_place_cells,
 * hc_checkpoint_restore and a change of hc_set_integration in between
 * discard it (HC_ERR_STATE until the next hc_adj_forward), since its reverse
 * sweep recomputes under the parameters and cells it ran with.  The
 * adjoint workspace is separate from the main one and sized by
 * hc_adj_query_workspace.
 * ------------------------------------------------------------------------- */
hc_status hc_adj_query_workspace(const hc_ctx* ctx, int32_t n_steps, int32_t ckpt_every,
                                 size_t* bytes);
hc_status hc_adj_bind_workspace(hc_ctx* ctx, void* dev_ptr, size_t bytes, int32_t n_steps,
                                int32_t ckpt_every);
/* targets [C][2] = (D_A*, D_T*); loss [C] float64. */
hc_status hc_adj_forward(hc_ctx* ctx, const double* targets, double* loss);
hc_status hc_adj_backward(hc_ctx* ctx, double* grad);

/* The same reverse-mode pair over n boxes at once (Sec. 2.3: fitting the
 * stiffness constants and relaxation time to many single-cell experiments):
 * ctxs[n] are contexts of one lattice shape and boundary kind, the same
 * mesh and cell count, each with its own adjoint workspace bound for the
 * same n_steps and ckpt_every; Euler moves with forces every step, the
 * 4-point kernel, no sheared images and no interior viscosity.  Every
 * per-step kernel runs as one launch over all boxes, on ctxs[0]'s stream
 * (the other streams are synchronised first); each box's loss and gradient
 * are those hc_adj_forward / hc_adj_backward give it alone, up to a few FP32
 * roundings (the same arithmetic in kernels compiled a second time).
 * targets [n][C][2], loss [n][C], grad [n][C][5] (host, row-major).  The
 * call returns after its work is done; errors are reported on ctxs[0]. */
hc_status hc_adj_multi_forward(hc_ctx* const* ctxs, int32_t n, const double* targets, double* loss);
hc_status hc_adj_multi_backward(hc_ctx* const* ctxs, int32_t n, double* grad);

/* ---------------------------------------------------------------------------
 * Batched form: n_boxes independent boxes, one cell each, advanced together
 * by ONE persistent kernel launch per hc_batch_run (replayed from a captured
 * hipGraph).  This is the calibration use of the model (Sec. 2.3 fits the
 * membrane parameters to single-cell stretching and shearing experiments):
 * every box may have its own size, boundaries, tau, stiffness and traction.
 * Each box is stepped exactly as hc_step steps a single lattice.
 *
 * Work split: every box owns a group of work-groups, sized in proportion to
 * its node count and kept on one XCD; tiles are full x rows by ty x tz rows.
 * hc_batch_set_tiling / hc_batch_autotune choose ty, tz and the work-group
 * size (256, 512 or 1024).  The grid never exceeds the resident capacity
 * reported by the occupancy API; group barriers spin with a bound, and a
 * timed-out barrier aborts the whole launch and surfaces at hc_batch_sync as
 * HC_ERR_DEVICE.  All boxes must use the same ibm_kernel.
 * Layouts per box: as for a single lattice.  Cell arrays are per box:
 * origin [B][3], offsets [B][V][3], k [B][4], traction [B][3] (or NULL).
 * ------------------------------------------------------------------------- */
typedef struct hc_batch hc_batch;
hc_status hc_batch_create(int32_t n_boxes, const hc_lattice_desc* boxes, const hc_mesh_desc* mesh,
                          hc_batch** out);
void hc_batch_destroy(hc_batch* b);
const char* hc_batch_last_error(const hc_batch* b);
hc_status hc_batch_set_stream(hc_batch* b, void* hip_stream);
hc_status hc_batch_query_workspace(const hc_batch* b, size_t* bytes);
/* Populations start at rest (f = w) when the workspace is bound. */
hc_status hc_batch_bind_workspace(hc_batch* b, void* dev_ptr, size_t bytes);
hc_status hc_batch_set_cells(hc_batch* b, const int32_t* origin, const float* offsets,
                             const float* k, const float* traction);
/* Interior viscosity per box (Sec. 1: cytosol five times more viscous than
 * plasma; Sec. 3.4: the internal ratio of stiffened cells): ratio [n_boxes]
 * host floats, finite and > 0; nodes inside box i's cell relax with
 * tau_in = 1/2 + ratio[i] (tau_i - 1/2), as hc_set_interior_viscosity does
 * for a single lattice (same inside test and limits; a cell beyond them
 * surfaces at hc_batch_sync as HC_ERR_UNSUPPORTED).  A ratio of 1 switches
 * the box's marking off.  HC_ERR_STATE before a workspace is bound. */
hc_status hc_batch_set_interior_viscosity(hc_batch* b, const float* ratio);
hc_status hc_batch_set_tiling(hc_batch* b, int32_t ty, int32_t tz, int32_t block);
hc_status hc_batch_get_tiling(const hc_batch* b, int32_t* ty, int32_t* tz, int32_t* block,
                              int32_t* grid);
/* Time every candidate tiling for trial_steps steps (the state is saved and
 * restored around each trial), keep the fastest and append it to the text
 * file cache_path (NULL: no cache) keyed by architecture and batch shape; a
 * cached entry is applied without timing. */
hc_status hc_batch_autotune(hc_batch* b, const char* cache_path, int32_t trial_steps, int32_t* ty,
                            int32_t* tz, int32_t* block);
/* Enqueue n_steps steps of every box: one kernel launch (graph replay). */
hc_status hc_batch_run(hc_batch* b, int32_t n_steps);
hc_status hc_batch_sync(hc_batch* b);
hc_status hc_batch_box_steps(hc_batch* b, int32_t box, int64_t* steps);
hc_status hc_batch_read_populations(hc_batch* b, int32_t box, float* host, int64_t count);
hc_status hc_batch_write_populations(hc_batch* b, int32_t box, const float* host, int64_t count);
/* Any pointer may be NULL; offsets/force/vel are [V][3] of the box's cell. */
hc_status hc_batch_read_vertices(hc_batch* b, int32_t box, int32_t* origin, float* offsets,
                                 float* force, float* vel);
hc_status hc_batch_launches(const hc_batch* b, int64_t* graph_launches);

#ifdef __cplusplus
}
#endif
#endif /* HEMO_H */
