/*
 * fluxlim.h -- C ABI of the MI355X (gfx950) flux-limited convective operator library.
 *
 * The operator is the algebraic flux limiter of Valle et al., "On the implementation of flux
 * limiters in algebraic frameworks" (arXiv 2110.03044):
 *   theta_f = theta_C + psi(r_f) (theta_D - theta_C) / 2,   r_f = d_U / d_u
 * (Section 3: Sweby form, gradient ratio, the algebraic operator theta_f = (Pi + F(r) Q E) theta
 * with F = (psi - 1)/2, and Algorithm 3), followed by the divergence of the face fluxes
 * a_f u_f theta_f and an explicit time step (Section 4.1, Algorithm 4), here forward Euler or
 * three-stage SSP Runge-Kutta.
 *
 * Mesh model (Section 2): a mesh is its oriented face-to-cell incidence.  Face f joins
 * own = face_cells[2f] and nbr = face_cells[2f+1]; its unit normal face_normal[3f..3f+2] points
 * from own into nbr (E_{C->F}[f][nbr] = +1, E_{C->F}[f][own] = -1).  u_f is the normal
 * velocity along that normal.  The velocity sign matrix Q(u_f) takes +1 where u_f > 0 and -1
 * otherwise (Table 1, signxty), so C = own where u_f > 0 and C = nbr where u_f <= 0.  The
 * upstream difference d_U = sum_j w_j (theta_C - theta_j) runs over the other faces j of C with
 * weights w_j = Q_f (n_f . t_j), t_j the normal of j oriented into C (the upstream adjacency
 * A^U_FF of Section 3.1 through the normal matrices: the rows of S_{C->F} and T_{C->F}), found
 * once at mesh creation.  On hexahedra, quadrilaterals and lines one face has weight 1 and the
 * rest 0, so d_U = theta_C - theta_U with U the cell across the face of C opposite to f; other
 * cells (triangles, tetrahedra, skewed cells) keep the list of weights and run on the face/cell
 * path (no adjoint, no batching for them).
 *
 * Conventions for every entry point:
 *   - all floating point is IEEE binary64 (double);
 *   - cell fields hold n_scalars values per cell, scalar index fastest: theta[c * S + s];
 *   - device pointers are plain HIP device allocations on the mesh's device (e.g. torch
 *     tensors), 8-byte aligned, not aliased unless stated; the caller owns them;
 *   - arrays are in MESH ORDER: the user's numbering, unless the mesh was created with
 *     FL_MESH_REORDER (then see fl_mesh_permutation);
 *   - hot-path calls (fl_convect_apply, fl_rk_step, fl_rk_steps, fl_convect_adjoint,
 *     fl_rk_step_adjoint, fl_batch_step) only enqueue work on the given HIP stream
 *     (hipStream_t passed as void*, NULL = the null stream): no host synchronisation, no
 *     allocation, O(1) argument checks (unless the opt-in finite check FL_OPT_CHECK_FINITE is
 *     on: it scans the inputs and synchronises the stream);
 *   - errors are returned as status codes (never abort, never throw); fl_last_error() gives a
 *     thread-local message for the last failing call of the calling thread;
 *   - results are bitwise deterministic from run to run (no atomics, fixed summation order).
 */
#ifndef FLUXLIM_H
#define FLUXLIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fl_status;
#define FL_OK 0
#define FL_E_INVALID -1     /* bad argument: null pointer, size, enum, alignment            */
#define FL_E_TOPOLOGY -2    /* incidence violates the mesh model (index range, own == nbr,
                               own == -1, two faces joining the same two cells)               */
#define FL_E_UNSUPPORTED -3 /* valid but outside this library: the adjoint on cells with
                               neither opposite face pairs nor projected-face lists; the
                               multi-step reverse sweep off the fused path; the algebraic
                               chain on meshes with boundary faces or face distances         */
#define FL_E_NOMEM -4       /* host or device allocation failed                              */
#define FL_E_HIP -5         /* a HIP runtime call failed (message in fl_last_error)          */
#define FL_E_NONFINITE -6   /* an input holds a NaN or an infinity (only reported while the
                               opt-in check FL_OPT_CHECK_FINITE is on)                        */
#define FL_E_NODEVICE -7    /* compute call on a host-only mesh (device = -1)                */

/* Limiters psi(r) (Sweby's family; superbee is the paper's, Table 1):
 *   FL_UPWIND    psi = 0 (first order upwind; the paper's F = -1/2)
 *   FL_MINMOD    max(0, min(1, r))
 *   FL_VANLEER   (r + |r|) / (1 + |r|)
 *   FL_VANALBADA (r^2 + r) / (r^2 + 1)  (not clipped; smooth)
 *   FL_SUPERBEE  max(0, min(1, 2r), min(r, 2))
 *   FL_SMART     max(0, min(2r, 1/4 + 3r/4, 4))
 *   FL_CENTRAL   psi = 1 (central differencing; the paper's F = 0)
 * theta_f = theta_C where theta_D == theta_C; |r| > 1e18 (and r = +-inf) takes psi(+-inf). */
enum { FL_UPWIND = 0, FL_MINMOD = 1, FL_VANLEER = 2, FL_VANALBADA = 3, FL_SUPERBEE = 4,
       FL_SMART = 5, FL_CENTRAL = 6, FL_NUM_LIMITERS = 7 };

/* Time schemes: forward Euler (Algorithm 4) and Shu-Osher SSP-RK3
 * theta1 = theta + dt L(theta); theta2 = 3/4 theta + 1/4 (theta1 + dt L(theta1));
 * theta+ = 1/3 theta + 2/3 (theta2 + dt L(theta2)). */
enum { FL_EULER = 1, FL_SSPRK3 = 3 };

/* fl_mesh_create flags */
enum {
    FL_MESH_REORDER = 1,     /* renumber cells along a space-filling (Morton) curve of the
                                lattice coordinates found by walking the face normals, and
                                faces by their lower cell, for gather locality                */
    FL_MESH_FACE_PATH = 2,   /* use the face-kernel + cell-gather pair even where the fused
                                cell-centric kernel applies                                   */
    FL_MESH_REORDER_BFS = 4  /* renumber cells breadth-first instead (any connected mesh)    */
};

/* Kernel paths reported by fl_mesh_info */
enum { FL_PATH_FACE_CELL = 1, FL_PATH_FUSED = 2 };

#define FL_MAX_SCALARS 8

typedef struct fl_mesh fl_mesh;
typedef struct fl_batch fl_batch;

typedef struct fl_mesh_info_t {
    int64_t n_cells, n_faces;
    int32_t max_degree;     /* faces per cell (max)                                          */
    int32_t pairs;          /* opposite-face pairs per cell if uniform (fused path), else 0  */
    int32_t path;           /* FL_PATH_FACE_CELL or FL_PATH_FUSED                            */
    int32_t device;         /* HIP device, -1 for a host-only mesh                           */
    int32_t reordered;      /* 1 if FL_MESH_REORDER renumbered the mesh                     */
    int32_t uniform_area;   /* 1 if all face areas are equal (then stored as one scalar)     */
    int32_t uniform_volume; /* 1 if all cell volumes are equal                               */
    int64_t device_bytes;   /* device memory held by the mesh                                */
    int32_t tile_cells;     /* cells per LDS-staged tile (fused path), 0 if no tile tables   */
    int32_t max_halo;       /* largest tile halo (cells outside a tile that it reads), -1   */
    int64_t halo_total;     /* halo entries summed over the tiles                            */
    int32_t general;        /* 1: some face side projects on several faces or with a weight */
                            /* other than 1 (triangles, tetrahedra, skewed cells)            */
    int32_t max_side;       /* most projected faces on one face side                         */
    int32_t aligned;        /* 1 if the opposite-face pairs line up from cell to cell (lattice */
                            /* meshes; the forward-rate stages, FL_OPT_FWD_RATES, apply)      */
    int32_t dist_weighted;  /* 1 if unequal face distances weight the upstream difference    */
    int64_t n_boundary;     /* boundary faces (one cell: nbr = -1)                           */
    int32_t compact;        /* 1 if the forward-rate stage's compact slot tables exist        */
    int32_t max_rated;      /* most leading halo entries of a tile whose rate the forward-rate */
                            /* stage stages (neighbours across backward slots), -1 if none   */
    int32_t max_nexts;      /* most leading halo entries of a tile whose next index it stages */
    int32_t side_entries;   /* general cells: side-list entries (projected faces), else 0   */
    int64_t halo_nexts;     /* those entries summed over the tiles                           */
} fl_mesh_info_t;

/* Checks an incidence against the mesh model without a GPU (Section 2).  face_cells: host
 * int32 [n_faces][2]; face_normal: host double [n_faces][3], unit length within 1e-12.
 * Returns FL_OK, FL_E_INVALID, FL_E_TOPOLOGY or FL_E_UNSUPPORTED. */
fl_status fl_mesh_validate(int64_t n_cells, int64_t n_faces, const int32_t *face_cells,
                           const double *face_normal);

/* Builds the mesh tables (far-upwind cell per face side, or its list of projected faces and
 * weights on general cells, cell -> face lists, and where every cell's faces form opposite
 * pairs, the per-cell slot tables and tile halos of the fused kernels) and copies them to
 * `device`.  Inputs are host arrays, read only during the call:
 *   face_cells  int32 [n_faces][2] (own, nbr), 0 <= index < n_cells, own != nbr; nbr = -1
 *               marks a boundary face (one cell, own; see fl_mesh_set_inflow).  A mesh with
 *               boundary faces runs the face path with the general kernel;
 *   face_normal double [n_faces][3], unit, own -> nbr (1-D and 2-D meshes pad with 0; out of
 *               the mesh on a boundary face);
 *   face_area   double [n_faces] or NULL (= 1);   cell_volume double [n_cells] or NULL (= 1).
 * device = -1 builds a host-only mesh (tables, validation and export work; compute calls
 * return FL_E_NODEVICE).  On success *out owns device memory until fl_mesh_destroy; apart from
 * its inflow values (fl_mesh_set_inflow) the mesh is immutable and may be used from several
 * streams at once.  The host loops run on the OpenMP
 * threads of the calling process (OMP_NUM_THREADS); the tables do not depend on their number.
 * With the environment variable FL_MESH_PROGRESS set, each phase reports its wall time on
 * stderr. */
fl_status fl_mesh_create(int64_t n_cells, int64_t n_faces, const int32_t *face_cells,
                         const double *face_normal, const double *face_area,
                         const double *cell_volume, int device, uint32_t flags, fl_mesh **out);
/* As fl_mesh_create, with the distance between the cells across each face (face_dist: host
 * double [n_faces], finite and positive; on a boundary face the distance from its cell to the
 * exterior cell, e.g. to the cell's mirror image).  The gradient ratio then weighs distances as
 * Algorithm 1D (r = (d_i / d_U)(theta_C - theta_U) / (theta_D - theta_C)) and Algorithm UNS
 * (each projected difference over the distance across its face, the face difference over d_i)
 * do: the upstream difference becomes d_U = sum_j w_j (d_f / d_j)(theta_C - theta_j).  Where all
 * distances are equal every ratio is 1 and the mesh is built as without them; otherwise it runs
 * the face path with the general kernel (the ratios sit in its side weights; the adjoint and
 * batches take it there).  face_dist = NULL is fl_mesh_create. */
fl_status fl_mesh_create_dist(int64_t n_cells, int64_t n_faces, const int32_t *face_cells,
                              const double *face_normal, const double *face_area,
                              const double *cell_volume, const double *face_dist, int device,
                              uint32_t flags, fl_mesh **out);
fl_status fl_mesh_destroy(fl_mesh *mesh);
fl_status fl_mesh_info(const fl_mesh *mesh, fl_mesh_info_t *info);

/* Boundary faces.  The paper states the operators on the mesh's graph, and its cell-to-face
 * shift (Section 2, S = D_FF^-1 |T_CF|) gives a face with a single cell that cell's value.  The
 * library reads a boundary face f (nbr = -1) as bordering an exterior cell with no other faces;
 * the face selection, differences, gradient ratio and limiter of Section 3 then apply as on
 * interior faces:
 *   - the exterior holds inflow[f][s] where the flow enters (u_f <= 0: the normal points out)
 *     and inflow values are set, and repeats the value of f's own cell otherwise;
 *   - an outflow face therefore takes theta_own (d_u = 0); an inflow face has C = the exterior
 *     and d_U = 0 (r = 0: the inflow value itself for every limiter with psi(0) = 0, half-way to
 *     theta_own for central differencing); a boundary face among the faces of an interior face's
 *     upwind cell adds w_j (theta_C - exterior value) to that face's d_U;
 *   - the flux a_f u_f theta_f of a boundary face leaves (or enters) its one cell.
 * inflow: device [n_faces][n_scalars] doubles in mesh order (only the boundary faces' rows are
 * read, and only where the flow enters), or NULL to clear (the exterior then repeats the cell's
 * value on every boundary face).  The mesh keeps the pointer: the caller keeps the memory alive
 * and unchanged while calls that read it are queued, and every compute call on the mesh must
 * then use n_scalars scalars (else FL_E_INVALID).  Not synchronised with calls running on other
 * threads.  Returns FL_E_NODEVICE on a host-only mesh. */
fl_status fl_mesh_set_inflow(fl_mesh *mesh, const double *inflow, int n_scalars);

/* Numbering maps of a reordered mesh (identity otherwise): cell_perm[user cell] = mesh cell,
 * face_perm[user face] = mesh face (host int32 arrays of n_cells / n_faces, or NULL to skip).
 * Face orientations are kept, so u_f moves without a sign change. */
fl_status fl_mesh_permutation(const fl_mesh *mesh, int32_t *cell_perm, int32_t *face_perm);

/* Host copies of the tables, in mesh order (any pointer may be NULL):
 *   face_far int32 [n_faces][2]: far-upwind cell when C = own, and when C = nbr (-1 on meshes
 *            of general cells: see fl_mesh_info_t.general);
 *   cf_ptr   int32 [n_cells + 1], cf_idx int32 [cf_ptr[n_cells]]: faces of each cell in
 *            ascending face order, encoded f for faces whose nbr is the cell and ~f (-f-1)
 *            for faces whose own is the cell. */
fl_status fl_mesh_export_tables(const fl_mesh *mesh, int32_t *face_far, int32_t *cf_ptr,
                                int32_t *cf_idx);

/* Reorders cell / face fields between user and mesh order on the device (to_mesh = 1: out =
 * in permuted into mesh order; 0: back).  in and out must not alias.  cells: [n_cells][S]
 * doubles; faces: [n_faces] doubles. */
fl_status fl_permute_cells(const fl_mesh *mesh, int to_mesh, int n_scalars, const double *in,
                           double *out, void *hip_stream);
fl_status fl_permute_faces(const fl_mesh *mesh, int to_mesh, const double *in, double *out,
                           void *hip_stream);

/* rhs = L(theta) = M U(u_f) theta_f (Algorithm 4's spatial operator):
 * rhs_c = (sum_{f: nbr_f = c} a_f u_f theta_f - sum_{f: own_f = c} a_f u_f theta_f) / V_c.
 * theta, rhs: device [n_cells][S]; u_f: device [n_faces]; 1 <= S <= FL_MAX_SCALARS.
 * rhs must not alias theta.  work: device workspace of fl_apply_workspace_bytes bytes (the face
 * fluxes of the face path; 0 bytes, work may be NULL, on the fused path). */
size_t fl_apply_workspace_bytes(const fl_mesh *mesh, int n_scalars);
fl_status fl_convect_apply(const fl_mesh *mesh, int limiter, int n_scalars, const double *theta,
                           const double *u_f, double *rhs, void *work, void *hip_stream);

/* Device workspace bytes needed by fl_rk_step / fl_rk_steps (256-byte aligned pointer). */
size_t fl_rk_workspace_bytes(const fl_mesh *mesh, int scheme, int n_scalars);

/* One (fl_rk_step) or n_steps (fl_rk_steps) explicit steps of size dt, theta updated in place.
 * work: device workspace of fl_rk_workspace_bytes bytes, owned by the caller, not shared by
 * calls that may run concurrently. */
fl_status fl_rk_step(const fl_mesh *mesh, int limiter, int scheme, double dt, int n_scalars,
                     double *theta, const double *u_f, void *work, void *hip_stream);
fl_status fl_rk_steps(const fl_mesh *mesh, int limiter, int scheme, double dt, int n_scalars,
                      int64_t n_steps, double *theta, const double *u_f, void *work,
                      void *hip_stream);

/* Explicit steps with a time-dependent velocity u(t) = s(t) u_f (the deformation benchmark of
 * Section 4.1 reverses its field with s = cos(pi t / T)).  u_scale: host array, read during
 * the call, of s at every stage: u_scale[i * stages + j] for stage j of step i (Euler: 1 stage;
 * SSP-RK3: 3 stages, evaluated at t_i, t_i + dt, t_i + dt/2).  Otherwise as fl_rk_steps. */
fl_status fl_rk_steps_scaled(const fl_mesh *mesh, int limiter, int scheme, double dt,
                             int n_scalars, int64_t n_steps, double *theta, const double *u_f,
                             const double *u_scale, void *work, void *hip_stream);

/* Adjoint of fl_convect_apply (discrete reverse mode; Q(u_f) and the branch of psi taken at
 * theta are held fixed):
 *   theta_bar += (dL/dtheta)^T rhs_bar,   u_bar += (dL/du_f)^T rhs_bar (skipped if NULL).
 * theta, rhs_bar, theta_bar: device [n_cells][S]; u_f, u_bar: device [n_faces].
 * Where theta_D == theta_C the limit of psi(d_U/d_u) d_u / 2 is differentiated (see the
 * readings: psi(+-inf)/2 along d_u for d_U != 0, psi(0)/2 where d_U == 0 too).  Cells with
 * opposite face pairs gather everything in one kernel (work may be NULL: 0 bytes); general cells
 * (fl_mesh_info_t.general) run a face kernel that writes each face's terms to work
 * (fl_adjoint_workspace_bytes bytes, 256-byte aligned) and a cell kernel that gathers them
 * through the cell's face list and the transposed projection lists (no atomics); so do meshes
 * with boundary faces (an inflow value is a constant; an exterior that repeats its face's own
 * cell passes that cell's cotangent on) and with face distances. */
size_t fl_adjoint_workspace_bytes(const fl_mesh *mesh, int n_scalars);
fl_status fl_convect_adjoint(const fl_mesh *mesh, int limiter, int n_scalars, const double *theta,
                             const double *u_f, const double *rhs_bar, double *theta_bar,
                             double *u_bar, void *work, void *hip_stream);

/* Reverse of one explicit step.  stages: device [n_stage][n_cells][S], the stage inputs of the
 * step (stage 0 is theta^n; SSP-RK3 also theta1, theta2).  lambda: device [n_cells][S], on entry
 * the cotangent of theta^{n+1}, on exit that of theta^n.  u_bar (+=, nullable): [n_faces].
 * work: fl_rk_adjoint_workspace_bytes bytes (on general cells it includes the face terms). */
size_t fl_rk_adjoint_workspace_bytes(const fl_mesh *mesh, int scheme, int n_scalars);
fl_status fl_rk_step_adjoint(const fl_mesh *mesh, int limiter, int scheme, double dt,
                             int n_scalars, const double *stages, const double *u_f,
                             double *lambda, double *u_bar, void *work, void *hip_stream);
/* Forward step that also stores its stage inputs (same layout as above) for the adjoint. */
fl_status fl_rk_step_store(const fl_mesh *mesh, int limiter, int scheme, double dt, int n_scalars,
                           double *theta, const double *u_f, double *stages, void *work,
                           void *hip_stream);
/* n_steps such steps in one call (the recompute of a checkpoint segment): stages: device
 * [n_steps][n_stage][n_cells][S], step i's stage inputs at stages[i]; theta advanced in place.
 * Results are bit-identical to n_steps calls of fl_rk_step_store.  work: fl_rk_workspace_bytes
 * bytes (two or more steps use its slot-rate table, see FL_OPT_SLOT_VELOCITY). */
fl_status fl_rk_steps_store(const fl_mesh *mesh, int limiter, int scheme, double dt,
                            int n_scalars, int64_t n_steps, double *theta, const double *u_f,
                            double *stages, void *work, void *hip_stream);

/* Reverse of n_steps steps of fl_rk_steps_store (the backward pass of a checkpoint segment):
 * stages: device [n_steps][n_stage][n_cells][S] as fl_rk_steps_store wrote them; lambda: device
 * [n_cells][S], on entry the cotangent of theta after the last step, on exit that of theta before
 * the first.  Identical arithmetic to n_steps calls of fl_rk_step_adjoint (same bits for lambda).
 * rates: the face velocities as a table of signed rates in cell-slot order, written once per
 * velocity field by fl_adjoint_rates (fl_adjoint_rates_bytes bytes, 16-byte aligned device
 * memory; a backward pass writes it once and passes it to every segment).  The face-velocity
 * cotangent is accumulated (+=) in u_acc, a device buffer of fl_adjoint_uacc_bytes bytes in the
 * mesh's cell-slot layout (each face is kept by exactly one of its cells), or skipped if u_acc
 * is NULL: zero it once, pass it to every call of a backward pass, then add it to a face-ordered
 * u_bar with fl_adjoint_uacc_scatter (u_bar += its entries; starting from u_bar = 0 this gives
 * the same bits as fl_rk_step_adjoint's u_bar).  work: fl_rk_steps_adjoint_workspace_bytes
 * bytes.  Needs a fused-path mesh (FL_E_UNSUPPORTED otherwise). */
size_t fl_adjoint_rates_bytes(const fl_mesh *mesh);
fl_status fl_adjoint_rates(const fl_mesh *mesh, const double *u_f, void *rates, void *hip_stream);
size_t fl_adjoint_uacc_bytes(const fl_mesh *mesh);
size_t fl_rk_steps_adjoint_workspace_bytes(const fl_mesh *mesh, int scheme, int n_scalars);
fl_status fl_rk_steps_adjoint(const fl_mesh *mesh, int limiter, int scheme, double dt,
                              int n_scalars, int64_t n_steps, const double *stages,
                              const void *rates, double *lambda, double *u_acc, void *work,
                              void *hip_stream);
fl_status fl_adjoint_uacc_scatter(const fl_mesh *mesh, const double *u_acc, double *u_bar,
                                  void *hip_stream);

/* Batched problems: n independent (mesh, limiter, S, dt, theta, u_f) problems advanced together
 * with one launch per Runge-Kutta stage for all the fused-path problems (one cell-centric kernel
 * over a work table of (problem, cell tile) entries) and two for all the face-path problems
 * (general cells, boundary faces with the inflow values the mesh holds when the batch is created,
 * face distances: one launch over their faces, one over their cells; the batch owns their flux
 * buffers).  device >= 0 and every
 * mesh created on it (a host-only mesh or device: FL_E_NODEVICE; a mesh on another device:
 * FL_E_INVALID; inflow values set for another scalar count: FL_E_INVALID); meshes may be shared
 * between problems.  theta[i] / u_f[i] are device pointers the batch keeps (not
 * owned) until fl_batch_destroy.  tile_cells > 0 fixes the tile size; 0 picks it here, at
 * creation, by timing the candidates (the first stage, which writes only the batch's own stage
 * buffers) after a device synchronisation, or reads the choice from the on-disk tuning cache:
 * the file named by the environment variable FL_TUNE_CACHE ("" or "0": no cache), by default
 * $XDG_CACHE_HOME/fluxlim/batch_tune.txt or $HOME/.cache/fluxlim/batch_tune.txt, one line per
 * batch shape (GPU architecture and CU count, scheme, tile order, every problem's cells, pairs,
 * scalars and limiter).  Creation then records one step's launches in a HIP graph.  Every tile
 * size gives the same bits. */
fl_status fl_batch_create(int n, fl_mesh *const *meshes, const int *limiter,
                          const int *n_scalars, const double *dt, int scheme,
                          double *const *theta, const double *const *u_f, int tile_cells,
                          int device, fl_batch **out);
/* Advances every problem by n_steps steps by replaying the graph recorded at creation on the
 * given stream: no synchronisation, no allocation. */
fl_status fl_batch_step(fl_batch *batch, int n_steps, void *hip_stream);
/* The same work as separate per-problem launches (no graph), for comparison. */
fl_status fl_batch_step_unbatched(fl_batch *batch, int n_steps, void *hip_stream);
/* The tile size in use, and whether the tiles are staged in LDS: the autotuner also times the
 * LDS-staged kernel (256-cell tiles, each tile's theta and halo in LDS, the mesh's tile tables;
 * FL_OPT_LDS_STAGE and every mesh's LDS need permitting); then fl_batch_step_unbatched runs the
 * same staged kernel per problem.  fl_batch_tuned_from_cache: 1 if the autotuner's choice was
 * read from the tuning cache instead of timed. */
fl_status fl_batch_tile(const fl_batch *batch, int *tile_cells);
fl_status fl_batch_lds(const fl_batch *batch, int *lds_staged);
fl_status fl_batch_tuned_from_cache(const fl_batch *batch, int *from_cache);
fl_status fl_batch_destroy(fl_batch *batch);

/* The paper's algebraic form of the same operator (Algorithms 3 and 4, Section 3.4), kept as a
 * second, literal implementation to compare with the fused path: the face differences
 * D_{C->F} = E_{C->F}, the unoriented and oriented upstream-difference matrices
 * UUD = T_{C->F} = N (I (x) A_FF) N^T E / 2 and OUD = -S_{C->F} = -N (I (x) A^D_FF) N^T E / 2,
 * so that d_U = Q UUD theta + OUD theta = theta_C - theta_U (the sign reading of the
 * upstream-difference equations that restores the one-dimensional gradient ratio), the
 * cell-to-face interpolation Pi_{C->F} = W^-1 B, and the divergence M = Omega^-1 E^T A_F.  Every
 * matrix is stored in ELLPACK format, 8-byte coefficient + 4-byte column per entry of its
 * structural pattern (zero coefficients included, as the paper counts them: 2k entries per row
 * of UUD and OUD), column-major [width][rows].  One scalar field (S = 1).
 *
 * fl_algebraic_create builds the matrices on the host from the mesh's tables and copies them to
 * the mesh's device (a host-only mesh, device -1, gives host-only matrices: export works,
 * compute returns FL_E_NODEVICE).  The mesh must outlive the object.  Errors as for
 * fl_mesh_create. */
typedef struct fl_algebraic fl_algebraic;
typedef struct {
    int64_t rows[5];      /* D, UUD, OUD, Pi, M */
    int32_t width[5];
    int64_t device_bytes; /* bytes of the ELLPACK arrays on the device */
} fl_algebraic_info_t;
enum { FL_ALG_D = 0, FL_ALG_UUD = 1, FL_ALG_OUD = 2, FL_ALG_PI = 3, FL_ALG_M = 4 };
fl_status fl_algebraic_create(const fl_mesh *mesh, fl_algebraic **out);
fl_status fl_algebraic_destroy(fl_algebraic *alg);
fl_status fl_algebraic_info(const fl_algebraic *alg, fl_algebraic_info_t *info);
/* Copies matrix `which` (FL_ALG_*) to host arrays val [width][rows] and col [width][rows]. */
fl_status fl_algebraic_export(const fl_algebraic *alg, int which, double *val, int32_t *col);
/* Device workspace bytes of fl_algebraic_face_values / fl_algebraic_rk_steps (256-byte aligned
 * pointer): three face vectors and three cell vectors. */
size_t fl_algebraic_workspace_bytes(const fl_algebraic *alg);
/* theta_f (device [n_faces]) of theta (device [n_cells]) by Algorithm 3: d_u = D theta (SpMV),
 * d_u = Q d_u (signxty), r = UUD theta (SpMV), r = Q r (signxty), r = r + OUD theta (SpMV),
 * r = r / d_u (axdy), theta_f = F(r) d_u (the limiter kbin, F = (psi - 1)/2), theta_f = theta_f
 * + Pi theta (SpMV).  Where d_u == 0 the two pointwise kernels give r = 0 and F(r) d_u = 0, so
 * theta_f = theta_C. */
fl_status fl_algebraic_face_values(const fl_algebraic *alg, int limiter, const double *theta,
                                   const double *u_f, double *theta_f, void *work,
                                   void *hip_stream);
/* n_steps explicit steps by Algorithm 4 per stage (theta_f by Algorithm 3, phi = U(u_f) theta_f
 * by kbin, rhs = M phi by SpMV, the stage combination by kbin): forward Euler as printed, or
 * SSP-RK3 with the same stage combination as fl_rk_steps.  theta updated in place. */
fl_status fl_algebraic_rk_steps(const fl_algebraic *alg, int limiter, int scheme, double dt,
                                int64_t n_steps, double *theta, const double *u_f, void *work,
                                void *hip_stream);

/* Process-wide launch tuning, read by later launches of the single-problem kernels:
 *   FL_OPT_XCD_REMAP  M in 2 .. 65536 (default 32): each XCD takes runs of M consecutive
 *                     256-cell tiles (grid padded to a multiple of 8 M), so the tiles sharing one
 *                     L2 are neighbours; 0: workgroups take cells in launch order (the hardware
 *                     deals consecutive workgroups to the 8 XCDs in turn); 1: the grid is padded
 *                     to a multiple of 8 and each XCD gets a contiguous eighth of the cells.
 *                     Results are bit-identical for every value.
 *   FL_OPT_SLOT_VELOCITY  1 (default): fl_rk_steps, fl_rk_steps_scaled and fl_rk_steps_store
 *                     calls of two or more steps on a mesh of the fused path first write one
 *                     16-byte record per cell slot (other cell, far-upwind cell, signed face rate
 *                     E a_f u_f) into their workspace and read only those records and theta;
 *                     0: every stage reads the mesh's slot tables and gathers u_f through the
 *                     face index.  Results are bit-identical either way (for time-dependent
 *                     velocity on meshes with face areas, up to the rounding of one product).
 *   FL_OPT_LDS_STAGE  1 (default): those multi-step calls, on meshes with tile tables
 *                     (fl_mesh_info_t.tile_cells > 0) and with (tile_cells + max_halo + 1) *
 *                     min(S, 2) * 8 bytes of LDS per tile at most 64 KiB, stage each tile's
 *                     theta and its halo in LDS (two scalars at a time) and read the per-call
 *                     rates E a_f u_f (8 bytes per slot) instead of the 16-byte records; the
 *                     adjoint stages (fl_convect_adjoint, fl_rk_step_adjoint) likewise stage theta
 *                     and lambda of all S scalars (and the cell volumes, where they differ)
 *                     where (tile_cells + max_halo + 1) * (2 S [+ 1]) * 8 bytes fit; 0: the records
 *                     and global gathers.  Results are bit-identical.
 *   FL_OPT_CHECK_FINITE  0 (default) or 1: the compute entry points (fl_convect_apply,
 *                     fl_rk_step(s), fl_rk_steps_scaled, fl_rk_step(s)_store, fl_convect_adjoint,
 *                     fl_rk_step_adjoint) first scan their floating-point inputs (theta or the
 *                     stage states, u_f, rhs_bar or lambda on the device; dt and u_scale on the
 *                     host) and return FL_E_NONFINITE, with nothing enqueued, if one holds a NaN
 *                     or an infinity.  The scan synchronises the caller's stream, so calls made
 *                     with the check on cannot be captured into a graph.  Batches and the
 *                     algebraic path are not checked.
 *   FL_OPT_FWD_RATES  1 (default): on meshes whose opposite-face pairs line up from cell to
 *                     cell (lattice meshes: the neighbour across a cell's slot k holds the shared
 *                     face in its slot k ^ 1), the LDS-staged stages of multi-step calls read the
 *                     per-call rates of each cell's forward faces only (every face once, half the
 *                     rate bytes) and take a backward face's rate from the neighbour that holds it
 *                     as its forward face, staged in LDS with the tile (and, for the tile's halo
 *                     entries, with their theta); 0: a rate per slot.  Likewise the tables of fl_adjoint_rates hold
 *                     one rate per face or two per slot (a table is read back under the setting
 *                     it was written with).  Results are bit-identical.
 *   FL_OPT_FACE_SHARE  1 (default): where FL_OPT_FWD_RATES applies and S <= 2, the reverse
 *                     stages of fl_rk_steps_adjoint evaluate each face a tile needs once and pass
 *                     its terms to the cells that need them through LDS (a face's limiter
 *                     partials otherwise come out three times: for both its cells and for its
 *                     far-upwind cell); 0: each cell evaluates every face it needs.  Every cell
 *                     adds the same terms in the same order either way: results are
 *                     bit-identical.
 * Returns FL_E_INVALID for an unknown option or value.  Not synchronised with launches running
 * on other threads. */
enum { FL_OPT_XCD_REMAP = 1, FL_OPT_SLOT_VELOCITY = 2, FL_OPT_LDS_STAGE = 3,
       FL_OPT_CHECK_FINITE = 4, FL_OPT_FWD_RATES = 5, FL_OPT_FACE_SHARE = 6 };
fl_status fl_set_option(int option, int value);

const char *fl_status_str(fl_status status);
const char *fl_last_error(void);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): fl_rk_steps with its workspace in a fixed device
 * array of FL_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it runs on until
 * the process ends, instead of a caller-provided buffer.  The caller still passes theta and u_f.
 * Returns FL_E_INVALID, with nothing enqueued, when fl_rk_workspace_bytes(mesh, scheme,
 * n_scalars) exceeds that size (about 1.2 M hexahedral cells at one scalar), and allocates
 * nothing.  All calls on one GPU share its array, so calls that may overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller.  Results are bit-identical to
 * fl_rk_steps. */
#define FL_NOALLOC_SCRATCH_BYTES (128u << 20)
fl_status fl_rk_steps_noalloc(const fl_mesh *mesh, int limiter, int scheme, double dt,
                              int n_scalars, int64_t n_steps, double *theta, const double *u_f,
                              void *hip_stream);

/* Test hook: runs the device face selection for u_f (device [n_faces]) and copies, per face,
 * (C, D, U) to cdu (host int32 [n_faces][3]).  Synchronises the stream. */
fl_status fl_debug_select(const fl_mesh *mesh, const double *u_f, int32_t *cdu, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* FLUXLIM_H */
