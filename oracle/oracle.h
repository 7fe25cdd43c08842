/*
 * oracle.h -- plain, slow FP64 CPU oracle of the flux-limited convective operator of
 * Valle et al., "On the implementation of flux limiters in algebraic frameworks".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this library.  The HIP library never includes, links or calls it, and it
 * shares no code with the HIP library.
 *
 * Conventions (Section 2 of the paper): face f joins cells own = fc[2f] and nbr = fc[2f+1];
 * its unit normal nrm[3f..3f+2] points from own into nbr; the oriented incidence is
 * E[f][nbr] = +1, E[f][own] = -1.  u[f] is the normal velocity along that normal.  Cell fields
 * hold S scalars per cell, scalar index fastest ([C][S]).
 *
 * Operator (Section 3, Sweby form and gradient ratio; Section 4.1, Algorithm 4):
 *   C, D : upwind and downwind cells of f, chosen by u_f > 0 (else the flow is taken as
 *          running from nbr to own, so u_f <= 0, -0.0 included, picks C = nbr);
 *   d_u  = theta_D - theta_C;
 *   d_U  = sum over the faces j != f of C of w_j (theta_C - theta_other(j)), where the
 *          projection weight w_j = s_f (n_f . t_j), s_f = +1 if u_f > 0 else -1, and t_j is
 *          n_j oriented from the other cell of j into C (upstream-difference projection of
 *          Section 3.1 with the velocity-sign correction; on hexahedra w_j is 1 for the face
 *          opposite f and 0 for the four side faces, giving d_U = theta_C - theta_U);
 *   theta_f = theta_C                           if d_u == 0,
 *           = theta_C + psi(d_U/d_u) d_u / 2    otherwise;
 *   rhs_c = (sum_{f: nbr_f=c} a_f u_f theta_f - sum_{f: own_f=c} a_f u_f theta_f) / V_c,
 *          summed over the faces of c in ascending face index.
 *
 * Boundary faces (a reading: the paper states the operators on the mesh's graph and notes that
 * its cell-to-face shift handles a face with a single cell by copying that cell, Section 2):
 * fc[2f+1] == -1 marks a face with one cell, own = fc[2f], its normal pointing out of the mesh.
 * Beyond it lies an exterior cell with no other faces whose value is the caller's inflow value
 * of f where the flow enters (u_f <= 0) and inflow values were given (orc_mesh_set_inflow), and
 * the value of own otherwise.  With that cell the rules above apply unchanged: an outflow face
 * takes theta_own (d_u = 0), an inflow face the exterior value (d_U = 0 upwind of it: r = 0),
 * and a boundary face among C's other faces adds w_j (theta_C - exterior value) to d_U.  Each
 * boundary flux a_f u_f theta_f leaves or enters its one cell.
 */
#ifndef FLUXLIM_ORACLE_H
#define FLUXLIM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* psi = 0 is first-order upwind (the paper's F = -1/2); psi = 1 is central differencing
 * (the paper's F = 0). */
enum { ORC_UPWIND = 0, ORC_MINMOD = 1, ORC_VANLEER = 2, ORC_VANALBADA = 3, ORC_SUPERBEE = 4,
       ORC_SMART = 5, ORC_CENTRAL = 6 };
enum { ORC_EULER = 1, ORC_SSPRK3 = 3 };

/* |r| above this is evaluated as the limiter's value at +-infinity. */
#define ORC_R_BIG 1.0e18

typedef struct orc_mesh orc_mesh;

/* Builds the cell -> faces lists.  Keeps the caller's arrays by pointer (they must outlive the
 * mesh).  Returns NULL on a face index out of range or own == nbr (nbr == -1 marks a boundary
 * face).  The derivative functions below cover boundary faces and face distances too: an
 * inflow value is a constant, an exterior that repeats its face's own cell passes that cell's
 * tangent and cotangent on. */
orc_mesh *orc_mesh_new(int64_t n_cells, int64_t n_faces, const int32_t *face_cells,
                       const double *face_normal, const double *face_area,
                       const double *cell_volume);
void orc_mesh_free(orc_mesh *m);
int64_t orc_cell_degree(const orc_mesh *m, int64_t c);
int64_t orc_boundary_faces(const orc_mesh *m);
/* Distance between the cells across each face ([F], kept by pointer; on a boundary face the
 * distance to the exterior cell), or NULL: d_U = d_f sum_j w_j (theta_C - theta_j) / d_j
 * (Algorithm 1D's distance ratio, Algorithm UNS's weighted upstream difference).  Without
 * distances every ratio d_f / d_j is taken as 1.  The derivative functions ignore them. */
void orc_mesh_set_distances(orc_mesh *m, const double *dist);
/* Inflow values of the boundary faces ([F][S], read at boundary faces only; kept by pointer),
 * or NULL: the exterior then repeats the cell's value on every boundary face. */
void orc_mesh_set_inflow(orc_mesh *m, const double *inflow, int S);

/* Limiter psi(r) and its derivative on the branch that the evaluation takes. */
double orc_psi(int limiter, double r);
double orc_dpsi(int limiter, double r);
double orc_psi_inf(int limiter, int sign);

/* Per face: C, D and the single far-upwind cell U (the other cell of the unique face of C with
 * a nonzero projection weight), or -2 when there is no such unique face. */
void orc_select(const orc_mesh *m, const double *u, int32_t *cdu);
/* Projection weights of face f on the side of cell C, one per face of C in ascending order
 * (0 for f itself); returns how many were written (<= cap). */
int orc_side_weights(const orc_mesh *m, int64_t f, int side_nbr, double *w, int32_t *faces,
                     int cap);

void orc_face_values(const orc_mesh *m, int limiter, int S, const double *theta, const double *u,
                     double *theta_f);
void orc_rhs(const orc_mesh *m, int limiter, int S, const double *theta, const double *u,
             double *rhs);
void orc_rhs_cells(const orc_mesh *m, int limiter, int S, const double *theta, const double *u,
                   int64_t n, const int64_t *cells, double *rhs);

/* In-place time integration: scheme ORC_EULER or ORC_SSPRK3, nsteps steps of size dt. */
int orc_run(const orc_mesh *m, int limiter, int scheme, double dt, int S, int64_t nsteps,
            double *theta, const double *u);

/* As orc_run with the time-dependent velocity u(t) = s(t) u (Section 4.1's deformation flow):
 * scales[i * stages + j] is s at stage j of step i (stages: Euler 1, SSP-RK3 3). */
int orc_run_scaled(const orc_mesh *m, int limiter, int scheme, double dt, int S, int64_t nsteps,
                   double *theta, const double *u, const double *scales);

/* Face values theta_f and their tangent along dtheta (u held fixed), [F][S] each. */
void orc_face_values_jvp(const orc_mesh *m, int limiter, int S, const double *theta,
                         const double *u, const double *dtheta, double *theta_f,
                         double *dtheta_f);
/* Tangent and adjoint of rhs = L(theta, u). */
void orc_rhs_jvp(const orc_mesh *m, int limiter, int S, const double *theta, const double *u,
                 const double *dtheta, const double *du, double *drhs);
void orc_rhs_vjp(const orc_mesh *m, int limiter, int S, const double *theta, const double *u,
                 const double *lam, double *theta_bar, double *u_bar);

/* Tangent of a whole run: theta (in/out) and dtheta (in/out) for a fixed du. */
int orc_run_tangent(const orc_mesh *m, int limiter, int scheme, double dt, int S, int64_t nsteps,
                    double *theta, double *dtheta, const double *u, const double *du);
/* Reverse sweep of a whole run storing every stage state: given theta0 and the cotangent of
 * the final state, writes theta0_bar and u_bar (both overwritten). */
int orc_run_adjoint(const orc_mesh *m, int limiter, int scheme, double dt, int S, int64_t nsteps,
                    const double *theta0, const double *u, const double *theta_bar_final,
                    double *theta0_bar, double *u_bar);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
