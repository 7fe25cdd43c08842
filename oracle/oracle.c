/*
 * oracle.c -- plain, slow FP64 CPU oracle of the flux-limited convective operator.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the benchmark's CPU
 * baseline; never by the HIP library.  Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math,
 * no FMA contraction).  OpenMP loops use a static schedule and every output element is written
 * by exactly one thread in a fixed order, so results do not depend on the thread count.
 *
 * Every function follows the paper's definitions directly (see oracle.h for the conventions):
 *   - face selection by the velocity sign matrix Q(u_f) (Section 3.1, sign equation and the
 *     signxty kernel of Table 1);
 *   - the face difference d_u (Section 3.1, face-difference equation);
 *   - the upstream difference d_U by visiting the faces of the upwind cell and projecting their
 *     differences on the face normal (Algorithm UNS of Section 3.3 and the upstream-difference
 *     equation of Section 3.1; see oracle.h for the orientation reading);
 *   - the gradient ratio r = d_U / d_u (Section 3, gradient-ratio equation);
 *   - the limited face value of the Sweby form theta_f = theta_C + psi(r)(theta_D - theta_C)/2
 *     (Section 3, first equation);
 *   - the advection update theta^{n+1} = theta^n + dt M U(u_f) theta_f (Algorithm 4), and its
 *     three-stage strong-stability-preserving Runge-Kutta extension.
 * Nothing is fused, blocked or precomputed beyond the cell -> faces lists.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct orc_mesh {
    int64_t nc, nf;
    const int32_t *fc;
    const double *nrm;
    const double *area;
    const double *vol;
    int64_t *cptr; /* [nc+1] */
    int64_t *cidx; /* faces of each cell, ascending (a boundary face in its one cell's list) */
    int64_t n_boundary;
    const double *inflow; /* [nf][inflow_S] or NULL (see exterior_value) */
    int inflow_S;
    const double *dist;   /* [nf] distance between the cells across each face, or NULL */
};

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

orc_mesh *orc_mesh_new(int64_t nc, int64_t nf, const int32_t *fc, const double *nrm,
                       const double *area, const double *vol) {
    if (nc <= 0 || nf <= 0 || !fc || !nrm || !area || !vol) return NULL;
    int64_t nb = 0;
    for (int64_t f = 0; f < nf; ++f) {
        int64_t a = fc[2 * f], b = fc[2 * f + 1];
        if (b == -1 && a >= 0 && a < nc) { /* boundary face: own is its cell */
            nb++;
            continue;
        }
        if (a < 0 || a >= nc || b < 0 || b >= nc || a == b) return NULL;
    }
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    m->nc = nc; m->nf = nf; m->fc = fc; m->nrm = nrm; m->area = area; m->vol = vol;
    m->n_boundary = nb;
    m->cptr = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    m->cidx = (int64_t *)malloc((size_t)(2 * nf) * sizeof(int64_t));
    for (int64_t f = 0; f < nf; ++f) {
        m->cptr[fc[2 * f] + 1]++;
        if (fc[2 * f + 1] >= 0) m->cptr[fc[2 * f + 1] + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) m->cptr[c + 1] += m->cptr[c];
    int64_t *fill = (int64_t *)malloc((size_t)nc * sizeof(int64_t));
    memcpy(fill, m->cptr, (size_t)nc * sizeof(int64_t));
    for (int64_t f = 0; f < nf; ++f) { /* ascending f => ascending lists */
        m->cidx[fill[fc[2 * f]]++] = f;
        if (fc[2 * f + 1] >= 0) m->cidx[fill[fc[2 * f + 1]]++] = f;
    }
    free(fill);
    return m;
}

int64_t orc_boundary_faces(const orc_mesh *m) { return m->n_boundary; }

void orc_mesh_set_distances(orc_mesh *m, const double *dist) { m->dist = dist; }

void orc_mesh_set_inflow(orc_mesh *m, const double *inflow, int S) {
    m->inflow = inflow;
    m->inflow_S = inflow ? S : 0;
}

void orc_mesh_free(orc_mesh *m) {
    if (!m) return;
    free(m->cptr);
    free(m->cidx);
    free(m);
}

int64_t orc_cell_degree(const orc_mesh *m, int64_t c) { return m->cptr[c + 1] - m->cptr[c]; }

/* ------------------------------------------------------------------------------------------
 * Limiters psi(r).  Superbee is the paper's (Table 1, superbeexty: F = (psi - 1)/2).  The
 * others are the standard forms of Sweby's family: minmod max(0, min(1, r)); van Leer
 * (r + |r|)/(1 + |r|); van Albada (r^2 + r)/(r^2 + 1), not clipped; SMART
 * max(0, min(2r, 1/4 + 3r/4, 4)); first-order upwind psi = 0; central differencing psi = 1.
 * ------------------------------------------------------------------------------------------ */
double orc_psi_inf(int lim, int sign) {
    if (sign > 0) {
        switch (lim) {
            case ORC_MINMOD: return 1.0;
            case ORC_VANLEER: return 2.0;
            case ORC_VANALBADA: return 1.0;
            case ORC_SUPERBEE: return 2.0;
            case ORC_SMART: return 4.0;
            case ORC_CENTRAL: return 1.0;
            default: return 0.0;
        }
    }
    return (lim == ORC_VANALBADA || lim == ORC_CENTRAL) ? 1.0 : 0.0;
}

double orc_psi(int lim, double r) {
    if (!(fabs(r) <= ORC_R_BIG)) return orc_psi_inf(lim, r > 0 ? 1 : -1);
    switch (lim) {
        case ORC_UPWIND: return 0.0;
        case ORC_MINMOD: return fmax(0.0, fmin(1.0, r));
        case ORC_VANLEER: return (r + fabs(r)) / (1.0 + fabs(r));
        case ORC_VANALBADA: return (r * r + r) / (r * r + 1.0);
        case ORC_SUPERBEE: return fmax(0.0, fmax(fmin(1.0, 2.0 * r), fmin(r, 2.0)));
        case ORC_SMART: return fmax(0.0, fmin(fmin(2.0 * r, 0.25 + 0.75 * r), 4.0));
        case ORC_CENTRAL: return 1.0;
        default: return 0.0;
    }
}

/* Derivative on the evaluated branch; at a break point the branch of the left-closed interval
 * listed first below is used. */
double orc_dpsi(int lim, double r) {
    if (!(fabs(r) <= ORC_R_BIG)) return 0.0;
    switch (lim) {
        case ORC_MINMOD: return (r > 0.0 && r < 1.0) ? 1.0 : 0.0;
        case ORC_VANLEER: return r > 0.0 ? 2.0 / ((1.0 + r) * (1.0 + r)) : 0.0;
        case ORC_VANALBADA: {
            double q = r * r + 1.0;
            return (1.0 + 2.0 * r - r * r) / (q * q);
        }
        case ORC_SUPERBEE:
            if (r <= 0.0) return 0.0;
            if (r <= 0.5) return 2.0;
            if (r <= 1.0) return 0.0;
            if (r <= 2.0) return 1.0;
            return 0.0;
        case ORC_SMART:
            if (r <= 0.0) return 0.0;
            if (r <= 0.2) return 2.0;
            if (r <= 5.0) return 0.75;
            return 0.0;
        default: return 0.0;
    }
}

/* ------------------------------------------------------------------------------------------
 * Face selection and projection weights.
 * ------------------------------------------------------------------------------------------ */
/* The cell across face j from c: -1 beyond a boundary face. */
static inline int64_t other_cell(const orc_mesh *m, int64_t j, int64_t c) {
    return m->fc[2 * j] == c ? m->fc[2 * j + 1] : m->fc[2 * j];
}

/* Value of the exterior beyond boundary face j, for scalar k.  The flow enters through j where
 * u_j <= 0 (the normal points out of the mesh): there the exterior holds the caller's inflow
 * value, if any; everywhere else (outflow, or no inflow values) it repeats the value of j's own
 * cell, as the cell-to-face shift of Section 2 does on a face with a single cell. */
static inline double exterior_value(const orc_mesh *m, int S, const double *th, const double *u,
                                    int64_t j, int k) {
    if (m->inflow && !(u[j] > 0.0)) return m->inflow[j * S + k];
    return th[m->fc[2 * j] * S + k];
}

/* theta of cell c (c >= 0) or of the exterior beyond boundary face j (c == -1). */
static inline double value_at(const orc_mesh *m, int S, const double *th, const double *u,
                              int64_t c, int64_t j, int k) {
    return c >= 0 ? th[c * S + k] : exterior_value(m, S, th, u, j, k);
}

/* Weight of face j of cell C for face f with flow sign s: s (n_f . t_j), t_j = n_j oriented
 * from other(j, C) into C. */
static inline double proj_weight(const orc_mesh *m, int64_t f, int64_t j, int64_t C, double s) {
    const double *nf = m->nrm + 3 * f, *nj = m->nrm + 3 * j;
    double dot = nf[0] * nj[0] + nf[1] * nj[1] + nf[2] * nj[2];
    double t = (m->fc[2 * j + 1] == C) ? 1.0 : -1.0;
    return s * (t * dot);
}

int orc_side_weights(const orc_mesh *m, int64_t f, int side_nbr, double *w, int32_t *faces,
                     int cap) {
    int64_t C = side_nbr ? m->fc[2 * f + 1] : m->fc[2 * f];
    double s = side_nbr ? -1.0 : 1.0;
    int k = 0;
    if (C < 0) return 0;
    for (int64_t p = m->cptr[C]; p < m->cptr[C + 1] && k < cap; ++p, ++k) {
        int64_t j = m->cidx[p];
        faces[k] = (int32_t)j;
        w[k] = (j == f) ? 0.0 : proj_weight(m, f, j, C, s);
    }
    return k;
}

/* Q(u_f): +1 if u_f > 0 else -1 (Table 1, signxty); C is own for +1, nbr for -1. */
typedef struct {
    int64_t C, D;
    double s;
} face_sel;

static inline face_sel select_face(const orc_mesh *m, const double *u, int64_t f) {
    face_sel fs;
    fs.s = (u[f] > 0.0) ? 1.0 : -1.0;
    fs.C = fs.s > 0 ? m->fc[2 * f] : m->fc[2 * f + 1];
    fs.D = fs.s > 0 ? m->fc[2 * f + 1] : m->fc[2 * f];
    return fs;
}

void orc_select(const orc_mesh *m, const double *u, int32_t *cdu) {
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < m->nf; ++f) {
        face_sel fs = select_face(m, u, f);
        int64_t U = -2;
        int nonzero = 0;
        for (int64_t p = fs.C >= 0 ? m->cptr[fs.C] : 0; fs.C >= 0 && p < m->cptr[fs.C + 1]; ++p) {
            int64_t j = m->cidx[p];
            if (j == f) continue;
            if (proj_weight(m, f, j, fs.C, fs.s) != 0.0) {
                nonzero++;
                U = other_cell(m, j, fs.C);
            }
        }
        cdu[3 * f] = (int32_t)fs.C;
        cdu[3 * f + 1] = (int32_t)fs.D;
        cdu[3 * f + 2] = (nonzero == 1) ? (int32_t)U : -2;
    }
}

/* The exterior upwind of an inflow face has no other faces: d_U = 0 there.  With face
 * distances (Algorithm 1D's d_i / d_U and Algorithm UNS), each projected difference is divided
 * by the distance d_j across its face and the sum is multiplied by the face's own distance d_f,
 * so that r = d_U / d_u equals Algorithm UNS's Delta_U / ((theta_D - theta_C) / d_f). */
static double upstream_difference(const orc_mesh *m, int S, const double *th, const double *u,
                                  int64_t f, face_sel fs, int k) {
    double dU = 0.0;
    if (fs.C < 0) return dU;
    double tC = th[fs.C * S + k];
    for (int64_t p = m->cptr[fs.C]; p < m->cptr[fs.C + 1]; ++p) {
        int64_t j = m->cidx[p];
        if (j == f) continue;
        double w = proj_weight(m, f, j, fs.C, fs.s);
        double diff = tC - value_at(m, S, th, u, other_cell(m, j, fs.C), j, k);
        if (m->dist) dU += w * diff / m->dist[j];
        else dU += w * diff;
    }
    if (m->dist) dU *= m->dist[f];
    return dU;
}

/* theta_f = theta_C + g(d_U, d_u), g(a, b) = psi(a/b) b / 2, and its partials ga = dg/da,
 * gb = dg/db.  Where d_u == 0, g vanishes for every d_U, so ga = 0; gb is the derivative along
 * d_u > 0, the limit of g(a, b)/b as b -> 0+: psi(+-inf)/2 with the sign of d_U, and psi(0)/2
 * where d_U is also 0 (g(0, b) = psi(0) b / 2: 0 for every limiter but central differencing).
 * Where |r| is taken as infinite, psi is constant, so ga = 0 and gb = psi(+-inf)/2. */
static double limited_value(int lim, double tC, double dU, double du, double *ga, double *gb) {
    if (du == 0.0) {
        if (ga) *ga = 0.0;
        if (gb) *gb = (dU == 0.0) ? 0.5 * orc_psi(lim, 0.0)
                                  : 0.5 * orc_psi_inf(lim, dU > 0 ? 1 : -1);
        return tC;
    }
    double r = dU / du;
    double psi = orc_psi(lim, r);
    if (ga || gb) {
        if (!(fabs(r) <= ORC_R_BIG)) {
            if (ga) *ga = 0.0;
            if (gb) *gb = 0.5 * psi;
        } else {
            double dp = orc_dpsi(lim, r);
            if (ga) *ga = 0.5 * dp;
            if (gb) *gb = 0.5 * (psi - r * dp);
        }
    }
    return tC + 0.5 * psi * du;
}

static double face_value(const orc_mesh *m, int lim, int S, const double *th, const double *u,
                         int64_t f, int k) {
    face_sel fs = select_face(m, u, f);
    double tC = value_at(m, S, th, u, fs.C, f, k), tD = value_at(m, S, th, u, fs.D, f, k);
    double du = tD - tC;
    double dU = upstream_difference(m, S, th, u, f, fs, k);
    return limited_value(lim, tC, dU, du, NULL, NULL);
}

void orc_face_values(const orc_mesh *m, int lim, int S, const double *th, const double *u,
                     double *tf) {
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < m->nf; ++f)
        for (int k = 0; k < S; ++k) tf[f * S + k] = face_value(m, lim, S, th, u, f, k);
}

/* Divergence of the face fluxes a_f u_f theta_f for cell c, ascending face order. */
static void cell_sum(const orc_mesh *m, int S, const double *u, const double *tf, int64_t c,
                     double *out) {
    for (int k = 0; k < S; ++k) {
        double acc = 0.0;
        for (int64_t p = m->cptr[c]; p < m->cptr[c + 1]; ++p) {
            int64_t f = m->cidx[p];
            double phi = m->area[f] * u[f] * tf[f * S + k];
            if (m->fc[2 * f + 1] == c) acc += phi;
            else acc -= phi;
        }
        out[k] = acc / m->vol[c];
    }
}

void orc_rhs(const orc_mesh *m, int lim, int S, const double *th, const double *u, double *rhs) {
    double *tf = (double *)malloc((size_t)(m->nf * S) * sizeof(double));
    orc_face_values(m, lim, S, th, u, tf);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < m->nc; ++c) cell_sum(m, S, u, tf, c, rhs + c * S);
    free(tf);
}

void orc_rhs_cells(const orc_mesh *m, int lim, int S, const double *th, const double *u,
                   int64_t n, const int64_t *cells, double *rhs) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = cells[i];
        for (int k = 0; k < S; ++k) {
            double acc = 0.0;
            for (int64_t p = m->cptr[c]; p < m->cptr[c + 1]; ++p) {
                int64_t f = m->cidx[p];
                double phi = m->area[f] * u[f] * face_value(m, lim, S, th, u, f, k);
                if (m->fc[2 * f + 1] == c) acc += phi;
                else acc -= phi;
            }
            rhs[i * S + k] = acc / m->vol[c];
        }
    }
}

/* ------------------------------------------------------------------------------------------
 * Time integration.  One stage: out = a theta_n + b (theta_s + dt L(theta_s)).
 * Euler: (a, b) = (0, 1).  SSP-RK3 (Shu-Osher): (0, 1), (3/4, 1/4), (1/3, 2/3).
 * ------------------------------------------------------------------------------------------ */
static const double RK3_A[3] = {0.0, 0.75, 1.0 / 3.0};
static const double RK3_B[3] = {1.0, 0.25, 2.0 / 3.0};

static void stage(const orc_mesh *m, int lim, int S, double dt, double a, double b,
                  const double *ts, const double *tn, const double *u, double *rhs, double *out) {
    orc_rhs(m, lim, S, ts, u, rhs);
    int64_t n = m->nc * S;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = a * tn[i] + b * (ts[i] + dt * rhs[i]);
}

int orc_run(const orc_mesh *m, int lim, int scheme, double dt, int S, int64_t nsteps,
            double *th, const double *u) {
    if (scheme != ORC_EULER && scheme != ORC_SSPRK3) return -1;
    size_t n = (size_t)(m->nc * S);
    double *rhs = (double *)malloc(n * sizeof(double));
    double *t1 = (double *)malloc(n * sizeof(double));
    double *t2 = (double *)malloc(n * sizeof(double));
    for (int64_t it = 0; it < nsteps; ++it) {
        if (scheme == ORC_EULER) {
            stage(m, lim, S, dt, 0.0, 1.0, th, th, u, rhs, t1);
            memcpy(th, t1, n * sizeof(double));
        } else {
            stage(m, lim, S, dt, RK3_A[0], RK3_B[0], th, th, u, rhs, t1);
            stage(m, lim, S, dt, RK3_A[1], RK3_B[1], t1, th, u, rhs, t2);
            stage(m, lim, S, dt, RK3_A[2], RK3_B[2], t2, th, u, rhs, t1);
            memcpy(th, t1, n * sizeof(double));
        }
    }
    free(rhs); free(t1); free(t2);
    return 0;
}

/* Time-dependent velocity u(t) = s(t) u: scales[i * stages + j] is s at stage j of step i.
 * Each stage forms the face velocities s u and applies the same stage as orc_run. */
int orc_run_scaled(const orc_mesh *m, int lim, int scheme, double dt, int S, int64_t nsteps,
                   double *th, const double *u, const double *scales) {
    if (scheme != ORC_EULER && scheme != ORC_SSPRK3) return -1;
    int ns = scheme == ORC_EULER ? 1 : 3;
    size_t n = (size_t)(m->nc * S);
    double *rhs = (double *)malloc(n * sizeof(double));
    double *t1 = (double *)malloc(n * sizeof(double));
    double *t2 = (double *)malloc(n * sizeof(double));
    double *us = (double *)malloc((size_t)m->nf * sizeof(double));
    for (int64_t it = 0; it < nsteps; ++it) {
        for (int st = 0; st < ns; ++st) {
            double s = scales[it * ns + st];
            for (int64_t f = 0; f < m->nf; ++f) us[f] = s * u[f];
            if (ns == 1) stage(m, lim, S, dt, 0.0, 1.0, th, th, us, rhs, t1);
            else if (st == 0) stage(m, lim, S, dt, RK3_A[0], RK3_B[0], th, th, us, rhs, t1);
            else if (st == 1) stage(m, lim, S, dt, RK3_A[1], RK3_B[1], t1, th, us, rhs, t2);
            else stage(m, lim, S, dt, RK3_A[2], RK3_B[2], t2, th, us, rhs, t1);
        }
        memcpy(th, t1, n * sizeof(double));
    }
    free(rhs); free(t1); free(t2); free(us);
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Tangent (forward mode) of L.  theta_f depends on theta_C, theta_D and the far cells through
 * d_U and d_u; the selection Q(u) is piecewise constant and contributes nothing.  The exterior
 * beyond a boundary face holds a constant inflow value (tangent 0) or repeats its face's own
 * cell (that cell's tangent).
 * ------------------------------------------------------------------------------------------ */
static inline double tangent_at(const orc_mesh *m, int S, const double *dth, const double *u,
                                int64_t c, int64_t j, int k) {
    if (c >= 0) return dth[c * S + k];
    if (m->inflow && !(u[j] > 0.0)) return 0.0;
    return dth[m->fc[2 * j] * S + k];
}

/* The tangent of d_U: the upstream difference is linear in the values it reads. */
static double upstream_difference_tangent(const orc_mesh *m, int S, const double *dth,
                                          const double *u, int64_t f, face_sel fs, int k) {
    double ddU = 0.0;
    if (fs.C < 0) return ddU;
    double dC = dth[fs.C * S + k];
    for (int64_t p = m->cptr[fs.C]; p < m->cptr[fs.C + 1]; ++p) {
        int64_t j = m->cidx[p];
        if (j == f) continue;
        double w = proj_weight(m, f, j, fs.C, fs.s);
        double diff = dC - tangent_at(m, S, dth, u, other_cell(m, j, fs.C), j, k);
        if (m->dist) ddU += w * diff / m->dist[j];
        else ddU += w * diff;
    }
    if (m->dist) ddU *= m->dist[f];
    return ddU;
}

static double face_value_tangent(const orc_mesh *m, int lim, int S, const double *th,
                                 const double *dth, const double *u, int64_t f, int k,
                                 double *dtf) {
    face_sel fs = select_face(m, u, f);
    double tC = value_at(m, S, th, u, fs.C, f, k), tD = value_at(m, S, th, u, fs.D, f, k);
    double dC = tangent_at(m, S, dth, u, fs.C, f, k), dD = tangent_at(m, S, dth, u, fs.D, f, k);
    double du = tD - tC, ddu = dD - dC;
    double dU = upstream_difference(m, S, th, u, f, fs, k);
    double ddU = upstream_difference_tangent(m, S, dth, u, f, fs, k);
    double ga, gb;
    double tf = limited_value(lim, tC, dU, du, &ga, &gb);
    *dtf = dC + ga * ddU + gb * ddu;
    return tf;
}

void orc_face_values_jvp(const orc_mesh *m, int lim, int S, const double *th, const double *u,
                         const double *dth, double *tf, double *dtf) {
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < m->nf; ++f)
        for (int k = 0; k < S; ++k)
            tf[f * S + k] = face_value_tangent(m, lim, S, th, dth, u, f, k, &dtf[f * S + k]);
}

void orc_rhs_jvp(const orc_mesh *m, int lim, int S, const double *th, const double *u,
                 const double *dth, const double *du, double *drhs) {
    double *dphi = (double *)malloc((size_t)(m->nf * S) * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < m->nf; ++f)
        for (int k = 0; k < S; ++k) {
            double dtf;
            double tf = face_value_tangent(m, lim, S, th, dth, u, f, k, &dtf);
            double dul = du ? du[f] : 0.0;
            dphi[f * S + k] = m->area[f] * (dul * tf + u[f] * dtf);
        }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < m->nc; ++c)
        for (int k = 0; k < S; ++k) {
            double acc = 0.0;
            for (int64_t p = m->cptr[c]; p < m->cptr[c + 1]; ++p) {
                int64_t f = m->cidx[p];
                if (m->fc[2 * f + 1] == c) acc += dphi[f * S + k];
                else acc -= dphi[f * S + k];
            }
            drhs[c * S + k] = acc / m->vol[c];
        }
    free(dphi);
}

/* ------------------------------------------------------------------------------------------
 * Adjoint (reverse mode) of L: theta_bar = J^T lam, u_bar = (dL/du)^T lam (both overwritten).
 * Serial scatter over faces: slow and plainly the transpose of the forward chain.  A cotangent
 * reaching the exterior beyond a boundary face goes to the face's own cell where the exterior
 * repeats it, and nowhere where it holds an inflow value.
 * ------------------------------------------------------------------------------------------ */
static inline void scatter_at(const orc_mesh *m, int S, double *tbar, const double *u, int64_t c,
                              int64_t j, int k, double v) {
    if (c >= 0) tbar[c * S + k] += v;
    else if (!(m->inflow && !(u[j] > 0.0))) tbar[m->fc[2 * j] * S + k] += v;
}

void orc_rhs_vjp(const orc_mesh *m, int lim, int S, const double *th, const double *u,
                 const double *lam, double *tbar, double *ubar) {
    memset(tbar, 0, (size_t)(m->nc * S) * sizeof(double));
    if (ubar) memset(ubar, 0, (size_t)m->nf * sizeof(double));
    for (int64_t f = 0; f < m->nf; ++f) {
        face_sel fs = select_face(m, u, f);
        int64_t own = m->fc[2 * f], nbr = m->fc[2 * f + 1];
        for (int k = 0; k < S; ++k) {
            /* rhs_nbr += a u tf / V_nbr, rhs_own -= a u tf / V_own (a boundary face has no nbr) */
            double mu = (nbr >= 0 ? lam[nbr * S + k] / m->vol[nbr] : 0.0) -
                        lam[own * S + k] / m->vol[own];
            double tC = value_at(m, S, th, u, fs.C, f, k), tD = value_at(m, S, th, u, fs.D, f, k);
            double du = tD - tC;
            double dU = upstream_difference(m, S, th, u, f, fs, k);
            double ga, gb;
            double tf = limited_value(lim, tC, dU, du, &ga, &gb);
            if (ubar) ubar[f] += m->area[f] * tf * mu;
            double z = m->area[f] * u[f] * mu; /* cotangent of theta_f */
            /* theta_f = theta_C + g(d_U, d_u) */
            scatter_at(m, S, tbar, u, fs.C, f, k, z);
            /* d_u = theta_D - theta_C */
            scatter_at(m, S, tbar, u, fs.D, f, k, z * gb);
            scatter_at(m, S, tbar, u, fs.C, f, k, -z * gb);
            /* d_U = d_f sum_j w_j (theta_C - theta_other(j)) / d_j (no distances: d = 1) */
            if (fs.C < 0) continue;
            for (int64_t p = m->cptr[fs.C]; p < m->cptr[fs.C + 1]; ++p) {
                int64_t j = m->cidx[p];
                if (j == f) continue;
                double w = proj_weight(m, f, j, fs.C, fs.s);
                if (m->dist) w = w / m->dist[j] * m->dist[f];
                int64_t o = other_cell(m, j, fs.C);
                tbar[fs.C * S + k] += z * ga * w;
                scatter_at(m, S, tbar, u, o, j, k, -z * ga * w);
            }
        }
    }
}

int orc_run_tangent(const orc_mesh *m, int lim, int scheme, double dt, int S, int64_t nsteps,
                    double *th, double *dth, const double *u, const double *du) {
    if (scheme != ORC_EULER && scheme != ORC_SSPRK3) return -1;
    size_t n = (size_t)(m->nc * S);
    int ns = scheme == ORC_EULER ? 1 : 3;
    double *rhs = (double *)malloc(n * sizeof(double));
    double *drhs = (double *)malloc(n * sizeof(double));
    double *ts = (double *)malloc(n * sizeof(double));
    double *dts = (double *)malloc(n * sizeof(double));
    double *to = (double *)malloc(n * sizeof(double));
    double *dto = (double *)malloc(n * sizeof(double));
    for (int64_t it = 0; it < nsteps; ++it) {
        memcpy(ts, th, n * sizeof(double));
        memcpy(dts, dth, n * sizeof(double));
        for (int st = 0; st < ns; ++st) {
            double a = ns == 1 ? 0.0 : RK3_A[st], b = ns == 1 ? 1.0 : RK3_B[st];
            orc_rhs(m, lim, S, ts, u, rhs);
            orc_rhs_jvp(m, lim, S, ts, u, dts, du, drhs);
            for (size_t i = 0; i < n; ++i) {
                to[i] = a * th[i] + b * (ts[i] + dt * rhs[i]);
                dto[i] = a * dth[i] + b * (dts[i] + dt * drhs[i]);
            }
            memcpy(ts, to, n * sizeof(double));
            memcpy(dts, dto, n * sizeof(double));
        }
        memcpy(th, ts, n * sizeof(double));
        memcpy(dth, dts, n * sizeof(double));
    }
    free(rhs); free(drhs); free(ts); free(dts); free(to); free(dto);
    return 0;
}

int orc_run_adjoint(const orc_mesh *m, int lim, int scheme, double dt, int S, int64_t nsteps,
                    const double *th0, const double *u, const double *tbar_final, double *th0_bar,
                    double *ubar) {
    if (scheme != ORC_EULER && scheme != ORC_SSPRK3) return -1;
    size_t n = (size_t)(m->nc * S);
    int ns = scheme == ORC_EULER ? 1 : 3;
    /* Forward pass storing every stage input: states[it][st] is the argument of L in stage st,
     * states[it][0] is also theta^n of that step. */
    double *states = (double *)malloc((size_t)nsteps * ns * n * sizeof(double));
    double *rhs = (double *)malloc(n * sizeof(double));
    double *cur = (double *)malloc(n * sizeof(double));
    double *nxt = (double *)malloc(n * sizeof(double));
    if (!states || !rhs || !cur || !nxt) {
        free(states); free(rhs); free(cur); free(nxt);
        return -4;
    }
    memcpy(cur, th0, n * sizeof(double));
    for (int64_t it = 0; it < nsteps; ++it) {
        const double *tn = states + ((size_t)it * ns) * n;
        memcpy(states + ((size_t)it * ns) * n, cur, n * sizeof(double));
        for (int st = 0; st < ns; ++st) {
            double a = ns == 1 ? 0.0 : RK3_A[st], b = ns == 1 ? 1.0 : RK3_B[st];
            const double *ts = states + ((size_t)it * ns + st) * n;
            orc_rhs(m, lim, S, ts, u, rhs);
            for (size_t i = 0; i < n; ++i) nxt[i] = a * tn[i] + b * (ts[i] + dt * rhs[i]);
            if (st + 1 < ns) memcpy(states + ((size_t)it * ns + st + 1) * n, nxt, n * sizeof(double));
        }
        memcpy(cur, nxt, n * sizeof(double));
    }
    /* Reverse pass.  Stage st: out = a tn + b (ts + dt L(ts)), so with out_bar = lam:
     * ts_bar += b (lam + dt J^T lam), tn_bar += a lam, u_bar += b dt (dL/du)^T lam. */
    double *lam = (double *)malloc(n * sizeof(double));
    double *lam_s = (double *)malloc(n * sizeof(double));
    double *tn_bar = (double *)malloc(n * sizeof(double));
    double *jt = (double *)malloc(n * sizeof(double));
    double *ub = (double *)malloc((size_t)m->nf * sizeof(double));
    memset(ubar, 0, (size_t)m->nf * sizeof(double));
    memcpy(lam, tbar_final, n * sizeof(double));
    for (int64_t it = nsteps - 1; it >= 0; --it) {
        memset(tn_bar, 0, n * sizeof(double));
        for (int st = ns - 1; st >= 0; --st) {
            double a = ns == 1 ? 0.0 : RK3_A[st], b = ns == 1 ? 1.0 : RK3_B[st];
            const double *ts = states + ((size_t)it * ns + st) * n;
            orc_rhs_vjp(m, lim, S, ts, u, lam, jt, ub);
            for (size_t i = 0; i < n; ++i) {
                tn_bar[i] += a * lam[i];
                lam_s[i] = b * (lam[i] + dt * jt[i]);
            }
            for (int64_t f = 0; f < m->nf; ++f) ubar[f] += b * dt * ub[f];
            memcpy(lam, lam_s, n * sizeof(double)); /* cotangent of this stage's input */
        }
        /* the first stage's input is theta^n itself */
        for (size_t i = 0; i < n; ++i) lam[i] += tn_bar[i];
    }
    memcpy(th0_bar, lam, n * sizeof(double));
    free(states); free(rhs); free(cur); free(nxt);
    free(lam); free(lam_s); free(tn_bar); free(jt); free(ub);
    return 0;
}
