// Face-path device routines: one face's flux (paired cells, or general cells with projected
// side lists and boundary faces) and one cell's divergence and stage combination.  The
// single-problem face and cell kernels and the batched ones call exactly these, so a problem
// advanced inside a batch gives the same bits as when advanced alone.
#pragma once

#include <hip/hip_runtime.h>

#include "fl_device.h"

namespace fl {
namespace dev {

template <int S>
__device__ __forceinline__ void load_cell(const double *__restrict__ th, int64_t c, double *v) {
#pragma unroll
    for (int k = 0; k < S; ++k) v[k] = th[c * S + k];
}

// Face f of a mesh with paired cells: {own, nbr, far_own, far_nbr} records; phi[f] = a_f u_f
// theta_f (u scaled by us, the time-dependent velocity factor; us = 1 is exact).
template <int S>
__device__ __forceinline__ void face_flux_one(int64_t f, const int4 *__restrict__ fc4,
                                              const double *__restrict__ u,
                                              const double *__restrict__ theta,
                                              const double *__restrict__ area, double area0,
                                              int lim, double *__restrict__ phi, double us) {
    const int4 e = fc4[f];
    const double uf = u[f] * us;
    const bool pos = uf > 0.0;
    const int64_t C = pos ? e.x : e.y;
    const int64_t D = pos ? e.y : e.x;
    const int64_t U = pos ? e.z : e.w;
    const double au = (area ? area[f] : area0) * uf;
    double tC[S], tD[S];
    load_cell<S>(theta, C, tC);
    load_cell<S>(theta, D, tD);
    if (lim == FL_UPWIND) {
#pragma unroll
        for (int k = 0; k < S; ++k) phi[f * S + k] = au * tC[k];
        return;
    }
    double tU[S];
    load_cell<S>(theta, U, tU);
#pragma unroll
    for (int k = 0; k < S; ++k) phi[f * S + k] = au * face_value(lim, tC[k], tD[k], tU[k]);
}

// General cells: the upstream difference of the upwind side sums its projected faces
// (side lists: far cells and weights, built at mesh creation).  Boundary faces (nbr = -1)
// border an exterior cell: it holds the inflow value of the face where the flow enters through
// it and inflow values are given, and repeats the face's own cell otherwise.  The exterior side
// of a boundary face has no side list (d_U = 0); a side-list entry ~j is the exterior beyond
// boundary face j of the upwind cell.
template <int S>
__device__ __forceinline__ void face_flux_general_one(
    int64_t f, const int4 *__restrict__ fc4, const int32_t *__restrict__ side_ptr,
    const int32_t *__restrict__ side_cell, const double *__restrict__ side_w,
    const double *__restrict__ u, const double *__restrict__ theta,
    const double *__restrict__ area, double area0, int lim, double *__restrict__ phi, double us,
    const double *__restrict__ inflow) {
    const int4 e = fc4[f];
    const double uf = u[f] * us;
    const bool pos = uf > 0.0;
    const int64_t C = pos ? e.x : e.y;  // -1: the exterior of an inflow face
    const int64_t D = pos ? e.y : e.x;  // -1: the exterior of an outflow face
    const double au = (area ? area[f] : area0) * uf;
    double tC[S], tD[S], dU[S];
    if (C >= 0) {
        load_cell<S>(theta, C, tC);
        if (D >= 0) load_cell<S>(theta, D, tD);
        else {
#pragma unroll
            for (int k = 0; k < S; ++k) tD[k] = tC[k];
        }
    } else {
        load_cell<S>(theta, D, tD);
        if (inflow) load_cell<S>(inflow, f, tC);
        else {
#pragma unroll
            for (int k = 0; k < S; ++k) tC[k] = tD[k];
        }
    }
    if (lim == FL_UPWIND) {
#pragma unroll
        for (int k = 0; k < S; ++k) phi[f * S + k] = au * tC[k];
        return;
    }
#pragma unroll
    for (int k = 0; k < S; ++k) dU[k] = 0.0;
    const int64_t side = 2 * f + (pos ? 0 : 1);
    for (int64_t p = side_ptr[side]; p < side_ptr[side + 1]; ++p) {
        const int64_t j = side_cell[p];
        const double w = side_w[p];
        if (j >= 0) {
#pragma unroll
            for (int k = 0; k < S; ++k) dU[k] += w * (tC[k] - theta[j * S + k]);
        } else {
            const int64_t jf = ~j;
            const bool in = inflow && !(u[jf] * us > 0.0);
#pragma unroll
            for (int k = 0; k < S; ++k) dU[k] += w * (tC[k] - (in ? inflow[jf * S + k] : tC[k]));
        }
    }
#pragma unroll
    for (int k = 0; k < S; ++k) phi[f * S + k] = au * face_value_d(lim, tC[k], tD[k] - tC[k], dU[k]);
}

// out = rhs (MODE_RHS), theta_s + dt rhs (MODE_EULER) or a theta_n + b (theta_s + dt rhs).
template <int S>
__device__ __forceinline__ void finish_cell(int64_t c, const double *acc, double V,
                                            const double *__restrict__ ts,
                                            const double *__restrict__ tn, double a, double b,
                                            double dt, int mode, double *__restrict__ out) {
    if (mode == MODE_RHS) {
#pragma unroll
        for (int k = 0; k < S; ++k) out[c * S + k] = acc[k] / V;
    } else if (mode == MODE_EULER) {
#pragma unroll
        for (int k = 0; k < S; ++k) out[c * S + k] = fma(dt, acc[k] / V, ts[c * S + k]);
    } else {
        // rounded as the fused stage rounds it (explicit fma)
#pragma unroll
        for (int k = 0; k < S; ++k)
            out[c * S + k] = fma(b, fma(dt, acc[k] / V, ts[c * S + k]), a * tn[c * S + k]);
    }
}

// Cell c: the divergence of its face fluxes (signed face list; K faces per cell where the list
// has no pointers) and the stage combination of mode.
template <int S>
__device__ __forceinline__ void cell_update_one(int64_t c, int K, const int32_t *__restrict__ cf_ptr,
                                                const int32_t *__restrict__ cf_idx,
                                                const double *__restrict__ phi,
                                                const double *__restrict__ vol, double vol0,
                                                const double *__restrict__ ts,
                                                const double *__restrict__ tn, double a, double b,
                                                double dt, int mode, double *__restrict__ out) {
    int64_t p0, p1;
    if (cf_ptr) {
        p0 = cf_ptr[c];
        p1 = cf_ptr[c + 1];
    } else {
        p0 = c * K;
        p1 = p0 + K;
    }
    double acc[S];
#pragma unroll
    for (int k = 0; k < S; ++k) acc[k] = 0.0;
    for (int64_t p = p0; p < p1; ++p) {
        const int32_t e = cf_idx[p];
        if (e >= 0) {
#pragma unroll
            for (int k = 0; k < S; ++k) acc[k] += phi[(int64_t)e * S + k];
        } else {
            const int64_t f = ~e;
#pragma unroll
            for (int k = 0; k < S; ++k) acc[k] -= phi[f * S + k];
        }
    }
    finish_cell<S>(c, acc, vol ? vol[c] : vol0, ts, tn, a, b, dt, mode, out);
}


}  // namespace dev
}  // namespace fl
