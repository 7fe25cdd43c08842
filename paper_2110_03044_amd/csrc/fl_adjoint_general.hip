// Discrete adjoint of the flux-limited operator on general cells (face path), gfx950, FP64.
//
// On general cells the upstream difference of a face side sums several projected faces,
// d_U = sum_j w_j (theta_C - theta_j), so a face's limiter partials reach C, D and every
// projected cell: with mu_f = lambda_nbr / V_nbr - lambda_own / V_own, z = a_f u_f mu_f and
// (g_a, g_b) the partials of theta_f = theta_C + g(d_U, d_u),
//   theta_bar_C += z (1 - g_b + g_a sum_j w_j),  theta_bar_D += z g_b,
//   theta_bar_j -= w_j z g_a,                      u_bar_f += a_f theta_f mu_f.
// No atomics: one thread per face forms its terms (for its own cell, its nbr, and z g_a on its
// upwind side), one thread per cell gathers them through its face list and the transposed side
// lists (the face sides whose d_U names the cell).  Q(u_f) and the limiter branch are held fixed,
// as on the paired path.
// Boundary faces (nbr = -1; the flux leaves or enters own alone, mu_f = -lambda_own / V_own):
// the exterior beyond one holds a constant inflow value (no cotangent) or repeats own, which then
// takes the exterior's share; a side-list entry ~j (the exterior beyond boundary face j of the
// upwind cell) is a constant inflow value, whose weight counts in sum_j w_j, or repeats the
// upwind cell itself, whose difference theta_C - theta_C is identically zero.  Face distances
// need nothing here: their ratios sit in the side weights.
#include <hip/hip_runtime.h>

#include "fl_adjoint_device.h"

namespace fl {
namespace adev {

// term[f][0][s]: the cell own's term, [1]: nbr's, [2 + side]: z g_a on the upwind side (0 on the
// other side).
template <int S, int LIM>
__global__ __launch_bounds__(kBlock) void adjoint_face_general_kernel(
    int64_t nf, const int4 *__restrict__ fc4, const int32_t *__restrict__ side_ptr,
    const int32_t *__restrict__ side_cell, const double *__restrict__ side_w,
    const double *__restrict__ u, const double *__restrict__ area, double area0,
    const double *__restrict__ vol, double ivol0, const double *__restrict__ th,
    const double *__restrict__ lam, const double *__restrict__ inflow, double scale,
    double *__restrict__ term, double *__restrict__ ubar) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= nf) return;
    const int4 e = fc4[f];
    const int64_t own = e.x, nbr = e.y;  // nbr = -1: a boundary face
    const bool bnd = nbr < 0;
    const double uf = u[f];
    const bool pos = uf > 0.0;
    const int64_t C = pos ? own : nbr, D = pos ? nbr : own;  // -1: the exterior
    const bool c_in = C < 0 && inflow;  // the exterior upwind holds the inflow value
    const double af = area ? area[f] : area0;
    const double ivo = vol ? 1.0 / vol[own] : ivol0;
    const double ivn = bnd ? 0.0 : (vol ? 1.0 / vol[nbr] : ivol0);
    const int64_t side = 2 * f + (pos ? 0 : 1);
    const int32_t p0 = side_ptr[side], p1 = side_ptr[side + 1];
    // the weights of the entries whose value does not follow theta_C
    double wsum = 0.0;
    for (int32_t p = p0; p < p1; ++p) {
        const int32_t j = side_cell[p];
        if (j >= 0 || (inflow && !(u[~j] > 0.0))) wsum += side_w[p];
    }
    double usum = 0.0;
    double *t = term + f * 4 * S;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        double tC, tD;
        if (C >= 0) {
            tC = th[C * S + s];
            tD = D >= 0 ? th[D * S + s] : tC;
        } else {
            tD = th[D * S + s];
            tC = c_in ? inflow[f * S + s] : tD;
        }
        double dU = 0.0;
        for (int32_t p = p0; p < p1; ++p) {
            const int32_t j = side_cell[p];
            double v = tC;
            if (j >= 0) v = th[(int64_t)j * S + s];
            else if (inflow && !(u[~j] > 0.0)) v = inflow[(int64_t)~j * S + s];
            dU += side_w[p] * (tC - v);
        }
        double ga, gb;
        const double tf = face_value_ab<LIM>(tC, dU, tD - tC, ga, gb);
        const double mu = cot_diff(bnd ? 0.0 : lam[nbr * S + s], ivn, lam[own * S + s], ivo);
        const double z = af * uf * mu;
        const double tc = mul_nc(z, 1.0 - gb + ga * wsum), td = mul_nc(z, gb);
        if (!bnd) {
            t[s] = pos ? tc : td;
            t[S + s] = pos ? td : tc;
        } else {
            // own takes the exterior's share where the exterior repeats it
            t[s] = pos ? tc + td : (c_in ? td : td + tc);
            t[S + s] = 0.0;
        }
        const double zg = mul_nc(z, ga);
        t[2 * S + s] = pos ? zg : 0.0;
        t[3 * S + s] = pos ? 0.0 : zg;
        usum += tf * mu;
    }
    if (ubar) ubar[f] = fma(scale, af * usum, ubar[f]);
}

// One cell x: J^T lambda from its faces' terms and the transposed side lists, then the stage
// combination of mode (as the paired path's per-step kernels).
template <int S>
__global__ __launch_bounds__(kBlock) void adjoint_cell_general_kernel(
    int64_t nc, int K, const int32_t *__restrict__ cf_ptr, const int32_t *__restrict__ cf_idx,
    const int32_t *__restrict__ rev_ptr, const int32_t *__restrict__ rev_side,
    const double *__restrict__ rev_w, const double *__restrict__ term,
    const double *__restrict__ lam, double a, double b, double dt, int mode,
    double *__restrict__ out, double *__restrict__ acc) {
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= nc) return;
    const int64_t q0 = cf_ptr ? cf_ptr[x] : x * K, q1 = cf_ptr ? cf_ptr[x + 1] : q0 + K;
    double jt[S];
#pragma unroll
    for (int s = 0; s < S; ++s) jt[s] = 0.0;
    for (int64_t q = q0; q < q1; ++q) {
        const int32_t fe = cf_idx[q];
        const bool is_own = fe < 0;
        const int64_t f = is_own ? ~fe : fe;
        const double *t = term + f * 4 * S + (is_own ? 0 : S);
#pragma unroll
        for (int s = 0; s < S; ++s) jt[s] += t[s];
    }
    for (int32_t p = rev_ptr[x]; p < rev_ptr[x + 1]; ++p) {
        const int64_t sd = rev_side[p];
        const double w = rev_w[p];
        const double *t = term + (sd >> 1) * 4 * S + (2 + (sd & 1)) * S;
#pragma unroll
        for (int s = 0; s < S; ++s) jt[s] -= mul_nc(w, t[s]);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t i = x * S + s;
        const double lx = lam[i];
        switch (mode) {
            case ADJ_APPLY: out[i] += jt[s]; break;
            case ADJ_EULER: out[i] = fma(dt, jt[s], lx); break;
            case ADJ_LAST:
                acc[i] = a * lx;
                out[i] = b * fma(dt, jt[s], lx);
                break;
            case ADJ_MID:
                acc[i] = fma(a, lx, acc[i]);
                out[i] = b * fma(dt, jt[s], lx);
                break;
            default: out[i] = fma(b, fma(dt, jt[s], lx), acc[i]); break;
        }
    }
}

}  // namespace adev

namespace {
template <int S, int LIM>
hipError_t launch_g2(const fl_mesh *m, const double *u, const double *th, const double *lam,
                     double a, double b, double dt, int mode, double *out, double *acc,
                     double *ubar, double *term, hipStream_t st) {
    const unsigned nbf = (unsigned)((m->h.nf + adev::kBlock - 1) / adev::kBlock);
    const unsigned nbc = (unsigned)((m->h.nc + adev::kBlock - 1) / adev::kBlock);
    const double scale = mode == ADJ_APPLY ? 1.0 : b * dt;
    adev::adjoint_face_general_kernel<S, LIM><<<nbf, adev::kBlock, 0, st>>>(
        m->h.nf, reinterpret_cast<const int4 *>(m->d_fc4), m->d_side_ptr, m->d_side_cell,
        m->d_side_w, u, m->d_area, m->h.area0, m->d_vol, 1.0 / m->h.vol0, th, lam, m->inflow,
        scale, term, ubar);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    adev::adjoint_cell_general_kernel<S><<<nbc, adev::kBlock, 0, st>>>(
        m->h.nc, m->h.max_degree, m->d_cf_ptr, m->d_cf_idx, m->d_rev_ptr, m->d_rev_side,
        m->d_rev_w, term, lam, a, b, dt, mode, out, acc);
    return hipGetLastError();
}

template <int S>
hipError_t launch_g1(const fl_mesh *m, int lim, const double *u, const double *th,
                     const double *lam, double a, double b, double dt, int mode, double *out,
                     double *acc, double *ubar, double *term, hipStream_t st) {
#define FL_AG(L) launch_g2<S, L>(m, u, th, lam, a, b, dt, mode, out, acc, ubar, term, st)
    switch (lim) {
        case FL_UPWIND: return FL_AG(FL_UPWIND);
        case FL_MINMOD: return FL_AG(FL_MINMOD);
        case FL_VANLEER: return FL_AG(FL_VANLEER);
        case FL_VANALBADA: return FL_AG(FL_VANALBADA);
        case FL_SUPERBEE: return FL_AG(FL_SUPERBEE);
        case FL_SMART: return FL_AG(FL_SMART);
        case FL_CENTRAL: return FL_AG(FL_CENTRAL);
        default: return hipErrorInvalidValue;
    }
#undef FL_AG
}
}  // namespace

size_t adjoint_general_term_bytes(const fl_mesh *m, int S) {
    return (size_t)m->h.nf * 4 * S * sizeof(double);
}

hipError_t launch_adjoint_general(const fl_mesh *m, int lim, int S, const double *u,
                                  const double *th, const double *lam, double a, double b,
                                  double dt, int mode, double *out, double *acc, double *ubar,
                                  double *term, hipStream_t st) {
#define FL_AG1(SS) launch_g1<SS>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, term, st)
    switch (S) {
        case 1: return FL_AG1(1);
        case 2: return FL_AG1(2);
        case 3: return FL_AG1(3);
        case 4: return FL_AG1(4);
        case 5: return FL_AG1(5);
        case 6: return FL_AG1(6);
        case 7: return FL_AG1(7);
        case 8: return FL_AG1(8);
        default: return hipErrorInvalidValue;
    }
#undef FL_AG1
}

}  // namespace fl
