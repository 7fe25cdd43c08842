// Discrete adjoint (reverse mode) of the flux-limited convective operator, gfx950, FP64.
//
// Forward, per face f with upwind C, downwind D and far-upwind U (selected by sign(u_f)):
//   theta_f = theta_C + g(d_U, d_u),  g = psi(d_U/d_u) d_u / 2,  d_U = theta_C - theta_U,
//   d_u = theta_D - theta_C,  rhs_c = sum_f E[f][c] a_f u_f theta_f / V_c.
// Reverse, for a cotangent lambda of rhs: mu_f = lambda_nbr/V_nbr - lambda_own/V_own and
// zeta_f = a_f u_f mu_f; then
//   theta_bar_C += zeta (1 + g_a - g_b),  theta_bar_D += zeta g_b,  theta_bar_U -= zeta g_a,
//   u_bar_f += a_f theta_f mu_f,
// with g_a = psi'(r)/2 and g_b = (psi(r) - r psi'(r))/2 (the limit values where d_u == 0 or
// |r| is beyond the range evaluated as infinity).  Q(u_f) and the limiter branch are held fixed.
//
// No atomics: one thread per cell x gathers every contribution it receives -- from its own
// faces (x is C or D there) and from the faces for which it is the far-upwind cell U (the face
// of each neighbour n opposite to the face shared with x, flow running from n away from x).
// u_bar of a face is written only by the thread of the face's own cell.
#include <hip/hip_runtime.h>

#include "fl_kernels.h"

namespace fl {
namespace adev {

constexpr int kBlock = 256;
constexpr double kRBig = 1.0e18;

__device__ __forceinline__ double psi_inf(int lim, bool pos) {
    switch (lim) {
        case FL_MINMOD: return pos ? 1.0 : 0.0;
        case FL_VANLEER: return pos ? 2.0 : 0.0;
        case FL_VANALBADA: return 1.0;
        case FL_SUPERBEE: return pos ? 2.0 : 0.0;
        case FL_SMART: return pos ? 4.0 : 0.0;
        case FL_CENTRAL: return 1.0;
        default: return 0.0;
    }
}

__device__ __forceinline__ double psi(int lim, double r) {
    switch (lim) {
        case FL_MINMOD: return fmax(0.0, fmin(1.0, r));
        case FL_VANLEER: {
            const double ar = fabs(r);
            return (r + ar) / (1.0 + ar);
        }
        case FL_VANALBADA: {
            const double r2 = r * r;
            return (r2 + r) / (r2 + 1.0);
        }
        case FL_SUPERBEE: return fmax(0.0, fmax(fmin(1.0, 2.0 * r), fmin(r, 2.0)));
        case FL_SMART: return fmax(0.0, fmin(fmin(2.0 * r, 0.25 + 0.75 * r), 4.0));
        case FL_CENTRAL: return 1.0;
        default: return 0.0;
    }
}

// psi'(r) on the branch the evaluation takes (left-closed pieces at break points).
__device__ __forceinline__ double dpsi(int lim, double r) {
    switch (lim) {
        case FL_MINMOD: return (r > 0.0 && r < 1.0) ? 1.0 : 0.0;
        case FL_VANLEER: {
            const double q = 1.0 + r;
            return r > 0.0 ? 2.0 / (q * q) : 0.0;
        }
        case FL_VANALBADA: {
            const double q = r * r + 1.0;
            return (1.0 + 2.0 * r - r * r) / (q * q);
        }
        case FL_SUPERBEE:
            return r <= 0.0 ? 0.0 : r <= 0.5 ? 2.0 : r <= 1.0 ? 0.0 : r <= 2.0 ? 1.0 : 0.0;
        case FL_SMART:
            return r <= 0.0 ? 0.0 : r <= 0.2 ? 2.0 : r <= 5.0 ? 0.75 : 0.0;
        default: return 0.0;
    }
}

// theta_f and its partials g_a = d theta_f / d d_U, g_b = d theta_f / d d_u.
__device__ __forceinline__ double face_value_d(int lim, double tC, double tD, double tU,
                                               double &ga, double &gb) {
    const double du = tD - tC;
    const double dU = tC - tU;
    if (du == 0.0) {
        ga = 0.0;
        gb = (dU == 0.0) ? 0.0 : 0.5 * psi_inf(lim, dU > 0.0);
        return tC;
    }
    if (lim == FL_UPWIND) {
        ga = 0.0;
        gb = 0.0;
        return tC;
    }
    const double r = dU / du;
    if (!(fabs(r) <= kRBig)) {
        const double p = psi_inf(lim, r > 0.0);
        ga = 0.0;
        gb = 0.5 * p;
        return tC + 0.5 * p * du;
    }
    const double p = psi(lim, r);
    const double dp = dpsi(lim, r);
    ga = 0.5 * dp;
    gb = 0.5 * (p - r * dp);
    return tC + 0.5 * p * du;
}

template <int S>
__device__ __forceinline__ void load(const double *__restrict__ a, int64_t c, double *v) {
#pragma unroll
    for (int s = 0; s < S; ++s) v[s] = a[c * S + s];
}

// mode: ADJ_APPLY    theta_bar[x] += J^T lam, u_bar += (dL/du)^T lam            (scale 1)
//       ADJ_EULER    out[x] = lam[x] + dt J^T lam                               (b = 1)
//       ADJ_LAST     acc[x] = a lam[x];  out[x] = b (lam[x] + dt J^T lam)
//       ADJ_MID      acc[x] += a lam[x]; out[x] = b (lam[x] + dt J^T lam)
//       ADJ_FIRST    out[x] = acc[x] + b (lam[x] + dt J^T lam)
// and u_bar += scale (dL/du)^T lam with scale = b dt (1 for ADJ_APPLY).
template <int S, int P>
__global__ __launch_bounds__(kBlock) void adjoint_stage_kernel(
    int64_t nc, const uint32_t *__restrict__ sface, const int32_t *__restrict__ snbr,
    const int32_t *__restrict__ sfar, const uint32_t *__restrict__ srev,
    const double *__restrict__ u, const double *__restrict__ area, double area0,
    const double *__restrict__ vol, double vol0, const double *__restrict__ th,
    const double *__restrict__ lam, double a, double b, double dt, int mode, int lim,
    double *__restrict__ out, double *__restrict__ acc, double *__restrict__ ubar) {
    constexpr int K = 2 * P;
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= nc) return;
    uint32_t fw[K], rw[K];
    int64_t nb[K], gf[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        fw[k] = sface[(int64_t)k * nc + x];
        rw[k] = srev[(int64_t)k * nc + x];
        nb[k] = snbr[(int64_t)k * nc + x];
        gf[k] = sfar[(int64_t)k * nc + x];
    }
    double tx[S], lx[S], tn[K][S];
    load<S>(th, x, tx);
    load<S>(lam, x, lx);
#pragma unroll
    for (int k = 0; k < K; ++k) load<S>(th, nb[k], tn[k]);
    const double vx = vol ? vol[x] : vol0;
    const double scale = (mode == ADJ_APPLY) ? 1.0 : b * dt;
    double jt[S];
#pragma unroll
    for (int s = 0; s < S; ++s) jt[s] = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t f = fw[k] & 0x7fffffffu, fr = rw[k] & 0x7fffffffu;
        const int64_t n = nb[k], g = gf[k];
        const double uf = u[f], ur = u[fr];
        const double af = area ? area[f] : area0, ar = area ? area[fr] : area0;
        const double vn = vol ? vol[n] : vol0, vg = vol ? vol[g] : vol0;
        double ln[S], lg[S], tg[S];
        load<S>(lam, n, ln);
        load<S>(lam, g, lg);
        load<S>(th, g, tg);
        // face f between x and n
        const bool x_own = (fw[k] >> 31) != 0;
        const bool x_up = ((uf > 0.0) == x_own);
        double usum = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            double ga, gb, tf;
            if (x_up) tf = face_value_d(lim, tx[s], tn[k][s], tn[k ^ 1][s], ga, gb);
            else tf = face_value_d(lim, tn[k][s], tx[s], tg[s], ga, gb);
            const double mu = x_own ? (ln[s] / vn - lx[s] / vx) : (lx[s] / vx - ln[s] / vn);
            const double z = af * uf * mu;
            jt[s] += x_up ? z * (1.0 + ga - gb) : z * gb;
            usum += tf * mu;
        }
        if (ubar != nullptr && x_own) ubar[f] += scale * (af * usum);
        // face fr between n and g, opposite to f in n: x is its far-upwind cell when the flow
        // runs from n to g
        const bool n_own = (rw[k] >> 31) != 0;
        if ((ur > 0.0) == n_own) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                double ga, gb;
                (void)face_value_d(lim, tn[k][s], tg[s], tx[s], ga, gb);
                const double mu = n_own ? (lg[s] / vg - ln[s] / vn) : (ln[s] / vn - lg[s] / vg);
                jt[s] -= (ar * ur * mu) * ga;
            }
        }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t i = x * S + s;
        switch (mode) {
            case ADJ_APPLY: out[i] += jt[s]; break;
            case ADJ_EULER: out[i] = lx[s] + dt * jt[s]; break;
            case ADJ_LAST:
                acc[i] = a * lx[s];
                out[i] = b * (lx[s] + dt * jt[s]);
                break;
            case ADJ_MID:
                acc[i] += a * lx[s];
                out[i] = b * (lx[s] + dt * jt[s]);
                break;
            default: out[i] = acc[i] + b * (lx[s] + dt * jt[s]); break;
        }
    }
}

}  // namespace adev

namespace {
template <int S>
hipError_t launch_adjoint_s(const fl_mesh *m, int lim, const double *u, const double *th,
                            const double *lam, double a, double b, double dt, int mode,
                            double *out, double *acc, double *ubar, hipStream_t st) {
    const unsigned nb = (unsigned)((m->h.nc + adev::kBlock - 1) / adev::kBlock);
    const uint32_t *rev = reinterpret_cast<const uint32_t *>(m->d_rev);
    switch (m->h.pairs) {
        case 1:
            adev::adjoint_stage_kernel<S, 1><<<nb, adev::kBlock, 0, st>>>(
                m->h.nc, m->d_slot_face, m->d_slot_nbr, m->d_slot_far, rev, u, m->d_area,
                m->h.area0, m->d_vol, m->h.vol0, th, lam, a, b, dt, mode, lim, out, acc, ubar);
            break;
        case 2:
            adev::adjoint_stage_kernel<S, 2><<<nb, adev::kBlock, 0, st>>>(
                m->h.nc, m->d_slot_face, m->d_slot_nbr, m->d_slot_far, rev, u, m->d_area,
                m->h.area0, m->d_vol, m->h.vol0, th, lam, a, b, dt, mode, lim, out, acc, ubar);
            break;
        case 3:
            adev::adjoint_stage_kernel<S, 3><<<nb, adev::kBlock, 0, st>>>(
                m->h.nc, m->d_slot_face, m->d_slot_nbr, m->d_slot_far, rev, u, m->d_area,
                m->h.area0, m->d_vol, m->h.vol0, th, lam, a, b, dt, mode, lim, out, acc, ubar);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_adjoint(const fl_mesh *m, int lim, int S, const double *u, const double *th,
                          const double *lam, double a, double b, double dt, int mode, double *out,
                          double *acc, double *ubar, hipStream_t st) {
    switch (S) {
        case 1: return launch_adjoint_s<1>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 2: return launch_adjoint_s<2>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 3: return launch_adjoint_s<3>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 4: return launch_adjoint_s<4>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 5: return launch_adjoint_s<5>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 6: return launch_adjoint_s<6>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 7: return launch_adjoint_s<7>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 8: return launch_adjoint_s<8>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fl
