// Device routines of the discrete adjoint shared by the per-step and the multi-step reverse
// kernels: the limiter with its derivative and the limited face value with its partials.
#pragma once

#include <hip/hip_runtime.h>

#include "fl_device.h"
#include "fl_kernels.h"

namespace fl {
namespace adev {

constexpr int kBlock = 256;
constexpr double kRBig = 1.0e18;

template <int LIM>
__device__ __forceinline__ double psi_inf(bool pos) {
    if constexpr (LIM == FL_MINMOD) return pos ? 1.0 : 0.0;
    else if constexpr (LIM == FL_VANLEER || LIM == FL_SUPERBEE) return pos ? 2.0 : 0.0;
    else if constexpr (LIM == FL_VANALBADA || LIM == FL_CENTRAL) return 1.0;
    else if constexpr (LIM == FL_SMART) return pos ? 4.0 : 0.0;
    else return 0.0;
}

// psi(r) and psi'(r) on the branch the evaluation takes (left-closed pieces at break points).
template <int LIM>
__device__ __forceinline__ void psi_dpsi(double r, double &p, double &dp) {
#pragma clang fp contract(off)
    if constexpr (LIM == FL_MINMOD) {
        p = fmax(0.0, fmin(1.0, r));
        dp = (r > 0.0 && r < 1.0) ? 1.0 : 0.0;
    } else if constexpr (LIM == FL_VANLEER) {
        const double q = 1.0 / (1.0 + fabs(r));
        p = (r + fabs(r)) * q;
        dp = r > 0.0 ? 2.0 * q * q : 0.0;
    } else if constexpr (LIM == FL_VANALBADA) {
        const double q = 1.0 / (r * r + 1.0);
        p = (r * r + r) * q;
        dp = (1.0 + 2.0 * r - r * r) * q * q;
    } else if constexpr (LIM == FL_SUPERBEE) {
        p = fmax(0.0, fmax(fmin(1.0, 2.0 * r), fmin(r, 2.0)));
        dp = r <= 0.0 ? 0.0 : r <= 0.5 ? 2.0 : r <= 1.0 ? 0.0 : r <= 2.0 ? 1.0 : 0.0;
    } else if constexpr (LIM == FL_SMART) {
        p = fmax(0.0, fmin(fmin(2.0 * r, 0.25 + 0.75 * r), 4.0));
        dp = r <= 0.0 ? 0.0 : r <= 0.2 ? 2.0 : r <= 5.0 ? 0.75 : 0.0;
    } else if constexpr (LIM == FL_CENTRAL) {
        p = 1.0;
        dp = 0.0;
    } else {
        p = 0.0;
        dp = 0.0;
    }
}

// theta_f and its partials g_a = d theta_f / d d_U, g_b = d theta_f / d d_u from theta_C and the
// differences a = d_U, b = d_u.  No multiply-add is fused here (contract off): the value and
// partials of a face come out with the same bits wherever the routine is inlined, whichever of
// its results the caller uses (the far-upwind term a neighbour hands over equals the one a cell
// forms itself).
template <int LIM>
__device__ __forceinline__ double face_value_ab(double tC, double a, double b, double &ga,
                                                double &gb) {
#pragma clang fp contract(off)
    if constexpr (LIM == FL_UPWIND) {
        ga = 0.0;
        gb = 0.0;
        return tC;
    }
    if (b == 0.0) {
        // g(., 0) = 0; along d_u > 0, g(a, b) / b -> psi(+-inf) / 2, and psi(0) / 2 where a = 0
        // (g(0, b) = psi(0) b / 2: 1/2 for central differencing, 0 for the others)
        ga = 0.0;
        gb = (a == 0.0) ? (LIM == FL_CENTRAL ? 0.5 : 0.0) : 0.5 * psi_inf<LIM>(a > 0.0);
        return tC;
    }
    if constexpr (LIM == FL_VANALBADA) {
        // psi(a/b) b / 2 = a b (a + b) / (2 (a^2 + b^2)): one reciprocal for value and partials
        const double q = a * a + b * b;
        if (q >= 1e-280 && q <= 1e280) {
            const double iq = 1.0 / q;
            const double iq2 = iq * iq;
            ga = 0.5 * (b * b) * (b * b + 2.0 * a * b - a * a) * iq2;
            gb = 0.5 * (a * a) * (a * a + 2.0 * a * b - b * b) * iq2;
            return tC + 0.5 * (a * b) * (a + b) * iq;
        }
    }
    const double r = a / b;
    if (!(fabs(r) <= kRBig)) {
        const double p = psi_inf<LIM>(r > 0.0);
        ga = 0.0;
        gb = 0.5 * p;
        return tC + 0.5 * p * b;
    }
    double p, dp;
    psi_dpsi<LIM>(r, p, dp);
    ga = 0.5 * dp;
    gb = 0.5 * (p - r * dp);
    return tC + 0.5 * p * b;
}

// The same from theta_C, theta_D and the far-upwind theta_U (d_U = theta_C - theta_U).
template <int LIM>
__device__ __forceinline__ double face_value_d(double tC, double tD, double tU, double &ga,
                                               double &gb) {
#pragma clang fp contract(off)
    const double b = tD - tC;  // d_u
    const double a = tC - tU;  // d_U
    return face_value_ab<LIM>(tC, a, b, ga, gb);
}

template <int S>
__device__ __forceinline__ void load(const double *__restrict__ a, int64_t c, double *v) {
#pragma unroll
    for (int s = 0; s < S; ++s) v[s] = a[c * S + s];
}

template <int S>
__device__ __forceinline__ void load_s(const double *src, int64_t i, int stride, double *v) {
#pragma unroll
    for (int s = 0; s < S; ++s) v[s] = src[i * stride + s];
}

// lambda_a / V_a - lambda_b / V_b as la * iva - lb * ivb with both products rounded and no fused
// multiply-add: swapping the two cells negates the result exactly, so the two cells of a face
// form its cotangent difference with the same bits (up to sign).
__device__ __forceinline__ double cot_diff(double la, double iva, double lb, double ivb) {
#pragma clang fp contract(off)
    return la * iva - lb * ivb;
}

// a * b rounded on its own: a term formed with it and added to a sum later is never fused into
// a multiply-add, so every reverse kernel adds the same rounded terms whatever it keeps in
// registers in between.
__device__ __forceinline__ double mul_nc(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}

// ------------------------------------------------------------------------------------------
// The reverse stage of one cell from signed slot rates (the multi-step reverse sweep).
// ------------------------------------------------------------------------------------------
// One slot of a cell for adj_cell_rate: the rates w, w' and the source indices of the
// neighbour n and the far cell g.
struct AdjSlot {
    double w, wp;
    int64_t n, g;
};

// theta / lambda / V of a cell with source index i: tsrc[i * stride + s], lsrc[i * stride + s],
// vsrc[i * vstride] (vsrc NULL: all volumes 1 / ivol0).  slot(k) gives slot k's AdjSlot (read
// where it is used, so that a kernel can keep its tables in LDS rather than in registers).
// jt = (J^T lambda)_x; ub(p, t) adds scale * t (one fused multiply-add) to the forward face p's
// velocity cotangent, t = a_f sum_s theta_f (lambda_n/V_n - lambda_x/V_x) (when UB), with af(p)
// that face's area.
template <int S, int P, int LIM, bool TNLDS, bool UB, class SlotFn, class AreaFn, class UbFn>
__device__ __forceinline__ void adj_cell_rate(int64_t xi, const SlotFn &slot, const double *tsrc,
                                              const double *lsrc, const double *vsrc, int stride,
                                              int vstride, double ivol0, const AreaFn &af,
                                              const UbFn &ub, double *jt, double *lx) {
    constexpr int K = 2 * P;
    double tx[S], tn[TNLDS ? 1 : K][S];
    load_s<S>(tsrc, xi, stride, tx);
    load_s<S>(lsrc, xi, stride, lx);
    if constexpr (!TNLDS) {
#pragma unroll
        for (int k = 0; k < K; ++k) load_s<S>(tsrc, slot(k).n, stride, tn[k]);
    }
    const double ivx = vsrc ? 1.0 / vsrc[xi * vstride] : ivol0;
#pragma unroll
    for (int s = 0; s < S; ++s) jt[s] = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const AdjSlot sl = slot(k);
        const double w = sl.w, wp = sl.wp;
        const double ivn = vsrc ? 1.0 / vsrc[sl.n * vstride] : ivol0;
        const double ivg = vsrc ? 1.0 / vsrc[sl.g * vstride] : ivol0;
        double tnk[S], tno[S];
        if constexpr (TNLDS) {
            load_s<S>(tsrc, sl.n, stride, tnk);
            load_s<S>(tsrc, slot(k ^ 1).n, stride, tno);
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                tnk[s] = tn[k][s];
                tno[s] = tn[k ^ 1][s];
            }
        }
        double ln[S], lg[S], tg[S];
        load_s<S>(lsrc, sl.n, stride, ln);
        load_s<S>(lsrc, sl.g, stride, lg);
        load_s<S>(tsrc, sl.g, stride, tg);
        // face f between x and n: x is its upwind cell where the flow leaves x (w > 0), or where
        // u_f is zero and x is the face's nbr (w = +0.0)
        const bool x_up = !signbit(w);
        double usum = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            double ga, gb;
            const double tC = x_up ? tx[s] : tnk[s];
            const double tD = x_up ? tnk[s] : tx[s];
            const double tU = x_up ? tno[s] : tg[s];
            const double tf = face_value_d<LIM>(tC, tD, tU, ga, gb);
            const double d = cot_diff(ln[s], ivn, lx[s], ivx);
            const double z = w * d;
            jt[s] += x_up ? mul_nc(z, 1.0 + ga - gb) : mul_nc(z, gb);
            if (UB && (k & 1) == 0) usum += tf * d;
        }
        if constexpr (UB) {
            if ((k & 1) == 0) ub(k >> 1, af(k >> 1) * usum);
        }
        // face fr between n and g: x is its far-upwind cell where the flow leaves n away from x
        if (wp > 0.0) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                double ga, gb;
                (void)face_value_d<LIM>(tnk[s], tg[s], tx[s], ga, gb);
                jt[s] -= mul_nc(wp * cot_diff(lg[s], ivg, ln[s], ivn), ga);
            }
        }
    }
}

// Stage combination of the multi-step reverse sweep (modes ADJ_EULER, ADJ_LAST, ADJ_MID,
// ADJ_FIRST): out = lambda + dt J^T lambda (Euler); out = b (lambda + dt J^T lambda) (the last
// and middle stages of SSP-RK3); for the first stage the cotangent of theta^n is completed with
// the terms of the two later stages, a3 lin + a2 l3 (lin: the step's input cotangent, l3: the
// last stage's output), in the order the per-step path accumulates them.
// (out may be lin: each thread reads lin only at its own cell before writing it.)
template <int S>
__device__ __forceinline__ void adj_combine(int64_t x, const double *jt, const double *lx, double a,
                                            double b, double a3, double dt, int mode,
                                            const double *lin, const double *__restrict__ l3,
                                            double *out) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t i = x * S + s;
        const double g = fma(dt, jt[s], lx[s]);
        if (mode == ADJ_EULER) out[i] = g;
        else if (mode == ADJ_FIRST) out[i] = fma(b, g, fma(a, l3[i], a3 * lin[i]));
        else out[i] = b * g;
    }
}

}  // namespace adev
}  // namespace fl
