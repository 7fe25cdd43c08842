// Forward kernels of the flux-limited convective operator for gfx950 (MI355X), FP64.
//
// The paper evaluates theta_f with four sparse matrix-vector products and four pointwise
// kernels (Algorithm 3) and the update with two more passes (Algorithm 4).  Here the whole
// chain -- sign selection Q(u_f), face difference d_u, upstream difference d_U, gradient ratio,
// limiter, face value, flux a_f u_f theta_f, divergence and the Runge-Kutta combination -- runs
// in one or two memory passes:
//   * face path: face_flux_kernel (one thread per face: coalesced u_f and {own, nbr, far_own,
//     far_nbr} records, three theta gathers, one flux store) + cell_update_kernel (one thread
//     per cell: its signed face list, flux gathers, divergence and stage combination, no
//     atomics);
//   * fused path (cells whose faces come in opposite pairs): fused_stage_kernel, one thread per
//     cell computing the fluxes of its own faces from the slot tables; every face is evaluated by
//     both of its cells with identical arithmetic, so the two contributions cancel exactly in
//     the global sum and no flux array is written.
// Launches use 256-thread workgroups; the grid is padded to a multiple of the 8 XCDs and block
// ids are remapped so each XCD sweeps one contiguous eighth of the mesh (its L2 then holds the
// neighbourhood of the cells it works on).
#include <hip/hip_runtime.h>

#include "fl_kernels.h"

namespace fl {
namespace dev {

constexpr int kBlock = 256;
constexpr double kRBig = 1.0e18;

__device__ __forceinline__ int64_t block_id(int remap) {
    if (!remap) return blockIdx.x;
    const int per = gridDim.x >> 3;
    return (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// psi at r = +inf (pos) or -inf.
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
    if (!(fabs(r) <= kRBig)) return psi_inf(lim, r > 0.0);
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

// Limited face value of the Sweby form from the upwind, downwind and far-upwind values.
__device__ __forceinline__ double face_value(int lim, double tC, double tD, double tU) {
    const double du = tD - tC;
    if (lim == FL_UPWIND || du == 0.0) return tC;
    const double r = (tC - tU) / du;
    return tC + 0.5 * psi(lim, r) * du;
}

template <int S>
__device__ __forceinline__ void load_cell(const double *__restrict__ th, int64_t c, double *v) {
#pragma unroll
    for (int k = 0; k < S; ++k) v[k] = th[c * S + k];
}

// ------------------------------------------------------------------------------------------
// Face path
// ------------------------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(kBlock) void face_flux_kernel(
    int64_t nf, const int4 *__restrict__ fc4, const double *__restrict__ u,
    const double *__restrict__ theta, const double *__restrict__ area, double area0, int lim,
    double *__restrict__ phi, int remap) {
    const int64_t f = block_id(remap) * kBlock + threadIdx.x;
    if (f >= nf) return;
    const int4 e = fc4[f];
    const double uf = u[f];
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
        for (int k = 0; k < S; ++k) out[c * S + k] = ts[c * S + k] + dt * (acc[k] / V);
    } else {
#pragma unroll
        for (int k = 0; k < S; ++k)
            out[c * S + k] = a * tn[c * S + k] + b * (ts[c * S + k] + dt * (acc[k] / V));
    }
}

template <int S>
__global__ __launch_bounds__(kBlock) void cell_update_kernel(
    int64_t nc, int K, const int32_t *__restrict__ cf_ptr, const int32_t *__restrict__ cf_idx,
    const double *__restrict__ phi, const double *__restrict__ vol, double vol0,
    const double *__restrict__ ts, const double *__restrict__ tn, double a, double b, double dt,
    int mode, double *__restrict__ out, int remap) {
    const int64_t c = block_id(remap) * kBlock + threadIdx.x;
    if (c >= nc) return;
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

// ------------------------------------------------------------------------------------------
// Fused path
// ------------------------------------------------------------------------------------------
// Contribution of one face of cell c: n is the other cell, g the far-upwind cell on n's side,
// o the neighbour across the opposite face of c (far-upwind on c's side).
template <int S>
__device__ __forceinline__ void fused_face(int lim, uint32_t fw, double uf, double au,
                                           const double *tc, const double *tn_,
                                           const double *to, const double *__restrict__ theta,
                                           int64_t g, double *acc) {
    const bool c_is_own = (fw >> 31) != 0;
    const bool pos = uf > 0.0;
    // Q(u_f): C = own where u_f > 0, nbr otherwise
    const bool c_upwind = (pos == c_is_own);
    double tf[S];
    if (c_upwind) {
#pragma unroll
        for (int k = 0; k < S; ++k) tf[k] = face_value(lim, tc[k], tn_[k], to[k]);
    } else if (lim == FL_UPWIND) {
#pragma unroll
        for (int k = 0; k < S; ++k) tf[k] = tn_[k];
    } else {
        double tg[S];
        load_cell<S>(theta, g, tg);
#pragma unroll
        for (int k = 0; k < S; ++k) tf[k] = face_value(lim, tn_[k], tc[k], tg[k]);
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const double ph = au * tf[k];
        if (c_is_own) acc[k] -= ph;
        else acc[k] += ph;
    }
}

template <int S>
__global__ __launch_bounds__(kBlock) void fused_stage_kernel(
    int64_t nc, int P, const uint32_t *__restrict__ sface, const int32_t *__restrict__ snbr,
    const int32_t *__restrict__ sfar, const double *__restrict__ u,
    const double *__restrict__ area, double area0, const double *__restrict__ vol, double vol0,
    const double *__restrict__ ts, const double *__restrict__ tn, double a, double b, double dt,
    int mode, int lim, double *__restrict__ out, int remap) {
    const int64_t c = block_id(remap) * kBlock + threadIdx.x;
    if (c >= nc) return;
    double tc[S], acc[S];
    load_cell<S>(ts, c, tc);
#pragma unroll
    for (int k = 0; k < S; ++k) acc[k] = 0.0;
    for (int p = 0; p < P; ++p) {
        const int64_t s0 = (int64_t)(2 * p) * nc + c, s1 = s0 + nc;
        const uint32_t f0 = sface[s0], f1 = sface[s1];
        const int64_t n0 = snbr[s0], n1 = snbr[s1];
        const int64_t i0 = f0 & 0x7fffffffu, i1 = f1 & 0x7fffffffu;
        const double u0 = u[i0], u1 = u[i1];
        double t0[S], t1[S];
        load_cell<S>(ts, n0, t0);
        load_cell<S>(ts, n1, t1);
        const double a0 = area ? area[i0] : area0, a1 = area ? area[i1] : area0;
        fused_face<S>(lim, f0, u0, a0 * u0, tc, t0, t1, ts, sfar[s0], acc);
        fused_face<S>(lim, f1, u1, a1 * u1, tc, t1, t0, ts, sfar[s1], acc);
    }
    finish_cell<S>(c, acc, vol ? vol[c] : vol0, ts, tn, a, b, dt, mode, out);
}

// ------------------------------------------------------------------------------------------
// Utilities
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void permute_kernel(int64_t n, int S,
                                                         const int32_t *__restrict__ perm,
                                                         int to_mesh, const double *__restrict__ in,
                                                         double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    if (to_mesh) {
        for (int k = 0; k < S; ++k) out[j * S + k] = in[i * S + k];
    } else {
        for (int k = 0; k < S; ++k) out[i * S + k] = in[j * S + k];
    }
}

__global__ __launch_bounds__(kBlock) void select_kernel(int64_t nf, const int4 *__restrict__ fc4,
                                                        const double *__restrict__ u,
                                                        int32_t *__restrict__ cdu) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= nf) return;
    const int4 e = fc4[f];
    const bool pos = u[f] > 0.0;
    cdu[3 * f] = pos ? e.x : e.y;
    cdu[3 * f + 1] = pos ? e.y : e.x;
    cdu[3 * f + 2] = pos ? e.z : e.w;
}

}  // namespace dev

// ------------------------------------------------------------------------------------------
// Launch wrappers
// ------------------------------------------------------------------------------------------
namespace {

struct Grid {
    unsigned blocks;
    int remap;
};

Grid grid_for(int64_t n, bool remap) {
    int64_t nb = (n + dev::kBlock - 1) / dev::kBlock;
    if (nb < 1) nb = 1;
    if (remap && nb >= 64) return {(unsigned)(((nb + 7) / 8) * 8), 1};
    return {(unsigned)nb, 0};
}

}  // namespace

#define FL_DISPATCH_S(S, CALL)                   \
    switch (S) {                                 \
        case 1: { constexpr int kS = 1; CALL; break; } \
        case 2: { constexpr int kS = 2; CALL; break; } \
        case 3: { constexpr int kS = 3; CALL; break; } \
        case 4: { constexpr int kS = 4; CALL; break; } \
        case 5: { constexpr int kS = 5; CALL; break; } \
        case 6: { constexpr int kS = 6; CALL; break; } \
        case 7: { constexpr int kS = 7; CALL; break; } \
        case 8: { constexpr int kS = 8; CALL; break; } \
        default: return hipErrorInvalidValue;    \
    }

int g_remap = 1;
void set_xcd_remap(int on) { g_remap = on; }

hipError_t launch_face_flux(const fl_mesh *m, int lim, int S, const double *theta,
                            const double *u, double *phi, hipStream_t st) {
    // Blocks beyond the face count exit at once (padding to a multiple of 8 XCDs).
    Grid g = grid_for(m->h.nf, g_remap);
    const int64_t nf_eff = g.remap ? m->h.nf : m->h.nf;
    FL_DISPATCH_S(S, (dev::face_flux_kernel<kS><<<g.blocks, dev::kBlock, 0, st>>>(
                         nf_eff, reinterpret_cast<const int4 *>(m->d_fc4), u, theta, m->d_area,
                         m->h.area0, lim, phi, g.remap)));
    return hipGetLastError();
}

hipError_t launch_cell_update(const fl_mesh *m, int S, const double *phi, const double *ts,
                              const double *tn, double a, double b, double dt, int mode,
                              double *out, hipStream_t st) {
    Grid g = grid_for(m->h.nc, g_remap);
    FL_DISPATCH_S(S, (dev::cell_update_kernel<kS><<<g.blocks, dev::kBlock, 0, st>>>(
                         m->h.nc, m->h.max_degree, m->d_cf_ptr, m->d_cf_idx, phi, m->d_vol,
                         m->h.vol0, ts, tn, a, b, dt, mode, out, g.remap)));
    return hipGetLastError();
}

hipError_t launch_fused(const fl_mesh *m, int lim, int S, const double *ts, const double *tn,
                        const double *u, double a, double b, double dt, int mode, double *out,
                        hipStream_t st) {
    Grid g = grid_for(m->h.nc, g_remap);
    FL_DISPATCH_S(S, (dev::fused_stage_kernel<kS><<<g.blocks, dev::kBlock, 0, st>>>(
                         m->h.nc, m->h.pairs, m->d_slot_face, m->d_slot_nbr, m->d_slot_far, u,
                         m->d_area, m->h.area0, m->d_vol, m->h.vol0, ts, tn, a, b, dt, mode, lim,
                         out, g.remap)));
    return hipGetLastError();
}

hipError_t launch_permute(int64_t n, int S, const int32_t *perm, int to_mesh, const double *in,
                          double *out, hipStream_t st) {
    const unsigned nb = (unsigned)((n + dev::kBlock - 1) / dev::kBlock);
    dev::permute_kernel<<<nb, dev::kBlock, 0, st>>>(n, S, perm, to_mesh, in, out);
    return hipGetLastError();
}

hipError_t launch_select(const fl_mesh *m, const double *u, int32_t *cdu, hipStream_t st) {
    const unsigned nb = (unsigned)((m->h.nf + dev::kBlock - 1) / dev::kBlock);
    dev::select_kernel<<<nb, dev::kBlock, 0, st>>>(
        m->h.nf, reinterpret_cast<const int4 *>(m->d_fc4), u, cdu);
    return hipGetLastError();
}

}  // namespace fl
