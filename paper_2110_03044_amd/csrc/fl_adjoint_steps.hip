// Multi-step reverse sweep of the flux-limited convective operator (fl_rk_steps_adjoint), gfx950,
// FP64: the reverse stages of a checkpoint segment with the face velocities read from a per-call
// table of signed rates in cell-slot order and the face-velocity cotangent accumulated in
// cell-slot order (each face kept by the one cell whose forward face it is).  The per-face
// arithmetic is the per-step reverse stage's (fl_adjoint.hip), so the two give the same bits.
#include <hip/hip_runtime.h>

#include "fl_adjoint_device.h"

namespace fl {

namespace adev {

// ------------------------------------------------------------------------------------------
// Multi-step reverse sweep (fl_rk_steps_adjoint): the same arithmetic as adj_cell, with the face
// terms read from a per-call table of signed rates in cell-slot order instead of gathered through
// face indices, and the face-velocity cotangent accumulated in cell-slot order.
//
// rates: two planes of [2P][C] doubles.  Plane 0, w[k][x] = E_f a_f u_f: the rate of slot k's
// face f out of x (E_f = +1 where x owns f; a zero u_f is taken as -0.0, so that the sign bit of
// w tells whether x is the upwind cell, as Q(u_f) chooses it, also where the flux vanishes).
// Plane 1, w'[k][x]: the rate out of n_k of the face fr of n_k opposite to f (x is fr's
// far-upwind cell where w' > 0).  With mu and z as in adj_cell: z = a_f u_f mu =
// w (lambda_n/V_n - lambda_x/V_x) and the U term a_r u_r mu' = w' (lambda_g/V_g - lambda_n/V_n),
// the same products as adj_cell's up to exact sign changes, so the two paths give the same bits.
// uacc[p][x]: slot 2p is x's forward face of pair p (each face is forward for exactly one of its
// cells); it accumulates scale a_f sum_s theta_f (lambda_n/V_n - lambda_x/V_x), which is E_f times
// adj_cell's u_bar term.  adjoint_uacc_scatter_kernel adds E_f uacc to u_bar once at the end.
// ------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void adjoint_rate_kernel(int64_t nc,
                                                              const int2 *__restrict__ fr,
                                                              const double *__restrict__ u,
                                                              const double *__restrict__ area,
                                                              double area0,
                                                              double *__restrict__ rates) {
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= nc) return;
    const int64_t plane = (int64_t)2 * P * nc;
#pragma unroll
    for (int k = 0; k < 2 * P; ++k) {
        const int2 r = fr[(int64_t)k * nc + x];
        const int64_t f = (uint32_t)r.x & 0x7fffffffu, g = (uint32_t)r.y & 0x7fffffffu;
        // a zero velocity enters as -0.0: the rate is then -0.0 seen from the face's own cell and
        // +0.0 from its nbr, so that the sign bit still names the upwind cell (nbr where u_f <= 0)
        const double uf = u[f] == 0.0 ? -0.0 : u[f], ug = u[g] == 0.0 ? -0.0 : u[g];
        const double w = (area ? area[f] : area0) * uf;
        const double v = (area ? area[g] : area0) * ug;
        rates[(int64_t)k * nc + x] = ((uint32_t)r.x >> 31) ? w : -w;
        rates[plane + (int64_t)k * nc + x] = ((uint32_t)r.y >> 31) ? v : -v;
    }
}

// Global-gather form (meshes without tile tables or without LDS room).  a is the middle stage's
// a (3/4) in ADJ_FIRST mode.
template <int S, int P, int LIM, bool UB>
__global__ __launch_bounds__(kBlock) void adjoint_rate_stage_kernel(
    int64_t nc, const double *__restrict__ wr, const int32_t *__restrict__ snbr,
    const int32_t *__restrict__ sfar, const uint32_t *__restrict__ sface,
    const double *__restrict__ area, double area0, const double *__restrict__ vol, double ivol0,
    const double *__restrict__ th, const double *__restrict__ lam, double a, double b,
    double a3, double dt, int mode, const double *lin, const double *__restrict__ l3,
    double *out, double *__restrict__ uacc) {
    constexpr int K = 2 * P;
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= nc) return;
    double2 wk[K];
    int64_t nb[K], gf[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        wk[k].x = wr[(int64_t)k * nc + x];
        wk[k].y = wr[(int64_t)(K + k) * nc + x];
        nb[k] = snbr[(int64_t)k * nc + x];
        gf[k] = sfar[(int64_t)k * nc + x];
    }
    double ubk[P];
    if constexpr (UB) {
#pragma unroll
        for (int p = 0; p < P; ++p) ubk[p] = uacc[(int64_t)p * nc + x];
    }
    auto af = [&](int p) {
        return area ? area[sface[(int64_t)(2 * p) * nc + x] & 0x7fffffffu] : area0;
    };
    double jt[S], lx[S];
    auto slot = [&](int k) { return AdjSlot{wk[k].x, wk[k].y, nb[k], gf[k]}; };
    const double scale = b * dt;
    auto ub = [&](int p, double t) { ubk[p] = fma(scale, t, ubk[p]); };
    adj_cell_rate<S, P, LIM, false, UB>(x, slot, th, lam, vol, S, 1, ivol0, af, ub, jt, lx);
    if constexpr (UB) {
#pragma unroll
        for (int p = 0; p < P; ++p) uacc[(int64_t)p * nc + x] = ubk[p];
    }
    adj_combine<S>(x, jt, lx, a, b, a3, dt, mode, lin, l3, out);
}

// LDS-staged form: the tile's and its halo's theta and lambda (and volumes, where they differ)
// staged as in adjoint_stage_lds_kernel; the slot rates, local indices and the forward faces'
// u-cotangent accumulators are requested before the staging barrier and stay in flight across it.
template <int S, int P, int LIM, bool UB>
__global__ __launch_bounds__(kBlock) void adjoint_rate_lds_kernel(
    int64_t nc, const double *__restrict__ wr, const int32_t *__restrict__ halo_ptr,
    const int32_t *__restrict__ halo, const uint32_t *__restrict__ slot_local,
    const uint32_t *__restrict__ sface, const double *__restrict__ area, double area0,
    const double *__restrict__ vol, double ivol0, const double *__restrict__ th,
    const double *__restrict__ lam, double a, double b, double a3, double dt, int mode,
    const double *lin, const double *__restrict__ l3, double *out, double *__restrict__ uacc,
    int remap) {
    extern __shared__ double lds[];
    constexpr int K = 2 * P;
    const int st = 2 * S + (vol ? 1 : 0);
    const int64_t tile = dev::block_id(remap);
    if (tile * kTileCells >= nc) return;
    const int64_t c0 = tile * kTileCells;
    const int64_t left = nc - c0;
    const int nt = left < kTileCells ? (int)left : kTileCells;
    const int h0 = halo_ptr[tile], nh = halo_ptr[tile + 1] - h0;
    const int tid = threadIdx.x;
    const int64_t xc = c0 + (tid < nt ? tid : 0);
    double tv[S], lv[S], ht[kHaloAhead][S], hl[kHaloAhead][S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        tv[s] = th[xc * S + s];
        lv[s] = lam[xc * S + s];
    }
#pragma unroll
    for (int j = 0; j < kHaloAhead; ++j) {
        const int i = tid + j * kTileCells;
        const int64_t h = halo[h0 + (i < nh ? i : 0)];
        const int64_t g = i < nh ? h : xc;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            ht[j][s] = th[g * S + s];
            hl[j][s] = lam[g * S + s];
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    double2 wk[K];
    uint32_t ll[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        ll[k] = slot_local[(int64_t)k * nc + xc];
        wk[k].x = wr[(int64_t)k * nc + xc];
        wk[k].y = wr[(int64_t)(K + k) * nc + xc];
    }
    double ubk[P];
    if constexpr (UB) {
#pragma unroll
        for (int p = 0; p < P; ++p) ubk[p] = uacc[(int64_t)p * nc + xc];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        lds[tid * st + s] = tv[s];
        lds[tid * st + S + s] = lv[s];
    }
#pragma unroll
    for (int j = 0; j < kHaloAhead; ++j) {
        const int i = tid + j * kTileCells;
        const int e = kTileCells + (i < nh ? i : nh);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            lds[e * st + s] = ht[j][s];
            lds[e * st + S + s] = hl[j][s];
        }
    }
    for (int i = tid + kHaloAhead * kTileCells; i < nh; i += kTileCells) {
        const int64_t g = halo[h0 + i];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            lds[(kTileCells + i) * st + s] = th[g * S + s];
            lds[(kTileCells + i) * st + S + s] = lam[g * S + s];
        }
    }
    if (vol) {
        if (tid < nt) lds[tid * st + 2 * S] = vol[c0 + tid];
        for (int i = tid; i < nh; i += kTileCells)
            lds[(kTileCells + i) * st + 2 * S] = vol[halo[h0 + i]];
    }
    __syncthreads();
    if (tid >= nt) return;
    const int64_t x = c0 + tid;
    int64_t nl[K], gl[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        nl[k] = ll[k] & 0xffffu;
        gl[k] = ll[k] >> 16;
    }
    auto af = [&](int p) {
        return area ? area[sface[(int64_t)(2 * p) * nc + x] & 0x7fffffffu] : area0;
    };
    double jt[S], lx[S];
    auto slot = [&](int k) { return AdjSlot{wk[k].x, wk[k].y, nl[k], gl[k]}; };
    const double scale = b * dt;
    auto ub = [&](int p, double t) { ubk[p] = fma(scale, t, ubk[p]); };
    adj_cell_rate<S, P, LIM, true, UB>(tid, slot, lds, lds + S, vol ? lds + 2 * S : nullptr, st,
                                       st, ivol0, af, ub, jt, lx);
    if constexpr (UB) {
#pragma unroll
        for (int p = 0; p < P; ++p) uacc[(int64_t)p * nc + x] = ubk[p];
    }
    adj_combine<S>(x, jt, lx, a, b, a3, dt, mode, lin, l3, out);
}

// u_bar[f] += E_f uacc[p][x] for the forward face f of pair p of every cell x (each face once).
template <int P>
__global__ __launch_bounds__(kBlock) void adjoint_uacc_scatter_kernel(
    int64_t nc, const uint32_t *__restrict__ sface, const double *__restrict__ uacc,
    double *__restrict__ ubar) {
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= nc) return;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t fw = sface[(int64_t)(2 * p) * nc + x];
        const double v = uacc[(int64_t)p * nc + x];
        const int64_t f = fw & 0x7fffffffu;
        ubar[f] += (fw >> 31) ? v : -v;
    }
}

}  // namespace adev

namespace {
template <int S, int P, int LIM>
hipError_t launch_rate3(const fl_mesh *m, const double *wr, const double *th, const double *lam,
                        double a, double b, double a3, double dt, int mode, const double *lin,
                        const double *l3, double *out, double *uacc, hipStream_t st) {
    const size_t lds = adjoint_lds_bytes(m, S);
    const double iv0 = 1.0 / m->h.vol0;
    if (lds > 0 && lds <= kMaxStageLds) {
        const Grid g = launch_grid(m->h.nc);
#define FL_ARL(UB)                                                                                \
    adev::adjoint_rate_lds_kernel<S, P, LIM, UB><<<g.blocks, adev::kBlock, lds, st>>>(            \
        m->h.nc, wr, m->d_halo_ptr, m->d_halo, m->d_slot_local, m->d_slot_face, m->d_area,       \
        m->h.area0, m->d_vol, iv0, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, g.remap)
        if (uacc) FL_ARL(true);
        else FL_ARL(false);
#undef FL_ARL
        return hipGetLastError();
    }
    const unsigned nb = (unsigned)((m->h.nc + adev::kBlock - 1) / adev::kBlock);
#define FL_ARG(UB)                                                                                \
    adev::adjoint_rate_stage_kernel<S, P, LIM, UB><<<nb, adev::kBlock, 0, st>>>(                  \
        m->h.nc, wr, m->d_slot_nbr, m->d_slot_far, m->d_slot_face, m->d_area, m->h.area0,        \
        m->d_vol, iv0, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc)
    if (uacc) FL_ARG(true);
    else FL_ARG(false);
#undef FL_ARG
    return hipGetLastError();
}

template <int S, int P>
hipError_t launch_rate2(const fl_mesh *m, int lim, const double *wr, const double *th,
                        const double *lam, double a, double b, double a3, double dt, int mode,
                        const double *lin, const double *l3, double *out, double *uacc,
                        hipStream_t st) {
#define FL_ARC(L) launch_rate3<S, P, L>(m, wr, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st)
    switch (lim) {
        case FL_UPWIND: return FL_ARC(FL_UPWIND);
        case FL_MINMOD: return FL_ARC(FL_MINMOD);
        case FL_VANLEER: return FL_ARC(FL_VANLEER);
        case FL_VANALBADA: return FL_ARC(FL_VANALBADA);
        case FL_SUPERBEE: return FL_ARC(FL_SUPERBEE);
        case FL_SMART: return FL_ARC(FL_SMART);
        case FL_CENTRAL: return FL_ARC(FL_CENTRAL);
        default: return hipErrorInvalidValue;
    }
#undef FL_ARC
}

template <int S>
hipError_t launch_rate1(const fl_mesh *m, int lim, const double *wr, const double *th,
                        const double *lam, double a, double b, double a3, double dt, int mode,
                        const double *lin, const double *l3, double *out, double *uacc,
                        hipStream_t st) {
    switch (m->h.pairs) {
        case 1: return launch_rate2<S, 1>(m, lim, wr, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 2: return launch_rate2<S, 2>(m, lim, wr, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 3: return launch_rate2<S, 3>(m, lim, wr, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_adjoint_rates(const fl_mesh *m, const double *u, void *wr, hipStream_t st) {
    const unsigned nb = (unsigned)((m->h.nc + adev::kBlock - 1) / adev::kBlock);
    const int2 *fr = reinterpret_cast<const int2 *>(m->d_adj_fr);
    double *w = static_cast<double *>(wr);
    if (!fr) return hipErrorInvalidValue;
    switch (m->h.pairs) {
        case 1: adev::adjoint_rate_kernel<1><<<nb, adev::kBlock, 0, st>>>(m->h.nc, fr, u, m->d_area, m->h.area0, w); break;
        case 2: adev::adjoint_rate_kernel<2><<<nb, adev::kBlock, 0, st>>>(m->h.nc, fr, u, m->d_area, m->h.area0, w); break;
        case 3: adev::adjoint_rate_kernel<3><<<nb, adev::kBlock, 0, st>>>(m->h.nc, fr, u, m->d_area, m->h.area0, w); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_rate_stage(const fl_mesh *m, int lim, int S, const void *wr,
                                     const double *th, const double *lam, double a, double b,
                                     double a3, double dt, int mode, const double *lin,
                                     const double *l3, double *out, double *uacc, hipStream_t st) {
    const double *w = static_cast<const double *>(wr);
    switch (S) {
        case 1: return launch_rate1<1>(m, lim, w, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 2: return launch_rate1<2>(m, lim, w, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 3: return launch_rate1<3>(m, lim, w, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 4: return launch_rate1<4>(m, lim, w, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 5: return launch_rate1<5>(m, lim, w, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 6: return launch_rate1<6>(m, lim, w, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 7: return launch_rate1<7>(m, lim, w, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 8: return launch_rate1<8>(m, lim, w, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_uacc_scatter(const fl_mesh *m, const double *uacc, double *ubar,
                                       hipStream_t st) {
    const unsigned nb = (unsigned)((m->h.nc + adev::kBlock - 1) / adev::kBlock);
    switch (m->h.pairs) {
        case 1: adev::adjoint_uacc_scatter_kernel<1><<<nb, adev::kBlock, 0, st>>>(m->h.nc, m->d_slot_face, uacc, ubar); break;
        case 2: adev::adjoint_uacc_scatter_kernel<2><<<nb, adev::kBlock, 0, st>>>(m->h.nc, m->d_slot_face, uacc, ubar); break;
        case 3: adev::adjoint_uacc_scatter_kernel<3><<<nb, adev::kBlock, 0, st>>>(m->h.nc, m->d_slot_face, uacc, ubar); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fl
