// Multi-step reverse sweep on meshes with aligned slots (the neighbour across slot k of a cell
// holds the shared face in its slot k ^ 1), gfx950, FP64: the face velocities enter as one signed
// rate per face, kept by the cell whose forward face it is, rf[p][x] = E_f a_f u_f of slot 2p (a
// quarter of the rate bytes of the two per-slot planes).  For slot k of x with neighbour n and
// far cell g the two rates the reverse stage needs follow from forward rates:
//   slot 2p (n across x's forward face):   w = rf[p][x],   w' = rf[p][n]   (n's forward face);
//   slot 2p + 1 (x across n's forward face): w = -rf[p][n], w' = -rf[p][g] (g's forward face is
//   the face of n beyond x, seen from n as its backward face).
// A negation is exact, so the rates, and the results, are the same bits as with the planes.  The
// LDS-staged kernel keeps the tile's forward rates and, for every halo entry (a cell reached
// along one pair's axis), that cell's forward rate of that pair beside its theta and lambda.
#include <hip/hip_runtime.h>

#include "fl_adjoint_device.h"

namespace fl {
namespace adev {

// rf[p][x] = E_f a_f u_f of x's forward face of pair p (a zero velocity as -0.0, as the planes).
template <int P>
__global__ __launch_bounds__(kBlock) void adjoint_fwd_rate_kernel(int64_t nc,
                                                                  const uint32_t *__restrict__ sface,
                                                                  const double *__restrict__ u,
                                                                  const double *__restrict__ area,
                                                                  double area0,
                                                                  double *__restrict__ rf) {
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= nc) return;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t fw = sface[(int64_t)(2 * p) * nc + x];
        const int64_t f = fw & 0x7fffffffu;
        const double uf = u[f] == 0.0 ? -0.0 : u[f];
        const double w = (area ? area[f] : area0) * uf;
        rf[(int64_t)p * nc + x] = (fw >> 31) ? w : -w;
    }
}

// Global-gather form (no tile tables or no LDS room): the neighbours' forward rates are gathered
// through the slot tables.
template <int S, int P, int LIM, bool UB>
__global__ __launch_bounds__(kBlock) void adjoint_fwd_stage_kernel(
    int64_t nc, const double *__restrict__ rf, const int32_t *__restrict__ snbr,
    const int32_t *__restrict__ sfar, const uint32_t *__restrict__ sface,
    const double *__restrict__ area, double area0, const double *__restrict__ vol, double ivol0,
    const double *__restrict__ th, const double *__restrict__ lam, double a, double b,
    double a3, double dt, int mode, const double *lin, const double *__restrict__ l3,
    double *out, double *__restrict__ uacc) {
    constexpr int K = 2 * P;
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= nc) return;
    int64_t nb[K], gf[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        nb[k] = snbr[(int64_t)k * nc + x];
        gf[k] = sfar[(int64_t)k * nc + x];
    }
    double2 wk[K];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int64_t row = (int64_t)p * nc;
        wk[2 * p].x = rf[row + x];
        wk[2 * p].y = rf[row + nb[2 * p]];
        wk[2 * p + 1].x = -rf[row + nb[2 * p + 1]];
        wk[2 * p + 1].y = -rf[row + gf[2 * p + 1]];
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

// LDS-staged form.  LDS: [0, rbase) theta, lambda (and V) of the tile and its halo, one entry
// per cell;
// then rates: the tile's forward rates [P][kTileCells], then one per halo
// entry (the entry's cell's forward rate of the entry's pair).  The tile's rates and the slot
// words and u-cotangent accumulators are requested after the theta / lambda gathers; the halo
// rates are gathered with the halo values.
template <int S, int P, int LIM, bool UB>
__global__ __launch_bounds__(kBlock) void adjoint_fwd_lds_kernel(
    int64_t nc, const double *__restrict__ rf, const int32_t *__restrict__ halo_ptr,
    const int32_t *__restrict__ halo, const uint8_t *__restrict__ halo_pair,
    const int32_t *__restrict__ halo_nrate, const uint32_t *__restrict__ slot_local,
    const uint32_t *__restrict__ sface,
    const double *__restrict__ area, double area0, const double *__restrict__ vol, double ivol0,
    const double *__restrict__ th, const double *__restrict__ lam, double a, double b, double a3,
    double dt, int mode, const double *lin, const double *__restrict__ l3, double *out,
    double *__restrict__ uacc, int rbase, int remap) {
    extern __shared__ double lds[];
    constexpr int K = 2 * P;
    const int st = 2 * S + (vol ? 1 : 0);  // LDS entry: theta [S], lambda [S], V
    const int64_t tile = dev::block_id(remap);
    if (tile * kTileCells >= nc) return;
    const int64_t c0 = tile * kTileCells;
    const int64_t left = nc - c0;
    const int nt = left < kTileCells ? (int)left : kTileCells;
    const int h0 = halo_ptr[tile], nh = halo_ptr[tile + 1] - h0;
    // the leading halo entries carry a needed rate (neighbours, and far cells of backward
    // slots); the others read their own cell's first rate instead (a line the tile reads anyway)
    const int nr = halo_nrate[2 * tile + 1];
    const int tid = threadIdx.x;
    double *rt = lds + rbase;                    // tile forward rates [P][kTileCells]
    double *rh = lds + rbase + P * kTileCells;  // one rate per halo entry
    const int64_t xc = c0 + (tid < nt ? tid : 0);
    double tv[S], lv[S], ht[kHaloAhead][S], hl[kHaloAhead][S], hr[kHaloAhead];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        tv[s] = th[xc * S + s];
        lv[s] = lam[xc * S + s];
    }
#pragma unroll
    for (int j = 0; j < kHaloAhead; ++j) {
        // a lane past the halo reads the halo's first entry (the arrays are padded) and its own
        // cell, and stores to the spare entry after the halo
        const int i = tid + j * kTileCells;
        const int ie = i < nh ? i : 0;
        const int64_t h = halo[h0 + ie];
        const int64_t pr = halo_pair[h0 + ie];
        const int64_t g = i < nh ? h : xc;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            ht[j][s] = th[g * S + s];
            hl[j][s] = lam[g * S + s];
        }
        hr[j] = rf[i < nr ? pr * nc + h : xc];
    }
    __builtin_amdgcn_sched_barrier(0);
    double rfv[P];
#pragma unroll
    for (int p = 0; p < P; ++p) rfv[p] = rf[(int64_t)p * nc + xc];
    __builtin_amdgcn_sched_barrier(0);
    uint32_t ll[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ll[k] = slot_local[(int64_t)k * nc + xc];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        lds[tid * st + s] = tv[s];
        lds[tid * st + S + s] = lv[s];
    }
#pragma unroll
    for (int j = 0; j < kHaloAhead; ++j) {
        const int i = tid + j * kTileCells;
        const int e = i < nh ? i : nh;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            lds[(kTileCells + e) * st + s] = ht[j][s];
            lds[(kTileCells + e) * st + S + s] = hl[j][s];
        }
        rh[e] = hr[j];
    }
#pragma unroll
    for (int p = 0; p < P; ++p) rt[p * kTileCells + tid] = rfv[p];
    for (int i = tid + kHaloAhead * kTileCells; i < nh; i += kTileCells) {
        const int64_t g = halo[h0 + i];
        const int64_t pr = halo_pair[h0 + i];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            lds[(kTileCells + i) * st + s] = th[g * S + s];
            lds[(kTileCells + i) * st + S + s] = lam[g * S + s];
        }
        if (i < nr) rh[i] = rf[pr * nc + g];
    }
    if (vol) {
        if (tid < nt) lds[tid * st + 2 * S] = vol[c0 + tid];
        for (int i = tid; i < nh; i += kTileCells)
            lds[(kTileCells + i) * st + 2 * S] = vol[halo[h0 + i]];
    }
    __syncthreads();
    if (tid >= nt) return;
    const int64_t x = c0 + tid;
    // forward rate of pair p of a cell with local index i (tile cell or halo entry of pair p)
    auto rate_of = [&](int p, uint32_t i) {
        return i < (uint32_t)kTileCells ? rt[p * kTileCells + i] : rh[i - kTileCells];
    };
    // slot k from its local word: rates from the LDS copies, read where they are used
    auto slot = [&](int k) {
        const uint32_t n = ll[k] & 0xffffu, g = ll[k] >> 16;
        const int p = k >> 1;
        if (k & 1) return AdjSlot{-rate_of(p, n), -rate_of(p, g), (int64_t)n, (int64_t)g};
        return AdjSlot{rate_of(p, (uint32_t)tid), rate_of(p, n), (int64_t)n, (int64_t)g};
    };
    auto af = [&](int p) {
        return area ? area[sface[(int64_t)(2 * p) * nc + x] & 0x7fffffffu] : area0;
    };
    double jt[S], lx[S];
    // the u cotangent is read and written where its term is formed (no accumulators held
    // through the cell's slots: registers decide this kernel's occupancy)
    const double scale = b * dt;
    auto ub = [&](int p, double t) {
        double &v = uacc[(int64_t)p * nc + x];
        v = fma(scale, t, v);
    };
    adj_cell_rate<S, P, LIM, true, UB>(tid, slot, lds, lds + S, vol ? lds + 2 * S : nullptr, st,
                                       st, ivol0, af, ub, jt, lx);
    adj_combine<S>(x, jt, lx, a, b, a3, dt, mode, lin, l3, out);
}

}  // namespace adev

namespace {
template <int S, int P, int LIM>
hipError_t launch_fwd3(const fl_mesh *m, const double *rf, const double *th, const double *lam,
                       double a, double b, double a3, double dt, int mode, const double *lin,
                       const double *l3, double *out, double *uacc, hipStream_t st) {
    const size_t lds = adjoint_lds_bytes(m, S);
    const double iv0 = 1.0 / m->h.vol0;
    const size_t flds =
        lds + ((size_t)P * kTileCells + m->h.max_halo + 1) * sizeof(double);
    if (lds > 0 && m->d_halo_pair && m->d_halo_nrate && flds <= kMaxStageLds) {
        const Grid g = launch_grid(m->h.nc);
        const int rbase = (int)(lds / sizeof(double));
#define FL_AFL(UB)                                                                                \
    adev::adjoint_fwd_lds_kernel<S, P, LIM, UB><<<g.blocks, adev::kBlock, flds, st>>>(            \
        m->h.nc, rf, m->d_halo_ptr, m->d_halo, m->d_halo_pair, m->d_halo_nrate, m->d_slot_local,  \
        m->d_slot_face,                                                                           \
        m->d_area, m->h.area0, m->d_vol, iv0, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc,   \
        rbase, g.remap)
        if (uacc) FL_AFL(true);
        else FL_AFL(false);
#undef FL_AFL
        return hipGetLastError();
    }
    const unsigned nb = (unsigned)((m->h.nc + adev::kBlock - 1) / adev::kBlock);
#define FL_AFG(UB)                                                                                \
    adev::adjoint_fwd_stage_kernel<S, P, LIM, UB><<<nb, adev::kBlock, 0, st>>>(                   \
        m->h.nc, rf, m->d_slot_nbr, m->d_slot_far, m->d_slot_face, m->d_area, m->h.area0,        \
        m->d_vol, iv0, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc)
    if (uacc) FL_AFG(true);
    else FL_AFG(false);
#undef FL_AFG
    return hipGetLastError();
}

template <int S, int P>
hipError_t launch_fwd2(const fl_mesh *m, int lim, const double *rf, const double *th,
                       const double *lam, double a, double b, double a3, double dt, int mode,
                       const double *lin, const double *l3, double *out, double *uacc,
                       hipStream_t st) {
#define FL_AFC(L) launch_fwd3<S, P, L>(m, rf, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st)
    switch (lim) {
        case FL_UPWIND: return FL_AFC(FL_UPWIND);
        case FL_MINMOD: return FL_AFC(FL_MINMOD);
        case FL_VANLEER: return FL_AFC(FL_VANLEER);
        case FL_VANALBADA: return FL_AFC(FL_VANALBADA);
        case FL_SUPERBEE: return FL_AFC(FL_SUPERBEE);
        case FL_SMART: return FL_AFC(FL_SMART);
        case FL_CENTRAL: return FL_AFC(FL_CENTRAL);
        default: return hipErrorInvalidValue;
    }
#undef FL_AFC
}

template <int S>
hipError_t launch_fwd1(const fl_mesh *m, int lim, const double *rf, const double *th,
                       const double *lam, double a, double b, double a3, double dt, int mode,
                       const double *lin, const double *l3, double *out, double *uacc,
                       hipStream_t st) {
    switch (m->h.pairs) {
        case 1: return launch_fwd2<S, 1>(m, lim, rf, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 2: return launch_fwd2<S, 2>(m, lim, rf, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 3: return launch_fwd2<S, 3>(m, lim, rf, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_adjoint_fwd_rates(const fl_mesh *m, const double *u, double *rf,
                                    hipStream_t st) {
    const unsigned nb = (unsigned)((m->h.nc + adev::kBlock - 1) / adev::kBlock);
    switch (m->h.pairs) {
        case 1: adev::adjoint_fwd_rate_kernel<1><<<nb, adev::kBlock, 0, st>>>(m->h.nc, m->d_slot_face, u, m->d_area, m->h.area0, rf); break;
        case 2: adev::adjoint_fwd_rate_kernel<2><<<nb, adev::kBlock, 0, st>>>(m->h.nc, m->d_slot_face, u, m->d_area, m->h.area0, rf); break;
        case 3: adev::adjoint_fwd_rate_kernel<3><<<nb, adev::kBlock, 0, st>>>(m->h.nc, m->d_slot_face, u, m->d_area, m->h.area0, rf); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_fwd_stage(const fl_mesh *m, int lim, int S, const double *rf,
                                    const double *th, const double *lam, double a, double b,
                                    double a3, double dt, int mode, const double *lin,
                                    const double *l3, double *out, double *uacc, hipStream_t st) {
    switch (S) {
        case 1: return launch_fwd1<1>(m, lim, rf, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 2: return launch_fwd1<2>(m, lim, rf, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 3: return launch_fwd1<3>(m, lim, rf, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 4: return launch_fwd1<4>(m, lim, rf, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 5: return launch_fwd1<5>(m, lim, rf, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 6: return launch_fwd1<6>(m, lim, rf, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 7: return launch_fwd1<7>(m, lim, rf, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        case 8: return launch_fwd1<8>(m, lim, rf, th, lam, a, b, a3, dt, mode, lin, l3, out, uacc, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fl
