// Discrete adjoint (reverse mode) of the flux-limited convective operator, gfx950, FP64.
//
// Forward, per face f with upwind C, downwind D and far-upwind U (selected by sign(u_f)):
//   theta_f = theta_C + g(d_U, d_u),  g = psi(d_U/d_u) d_u / 2,  d_U = theta_C - theta_U,
//   d_u = theta_D - theta_C,  rhs_c = sum_f E[f][c] a_f u_f theta_f / V_c.
// Reverse, for a cotangent lambda of rhs: mu_f = lambda_nbr/V_nbr - lambda_own/V_own and
// zeta_f = a_f u_f mu_f; then
//   theta_bar_C += zeta (1 + g_a - g_b),  theta_bar_D += zeta g_b,  theta_bar_U -= zeta g_a,
//   u_bar_f += a_f theta_f mu_f,
// with g_a = psi'(r)/2 and g_b = (psi(r) - r psi'(r))/2 (where d_u == 0: g_a = 0 and g_b the
// derivative along d_u > 0; where |r| is beyond the range evaluated as infinity, psi is
// constant: g_a = 0, g_b = psi(+-inf)/2).  Q(u_f) and the limiter branch are held fixed.
//
// No atomics: one thread per cell x gathers every contribution it receives -- from its own
// faces (x is C or D there) and from the faces for which it is the far-upwind cell U (the face
// of each neighbour n opposite to the face shared with x, flow running from n away from x).
// u_bar of a face is written only by the thread of the face's own cell.
#include <hip/hip_runtime.h>

#include "fl_adjoint_device.h"

namespace fl {
namespace adev {

// Face velocities and the u_bar entries of the faces the cell owns, requested before the slot
// loop (the per-slot theta / lambda reads stay next to their use: hoisting them as well raised
// register use and measured slower at 128^3).  u_bar is read once and written once per face
// (the slot faces are distinct, so the loads need not wait for earlier slots' stores).
template <int P>
__device__ __forceinline__ void adj_velocities(const uint32_t *fw, const uint32_t *rw,
                                               const double *__restrict__ u,
                                               const double *__restrict__ ubar, double *ufk,
                                               double *urk, double *ubk) {
#pragma unroll
    for (int k = 0; k < 2 * P; ++k) {
        ufk[k] = u[fw[k] & 0x7fffffffu];
        urk[k] = u[rw[k] & 0x7fffffffu];
        ubk[k] = (ubar != nullptr && (fw[k] >> 31)) ? ubar[fw[k] & 0x7fffffffu] : 0.0;
    }
}

// mode: ADJ_APPLY    theta_bar[x] += J^T lam, u_bar += (dL/du)^T lam            (scale 1)
//       ADJ_EULER    out[x] = lam[x] + dt J^T lam                               (b = 1)
//       ADJ_LAST     acc[x] = a lam[x];  out[x] = b (lam[x] + dt J^T lam)
//       ADJ_MID      acc[x] += a lam[x]; out[x] = b (lam[x] + dt J^T lam)
//       ADJ_FIRST    out[x] = acc[x] + b (lam[x] + dt J^T lam)
// and u_bar += scale (dL/du)^T lam with scale = b dt (1 for ADJ_APPLY).
//
// One cell x.  Slot k: face fw[k] (bit 31: x owns it), the face rw[k] of the neighbour opposite
// to it (bit 31: the neighbour owns that one), the neighbour and the far-upwind cell on its side
// with source indices nbi/gfi.  theta, lambda and the volume of a cell with source index i are
// tsrc[i * stride + s], lsrc[i * stride + s] and vsrc[i * vstride] (vsrc NULL: all volumes are
// 1 / ivol0): the global arrays (stride S, vstride 1, source index = global index) or a tile's
// LDS copy (interleaved per cell).
// ufk, urk, ubk0: slot k's face velocity, the opposite face's velocity and the face's u_bar
// entry (0 where x does not own it), loaded by adj_velocities.
// TNLDS: theta of the slot neighbours is read where it is used (cheap LDS reads in the staged
// kernel; keeping all 2P of them in registers would cost that kernel a wave per SIMD), else
// gathered once up front.
template <int S, int P, int LIM, bool TNLDS>
__device__ __forceinline__ void adj_cell(
    int64_t nc, int64_t x, int64_t xi, const uint32_t *fw, const uint32_t *rw,
    const int64_t *nbi, const int64_t *gfi, const double *tsrc, const double *lsrc,
    const double *vsrc, int stride, int vstride, const double *ufk, const double *urk,
    const double *ubk0, const double *__restrict__ area, double area0, double ivol0, double a,
    double b, double dt, int mode, double *__restrict__ out, double *__restrict__ acc,
    double *__restrict__ ubar) {
    constexpr int K = 2 * P;
    double tx[S], lx[S], tn[TNLDS ? 1 : K][S];
    load_s<S>(tsrc, xi, stride, tx);
    load_s<S>(lsrc, xi, stride, lx);
    if constexpr (!TNLDS) {
#pragma unroll
        for (int k = 0; k < K; ++k) load_s<S>(tsrc, nbi[k], stride, tn[k]);
    }
    // lambda / V appears in every face term: multiply by reciprocal volumes
    const double ivx = vsrc ? 1.0 / vsrc[xi * vstride] : ivol0;
    const double scale = (mode == ADJ_APPLY) ? 1.0 : b * dt;
    double jt[S];
#pragma unroll
    for (int s = 0; s < S; ++s) jt[s] = 0.0;
    double ubk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ubk[k] = ubk0[k];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t f = fw[k] & 0x7fffffffu, fr = rw[k] & 0x7fffffffu;
        const double uf = ufk[k], ur = urk[k];
        const double af = area ? area[f] : area0, ar = area ? area[fr] : area0;
        const double ivn = vsrc ? 1.0 / vsrc[nbi[k] * vstride] : ivol0;
        const double ivg = vsrc ? 1.0 / vsrc[gfi[k] * vstride] : ivol0;
        // theta of the neighbour across slot k and of the one across the opposite slot
        double tnk[S], tno[S];
        if constexpr (TNLDS) {
            load_s<S>(tsrc, nbi[k], stride, tnk);
            load_s<S>(tsrc, nbi[k ^ 1], stride, tno);
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                tnk[s] = tn[k][s];
                tno[s] = tn[k ^ 1][s];
            }
        }
        double ln[S], lg[S], tg[S];
        load_s<S>(lsrc, nbi[k], stride, ln);
        load_s<S>(lsrc, gfi[k], stride, lg);
        load_s<S>(tsrc, gfi[k], stride, tg);
        // face f between x and n
        const bool x_own = (fw[k] >> 31) != 0;
        const bool x_up = ((uf > 0.0) == x_own);
        double usum = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            double ga, gb;
            // pick (theta_C, theta_D, theta_U) first: one evaluation even where lanes diverge
            const double tC = x_up ? tx[s] : tnk[s];
            const double tD = x_up ? tnk[s] : tx[s];
            const double tU = x_up ? tno[s] : tg[s];
            const double tf = face_value_d<LIM>(tC, tD, tU, ga, gb);
            // one rounding of the difference, then the sign (the same bits from either cell)
            const double d = cot_diff(ln[s], ivn, lx[s], ivx);
            const double mu = x_own ? d : -d;
            const double z = af * uf * mu;
            jt[s] += x_up ? mul_nc(z, 1.0 + ga - gb) : mul_nc(z, gb);
            usum += tf * mu;
        }
        ubk[k] = fma(scale, af * usum, ubk[k]);
        // face fr between n and g, opposite to f in n: x is its far-upwind cell when the flow
        // runs from n to g
        const bool n_own = (rw[k] >> 31) != 0;
        if ((ur > 0.0) == n_own) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                double ga, gb;
                (void)face_value_d<LIM>(tnk[s], tg[s], tx[s], ga, gb);
                const double d = cot_diff(lg[s], ivg, ln[s], ivn);
                const double mu = n_own ? d : -d;
                jt[s] -= mul_nc(ar * ur * mu, ga);
            }
        }
    }
    if (ubar != nullptr) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (fw[k] >> 31) ubar[fw[k] & 0x7fffffffu] = ubk[k];
    }
    // the roundings written out (explicit fma), as in adj_combine
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t i = x * S + s;
        switch (mode) {
            case ADJ_APPLY: out[i] += jt[s]; break;
            case ADJ_EULER: out[i] = fma(dt, jt[s], lx[s]); break;
            case ADJ_LAST:
                acc[i] = a * lx[s];
                out[i] = b * fma(dt, jt[s], lx[s]);
                break;
            case ADJ_MID:
                acc[i] = fma(a, lx[s], acc[i]);
                out[i] = b * fma(dt, jt[s], lx[s]);
                break;
            default: out[i] = fma(b, fma(dt, jt[s], lx[s]), acc[i]); break;
        }
    }
}

// rec[k][x] = {face of slot k | bit 31 if x owns it, face of the neighbour n_k opposite to it |
// bit 31 if n_k owns that one, n_k, far-upwind cell on n_k's side}: one 16-byte load per slot.
template <int P>
__device__ __forceinline__ void read_rec(int64_t nc, int64_t x, const int4 *__restrict__ rec,
                                         uint32_t *fw, uint32_t *rw, int64_t *nb, int64_t *gf) {
#pragma unroll
    for (int k = 0; k < 2 * P; ++k) {
        const int4 r = rec[(int64_t)k * nc + x];
        fw[k] = (uint32_t)r.x;
        rw[k] = (uint32_t)r.y;
        nb[k] = r.z;
        gf[k] = r.w;
    }
}

// One thread per cell, theta and lambda gathered from global memory.
template <int S, int P, int LIM>
__global__ __launch_bounds__(kBlock) void adjoint_stage_kernel(
    int64_t nc, const int4 *__restrict__ rec, const double *__restrict__ u,
    const double *__restrict__ area, double area0, const double *__restrict__ vol, double ivol0,
    const double *__restrict__ th, const double *__restrict__ lam, double a, double b, double dt,
    int mode, double *__restrict__ out, double *__restrict__ acc, double *__restrict__ ubar) {
    constexpr int K = 2 * P;
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= nc) return;
    uint32_t fw[K], rw[K];
    int64_t nb[K], gf[K];
    read_rec<P>(nc, x, rec, fw, rw, nb, gf);
    double ufk[K], urk[K], ubk[K];
    adj_velocities<P>(fw, rw, u, ubar, ufk, urk, ubk);
    adj_cell<S, P, LIM, false>(nc, x, x, fw, rw, nb, gf, th, lam, vol, S, 1, ufk, urk, ubk, area,
                               area0, ivol0, a, b, dt, mode, out, acc, ubar);
}

// One workgroup per tile of kTileCells cells: theta, lambda (and the volume, where volumes
// differ) of the tile and of its halo are staged in LDS, interleaved per cell, each read from
// global memory once per tile; then every cell reads them there through the 16-bit local slot
// indices of the forward's tile tables, and its faces from 8-byte {face, opposite face} records.
// Dynamic LDS of (kTileCells + max halo + 1) * (2 S + [1]) doubles.  Same arithmetic as
// adjoint_stage_kernel, so the results are bit-identical.
template <int S, int P, int LIM>
__global__ __launch_bounds__(kBlock) void adjoint_stage_lds_kernel(
    int64_t nc, const int2 *__restrict__ fr, const int32_t *__restrict__ halo_ptr,
    const int32_t *__restrict__ halo, const uint32_t *__restrict__ slot_local,
    const double *__restrict__ u, const double *__restrict__ area, double area0,
    const double *__restrict__ vol, double ivol0, const double *__restrict__ th,
    const double *__restrict__ lam, double a, double b, double dt, int mode,
    double *__restrict__ out, double *__restrict__ acc, double *__restrict__ ubar, int remap) {
    extern __shared__ double lds[];
    constexpr int K = 2 * P;
    const int st = 2 * S + (vol ? 1 : 0);
    // the tile is the same for the whole workgroup: padding workgroups leave before the barrier
    const int64_t tile = dev::block_id(remap);
    if (tile * kTileCells >= nc) return;
    const int64_t c0 = tile * kTileCells;
    const int64_t left = nc - c0;
    const int nt = left < kTileCells ? (int)left : kTileCells;
    const int h0 = halo_ptr[tile], nh = halo_ptr[tile + 1] - h0;
    const int tid = threadIdx.x;
    // As the forward's first chunk: theta and lambda of the tile cell and of the first
    // kHaloAhead halo entries are gathered, then the slot records are loaded, then the gathered
    // values are stored.  No load sits in a branch, so the records stay in flight across the
    // barrier: a lane past the tile reads its first cell, one past the halo the halo's first
    // entry (the array is padded) and its own cell, and stores to the spare entry after the halo.
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
    int2 rr[K];
    uint32_t ll[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        rr[k] = fr[(int64_t)k * nc + xc];
        ll[k] = slot_local[(int64_t)k * nc + xc];
    }
    // the records are needed now: their velocity and u_bar gathers then stay in flight across
    // the barrier as well (the records arrive right behind the theta / lambda gathers)
    uint32_t fw[K], rw[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        fw[k] = (uint32_t)rr[k].x;
        rw[k] = (uint32_t)rr[k].y;
    }
    double ufk[K], urk[K], ubk[K];
    adj_velocities<P>(fw, rw, u, ubar, ufk, urk, ubk);
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
    adj_cell<S, P, LIM, true>(nc, x, tid, fw, rw, nl, gl, lds, lds + S, vol ? lds + 2 * S : nullptr,
                              st, st, ufk, urk, ubk, area, area0, ivol0, a, b, dt, mode, out, acc,
                              ubar);
}

}  // namespace adev

namespace {
template <int S, int P, int LIM>
hipError_t launch3(const fl_mesh *m, const double *u, const double *th, const double *lam,
                   double a, double b, double dt, int mode, double *out, double *acc,
                   double *ubar, hipStream_t st) {
    const size_t lds = adjoint_lds_bytes(m, S);
    if (lds > 0 && lds <= kMaxStageLds) {
        const Grid g = launch_grid(m->h.nc);  // one workgroup per tile (kBlock == kTileCells)
        adev::adjoint_stage_lds_kernel<S, P, LIM><<<g.blocks, adev::kBlock, lds, st>>>(
            m->h.nc, reinterpret_cast<const int2 *>(m->d_adj_fr), m->d_halo_ptr, m->d_halo,
            m->d_slot_local, u, m->d_area, m->h.area0, m->d_vol, 1.0 / m->h.vol0, th, lam, a, b,
            dt, mode, out, acc, ubar, g.remap);
        return hipGetLastError();
    }
    const unsigned nb = (unsigned)((m->h.nc + adev::kBlock - 1) / adev::kBlock);
    adev::adjoint_stage_kernel<S, P, LIM><<<nb, adev::kBlock, 0, st>>>(
        m->h.nc, reinterpret_cast<const int4 *>(m->d_adj_rec), u, m->d_area, m->h.area0,
        m->d_vol, 1.0 / m->h.vol0, th, lam, a, b, dt, mode, out, acc, ubar);
    return hipGetLastError();
}

template <int S, int P>
hipError_t launch2(const fl_mesh *m, int lim, const double *u, const double *th,
                   const double *lam, double a, double b, double dt, int mode, double *out,
                   double *acc, double *ubar, hipStream_t st) {
    switch (lim) {
        case FL_UPWIND: return launch3<S, P, FL_UPWIND>(m, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case FL_MINMOD: return launch3<S, P, FL_MINMOD>(m, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case FL_VANLEER: return launch3<S, P, FL_VANLEER>(m, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case FL_VANALBADA: return launch3<S, P, FL_VANALBADA>(m, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case FL_SUPERBEE: return launch3<S, P, FL_SUPERBEE>(m, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case FL_SMART: return launch3<S, P, FL_SMART>(m, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case FL_CENTRAL: return launch3<S, P, FL_CENTRAL>(m, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        default: return hipErrorInvalidValue;
    }
}

template <int S>
hipError_t launch1(const fl_mesh *m, int lim, const double *u, const double *th,
                   const double *lam, double a, double b, double dt, int mode, double *out,
                   double *acc, double *ubar, hipStream_t st) {
    switch (m->h.pairs) {
        case 1: return launch2<S, 1>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 2: return launch2<S, 2>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 3: return launch2<S, 3>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_adjoint(const fl_mesh *m, int lim, int S, const double *u, const double *th,
                          const double *lam, double a, double b, double dt, int mode, double *out,
                          double *acc, double *ubar, hipStream_t st) {
    switch (S) {
        case 1: return launch1<1>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 2: return launch1<2>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 3: return launch1<3>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 4: return launch1<4>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 5: return launch1<5>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 6: return launch1<6>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 7: return launch1<7>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        case 8: return launch1<8>(m, lim, u, th, lam, a, b, dt, mode, out, acc, ubar, st);
        default: return hipErrorInvalidValue;
    }
}


}  // namespace fl
