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

// LDS-staged forms.  LDS: [0, rbase) theta, lambda (and V) of the tile and its halo, one entry
// per cell (st doubles); then rates: the tile's forward rates [P][kTileCells], then one per halo
// entry (the entry's cell's forward rate of the entry's pair).  The tile's rates and the slot
// words are requested after the theta / lambda gathers; the halo rates are gathered with the
// halo values (only the leading nr entries carry a rate these stages read: neighbours, and far
// cells of backward slots; the others read their own cell's first rate, a line the tile reads
// anyway).  Ends without a barrier; ll receives the thread's slot words.
template <int S, int P>
__device__ __forceinline__ void adj_stage_fwd(double *lds, int st, int rbase, int64_t nc,
                                              int64_t c0, int nt, int h0, int nh, int nr,
                                              const double *__restrict__ rf,
                                              const int32_t *__restrict__ halo,
                                              const uint8_t *__restrict__ halo_pair,
                                              const uint32_t *__restrict__ slot_local,
                                              const double *__restrict__ vol,
                                              const double *__restrict__ th,
                                              const double *__restrict__ lam, uint32_t *ll) {
    constexpr int K = 2 * P;
    const int tid = threadIdx.x;
    double *rt = lds + rbase;                   // tile forward rates [P][kTileCells]
    double *rh = lds + rbase + P * kTileCells;  // one rate per rated halo entry
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
#pragma unroll
    for (int k = 0; k < K; ++k) ll[k] = slot_local[(int64_t)k * nc + xc];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        lds[tid * st + s] = tv[s];
        lds[tid * st + S + s] = lv[s];
    }
    // (lanes past the halo, or past its rated entries, store nothing: no spare entries)
#pragma unroll
    for (int j = 0; j < kHaloAhead; ++j) {
        const int i = tid + j * kTileCells;
        if (i < nh) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                lds[(kTileCells + i) * st + s] = ht[j][s];
                lds[(kTileCells + i) * st + S + s] = hl[j][s];
            }
        }
        if (i < nr) rh[i] = hr[j];
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
}

// Cell-wise form: every thread evaluates all its slots' faces (and the faces beyond its
// neighbours of which it is the far-upwind cell) from the staged values.
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
    const int nr = halo_nrate[2 * tile + 1];
    const int tid = threadIdx.x;
    uint32_t ll[K];
    adj_stage_fwd<S, P>(lds, st, rbase, nc, c0, nt, h0, nh, nr, rf, halo, halo_pair, slot_local,
                        vol, th, lam, ll);
    __syncthreads();
    if (tid >= nt) return;
    const double *rt = lds + rbase;
    const double *rh = lds + rbase + P * kTileCells;
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

// Face-wise form: each face the tile needs is evaluated once and its terms are shared through
// LDS, then every cell sums its terms in the cell-wise form's order (the same bits).
//  * Each tile cell evaluates its P forward faces: its own term, its forward neighbour's term
//    (rn) and the far-upwind term (ru, subtracted by whichever cell is the face's far-upwind
//    cell).
//  * A face owned by a halo entry (the entry's cell's forward face of the entry's pair) is an
//    item: the leading nr entries are the only ones whose face a tile cell can need (the backward
//    neighbours, whose face gives that tile cell's own term, and the cells beyond a neighbour,
//    whose face gives a far-upwind term).  The tile cell that needs an item writes its
//    descriptor (the face's other cell and its far-upwind cell for the face's flow direction);
//    the items are then spread over all threads (no thread evaluates a tile-boundary face for
//    its own cell alone, which would hold a whole wave).
//  * After the last read of the staged values, the terms go to LDS over the staged values and
//    each cell gathers its slots' terms.
// Needs S <= 2 (the terms live in registers across the barriers) and nr <= J kTileCells.
constexpr uint32_t kNoItem = 0xffffffffu;

template <int S, int P, int LIM, bool UB, int J>
__global__ __launch_bounds__(kBlock) void adjoint_fwd_share_kernel(
    int64_t nc, const double *__restrict__ rf, const int32_t *__restrict__ halo_ptr,
    const int32_t *__restrict__ halo, const uint8_t *__restrict__ halo_pair,
    const int32_t *__restrict__ halo_nrate, const uint32_t *__restrict__ slot_local,
    const uint32_t *__restrict__ sface,
    const double *__restrict__ area, double area0, const double *__restrict__ vol, double ivol0,
    const double *__restrict__ th, const double *__restrict__ lam, double a, double b, double a3,
    double dt, int mode, const double *lin, const double *__restrict__ l3, double *out,
    double *__restrict__ uacc, int rbase, int dbase, int remap) {
    extern __shared__ double lds[];
    constexpr int K = 2 * P;
    constexpr uint32_t T = kTileCells;
    const int st = 2 * S + (vol ? 1 : 0);
    const int64_t tile = dev::block_id(remap);
    if (tile * kTileCells >= nc) return;
    const int64_t c0 = tile * kTileCells;
    const int64_t left = nc - c0;
    const int nt = left < kTileCells ? (int)left : kTileCells;
    const int h0 = halo_ptr[tile], nh = halo_ptr[tile + 1] - h0;
    const int n0 = halo_nrate[2 * tile], nr = halo_nrate[2 * tile + 1];
    const int tid = threadIdx.x;
    uint32_t *desc = reinterpret_cast<uint32_t *>(lds + dbase);  // one per item (nr)
    uint32_t ll[K];
    adj_stage_fwd<S, P>(lds, st, rbase, nc, c0, nt, h0, nh, nr, rf, halo, halo_pair, slot_local,
                        vol, th, lam, ll);
    for (int e = tid; e < nr; e += kTileCells) desc[e] = kNoItem;
    __syncthreads();
    const double *rt = lds + rbase;
    const double *rh = lds + rbase + P * kTileCells;
    auto rate_of = [&](int p, uint32_t i) {
        return i < T ? rt[p * kTileCells + i] : rh[i - T];
    };
    auto tv = [&](uint32_t i, int s) { return lds[i * st + s]; };
    auto lv = [&](uint32_t i, int s) { return lds[i * st + S + s]; };
    auto iv = [&](uint32_t i) { return vol ? 1.0 / lds[i * st + 2 * S] : ivol0; };
    const bool live = tid < nt;
    const int64_t x = c0 + tid;
    double own[P][S], rn[P][S], ru[P][S], lx[S];
    uint32_t frm = 0;  // bit k: slot k's far-upwind term applies (w' > 0)
    if (live) {
        double tx[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            tx[s] = tv(tid, s);
            lx[s] = lv(tid, s);
        }
        const double ivx = iv(tid);
        const double scale = b * dt;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint32_t n = ll[2 * p] & 0xffffu, g = ll[2 * p] >> 16;
            const uint32_t bn = ll[2 * p + 1] & 0xffffu, bg = ll[2 * p + 1] >> 16;
            // the forward face (x, n): x is its upwind cell where !signbit(w)
            const double w = rt[p * kTileCells + tid];
            const bool x_up = !signbit(w);
            const uint32_t u = x_up ? bn : g;
            const double ivn = iv(n);
            double usum = 0.0;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                double ga, gb;
                const double tn = tv(n, s);
                const double tf =
                    face_value_d<LIM>(x_up ? tx[s] : tn, x_up ? tn : tx[s], tv(u, s), ga, gb);
                const double d = cot_diff(lv(n, s), ivn, lx[s], ivx);
                const double z = w * d;
                const double up = mul_nc(z, 1.0 + ga - gb), dn = mul_nc(z, gb);
                own[p][s] = x_up ? up : dn;
                rn[p][s] = x_up ? dn : up;
                ru[p][s] = mul_nc(z, ga);
                if (UB) usum += tf * d;
            }
            if constexpr (UB) {
                const double af = area ? area[sface[(int64_t)(2 * p) * nc + x] & 0x7fffffffu]
                                       : area0;
                double &v = uacc[(int64_t)p * nc + x];
                v = fma(scale, af * usum, v);
            }
            const double wpf = rate_of(p, n), wpb = -rate_of(p, bg);
            if (wpf > 0.0) frm |= 1u << (2 * p);
            if (wpb > 0.0) frm |= 1u << (2 * p + 1);
            // items: the backward face (bn, x) when bn is a halo entry (x's own term; its
            // far-upwind cell: x's forward neighbour where x is upwind, else bg)
            if (bn >= T) desc[bn - T] = (uint32_t)tid | (signbit(rate_of(p, bn)) ? n : bg) << 16;
            // the face (n, g) where the flow leaves n towards g (x is its far-upwind cell), and
            // the face (bg, bn) where it leaves bn towards bg, when not an item already
            if (n >= T && (int)(n - T) >= n0 && wpf > 0.0) desc[n - T] = g | (uint32_t)tid << 16;
            if (bg >= T && (int)(bg - T) >= n0 && wpb > 0.0)
                desc[bg - T] = bn | (uint32_t)tid << 16;
        }
    }
    __syncthreads();
    // items: face (h, hf) of halo entry e = h - T with its far-upwind cell fu; io: the term of
    // hf (a tile cell where the item came from a backward face), ifr: the far-upwind term
    double io[J][S], ifr[J][S];
    bool has[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int e = tid + j * kTileCells;
        const uint32_t dw = e < nr ? desc[e] : kNoItem;
        has[j] = dw != kNoItem;
        if (has[j]) {
            const uint32_t h = T + (uint32_t)e, hf = dw & 0xffffu, fu = dw >> 16;
            const double wh = rh[e];
            const bool h_up = !signbit(wh);
            const uint32_t cc = h_up ? h : hf, cd = h_up ? hf : h;
            const double ivh = iv(h), ivf = iv(hf);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                double ga, gb;
                (void)face_value_d<LIM>(tv(cc, s), tv(cd, s), tv(fu, s), ga, gb);
                const double z = wh * cot_diff(lv(hf, s), ivf, lv(h, s), ivh);
                io[j][s] = h_up ? mul_nc(z, gb) : mul_nc(z, 1.0 + ga - gb);
                ifr[j][s] = mul_nc(z, ga);
            }
        }
    }
    __syncthreads();
    // terms over the staged values: rn [P][T][S], ru [P][T][S], item terms [nr][S] twice
    double *trn = lds, *tru = lds + P * kTileCells * S;
    double *tio = lds + 2 * P * kTileCells * S, *tif = tio + nr * S;
    if (live) {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int s = 0; s < S; ++s) {
                trn[(p * kTileCells + tid) * S + s] = rn[p][s];
                tru[(p * kTileCells + tid) * S + s] = ru[p][s];
            }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int e = tid + j * kTileCells;
        if (has[j]) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                tio[e * S + s] = io[j][s];
                tif[e * S + s] = ifr[j][s];
            }
        }
    }
    __syncthreads();
    if (!live) return;
    // far-upwind term of the forward face of local cell i (tile cell or item) of pair p
    auto fr_of = [&](int p, uint32_t i, int s) {
        return i < T ? tru[(p * kTileCells + i) * S + s] : tif[(i - T) * S + s];
    };
    double jt[S];
#pragma unroll
    for (int s = 0; s < S; ++s) jt[s] = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t n = ll[2 * p] & 0xffffu;
        const uint32_t bn = ll[2 * p + 1] & 0xffffu, bg = ll[2 * p + 1] >> 16;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            jt[s] += own[p][s];
            if (frm >> (2 * p) & 1u) jt[s] -= fr_of(p, n, s);
            jt[s] += bn < T ? trn[(p * kTileCells + bn) * S + s] : tio[(bn - T) * S + s];
            if (frm >> (2 * p + 1) & 1u) jt[s] -= fr_of(p, bg, s);
        }
    }
    adj_combine<S>(x, jt, lx, a, b, a3, dt, mode, lin, l3, out);
}

}  // namespace adev

namespace {
int g_adjoint_share = 1;  // FL_OPT_FACE_SHARE

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
        if constexpr (S <= 2) {
            // face-wise form: the staged values and the rates of the rated halo entries with no
            // spare entries (a workgroup per CU more on brick tiles), descriptors after them;
            // the terms over all of it
            const int nr = m->h.max_nrate;
            const int per = 2 * S + (m->d_vol ? 1 : 0);  // doubles per staged entry
            const size_t vlds = (size_t)(kTileCells + m->h.max_halo) * per * sizeof(double);
            const size_t flds2 = vlds + ((size_t)P * kTileCells + (nr > 0 ? nr : 0)) * sizeof(double);
            const size_t dlds = flds2 + ((size_t)nr * sizeof(uint32_t) + 7) / 8 * 8;
            const size_t tlds = ((size_t)2 * P * kTileCells + 2 * (size_t)nr) * S * sizeof(double);
            const size_t slds = dlds > tlds ? dlds : tlds;
            if (g_adjoint_share && nr >= 0 && nr <= 2 * kTileCells && slds <= kMaxStageLds) {
                const int sbase = (int)(vlds / sizeof(double));
                const int dbase = (int)(flds2 / sizeof(double));
#define FL_AFS(UB, J)                                                                             \
    adev::adjoint_fwd_share_kernel<S, P, LIM, UB, J><<<g.blocks, adev::kBlock, slds, st>>>(       \
        m->h.nc, rf, m->d_halo_ptr, m->d_halo, m->d_halo_pair, m->d_halo_nrate, m->d_slot_local,  \
        m->d_slot_face, m->d_area, m->h.area0, m->d_vol, iv0, th, lam, a, b, a3, dt, mode, lin,   \
        l3, out, uacc, sbase, dbase, g.remap)
                if (nr <= kTileCells) {
                    if (uacc) FL_AFS(true, 1);
                    else FL_AFS(false, 1);
                } else {
                    if (uacc) FL_AFS(true, 2);
                    else FL_AFS(false, 2);
                }
#undef FL_AFS
                return hipGetLastError();
            }
        }
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

void set_adjoint_share(int on) { g_adjoint_share = on; }

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
