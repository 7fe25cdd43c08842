// Device routines shared by the single-problem and the batched kernels: the limiter, the
// limited face value and the fused per-cell stage.  Both launch paths call exactly this code, so
// a problem advanced inside a batch gives the same bits as when advanced alone.
#pragma once

#include <hip/hip_runtime.h>

#include "fl_kernels.h"

namespace fl {
namespace dev {

// Workgroup -> cell tile.  Dispatch sends workgroup d to XCD d mod 8; with chunk M > 0 (the grid
// padded to a multiple of 8 M) XCD x takes runs of M consecutive tiles, so the tiles one XCD
// (one L2) works on at a time are neighbours on the cell curve.  M = grid / 8 gives each XCD a
// contiguous eighth of the mesh.
__device__ __forceinline__ int64_t block_id(int chunk) {
    if (!chunk) return blockIdx.x;
    const int64_t d = blockIdx.x, xcd = d & 7, local = d >> 3;
    return (local / chunk) * (8 * (int64_t)chunk) + xcd * chunk + local % chunk;
}

constexpr double kRBig = 1.0e18;

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

// Limiters of Sweby's family (superbee as in Table 1 of the paper).
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

// The limited correction psi(r) b / 2 of the Sweby form, r = a / b (a = d_U, b = d_u != 0),
// written so that the limiter needs no division where its form allows: for r > 0, with
// A = |a|, B = |b| and s the sign of b (r = A / B), psi(r) B is min(A, B) for minmod,
// max(min(B, 2A), min(A, 2B)) for superbee and min(2A, B/4 + 3A/4, 4B) for SMART, and
// psi(r) b / 2 = a b / (a + b) for van Leer; all of them vanish for r <= 0.  Van Albada gives
// a b (a + b) / (2 (a^2 + b^2)) for every r (one reciprocal; the ratio where a^2 + b^2 would
// under- or overflow).  Each form tends to psi(+-inf) b / 2 as |r| grows, as the ratio form does
// past |r| = 1e18.
__device__ __forceinline__ double limited_half(int lim, double a, double b) {
    const bool same = (a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0);  // r > 0
    const double A = fabs(a), B = fabs(b);
    const double s = b > 0.0 ? 0.5 : -0.5;
    switch (lim) {
        case FL_MINMOD: return same ? s * fmin(A, B) : 0.0;
        case FL_SUPERBEE: return same ? s * fmax(fmin(B, 2.0 * A), fmin(A, 2.0 * B)) : 0.0;
        case FL_SMART: return same ? s * fmin(fmin(2.0 * A, 0.25 * B + 0.75 * A), 4.0 * B) : 0.0;
        case FL_VANLEER: return same ? a * (b / (a + b)) : 0.0;
        case FL_VANALBADA: {
            const double q = a * a + b * b;
            if (q >= 1e-280 && q <= 1e280) return 0.5 * (a * b) * (a + b) / q;
            return 0.5 * psi(lim, a / b) * b;
        }
        case FL_CENTRAL: return 0.5 * b;
        default: return 0.0;
    }
}

// Limited face value of the Sweby form from the upwind, downwind and far-upwind values:
// theta_C + psi(r) (theta_D - theta_C) / 2, r = (theta_C - theta_U) / (theta_D - theta_C).
__device__ __forceinline__ double face_value(int lim, double tC, double tD, double tU) {
    const double du = tD - tC;
    if (lim == FL_UPWIND || du == 0.0) return tC;
    return tC + limited_half(lim, tC - tU, du);
}

// The same from the differences themselves, for cells whose upstream difference projects on
// several faces: d_U = sum_j w_j (theta_C - theta_j), d_u = theta_D - theta_C.
__device__ __forceinline__ double face_value_d(int lim, double tC, double du, double dU) {
    if (lim == FL_UPWIND || du == 0.0) return tC;
    return tC + limited_half(lim, dU, du);
}

// Scalars S0 .. S0+CS-1 of cell c.  theta_s of a cell with source index i is
// src[i * SST + SOFF + s] for s < CS: src is theta_s itself (SST = S, SOFF = S0, global indices)
// or a tile's LDS copy of this chunk (SST = CS, SOFF = 0, local indices); tn and out are indexed
// by the global cell c.
// PRE: theta_n of the chunk was loaded ahead into tnv (stage-combination mode only).  IDX: the
// index type (64-bit global cell indices, or 32-bit tile-local ones, fewer registers to keep
// across the chunks of many scalars).
template <int S, int P, int S0, int CS, int SST, int SOFF, bool PRE = false,
          typename IDX = int64_t>
__device__ __forceinline__ void fused_chunk(int64_t c, int64_t cs, const double *src,
                                            const double *w, const IDX *nb, const IDX *gf,
                                            double V, const double *__restrict__ tn, double a,
                                            double b, double dt, int mode, int lim,
                                            double *__restrict__ out,
                                            const double *tnv = nullptr) {
    constexpr int K = 2 * P;
    double tc[CS], acc[CS];
#pragma unroll
    for (int i = 0; i < CS; ++i) tc[i] = src[cs * SST + SOFF + i];
#pragma unroll
    for (int i = 0; i < CS; ++i) acc[i] = 0.0;
    // Face k of the cell: Q(u_f) makes c the upwind cell C where the flow leaves c (w_k > 0;
    // where w_k == 0 the flux vanishes whichever cell is taken).  tnk: the neighbour across k,
    // tno: across the opposite slot k ^ 1, tgk: the far cell beyond the neighbour.
    auto face = [&](int k, const double *tnk, const double *tno, const double *tgk) {
        const bool c_upwind = w[k] > 0.0;
#pragma unroll
        for (int i = 0; i < CS; ++i) {
            // pick (theta_C, theta_D, theta_U) first: one evaluation where lanes diverge
            const double tC = c_upwind ? tc[i] : tnk[i];
            const double tD = c_upwind ? tnk[i] : tc[i];
            const double tU = c_upwind ? tno[i] : tgk[i];
            acc[i] -= w[k] * face_value(lim, tC, tD, tU);
        }
    };
    if constexpr (S <= 2) {
        // one chunk: every gather issued ahead
        double tnb[K][CS], tg[K][CS];
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int i = 0; i < CS; ++i) tnb[k][i] = src[nb[k] * SST + SOFF + i];
            if (lim != FL_UPWIND) {
#pragma unroll
                for (int i = 0; i < CS; ++i) tg[k][i] = src[gf[k] * SST + SOFF + i];
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) face(k, tnb[k], tnb[k ^ 1], tg[k]);
    } else {
        // several chunks: the gathers of one slot pair at a time (the slot tables stay live
        // across the chunks; fewer registers keep more waves resident); same order of the sum
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double t0[CS], t1[CS], g0[CS], g1[CS];
#pragma unroll
            for (int i = 0; i < CS; ++i) {
                t0[i] = src[nb[2 * p] * SST + SOFF + i];
                t1[i] = src[nb[2 * p + 1] * SST + SOFF + i];
            }
            if (lim != FL_UPWIND) {
#pragma unroll
                for (int i = 0; i < CS; ++i) {
                    g0[i] = src[gf[2 * p] * SST + SOFF + i];
                    g1[i] = src[gf[2 * p + 1] * SST + SOFF + i];
                }
            }
            face(2 * p, t0, t1, g0);
            face(2 * p + 1, t1, t0, g1);
        }
    }
    // The stage combination with its roundings written out (explicit fma), so that every kernel
    // built on this routine rounds it alike whatever the compiler would contract.
#pragma unroll
    for (int i = 0; i < CS; ++i) {
        const int64_t j = c * S + S0 + i;
        const double rhs = acc[i] / V;
        if (mode == MODE_RHS) out[j] = rhs;
        else if (mode == MODE_EULER) out[j] = fma(dt, rhs, tc[i]);
        else out[j] = fma(b, fma(dt, rhs, tc[i]), a * (PRE ? tnv[i] : tn[j]));
    }
}

// All scalars of cell c from global memory, in chunks of at most two (the gathered values of a
// chunk stay in registers for any S).
template <int S, int P, int S0>
__device__ __forceinline__ void fused_chunks(int64_t c, int64_t cs, const double *src,
                                             const double *w, const int64_t *nb,
                                             const int64_t *gf, double V,
                                             const double *__restrict__ tn, double a, double b,
                                             double dt, int mode, int lim,
                                             double *__restrict__ out) {
    if constexpr (S0 < S) {
        constexpr int CS = (S - S0) >= 2 ? 2 : 1;
        fused_chunk<S, P, S0, CS, S, S0>(c, cs, src, w, nb, gf, V, tn, a, b, dt, mode, lim, out);
        fused_chunks<S, P, S0 + CS>(c, cs, src, w, nb, gf, V, tn, a, b, dt, mode, lim, out);
    }
}

// One stage for cell c with P opposite-face pairs (slots 2p and 2p+1 are opposite faces).
// Slot k gives the face f_k (bit 31: c is its own), the other cell n_k and the far-upwind cell
// g_k on n_k's side; the far-upwind cell on c's side of f_k is n_{k^1}.  The face terms enter as
// w_k = a_f u_f E, the signed rate out of c (E = +1 where c is the face's own cell, -1 where it
// is the nbr), so rhs_c = -sum_k w_k theta_f,k / V_c.  The table entries and velocities are read
// once for all scalars, then every gather of a chunk is issued before its arithmetic (the kernel
// is bound by gather latency and L2 misses, not by arithmetic).
// out = rhs (MODE_RHS), theta_s + dt rhs (MODE_EULER) or a theta_n + b (theta_s + dt rhs);
// the face velocities are us * u.
template <int S, int P>
__device__ __forceinline__ void fused_cell(int64_t c, int64_t nc, const uint32_t *__restrict__ sface,
                                           const int32_t *__restrict__ snbr,
                                           const int32_t *__restrict__ sfar,
                                           const double *__restrict__ u,
                                           const double *__restrict__ area, double area0,
                                           const double *__restrict__ vol, double vol0,
                                           const double *__restrict__ ts,
                                           const double *__restrict__ tn, double a, double b,
                                           double dt, int mode, int lim,
                                           double *__restrict__ out, double us) {
    constexpr int K = 2 * P;
    uint32_t fw[K];
    int64_t nb[K], gf[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        fw[k] = sface[(int64_t)k * nc + c];
        nb[k] = snbr[(int64_t)k * nc + c];
        gf[k] = sfar[(int64_t)k * nc + c];
    }
    double w[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t f = fw[k] & 0x7fffffffu;
        // time-dependent velocity u(t) = us u_f; us = 1 is exact
        const double au = (area ? area[f] : area0) * (u[f] * us);
        w[k] = (fw[k] >> 31) ? au : -au;
    }
    const double V = vol ? vol[c] : vol0;
    fused_chunks<S, P, 0>(c, c, ts, w, nb, gf, V, tn, a, b, dt, mode, lim, out);
}

// One slot of the per-call record table of multi-step calls: the other cell, the far-upwind cell
// on its side and the signed face rate E a_f u_f (E u_f where all areas are area0), 16 bytes so
// that one load brings all three.
struct alignas(16) SlotRec {
    int32_t nbr, far;
    double rate;
};

// The same stage reading the slot records rec[k][c] built once per call (slot_record_kernel):
// every operand then streams in cell order except the theta gathers, with one 16-byte load per
// slot (the kernel is bound by the address processing of its loads, so fewer, wider loads pay).
// For us = 1 the rates w_k, and so the results, are bit-identical to fused_cell's.
template <int S, int P>
__device__ __forceinline__ void fused_cell_rec(int64_t c, int64_t nc,
                                               const SlotRec *__restrict__ rec, bool has_area,
                                               double area0, const double *__restrict__ vol,
                                               double vol0, const double *__restrict__ ts,
                                               const double *__restrict__ tn, double a, double b,
                                               double dt, int mode, int lim,
                                               double *__restrict__ out, double us) {
    constexpr int K = 2 * P;
    int64_t nb[K], gf[K];
    double w[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int4 raw = *reinterpret_cast<const int4 *>(rec + (int64_t)k * nc + c);
        nb[k] = raw.x;
        gf[k] = raw.y;
        const double v = __hiloint2double(raw.w, raw.z) * us;
        w[k] = has_area ? v : area0 * v;
    }
    const double V = vol ? vol[c] : vol0;
    fused_chunks<S, P, 0>(c, c, ts, w, nb, gf, V, tn, a, b, dt, mode, lim, out);
}

// Copies scalars S0 .. S0+CS-1 of theta_s of tile `tile` (kTileCells consecutive cells) and of
// its halo (the cells outside it that its slots name, ascending) to LDS: [tile cells | halo], CS
// values per cell, each read from global memory once per tile.  Every thread of the workgroup
// takes part; the caller puts a barrier between this and the reads.  Returns the number of cells
// in the tile.
template <int S, int S0, int CS>
__device__ __forceinline__ int tile_stage(int64_t nc, int64_t tile, double *lds,
                                          const int32_t *__restrict__ halo_ptr,
                                          const int32_t *__restrict__ halo,
                                          const double *__restrict__ ts) {
    const int64_t c0 = tile * kTileCells;
    const int64_t left = nc - c0;
    const int nt = left < kTileCells ? (int)left : kTileCells;
    const int h0 = halo_ptr[tile], nh = halo_ptr[tile + 1] - h0;
    for (int i = threadIdx.x; i < nt; i += blockDim.x) {
#pragma unroll
        for (int s = 0; s < CS; ++s) lds[i * CS + s] = ts[(c0 + i) * S + S0 + s];
    }
    for (int i = threadIdx.x; i < nh; i += blockDim.x) {
        const int64_t g = halo[h0 + i];
#pragma unroll
        for (int s = 0; s < CS; ++s) lds[(kTileCells + i) * CS + s] = ts[g * S + S0 + s];
    }
    return nt;
}

// The first chunk (CS scalars) of one tile staged as tile_stage does, with the cell's raw slot
// words loaded after the theta gathers of the tile cell and of its first kHaloAhead halo
// entries and before their LDS stores.  Loads complete in issue order, so the stores wait for
// the gathers only and the slot words stay in flight across the barrier that follows
// (tile_slots_finish decodes them after it).  No load sits in a branch, so that the compiler's
// count of outstanding loads stays exact: a lane past the tile's cells reads the tile's first
// cell, one past its halo the halo's first entry (the device array is padded by kHaloPad
// entries, so that entry exists even for an empty halo at the end).
template <int P, bool RATES>
struct SlotRaw {
    uint32_t l[2 * P];                 // local indices: neighbour | far cell << 16
    double r[RATES ? 2 * P : 1];       // per-call rates (RATES)
    uint32_t fw[RATES ? 1 : 2 * P];    // face | own bit (face-index form)
};

template <int S, int CS, int P, bool RATES, bool PRE>
__device__ __forceinline__ int tile_stage_slots(int64_t nc, int64_t tile, double *lds,
                                                const int32_t *__restrict__ halo_ptr,
                                                const int32_t *__restrict__ halo,
                                                const double *__restrict__ ts,
                                                const uint32_t *__restrict__ slot_local,
                                                const double *__restrict__ rate,
                                                const uint32_t *__restrict__ sface,
                                                const double *__restrict__ tn, double *tnv,
                                                SlotRaw<P, RATES> &raw) {
    const int64_t c0 = tile * kTileCells;
    const int64_t left = nc - c0;
    const int nt = left < kTileCells ? (int)left : kTileCells;
    const int h0 = halo_ptr[tile], nh = halo_ptr[tile + 1] - h0;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int64_t c = c0 + (tid < nt ? tid : 0);
    double tv[CS], hv[kHaloAhead][CS];
#pragma unroll
    for (int s = 0; s < CS; ++s) tv[s] = ts[c * S + s];
    // a lane past the halo re-reads the halo's first entry and gathers its own cell: lines the
    // tile reads anyway
#pragma unroll
    for (int j = 0; j < kHaloAhead; ++j) {
        const int i = tid + j * nthr;
        const int64_t h = halo[h0 + (i < nh ? i : 0)];
        const int64_t g = i < nh ? h : c;
#pragma unroll
        for (int s = 0; s < CS; ++s) hv[j][s] = ts[g * S + s];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 2 * P; ++k) {
        raw.l[k] = slot_local[(int64_t)k * nc + c];
        if constexpr (RATES) raw.r[k] = rate[(int64_t)k * nc + c];
        else raw.fw[k] = sface[(int64_t)k * nc + c];
    }
    // PRE: theta_n of the chunk (used by the stage combination only; Euler stages pass tn == ts)
    if constexpr (PRE) {
        const double *tnp = tn ? tn : ts;
#pragma unroll
        for (int s = 0; s < CS; ++s) tnv[s] = tnp[c * S + s];
    }
    __builtin_amdgcn_sched_barrier(0);
    // every lane stores (tid < kTileCells): entries past nt are never read
#pragma unroll
    for (int s = 0; s < CS; ++s) lds[tid * CS + s] = tv[s];
    // lanes past the halo store to the spare entry just after it (never read; the LDS holds
    // kTileCells + max halo + 1 entries), so that no gather is sunk into a branch
#pragma unroll
    for (int j = 0; j < kHaloAhead; ++j) {
        const int i = tid + j * nthr;
        const int e = kTileCells + (i < nh ? i : nh);
#pragma unroll
        for (int s = 0; s < CS; ++s) lds[e * CS + s] = hv[j][s];
    }
    for (int i = tid + kHaloAhead * nthr; i < nh; i += nthr) {
        const int64_t g = halo[h0 + i];
#pragma unroll
        for (int s = 0; s < CS; ++s) lds[(kTileCells + i) * CS + s] = ts[g * S + s];
    }
    return nt;
}

// Local slot indices and signed face rates of the cell from its raw slot words.  The face terms
// come from the per-call rates (RATES) or, as in fused_cell, from u through the face index;
// either way the rates w_k, and so the results, are bit-identical to fused_cell's for us = 1.
template <int P, bool RATES>
__device__ __forceinline__ void tile_slots_finish(const SlotRaw<P, RATES> &raw,
                                                  const double *__restrict__ u,
                                                  const double *__restrict__ area, bool has_area,
                                                  double area0, double us, int32_t *nb,
                                                  int32_t *gf, double *w) {
#pragma unroll
    for (int k = 0; k < 2 * P; ++k) {
        nb[k] = raw.l[k] & 0xffffu;
        gf[k] = raw.l[k] >> 16;
        if constexpr (RATES) {
            const double v = raw.r[k] * us;
            w[k] = has_area ? v : area0 * v;
        } else {
            const uint32_t fw = raw.fw[k];
            const int64_t f = fw & 0x7fffffffu;
            const double au = (area ? area[f] : area0) * (u[f] * us);
            w[k] = (fw >> 31) ? au : -au;
        }
    }
}

// Chunks S0.. (S0 > 0) of one tile: barrier (the previous chunk's LDS reads are done), stage the
// chunk (all threads), barrier, each cell of the tile computes it from LDS.  Chunks of at most
// CMAX scalars.
template <int S, int P, int S0, int CMAX = 2>
__device__ __forceinline__ void tile_chunks(int64_t nc, int64_t tile, double *lds,
                                            const int32_t *__restrict__ halo_ptr,
                                            const int32_t *__restrict__ halo,
                                            const double *__restrict__ ts, bool active, int64_t c,
                                            const double *w, const int32_t *nb, const int32_t *gf,
                                            double V, const double *__restrict__ tn, double a,
                                            double b, double dt, int mode, int lim,
                                            double *__restrict__ out) {
    if constexpr (S0 < S) {
        constexpr int CS = (S - S0) >= CMAX ? CMAX : S - S0;
        __syncthreads();
        tile_stage<S, S0, CS>(nc, tile, lds, halo_ptr, halo, ts);
        __syncthreads();
        if (active)
            fused_chunk<S, P, S0, CS, CS, 0>(c, threadIdx.x, lds, w, nb, gf, V, tn, a, b, dt, mode,
                                             lim, out);
        tile_chunks<S, P, S0 + CS, CMAX>(nc, tile, lds, halo_ptr, halo, ts, active, c, w, nb, gf,
                                         V, tn, a, b, dt, mode, lim, out);
    }
}

// The whole stage of one tile, one thread per cell (kTileCells threads).  Face terms from
// `rate` (RATES), or from u through the face index.  LDS: (kTileCells + max halo + 1) * min(S,
// 2) doubles.  Every thread of the workgroup must call it (barriers).  The slot loads are
// issued while the first chunk is being staged (tile_stage_slots), and with PRE the first
// chunk's theta_n too (4 more VGPRs at most: kernels whose occupancy they would lower pass
// false).
template <int S, int P, bool RATES, bool PRE = true>
__device__ __forceinline__ void fused_tile(int64_t nc, int64_t tile, double *lds,
                                           const int32_t *__restrict__ halo_ptr,
                                           const int32_t *__restrict__ halo,
                                           const uint32_t *__restrict__ slot_local,
                                           const double *__restrict__ rate,
                                           const uint32_t *__restrict__ sface,
                                           const double *__restrict__ u,
                                           const double *__restrict__ area, double area0,
                                           const double *__restrict__ vol, double vol0,
                                           const double *__restrict__ ts,
                                           const double *__restrict__ tn, double a, double b,
                                           double dt, int mode, int lim,
                                           double *__restrict__ out, double us) {
    constexpr int K = 2 * P;
    constexpr int CS0 = fwd_chunk(S);
    int32_t nb[K], gf[K];  // tile-local indices
    double w[K];
    SlotRaw<P, RATES> raw;
    double tnv[CS0];
    const int nt = tile_stage_slots<S, CS0, P, RATES, PRE>(nc, tile, lds, halo_ptr, halo, ts,
                                                           slot_local, rate, sface, tn, tnv, raw);
    __syncthreads();
    const bool active = (int)threadIdx.x < nt;
    const int64_t c = tile * kTileCells + threadIdx.x;
    double V = vol0;
    if (active) {
        tile_slots_finish<P, RATES>(raw, u, area, area != nullptr, area0, us, nb, gf, w);
        if (vol) V = vol[c];
        fused_chunk<S, P, 0, CS0, CS0, 0, PRE>(c, threadIdx.x, lds, w, nb, gf, V, tn, a, b, dt,
                                               mode, lim, out, tnv);
    }
    tile_chunks<S, P, CS0, fwd_chunk(S)>(nc, tile, lds, halo_ptr, halo, ts, active, c, w, nb, gf,
                                         V, tn, a, b, dt, mode, lim, out);
}

// The stage of one tile on a mesh with aligned slots (the neighbour across slot k of a cell holds
// the shared face in its slot k ^ 1), reading per-call rates of each cell's forward faces only:
// rf[p][c] = E a_f u_f (E u_f where all areas are area0) of slot 2p.  The rate of a backward slot
// 2p + 1 is the negated forward rate of the neighbour across it (whose slot 2p is the shared
// face), read from the tile's LDS copy of the forward rates or, for a neighbour outside the
// tile, from the LDS copy of the halo entries' rates (a halo entry is a (cell, pair) reference;
// the leading ones, the neighbours across backward slots, carry that cell's forward rate of that
// pair, gathered with its theta): half the rate bytes of fused_tile<RATES>, the same rates w_k
// (a negation is exact), so the same bits.
// Compact tables: a cell reads only its neighbours' 16-bit local indices (slot_nb, one word per
// pair); the far cell beyond a neighbour is that neighbour's own neighbour in the same direction,
// read from the tile's LDS copy of the words or, for a halo neighbour, from the LDS copy of the
// halo's next indices (halo_next, the leading halo_nrate[2 tile + 1] entries); halo cells and
// their pairs come packed in one word (halo_pk).  The tile's rates and words are loaded between
// the theta gathers and the LDS stores, so that the stores wait only for the gathers and the
// rest stays in flight across the barrier.
// LDS (doubles): the chunk area [0, rbase); tile rates [P][kTileCells] at rbase, then one rate
// per leading halo entry (halo_nrate[2 tile] of them, and a spare); at nbase the tile's words
// (uint32 [P][kTileCells]), then the halo's next indices (uint16, halo_nrate[2 tile + 1] and a
// spare).
template <int S, int P, bool PRE = true>
__device__ __forceinline__ void fused_tile_fwd(int64_t nc, int64_t tile, double *lds, int rbase,
                                               int nbase, const int32_t *__restrict__ halo_ptr,
                                               const int32_t *__restrict__ halo,
                                               const int32_t *__restrict__ halo_pk,
                                               const uint16_t *__restrict__ halo_next,
                                               const int32_t *__restrict__ halo_nrate,
                                               const uint32_t *__restrict__ slot_nb,
                                               const double *__restrict__ rf, bool has_area,
                                               double area0, const double *__restrict__ vol,
                                               double vol0, const double *__restrict__ ts,
                                               const double *__restrict__ tn, double a, double b,
                                               double dt, int mode, int lim,
                                               double *__restrict__ out, double us) {
    constexpr int K = 2 * P;
    constexpr int CS = fwd_chunk(S);
    constexpr uint32_t T = kTileCells;
    const int64_t c0 = tile * kTileCells;
    const int64_t left = nc - c0;
    const int nt = left < kTileCells ? (int)left : kTileCells;
    const int h0 = halo_ptr[tile], nh = halo_ptr[tile + 1] - h0;
    // the leading halo entries (neighbours across backward slots) need their rate, the leading
    // nx (also neighbours across forward slots) their next index; the other lanes read their own
    // cell's first rate and the halo's first index instead (lines the tile reads anyway)
    const int nr = halo_nrate[2 * tile], nx = halo_nrate[2 * tile + 1];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int64_t c = c0 + (tid < nt ? tid : 0);
    double tv[CS], hv[kHaloAhead][CS], hr[kHaloAhead];
    uint32_t hn[kHaloAhead];
#pragma unroll
    for (int s = 0; s < CS; ++s) tv[s] = ts[c * S + s];
#pragma unroll
    for (int j = 0; j < kHaloAhead; ++j) {
        const int i = tid + j * nthr;
        const int ie = i < nh ? i : 0;  // (the arrays are padded: entry 0 exists)
        const uint32_t hw = (uint32_t)halo_pk[h0 + ie];
        const int64_t h = hw & 0x3fffffffu;
        const int64_t pr = hw >> 30;
        const int64_t g = i < nh ? h : c;
#pragma unroll
        for (int s = 0; s < CS; ++s) hv[j][s] = ts[g * S + s];
        hr[j] = rf[i < nr ? pr * nc + h : c];
        hn[j] = halo_next[h0 + (i < nx ? i : 0)];
    }
    __builtin_amdgcn_sched_barrier(0);
    double rfv[P];
    uint32_t l[P];
#pragma unroll
    for (int p = 0; p < P; ++p) rfv[p] = rf[(int64_t)p * nc + c];
#pragma unroll
    for (int p = 0; p < P; ++p) l[p] = slot_nb[(int64_t)p * nc + c];
    double tnv[CS];
    if constexpr (PRE) {
        const double *tnp = tn ? tn : ts;
#pragma unroll
        for (int s = 0; s < CS; ++s) tnv[s] = tnp[c * S + s];
    }
    __builtin_amdgcn_sched_barrier(0);
    double *rt = lds + rbase;                   // tile forward rates [P][kTileCells]
    double *rh = lds + rbase + P * kTileCells;  // rates of the leading halo entries
    uint32_t *nw = reinterpret_cast<uint32_t *>(lds + nbase);  // tile words [P][kTileCells]
    uint16_t *nxt = reinterpret_cast<uint16_t *>(nw + P * kTileCells);
#pragma unroll
    for (int s = 0; s < CS; ++s) lds[tid * CS + s] = tv[s];
#pragma unroll
    for (int j = 0; j < kHaloAhead; ++j) {
        const int i = tid + j * nthr;
        const int e = kTileCells + (i < nh ? i : nh);
#pragma unroll
        for (int s = 0; s < CS; ++s) lds[e * CS + s] = hv[j][s];
        rh[i < nr ? i : nr] = hr[j];
        nxt[i < nx ? i : nx] = (uint16_t)hn[j];
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        rt[p * kTileCells + tid] = rfv[p];
        nw[p * kTileCells + tid] = l[p];
    }
    for (int i = tid + kHaloAhead * nthr; i < nh; i += nthr) {
        const uint32_t hw = (uint32_t)halo_pk[h0 + i];
        const int64_t g = hw & 0x3fffffffu;
#pragma unroll
        for (int s = 0; s < CS; ++s) lds[(kTileCells + i) * CS + s] = ts[g * S + s];
        if (i < nr) rh[i] = rf[(int64_t)(hw >> 30) * nc + g];
        if (i < nx) nxt[i] = halo_next[h0 + i];
    }
    __syncthreads();
    const bool active = tid < nt;
    const int64_t cc = c0 + tid;
    int32_t nb[K], gf[K];  // tile-local indices
    double w[K];
    double V = vol0;
    if (active) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint32_t n0 = l[p] & 0xffffu, n1 = l[p] >> 16;
            nb[2 * p] = n0;
            nb[2 * p + 1] = n1;
            // the far cell beyond a neighbour: the neighbour's own neighbour in that direction
            gf[2 * p] = n0 < T ? (nw[p * kTileCells + n0] & 0xffffu) : nxt[n0 - T];
            gf[2 * p + 1] = n1 < T ? (nw[p * kTileCells + n1] >> 16) : nxt[n1 - T];
            const double v = rfv[p] * us;
            w[2 * p] = has_area ? v : area0 * v;
            const double r = n1 < T ? rt[p * kTileCells + n1] : rh[n1 - T];
            const double vb = (-r) * us;
            w[2 * p + 1] = has_area ? vb : area0 * vb;
        }
        if (vol) V = vol[cc];
        fused_chunk<S, P, 0, CS, CS, 0, PRE>(cc, tid, lds, w, nb, gf, V, tn, a, b, dt, mode, lim,
                                             out, tnv);
    }
    tile_chunks<S, P, CS, fwd_chunk(S)>(nc, tile, lds, halo_ptr, halo, ts, active, cc, w, nb, gf, V,
                                     tn, a, b, dt, mode, lim, out);
}

}  // namespace dev
}  // namespace fl
