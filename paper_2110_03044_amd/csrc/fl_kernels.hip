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
// Launches use 256-thread workgroups, one thread per face or cell.  The fused kernel is bound by
// its gathers, not by arithmetic: at 256^3 with a locality-ordered mesh the bytes it fetches
// past L2 equal its compulsory traffic, so the mesh ordering (see mesh.cpp) is what keeps it
// near the memory roofline.
#include <hip/hip_runtime.h>

#include "fl_device.h"
#include "fl_face_device.h"

namespace fl {
namespace dev {

constexpr int kBlock = 256;
static_assert(kBlock == kTileCells, "one thread per cell of an LDS-staged tile");


template <int S>
__global__ __launch_bounds__(kBlock) void face_flux_kernel(
    int64_t nf, const int4 *__restrict__ fc4, const double *__restrict__ u,
    const double *__restrict__ theta, const double *__restrict__ area, double area0, int lim,
    double *__restrict__ phi, int remap, double us) {
    const int64_t f = block_id(remap) * kBlock + threadIdx.x;
    if (f >= nf) return;
    face_flux_one<S>(f, fc4, u, theta, area, area0, lim, phi, us);
}

template <int S>
__global__ __launch_bounds__(kBlock) void face_flux_general_kernel(
    int64_t nf, const int4 *__restrict__ fc4, const int32_t *__restrict__ side_ptr,
    const int32_t *__restrict__ side_cell, const double *__restrict__ side_w,
    const double *__restrict__ u, const double *__restrict__ theta,
    const double *__restrict__ area, double area0, int lim, double *__restrict__ phi, double us,
    const double *__restrict__ inflow) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= nf) return;
    face_flux_general_one<S>(f, fc4, side_ptr, side_cell, side_w, u, theta, area, area0, lim,
                             phi, us, inflow);
}

template <int S>
__global__ __launch_bounds__(kBlock) void cell_update_kernel(
    int64_t nc, int K, const int32_t *__restrict__ cf_ptr, const int32_t *__restrict__ cf_idx,
    const double *__restrict__ phi, const double *__restrict__ vol, double vol0,
    const double *__restrict__ ts, const double *__restrict__ tn, double a, double b, double dt,
    int mode, double *__restrict__ out, int remap) {
    const int64_t c = block_id(remap) * kBlock + threadIdx.x;
    if (c >= nc) return;
    cell_update_one<S>(c, K, cf_ptr, cf_idx, phi, vol, vol0, ts, tn, a, b, dt, mode, out);
}

// ------------------------------------------------------------------------------------------
// Fused path (the per-cell routine is in fl_device.h, shared with the batched kernel)
// ------------------------------------------------------------------------------------------
template <int S, int P>
__global__ __launch_bounds__(kBlock) void fused_stage_kernel(
    int64_t nc, const uint32_t *__restrict__ sface, const int32_t *__restrict__ snbr,
    const int32_t *__restrict__ sfar, const double *__restrict__ u,
    const double *__restrict__ area, double area0, const double *__restrict__ vol, double vol0,
    const double *__restrict__ ts, const double *__restrict__ tn, double a, double b, double dt,
    int mode, int lim, double *__restrict__ out, int remap, double us) {
    const int64_t c = block_id(remap) * kBlock + threadIdx.x;
    if (c >= nc) return;
    fused_cell<S, P>(c, nc, sface, snbr, sfar, u, area, area0, vol, vol0, ts, tn, a, b, dt, mode,
                     lim, out, us);
}

// rec[k][c] = {n_k, g_k, E a_f u_f} (E = +1 where c is the own cell of its slot-k face, -1 where
// it is the nbr; a_f omitted where the mesh has no face areas).  Built once per multi-step call.
template <int P>
__global__ __launch_bounds__(kBlock) void slot_record_kernel(
    int64_t nc, const uint32_t *__restrict__ sface, const int32_t *__restrict__ snbr,
    const int32_t *__restrict__ sfar, const double *__restrict__ u,
    const double *__restrict__ area, SlotRec *__restrict__ rec) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= nc) return;
#pragma unroll
    for (int k = 0; k < 2 * P; ++k) {
        const int64_t at = (int64_t)k * nc + c;
        const uint32_t fw = sface[at];
        const int64_t f = fw & 0x7fffffffu;
        const double x = area ? area[f] * u[f] : u[f];
        SlotRec r;
        r.nbr = snbr[at];
        r.far = sfar[at];
        r.rate = (fw >> 31) ? x : -x;
        rec[at] = r;
    }
}

template <int S, int P>
__global__ __launch_bounds__(kBlock) void fused_stage_rec_kernel(
    int64_t nc, const SlotRec *__restrict__ rec, int has_area, double area0,
    const double *__restrict__ vol, double vol0, const double *__restrict__ ts,
    const double *__restrict__ tn, double a, double b, double dt, int mode, int lim,
    double *__restrict__ out, int remap, double us) {
    const int64_t c = block_id(remap) * kBlock + threadIdx.x;
    if (c >= nc) return;
    fused_cell_rec<S, P>(c, nc, rec, has_area != 0, area0, vol, vol0, ts, tn, a, b, dt, mode,
                         lim, out, us);
}

// rate[k][c] = E a_f u_f of slot k (the rate part of the slot records), for the LDS-staged stage.
// All face words first, then all gathers, then the stores: one dependent round trip per cell
// rather than one per slot.  AREA: per-face areas (uniform areas enter later, as one scalar).
template <int P, bool AREA>
__global__ __launch_bounds__(kBlock) void slot_rate_kernel(int64_t nc,
                                                           const uint32_t *__restrict__ sface,
                                                           const double *__restrict__ u,
                                                           const double *__restrict__ area,
                                                           double *__restrict__ rate) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= nc) return;
    constexpr int K = 2 * P;
    uint32_t fw[K];
    double x[K];
#pragma unroll
    for (int k = 0; k < K; ++k) fw[k] = sface[(int64_t)k * nc + c];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t f = fw[k] & 0x7fffffffu;
        if constexpr (AREA) x[k] = area[f] * u[f];
        else x[k] = u[f];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) rate[(int64_t)k * nc + c] = (fw[k] >> 31) ? x[k] : -x[k];
}

// rf[p][c] = E a_f u_f of slot 2p (each cell's forward faces: every face once), for the
// forward-rate stage of meshes with aligned slots.
template <int P, bool AREA>
__global__ __launch_bounds__(kBlock) void slot_rate_fwd_kernel(int64_t nc,
                                                               const uint32_t *__restrict__ sface,
                                                               const double *__restrict__ u,
                                                               const double *__restrict__ area,
                                                               double *__restrict__ rf) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= nc) return;
    uint32_t fw[P];
    double x[P];
#pragma unroll
    for (int p = 0; p < P; ++p) fw[p] = sface[(int64_t)(2 * p) * nc + c];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int64_t f = fw[p] & 0x7fffffffu;
        if constexpr (AREA) x[p] = area[f] * u[f];
        else x[p] = u[f];
    }
#pragma unroll
    for (int p = 0; p < P; ++p) rf[(int64_t)p * nc + c] = (fw[p] >> 31) ? x[p] : -x[p];
}

// The LDS-staged stage reading forward rates and the compact slot tables (fused_tile_fwd);
// dynamic LDS as lds_fwd_bytes.  The limiter is fixed at compile time, so that the face
// evaluations of a cell carry no limiter branch and schedule together.
template <int S, int P, int LIM>
__global__ __launch_bounds__(kBlock) void fused_stage_lds_fwd_kernel(
    int64_t nc, const int32_t *__restrict__ halo_ptr, const int32_t *__restrict__ halo,
    const int32_t *__restrict__ halo_pk, const uint16_t *__restrict__ halo_next,
    const int32_t *__restrict__ halo_nrate, const uint32_t *__restrict__ slot_nb,
    const double *__restrict__ rf, int has_area, double area0, const double *__restrict__ vol,
    double vol0, const double *__restrict__ ts, const double *__restrict__ tn, double a,
    double b, double dt, int mode, double *__restrict__ out, double us, int rbase, int nbase,
    int remap) {
    extern __shared__ double lds[];
    const int64_t tile = block_id(remap);
    if (tile * kTileCells >= nc) return;
    fused_tile_fwd<S, P>(nc, tile, lds, rbase, nbase, halo_ptr, halo, halo_pk, halo_next,
                         halo_nrate, slot_nb, rf, has_area != 0, area0, vol, vol0, ts, tn, a, b,
                         dt, mode, LIM, out, us);
}

// One workgroup per tile of kTileCells cells; dynamic LDS of (kTileCells + max halo + 1) *
// fwd_chunk(S) doubles.
template <int S, int P, bool RATES>
__global__ __launch_bounds__(kBlock) void fused_stage_lds_kernel(
    int64_t nc, const int32_t *__restrict__ halo_ptr, const int32_t *__restrict__ halo,
    const uint32_t *__restrict__ slot_local, const double *__restrict__ rate,
    const uint32_t *__restrict__ sface, const double *__restrict__ u,
    const double *__restrict__ area, double area0, const double *__restrict__ vol, double vol0,
    const double *__restrict__ ts, const double *__restrict__ tn, double a, double b, double dt,
    int mode, int lim, double *__restrict__ out, double us, int remap) {
    extern __shared__ double lds[];
    // the tile is the same for the whole workgroup: padding workgroups leave before any barrier
    const int64_t tile = block_id(remap);
    if (tile * kTileCells >= nc) return;
    fused_tile<S, P, RATES>(nc, tile, lds, halo_ptr, halo, slot_local, rate, sface, u, area, area0,
                            vol, vol0, ts, tn, a, b, dt, mode, lim, out, us);
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

// (C, D, U) per face; U = -2 where the upwind side projects on more than one face (general
// cells, side lists given).
__global__ __launch_bounds__(kBlock) void select_kernel(int64_t nf, const int4 *__restrict__ fc4,
                                                        const int32_t *__restrict__ side_ptr,
                                                        const int32_t *__restrict__ side_cell,
                                                        const double *__restrict__ u,
                                                        int32_t *__restrict__ cdu) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= nf) return;
    const int4 e = fc4[f];
    const bool pos = u[f] > 0.0;
    cdu[3 * f] = pos ? e.x : e.y;
    cdu[3 * f + 1] = pos ? e.y : e.x;
    if (side_ptr) {
        const int64_t side = 2 * f + (pos ? 0 : 1);
        const int32_t p0 = side_ptr[side], n = side_ptr[side + 1] - p0;
        cdu[3 * f + 2] = n == 1 ? side_cell[p0] : -2;
    } else {
        cdu[3 * f + 2] = pos ? e.z : e.w;
    }
}

}  // namespace dev

// ------------------------------------------------------------------------------------------
// Launch wrappers
// ------------------------------------------------------------------------------------------
namespace {

// remap: 0 launch order; 1 contiguous eighths; M >= 2 runs of M tiles per XCD.
Grid grid_for(int64_t n, int remap) {
    int64_t nb = (n + dev::kBlock - 1) / dev::kBlock;
    if (nb < 1) nb = 1;
    if (remap <= 0 || nb < 64) return {(unsigned)nb, 0};
    const int64_t chunk = remap == 1 ? (nb + 7) / 8 : remap;
    const int64_t span = 8 * chunk;
    return {(unsigned)(((nb + span - 1) / span) * span), (int)chunk};
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

// Block ids map to cells through dev::block_id: runs of 32 consecutive tiles per XCD by default
// (the tiles sharing one L2 are then neighbours), launch order with FL_OPT_XCD_REMAP = 0.
int g_remap = 32;
void set_xcd_remap(int value) { g_remap = value; }
Grid launch_grid(int64_t n) { return grid_for(n, g_remap); }
int xcd_remap() { return g_remap; }

hipError_t launch_face_flux(const fl_mesh *m, int lim, int S, const double *theta,
                            const double *u, double *phi, hipStream_t st, double us) {
    // Blocks beyond the face count exit at once (padding to a multiple of 8 XCDs).
    if (m->h.general) {
        const unsigned nb = (unsigned)((m->h.nf + dev::kBlock - 1) / dev::kBlock);
        FL_DISPATCH_S(S, (dev::face_flux_general_kernel<kS><<<nb, dev::kBlock, 0, st>>>(
                             m->h.nf, reinterpret_cast<const int4 *>(m->d_fc4), m->d_side_ptr,
                             m->d_side_cell, m->d_side_w, u, theta, m->d_area, m->h.area0, lim,
                             phi, us, m->inflow)));
        return hipGetLastError();
    }
    Grid g = grid_for(m->h.nf, g_remap);
    FL_DISPATCH_S(S, (dev::face_flux_kernel<kS><<<g.blocks, dev::kBlock, 0, st>>>(
                         m->h.nf, reinterpret_cast<const int4 *>(m->d_fc4), u, theta, m->d_area,
                         m->h.area0, lim, phi, g.remap, us)));
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
                        hipStream_t st, double us) {
    Grid g = grid_for(m->h.nc, g_remap);
#define FL_FUSED(P)                                                                           \
    FL_DISPATCH_S(S, (dev::fused_stage_kernel<kS, P><<<g.blocks, dev::kBlock, 0, st>>>(       \
                         m->h.nc, m->d_slot_face, m->d_slot_nbr, m->d_slot_far, u, m->d_area, \
                         m->h.area0, m->d_vol, m->h.vol0, ts, tn, a, b, dt, mode, lim, out,   \
                         g.remap, us)))
    switch (m->h.pairs) {
        case 1: FL_FUSED(1); break;
        case 2: FL_FUSED(2); break;
        case 3: FL_FUSED(3); break;
        default: return hipErrorInvalidValue;
    }
#undef FL_FUSED
    return hipGetLastError();
}

hipError_t launch_slot_records(const fl_mesh *m, const double *u, void *rec, hipStream_t st) {
    const unsigned nb = (unsigned)((m->h.nc + dev::kBlock - 1) / dev::kBlock);
    dev::SlotRec *r = static_cast<dev::SlotRec *>(rec);
    switch (m->h.pairs) {
        case 1: dev::slot_record_kernel<1><<<nb, dev::kBlock, 0, st>>>(m->h.nc, m->d_slot_face, m->d_slot_nbr, m->d_slot_far, u, m->d_area, r); break;
        case 2: dev::slot_record_kernel<2><<<nb, dev::kBlock, 0, st>>>(m->h.nc, m->d_slot_face, m->d_slot_nbr, m->d_slot_far, u, m->d_area, r); break;
        case 3: dev::slot_record_kernel<3><<<nb, dev::kBlock, 0, st>>>(m->h.nc, m->d_slot_face, m->d_slot_nbr, m->d_slot_far, u, m->d_area, r); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fused_rec(const fl_mesh *m, int lim, int S, const double *ts, const double *tn,
                            const void *rec, double a, double b, double dt, int mode, double *out,
                            hipStream_t st, double us) {
    Grid g = grid_for(m->h.nc, g_remap);
    const int has_area = m->d_area != nullptr;
    const dev::SlotRec *r = static_cast<const dev::SlotRec *>(rec);
#define FL_FUSED_REC(P)                                                                        \
    FL_DISPATCH_S(S, (dev::fused_stage_rec_kernel<kS, P><<<g.blocks, dev::kBlock, 0, st>>>(    \
                         m->h.nc, r, has_area, m->h.area0, m->d_vol, m->h.vol0, ts, tn, a, b,   \
                         dt, mode, lim, out, g.remap, us)))
    switch (m->h.pairs) {
        case 1: FL_FUSED_REC(1); break;
        case 2: FL_FUSED_REC(2); break;
        case 3: FL_FUSED_REC(3); break;
        default: return hipErrorInvalidValue;
    }
#undef FL_FUSED_REC
    return hipGetLastError();
}

int g_lds_stage = 1;
void set_lds_stage(int on) { g_lds_stage = on; }

// The forward LDS stages stage fwd_chunk(S) scalars at a time; the adjoint stages theta and
// lambda of every scalar at once.
size_t lds_stage_bytes(const fl_mesh *m, int S) {
    if (!g_lds_stage || m->path != FL_PATH_FUSED || m->h.max_halo < 0 || !m->d_slot_local) return 0;
    return (size_t)(kTileCells + m->h.max_halo + 1) * fwd_chunk(S) * sizeof(double);
}

size_t adjoint_lds_bytes(const fl_mesh *m, int S) {
    if (!g_lds_stage || m->path != FL_PATH_FUSED || m->h.max_halo < 0 || !m->d_slot_local ||
        !m->d_adj_fr)
        return 0;
    return (size_t)(kTileCells + m->h.max_halo + 1) * (2 * S + (m->d_vol ? 1 : 0)) * sizeof(double);
}

hipError_t launch_slot_rates(const fl_mesh *m, const double *u, double *rate, hipStream_t st) {
    const unsigned nb = (unsigned)((m->h.nc + dev::kBlock - 1) / dev::kBlock);
#define FL_RATES(P)                                                                            \
    (m->d_area ? dev::slot_rate_kernel<P, true><<<nb, dev::kBlock, 0, st>>>(                   \
                     m->h.nc, m->d_slot_face, u, m->d_area, rate)                              \
               : dev::slot_rate_kernel<P, false><<<nb, dev::kBlock, 0, st>>>(                  \
                     m->h.nc, m->d_slot_face, u, nullptr, rate))
    switch (m->h.pairs) {
        case 1: FL_RATES(1); break;
        case 2: FL_RATES(2); break;
        case 3: FL_RATES(3); break;
        default: return hipErrorInvalidValue;
    }
#undef FL_RATES
    return hipGetLastError();
}

hipError_t launch_fused_lds(const fl_mesh *m, int lim, int S, const double *ts, const double *tn,
                            const double *rate, double a, double b, double dt, int mode,
                            double *out, hipStream_t st, double us, const double *u) {
    const size_t lds = lds_stage_bytes(m, S);
    if (lds == 0 || lds > kMaxStageLds || (!rate && !u)) return hipErrorInvalidValue;
    const Grid g = grid_for(m->h.nc, g_remap);  // one workgroup per tile (kBlock == kTileCells)
#define FL_FUSED_LDS_R(P, R)                                                                     \
    FL_DISPATCH_S(S, (dev::fused_stage_lds_kernel<kS, P, R><<<g.blocks, dev::kBlock, lds, st>>>( \
                         m->h.nc, m->d_halo_ptr, m->d_halo, m->d_slot_local, rate,                \
                         m->d_slot_face, u, m->d_area, m->h.area0, m->d_vol, m->h.vol0, ts, tn,   \
                         a, b, dt, mode, lim, out, us, g.remap)))
#define FL_FUSED_LDS(P)            \
    if (rate) {                    \
        FL_FUSED_LDS_R(P, true);   \
    } else {                       \
        FL_FUSED_LDS_R(P, false);  \
    }
    switch (m->h.pairs) {
        case 1: FL_FUSED_LDS(1); break;
        case 2: FL_FUSED_LDS(2); break;
        case 3: FL_FUSED_LDS(3); break;
        default: return hipErrorInvalidValue;
    }
#undef FL_FUSED_LDS
#undef FL_FUSED_LDS_R
    return hipGetLastError();
}

// The forward-rate stage's chunk area (doubles): fwd_chunk(S) scalars per cell.
static size_t fwd_theta_doubles(const fl_mesh *m, int S) {
    return (size_t)(kTileCells + m->h.max_halo + 1) * fwd_chunk(S);
}

// Offset (in doubles) of the tile words in the forward-rate stage's LDS.
static size_t fwd_nbase(const fl_mesh *m, int S) {
    return fwd_theta_doubles(m, S) + (size_t)m->h.pairs * kTileCells + m->h.max_nrate0 + 1;
}

size_t lds_fwd_bytes(const fl_mesh *m, int S) {
    const size_t lds = lds_stage_bytes(m, S);
    if (lds == 0 || !m->h.aligned_slots || !m->d_slot_nb || !m->d_halo_nrate) return 0;
    const size_t words = (size_t)m->h.pairs * kTileCells * sizeof(uint32_t) +
                         ((size_t)m->h.max_nrate + 1) * sizeof(uint16_t);
    const size_t b = fwd_nbase(m, S) * sizeof(double) + (words + 7) / 8 * 8;
    // large halos (meshes not renumbered for locality) gain nothing from the rate staging and
    // would cost occupancy: the per-slot rates serve them
    return b <= kMaxFwdLds ? b : 0;
}

hipError_t launch_slot_rates_fwd(const fl_mesh *m, const double *u, double *rf, hipStream_t st) {
    const unsigned nb = (unsigned)((m->h.nc + dev::kBlock - 1) / dev::kBlock);
#define FL_RATES_FWD(P)                                                                         \
    (m->d_area ? dev::slot_rate_fwd_kernel<P, true><<<nb, dev::kBlock, 0, st>>>(                \
                     m->h.nc, m->d_slot_face, u, m->d_area, rf)                                 \
               : dev::slot_rate_fwd_kernel<P, false><<<nb, dev::kBlock, 0, st>>>(               \
                     m->h.nc, m->d_slot_face, u, nullptr, rf))
    switch (m->h.pairs) {
        case 1: FL_RATES_FWD(1); break;
        case 2: FL_RATES_FWD(2); break;
        case 3: FL_RATES_FWD(3); break;
        default: return hipErrorInvalidValue;
    }
#undef FL_RATES_FWD
    return hipGetLastError();
}

hipError_t launch_fused_lds_fwd(const fl_mesh *m, int lim, int S, const double *ts,
                                const double *tn, const double *rf, double a, double b, double dt,
                                int mode, double *out, hipStream_t st, double us) {
    const size_t lds = lds_fwd_bytes(m, S);
    if (lds == 0 || lds > kMaxStageLds || !rf) return hipErrorInvalidValue;
    const int rbase = (int)fwd_theta_doubles(m, S);
    const int nbase = (int)fwd_nbase(m, S);
    const Grid g = grid_for(m->h.nc, g_remap);
#define FL_FWD_K(SS, P, L)                                                                     \
    dev::fused_stage_lds_fwd_kernel<SS, P, L><<<g.blocks, dev::kBlock, lds, st>>>(             \
        m->h.nc, m->d_halo_ptr, m->d_halo, m->d_halo_pk, m->d_halo_next, m->d_halo_nrate,     \
        m->d_slot_nb, rf, m->d_area ? 1 : 0, m->h.area0, m->d_vol, m->h.vol0, ts, tn, a, b,   \
        dt, mode, out, us, rbase, nbase, g.remap)
#define FL_FWD_LIM(SS, P)                                                  \
    switch (lim) {                                                         \
        case FL_UPWIND: FL_FWD_K(SS, P, FL_UPWIND); break;                 \
        case FL_MINMOD: FL_FWD_K(SS, P, FL_MINMOD); break;                 \
        case FL_VANLEER: FL_FWD_K(SS, P, FL_VANLEER); break;               \
        case FL_VANALBADA: FL_FWD_K(SS, P, FL_VANALBADA); break;           \
        case FL_SUPERBEE: FL_FWD_K(SS, P, FL_SUPERBEE); break;             \
        case FL_SMART: FL_FWD_K(SS, P, FL_SMART); break;                   \
        case FL_CENTRAL: FL_FWD_K(SS, P, FL_CENTRAL); break;               \
        default: return hipErrorInvalidValue;                              \
    }
#define FL_FUSED_FWD(P) FL_DISPATCH_S(S, FL_FWD_LIM(kS, P))
    switch (m->h.pairs) {
        case 1: FL_FUSED_FWD(1); break;
        case 2: FL_FUSED_FWD(2); break;
        case 3: FL_FUSED_FWD(3); break;
        default: return hipErrorInvalidValue;
    }
#undef FL_FUSED_FWD
#undef FL_FWD_LIM
#undef FL_FWD_K
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
        m->h.nf, reinterpret_cast<const int4 *>(m->d_fc4), m->h.general ? m->d_side_ptr : nullptr,
        m->d_side_cell, u, cdu);
    return hipGetLastError();
}

}  // namespace fl
