// Launch wrappers of the HIP kernels (host side).
#pragma once

#include <hip/hip_runtime_api.h>

#include "fl_internal.h"

namespace fl {

// Cell-stage modes: write rhs, theta_s + dt rhs, or a theta_n + b (theta_s + dt rhs).
enum { MODE_RHS = 0, MODE_EULER = 1, MODE_RK = 2 };

// Adjoint-stage modes (see fl_adjoint.hip).
enum { ADJ_APPLY = 0, ADJ_EULER = 1, ADJ_LAST = 2, ADJ_MID = 3, ADJ_FIRST = 4 };

// 0: launch order; 1: each XCD a contiguous eighth of the tiles; M >= 2: runs of M tiles per XCD
// (default 32).
void set_xcd_remap(int value);

// Grid of 256-thread workgroups for n cells or faces in the current XCD order: `blocks`
// workgroups (padded to a multiple of 8 remap when remapping), decoded by dev::block_id(remap).
struct Grid {
    unsigned blocks;
    int remap;  // chunk M of block_id, 0 = launch order
};
Grid launch_grid(int64_t n);
int xcd_remap();  // the current FL_OPT_XCD_REMAP value

hipError_t launch_adjoint(const fl_mesh *m, int lim, int S, const double *u, const double *th,
                          const double *lam, double a, double b, double dt, int mode, double *out,
                          double *acc, double *ubar, hipStream_t st);
// The same on general cells (fl_adjoint_general.hip): a face kernel writes each face's terms to
// term (adjoint_general_term_bytes), a cell kernel gathers them.
size_t adjoint_general_term_bytes(const fl_mesh *m, int S);
hipError_t launch_adjoint_general(const fl_mesh *m, int lim, int S, const double *u,
                                  const double *th, const double *lam, double a, double b,
                                  double dt, int mode, double *out, double *acc, double *ubar,
                                  double *term, hipStream_t st);

// Multi-step reverse sweep (fl_rk_steps_adjoint): per-call slot rates {w, w'} (16 bytes per slot,
// kAdjRateBytes) from u; one reverse stage in mode ADJ_EULER / ADJ_LAST / ADJ_MID / ADJ_FIRST
// (FIRST: a = the middle stage's a, a3 = the last stage's, lin / l3 the step's input cotangent
// and the last stage's output); uacc: the forward faces' u cotangent [P][C] (+=, or NULL); and
// u_bar[f] += E_f uacc.
constexpr size_t kAdjRateBytes = 16;

hipError_t launch_adjoint_rates(const fl_mesh *m, const double *u, void *wr, hipStream_t st);
hipError_t launch_adjoint_rate_stage(const fl_mesh *m, int lim, int S, const void *wr,
                                     const double *th, const double *lam, double a, double b,
                                     double a3, double dt, int mode, const double *lin,
                                     const double *l3, double *out, double *uacc, hipStream_t st);
hipError_t launch_adjoint_uacc_scatter(const fl_mesh *m, const double *uacc, double *ubar,
                                       hipStream_t st);
// The same reverse stage on meshes with aligned slots from the forward rates rf[P][C] (one per
// face; fl_adjoint_fwd.hip).
hipError_t launch_adjoint_fwd_rates(const fl_mesh *m, const double *u, double *rf,
                                    hipStream_t st);
hipError_t launch_adjoint_fwd_stage(const fl_mesh *m, int lim, int S, const double *rf,
                                    const double *th, const double *lam, double a, double b,
                                    double a3, double dt, int mode, const double *lin,
                                    const double *l3, double *out, double *uacc, hipStream_t st);
// 1 (default): the LDS-staged form evaluates each face once per tile and shares its terms
// (FL_OPT_FACE_SHARE); 0: each cell evaluates every face it needs.
void set_adjoint_share(int on);

// us scales the face velocities (time-dependent velocity); 1 leaves them untouched.
hipError_t launch_face_flux(const fl_mesh *m, int lim, int S, const double *theta,
                            const double *u, double *phi, hipStream_t st, double us = 1.0);
hipError_t launch_cell_update(const fl_mesh *m, int S, const double *phi, const double *ts,
                              const double *tn, double a, double b, double dt, int mode,
                              double *out, hipStream_t st);
hipError_t launch_fused(const fl_mesh *m, int lim, int S, const double *ts, const double *tn,
                        const double *u, double a, double b, double dt, int mode, double *out,
                        hipStream_t st, double us = 1.0);
// Per-call slot records rec[2P][C] (16 bytes each: other cell, far cell, signed face rate) for
// launch_fused_rec (fused-path meshes only).
constexpr size_t kSlotRecBytes = 16;
hipError_t launch_slot_records(const fl_mesh *m, const double *u, void *rec, hipStream_t st);
hipError_t launch_fused_rec(const fl_mesh *m, int lim, int S, const double *ts, const double *tn,
                            const void *rec, double a, double b, double dt, int mode, double *out,
                            hipStream_t st, double us = 1.0);
// LDS-staged stage (fused path with tile tables): per-call rates rate[2P][C] (8 bytes per slot)
// and one workgroup per tile with lds_stage_bytes(m, S) = (tile + max halo + 1) * fwd_chunk(S)
// doubles of dynamic LDS (fwd_chunk(S) scalars staged at a time); used while that is at most
// kMaxStageLds (0 = no tile tables).
// The adjoint stage stages theta and lambda: adjoint_lds_bytes(m, S).  Both are 0 while
// FL_OPT_LDS_STAGE is off (set_lds_stage).
constexpr size_t kMaxStageLds = 64 * 1024;
void set_lds_stage(int on);
size_t lds_stage_bytes(const fl_mesh *m, int S);
size_t adjoint_lds_bytes(const fl_mesh *m, int S);
hipError_t launch_slot_rates(const fl_mesh *m, const double *u, double *rate, hipStream_t st);
// rate: the per-call signed face rates, or NULL to read u (then non-NULL) through the face index.
hipError_t launch_fused_lds(const fl_mesh *m, int lim, int S, const double *ts, const double *tn,
                            const double *rate, double a, double b, double dt, int mode,
                            double *out, hipStream_t st, double us = 1.0,
                            const double *u = nullptr);
// Forward-rate stage (meshes with aligned slots, fused_tile_fwd): per-call rates of the forward
// faces rf[P][C]; LDS of lds_fwd_bytes(m, S) (0: not available).
constexpr size_t kMaxFwdLds = 32 * 1024;
// Scalars the LDS-staged forward stages (single-problem and batched) stage at a time: three,
// which halves the barriers and round trips per tile at S = 6, 8 and makes S = 3 one chunk; at
// S = 4 two chunks of two keep a wave per SIMD more than 3 + 1 (measured on 128^3 boxes).
constexpr int fwd_chunk(int S) { return S == 4 ? 2 : (S < 3 ? S : 3); }
size_t lds_fwd_bytes(const fl_mesh *m, int S);
hipError_t launch_slot_rates_fwd(const fl_mesh *m, const double *u, double *rf, hipStream_t st);
hipError_t launch_fused_lds_fwd(const fl_mesh *m, int lim, int S, const double *ts,
                                const double *tn, const double *rf, double a, double b, double dt,
                                int mode, double *out, hipStream_t st, double us = 1.0);
hipError_t launch_permute(int64_t n, int S, const int32_t *perm, int to_mesh, const double *in,
                          double *out, hipStream_t st);
hipError_t launch_select(const fl_mesh *m, const double *u, int32_t *cdu, hipStream_t st);

// Opt-in finite check of a call's device inputs (FL_OPT_CHECK_FINITE): FL_OK, FL_E_NONFINITE or
// FL_E_HIP.  The device must be current; synchronises st.
struct FiniteSpan {
    const double *p;
    int64_t n;
};
void set_check_finite(int on);
bool check_finite_enabled();
fl_status check_finite(int device, const FiniteSpan *spans, int n_spans, hipStream_t st);

}  // namespace fl
