// C ABI entry points: mesh lifetime, forward operator and explicit time steps.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
#include <initializer_list>
#include <new>
#include <sstream>

#include "fl_internal.h"
#include "fl_kernels.h"

namespace fl {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string &msg) { g_error = msg; }

fl_status fail(fl_status st, const std::string &msg) {
    g_error = msg;
    return st;
}

namespace {

fl_status hip_fail(hipError_t e, const char *what) {
    std::ostringstream os;
    os << what << ": " << hipGetErrorName(e) << " (" << hipGetErrorString(e) << ")";
    return fail(FL_E_HIP, os.str());
}

// Makes the mesh's device current for the scope of a call and restores the caller's device.
struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) {
            err = hipSetDevice(dev);
            changed = (err == hipSuccess);
        }
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

template <class T>
fl_status upload(T **dst, const T *src, size_t n, int64_t &bytes, const char *what) {
    *dst = nullptr;
    if (n == 0) return FL_OK;
    hipError_t e = hipMalloc((void **)dst, n * sizeof(T));
    if (e != hipSuccess) {
        *dst = nullptr;
        std::ostringstream os;
        os << "hipMalloc of " << what << " (" << n * sizeof(T) << " bytes) failed";
        return fail(e == hipErrorOutOfMemory ? FL_E_NOMEM : FL_E_HIP, os.str());
    }
    bytes += (int64_t)(n * sizeof(T));
    e = hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, what);
    return FL_OK;
}

void free_device(fl_mesh *m) {
    void *ptrs[] = {m->d_fc4,      m->d_cf_ptr,  m->d_cf_idx, m->d_slot_face, m->d_slot_nbr,
                    m->d_slot_far, m->d_adj_rec, m->d_area,   m->d_vol,       m->d_cell_perm,
                    m->d_face_perm, m->d_halo_ptr, m->d_halo, m->d_slot_local, m->d_side_ptr,
                    m->d_side_cell, m->d_side_w, m->d_adj_fr, m->d_halo_pair,
                    m->d_halo_nrate, m->d_slot_nb, m->d_halo_pk, m->d_halo_next,
                    m->d_rev_ptr, m->d_rev_side, m->d_rev_w};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    m->d_fc4 = m->d_cf_ptr = m->d_cf_idx = nullptr;
    m->d_slot_face = nullptr;
    m->d_slot_nbr = m->d_slot_far = nullptr;
    m->d_adj_rec = nullptr;
    m->d_adj_fr = nullptr;
    m->d_halo_ptr = m->d_halo = nullptr;
    m->d_slot_local = nullptr;
    m->d_halo_pair = nullptr;
    m->d_halo_nrate = nullptr;
    m->d_slot_nb = nullptr;
    m->d_halo_pk = nullptr;
    m->d_halo_next = nullptr;
    m->d_rev_ptr = m->d_rev_side = nullptr;
    m->d_rev_w = nullptr;
    m->d_side_ptr = m->d_side_cell = nullptr;
    m->d_side_w = nullptr;
    m->d_area = m->d_vol = nullptr;
    m->d_cell_perm = m->d_face_perm = nullptr;
}

fl_status check_compute(const fl_mesh *m, int lim, int S) {
    if (!m) return fail(FL_E_INVALID, "mesh is NULL");
    if (m->device < 0) return fail(FL_E_NODEVICE, "the mesh was created host-only (device = -1)");
    if (lim < 0 || lim >= FL_NUM_LIMITERS) return fail(FL_E_INVALID, "unknown limiter");
    if (S < 1 || S > FL_MAX_SCALARS) return fail(FL_E_INVALID, "n_scalars must be in [1, 8]");
    if (m->inflow && S != m->inflow_S)
        return fail(FL_E_INVALID, "the mesh's inflow values hold another number of scalars");
    return FL_OK;
}

bool misaligned(const void *p) { return ((uintptr_t)p & 7u) != 0; }

// The opt-in finite check of a call's inputs (nothing runs while FL_OPT_CHECK_FINITE is off).
fl_status finite_inputs(const fl_mesh *m, std::initializer_list<FiniteSpan> spans, double dt,
                        hipStream_t st) {
    if (!check_finite_enabled()) return FL_OK;
    if (!std::isfinite(dt)) return fail(FL_E_NONFINITE, "dt is not finite");
    return check_finite(m->device, spans.begin(), (int)spans.size(), st);
}

constexpr double kRk3A[3] = {0.0, 0.75, 1.0 / 3.0};
constexpr double kRk3B[3] = {1.0, 0.25, 2.0 / 3.0};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Multi-step calls on fused-path meshes build per-call slot tables once (FL_OPT_SLOT_VELOCITY)
// and, where the mesh has tile tables and the tile fits in LDS, run the LDS-staged stage
// (FL_OPT_LDS_STAGE).
int g_slot_velocity = 1;

// How the stages of one call read the face velocities: gathered through the face index
// (PLAN_GATHER), from per-call slot records (PLAN_RECORDS), or from per-call rates with the
// LDS-staged stage (PLAN_LDS).
enum { PLAN_GATHER = 0, PLAN_RECORDS = 1, PLAN_LDS = 2, PLAN_LDS_FWD = 3 };
int g_fwd_rates = 1;  // FL_OPT_FWD_RATES
struct Plan {
    int kind = PLAN_GATHER;
    void *table = nullptr;
};

// One stage: out = a tn + b (ts + dt L(ts)) in the given mode.
hipError_t stage(const fl_mesh *m, int lim, int S, double dt, double a, double b, int mode,
                 const double *ts, const double *tn, const double *u, double *out, double *phi,
                 hipStream_t st, double us = 1.0, const Plan &pl = Plan()) {
    if (m->path == FL_PATH_FUSED) {
        if (pl.kind == PLAN_LDS_FWD)
            return launch_fused_lds_fwd(m, lim, S, ts, tn, static_cast<const double *>(pl.table),
                                        a, b, dt, mode, out, st, us);
        if (pl.kind == PLAN_LDS)
            return launch_fused_lds(m, lim, S, ts, tn, static_cast<const double *>(pl.table), a,
                                    b, dt, mode, out, st, us);
        if (pl.kind == PLAN_RECORDS)
            return launch_fused_rec(m, lim, S, ts, tn, pl.table, a, b, dt, mode, out, st, us);
        return launch_fused(m, lim, S, ts, tn, u, a, b, dt, mode, out, st, us);
    }
    hipError_t e = launch_face_flux(m, lim, S, ts, u, phi, st, us);
    if (e != hipSuccess) return e;
    return launch_cell_update(m, S, phi, ts, tn, a, b, dt, mode, out, st);
}

struct Work {
    double *phi = nullptr, *t1 = nullptr, *t2 = nullptr;
    void *vs = nullptr;
};

// Workspace of fl_rk_steps: [phi (face path)] t1 t2 [slot records (fused path)].
size_t slot_velocity_bytes(const fl_mesh *m) {
    return m->path == FL_PATH_FUSED ? align256((size_t)2 * m->h.pairs * m->h.nc * kSlotRecBytes)
                                    : 0;
}

Work carve(const fl_mesh *m, int S, void *work) {
    Work w;
    char *p = (char *)work;
    const size_t cell = align256((size_t)m->h.nc * S * sizeof(double));
    if (m->path == FL_PATH_FACE_CELL) {
        w.phi = (double *)p;
        p += align256((size_t)m->h.nf * S * sizeof(double));
    }
    w.t1 = (double *)p;
    p += cell;
    w.t2 = (double *)p;
    p += cell;
    if (m->path == FL_PATH_FUSED) w.vs = p;
    return w;
}

// The per-call tables of a multi-step call (single steps gather u directly: the tables cost
// about one stage's table traffic to build).
hipError_t prepare_rates(const fl_mesh *m, const double *u, int S, int64_t n_steps,
                         const Work &w, hipStream_t st, Plan *pl) {
    *pl = Plan();
    if (m->path != FL_PATH_FUSED || !g_slot_velocity || n_steps < 2) return hipSuccess;
    const size_t fl = lds_fwd_bytes(m, S);
    if (g_fwd_rates && fl > 0 && fl <= kMaxStageLds) {
        hipError_t e = launch_slot_rates_fwd(m, u, static_cast<double *>(w.vs), st);
        if (e == hipSuccess) *pl = Plan{PLAN_LDS_FWD, w.vs};
        return e;
    }
    const size_t lds = lds_stage_bytes(m, S);
    if (lds > 0 && lds <= kMaxStageLds) {
        hipError_t e = launch_slot_rates(m, u, static_cast<double *>(w.vs), st);
        if (e == hipSuccess) *pl = Plan{PLAN_LDS, w.vs};
        return e;
    }
    hipError_t e = launch_slot_records(m, u, w.vs, st);
    if (e == hipSuccess) *pl = Plan{PLAN_RECORDS, w.vs};
    return e;
}

}  // namespace
}  // namespace fl

using namespace fl;

extern "C" {

const char *fl_status_str(fl_status s) {
    switch (s) {
        case FL_OK: return "FL_OK";
        case FL_E_INVALID: return "FL_E_INVALID";
        case FL_E_TOPOLOGY: return "FL_E_TOPOLOGY";
        case FL_E_UNSUPPORTED: return "FL_E_UNSUPPORTED";
        case FL_E_NOMEM: return "FL_E_NOMEM";
        case FL_E_HIP: return "FL_E_HIP";
        case FL_E_NONFINITE: return "FL_E_NONFINITE";
        case FL_E_NODEVICE: return "FL_E_NODEVICE";
        default: return "FL_E_UNKNOWN";
    }
}

const char *fl_last_error(void) { return g_error.c_str(); }

fl_status fl_set_option(int option, int value) {
    if (option == FL_OPT_XCD_REMAP && value >= 0 && value <= (1 << 16)) {
        set_xcd_remap(value);
        return FL_OK;
    }
    if (option == FL_OPT_SLOT_VELOCITY && (value == 0 || value == 1)) {
        g_slot_velocity = value;
        return FL_OK;
    }
    if (option == FL_OPT_LDS_STAGE && (value == 0 || value == 1)) {
        set_lds_stage(value);
        return FL_OK;
    }
    if (option == FL_OPT_FWD_RATES && (value == 0 || value == 1)) {
        g_fwd_rates = value;
        return FL_OK;
    }
    if (option == FL_OPT_FACE_SHARE && (value == 0 || value == 1)) {
        set_adjoint_share(value);
        return FL_OK;
    }
    if (option == FL_OPT_CHECK_FINITE && (value == 0 || value == 1)) {
        set_check_finite(value);
        return FL_OK;
    }
    return fail(FL_E_INVALID, "unknown option or value");
}

fl_status fl_mesh_validate(int64_t n_cells, int64_t n_faces, const int32_t *face_cells,
                           const double *face_normal) {
    try {
        HostTables t;
        return build_host_tables(n_cells, n_faces, face_cells, face_normal, nullptr, nullptr,
                                 nullptr, REORDER_NONE, t);
    } catch (const std::bad_alloc &) {
        return fail(FL_E_NOMEM, "host allocation failed");
    }
}

fl_status fl_mesh_create(int64_t n_cells, int64_t n_faces, const int32_t *face_cells,
                         const double *face_normal, const double *face_area,
                         const double *cell_volume, int device, uint32_t flags, fl_mesh **out) {
    return fl_mesh_create_dist(n_cells, n_faces, face_cells, face_normal, face_area, cell_volume,
                               nullptr, device, flags, out);
}

fl_status fl_mesh_create_dist(int64_t n_cells, int64_t n_faces, const int32_t *face_cells,
                              const double *face_normal, const double *face_area,
                              const double *cell_volume, const double *face_dist, int device,
                              uint32_t flags, fl_mesh **out) {
    if (!out) return fail(FL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (flags & ~(uint32_t)(FL_MESH_REORDER | FL_MESH_FACE_PATH | FL_MESH_REORDER_BFS))
        return fail(FL_E_INVALID, "unknown flag");
    if ((flags & FL_MESH_REORDER) && (flags & FL_MESH_REORDER_BFS))
        return fail(FL_E_INVALID, "FL_MESH_REORDER and FL_MESH_REORDER_BFS are exclusive");
    const int reorder = (flags & FL_MESH_REORDER) ? REORDER_CURVE
                        : (flags & FL_MESH_REORDER_BFS) ? REORDER_BFS : REORDER_NONE;
    if (device < -1) return fail(FL_E_INVALID, "device must be >= -1");
    fl_mesh *m = nullptr;
    try {
        m = new fl_mesh();
        fl_status st = build_host_tables(n_cells, n_faces, face_cells, face_normal, face_area,
                                         cell_volume, face_dist, reorder, m->h);
        if (st != FL_OK) {
            delete m;
            return st;
        }
        m->reordered = reorder != REORDER_NONE;
        m->path = (m->h.pairs > 0 && !(flags & FL_MESH_FACE_PATH)) ? FL_PATH_FUSED
                                                                    : FL_PATH_FACE_CELL;
        m->device = device;
        if (device >= 0) {
            int ndev = 0;
            hipError_t e = hipGetDeviceCount(&ndev);
            if (e != hipSuccess || device >= ndev) {
                delete m;
                return fail(FL_E_HIP, "no such HIP device");
            }
            DeviceGuard g(device);
            if (g.err != hipSuccess) {
                delete m;
                return hip_fail(g.err, "hipSetDevice");
            }
            const HostTables &h = m->h;
            std::vector<int32_t> fc4((size_t)h.nf * 4);
#pragma omp parallel for schedule(static)
            for (int64_t f = 0; f < h.nf; ++f) {
                fc4[4 * f] = h.fc[2 * f];
                fc4[4 * f + 1] = h.fc[2 * f + 1];
                fc4[4 * f + 2] = h.far[2 * f];
                fc4[4 * f + 3] = h.far[2 * f + 1];
            }
            int64_t &B = m->device_bytes;
            st = upload(&m->d_fc4, fc4.data(), fc4.size(), B, "face records");
            if (st == FL_OK && h.general) {
                st = upload(&m->d_side_ptr, h.side_ptr.data(), h.side_ptr.size(), B, "side pointers");
                if (st == FL_OK) st = upload(&m->d_side_cell, h.side_cell.data(), h.side_cell.size(), B, "side cells");
                if (st == FL_OK) st = upload(&m->d_side_w, h.side_w.data(), h.side_w.size(), B, "side weights");
                if (st == FL_OK) st = upload(&m->d_rev_ptr, h.rev_ptr.data(), h.rev_ptr.size(), B, "transposed side pointers");
                if (st == FL_OK && !h.rev_side.empty()) {
                    st = upload(&m->d_rev_side, h.rev_side.data(), h.rev_side.size(), B, "transposed sides");
                    if (st == FL_OK) st = upload(&m->d_rev_w, h.rev_w.data(), h.rev_w.size(), B, "transposed weights");
                }
            }
            if (st == FL_OK && !h.uniform_degree)
                st = upload(&m->d_cf_ptr, h.cf_ptr.data(), h.cf_ptr.size(), B, "cell pointers");
            if (st == FL_OK) st = upload(&m->d_cf_idx, h.cf_idx.data(), h.cf_idx.size(), B, "cell faces");
            if (st == FL_OK && h.pairs > 0) {
                st = upload(&m->d_slot_face, h.slot_face.data(), h.slot_face.size(), B, "slot faces");
                if (st == FL_OK) st = upload(&m->d_slot_nbr, h.slot_nbr.data(), h.slot_nbr.size(), B, "slot cells");
                if (st == FL_OK) st = upload(&m->d_slot_far, h.slot_far.data(), h.slot_far.size(), B, "slot far cells");
                if (st == FL_OK) {
                    // adjoint records {face | own bit, opposite face of the neighbour | its own
                    // bit, neighbour, far cell}: one 16-byte load per slot in the reverse kernel
                    const size_t n = h.slot_face.size();
                    std::vector<int32_t> rec(4 * n);
#pragma omp parallel for schedule(static)
                    for (size_t i = 0; i < n; ++i) {
                        rec[4 * i] = (int32_t)h.slot_face[i];
                        rec[4 * i + 1] = (int32_t)h.slot_rev[i];
                        rec[4 * i + 2] = h.slot_nbr[i];
                        rec[4 * i + 3] = h.slot_far[i];
                    }
                    st = upload(&m->d_adj_rec, rec.data(), rec.size(), B, "adjoint slot records");
                }
                if (st == FL_OK && h.max_halo >= 0) {
                    const size_t n = h.slot_face.size();
                    std::vector<int32_t> fr(2 * n);
#pragma omp parallel for schedule(static)
                    for (size_t i = 0; i < n; ++i) {
                        fr[2 * i] = (int32_t)h.slot_face[i];
                        fr[2 * i + 1] = (int32_t)h.slot_rev[i];
                    }
                    st = upload(&m->d_adj_fr, fr.data(), fr.size(), B, "adjoint face pairs");
                }
                if (st == FL_OK && h.max_halo >= 0) {
                    st = upload(&m->d_halo_ptr, h.halo_ptr.data(), h.halo_ptr.size(), B, "tile halo pointers");
                    if (st == FL_OK) {
                        // padded: the staging reads each tile's first entry, also where its
                        // halo is empty
                        std::vector<int32_t> hp(h.halo);
                        hp.resize(h.halo.size() + kHaloPad, 0);
                        st = upload(&m->d_halo, hp.data(), hp.size(), B, "tile halos");
                    }
                    if (st == FL_OK)
                        st = upload(&m->d_slot_local, h.slot_local.data(), h.slot_local.size(), B,
                                    "local slot indices");
                    if (st == FL_OK && !h.halo_pair.empty()) {
                        std::vector<uint8_t> hp(h.halo_pair);
                        hp.resize(h.halo_pair.size() + kHaloPad, 0);
                        st = upload(&m->d_halo_pair, hp.data(), hp.size(), B, "tile halo pairs");
                        if (st == FL_OK)
                            st = upload(&m->d_halo_nrate, h.halo_nrate.data(), h.halo_nrate.size(),
                                        B, "tile halo rate counts");
                    }
                    if (st == FL_OK && !h.slot_nb.empty()) {
                        st = upload(&m->d_slot_nb, h.slot_nb.data(), h.slot_nb.size(), B,
                                    "compact slot words");
                        std::vector<int32_t> pk(h.halo_pk);
                        pk.resize(h.halo_pk.size() + kHaloPad, 0);
                        if (st == FL_OK)
                            st = upload(&m->d_halo_pk, pk.data(), pk.size(), B, "packed tile halos");
                        std::vector<uint16_t> nx(h.halo_next);
                        nx.resize(h.halo_next.size() + kHaloPad, 0);
                        if (st == FL_OK)
                            st = upload(&m->d_halo_next, nx.data(), nx.size(), B, "tile halo next");
                    }
                }
            }
            if (st == FL_OK && !h.uni_area) st = upload(&m->d_area, h.area.data(), h.area.size(), B, "areas");
            if (st == FL_OK && !h.uni_vol) st = upload(&m->d_vol, h.vol.data(), h.vol.size(), B, "volumes");
            if (st == FL_OK && m->reordered) {
                st = upload(&m->d_cell_perm, h.cell_perm.data(), h.cell_perm.size(), B, "cell permutation");
                if (st == FL_OK)
                    st = upload(&m->d_face_perm, h.face_perm.data(), h.face_perm.size(), B, "face permutation");
            }
            if (st != FL_OK) {
                free_device(m);
                delete m;
                return st;
            }
        }
        *out = m;
        return FL_OK;
    } catch (const std::bad_alloc &) {
        if (m) {
            free_device(m);
            delete m;
        }
        return fail(FL_E_NOMEM, "host allocation failed");
    }
}

fl_status fl_mesh_destroy(fl_mesh *m) {
    if (!m) return FL_OK;
    if (m->device >= 0) {
        DeviceGuard g(m->device);
        free_device(m);
    }
    delete m;
    return FL_OK;
}

fl_status fl_mesh_info(const fl_mesh *m, fl_mesh_info_t *info) {
    if (!m || !info) return fail(FL_E_INVALID, "NULL argument");
    info->n_cells = m->h.nc;
    info->n_faces = m->h.nf;
    info->max_degree = m->h.max_degree;
    info->pairs = m->h.pairs;
    info->path = m->path;
    info->device = m->device;
    info->reordered = m->reordered ? 1 : 0;
    info->uniform_area = m->h.uni_area ? 1 : 0;
    info->uniform_volume = m->h.uni_vol ? 1 : 0;
    info->device_bytes = m->device_bytes;
    info->tile_cells = m->h.max_halo >= 0 ? kTileCells : 0;
    info->max_halo = m->h.max_halo;
    info->halo_total = (int64_t)m->h.halo.size();
    info->general = m->h.general ? 1 : 0;
    int32_t ms = 0;
    for (size_t i = 0; i + 1 < m->h.side_ptr.size(); ++i)
        ms = std::max(ms, m->h.side_ptr[i + 1] - m->h.side_ptr[i]);
    info->max_side = m->h.general ? ms : 1;
    info->aligned = m->h.aligned_slots ? 1 : 0;
    info->dist_weighted = m->h.dist_weighted ? 1 : 0;
    info->n_boundary = m->h.n_boundary;
    info->compact = m->d_slot_nb || !m->h.slot_nb.empty() ? 1 : 0;
    info->max_rated = m->h.max_nrate0;
    info->max_nexts = m->h.max_nrate;
    info->side_entries = m->h.general && !m->h.side_ptr.empty() ? m->h.side_ptr.back() : 0;
    int64_t nx = 0;
    for (size_t t = 1; t < m->h.halo_nrate.size(); t += 2) nx += m->h.halo_nrate[t];
    info->halo_nexts = nx;
    return FL_OK;
}

fl_status fl_mesh_set_inflow(fl_mesh *m, const double *inflow, int n_scalars) {
    if (!m) return fail(FL_E_INVALID, "mesh is NULL");
    if (!inflow) {
        m->inflow = nullptr;
        m->inflow_S = 0;
        return FL_OK;
    }
    if (m->device < 0) return fail(FL_E_NODEVICE, "the mesh was created host-only (device = -1)");
    if (n_scalars < 1 || n_scalars > FL_MAX_SCALARS)
        return fail(FL_E_INVALID, "n_scalars must be in [1, 8]");
    if (misaligned(inflow)) return fail(FL_E_INVALID, "inflow must be 8-byte aligned");
    m->inflow = inflow;
    m->inflow_S = n_scalars;
    return FL_OK;
}

fl_status fl_mesh_permutation(const fl_mesh *m, int32_t *cell_perm, int32_t *face_perm) {
    if (!m) return fail(FL_E_INVALID, "mesh is NULL");
    if (cell_perm) {
        if (m->reordered) std::memcpy(cell_perm, m->h.cell_perm.data(), m->h.nc * sizeof(int32_t));
        else for (int64_t c = 0; c < m->h.nc; ++c) cell_perm[c] = (int32_t)c;
    }
    if (face_perm) {
        if (m->reordered) std::memcpy(face_perm, m->h.face_perm.data(), m->h.nf * sizeof(int32_t));
        else for (int64_t f = 0; f < m->h.nf; ++f) face_perm[f] = (int32_t)f;
    }
    return FL_OK;
}

fl_status fl_mesh_export_tables(const fl_mesh *m, int32_t *face_far, int32_t *cf_ptr,
                                int32_t *cf_idx) {
    if (!m) return fail(FL_E_INVALID, "mesh is NULL");
    if (face_far) std::memcpy(face_far, m->h.far.data(), m->h.far.size() * sizeof(int32_t));
    if (cf_ptr) std::memcpy(cf_ptr, m->h.cf_ptr.data(), m->h.cf_ptr.size() * sizeof(int32_t));
    if (cf_idx) std::memcpy(cf_idx, m->h.cf_idx.data(), m->h.cf_idx.size() * sizeof(int32_t));
    return FL_OK;
}

fl_status fl_permute_cells(const fl_mesh *m, int to_mesh, int S, const double *in, double *out,
                           void *stream) {
    fl_status s = check_compute(m, 0, S);
    if (s != FL_OK) return s;
    if (!in || !out || in == out) return fail(FL_E_INVALID, "in/out must be distinct non-NULL");
    DeviceGuard g(m->device);
    hipError_t e;
    if (!m->reordered)
        e = hipMemcpyAsync(out, in, m->h.nc * S * sizeof(double), hipMemcpyDeviceToDevice,
                           (hipStream_t)stream);
    else
        e = launch_permute(m->h.nc, S, m->d_cell_perm, to_mesh, in, out, (hipStream_t)stream);
    return e == hipSuccess ? FL_OK : hip_fail(e, "permute cells");
}

fl_status fl_permute_faces(const fl_mesh *m, int to_mesh, const double *in, double *out,
                           void *stream) {
    fl_status s = check_compute(m, 0, 1);
    if (s != FL_OK) return s;
    if (!in || !out || in == out) return fail(FL_E_INVALID, "in/out must be distinct non-NULL");
    DeviceGuard g(m->device);
    hipError_t e;
    if (!m->reordered)
        e = hipMemcpyAsync(out, in, m->h.nf * sizeof(double), hipMemcpyDeviceToDevice,
                           (hipStream_t)stream);
    else
        e = launch_permute(m->h.nf, 1, m->d_face_perm, to_mesh, in, out, (hipStream_t)stream);
    return e == hipSuccess ? FL_OK : hip_fail(e, "permute faces");
}

size_t fl_apply_workspace_bytes(const fl_mesh *m, int S) {
    if (!m || S < 1 || S > FL_MAX_SCALARS) return 0;
    return m->path == FL_PATH_FACE_CELL ? align256((size_t)m->h.nf * S * sizeof(double)) : 0;
}

fl_status fl_convect_apply(const fl_mesh *m, int lim, int S, const double *theta,
                           const double *u, double *rhs, void *work, void *stream) {
    fl_status s = check_compute(m, lim, S);
    if (s != FL_OK) return s;
    if (!theta || !u || !rhs) return fail(FL_E_INVALID, "NULL device pointer");
    if (misaligned(theta) || misaligned(u) || misaligned(rhs))
        return fail(FL_E_INVALID, "device pointers must be 8-byte aligned");
    if (rhs == theta) return fail(FL_E_INVALID, "rhs must not alias theta");
    DeviceGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    s = finite_inputs(m, {{theta, m->h.nc * S}, {u, m->h.nf}}, 0.0, st);
    if (s != FL_OK) return s;
    hipError_t e;
    if (m->path == FL_PATH_FUSED) {
        e = launch_fused(m, lim, S, theta, theta, u, 0.0, 1.0, 0.0, MODE_RHS, rhs, st);
    } else {
        if (!work || ((uintptr_t)work & 255u))
            return fail(FL_E_INVALID, "face-path meshes need a 256-byte aligned workspace");
        double *phi = (double *)work;
        e = launch_face_flux(m, lim, S, theta, u, phi, st);
        if (e == hipSuccess)
            e = launch_cell_update(m, S, phi, theta, theta, 0.0, 1.0, 0.0, MODE_RHS, rhs, st);
    }
    return e == hipSuccess ? FL_OK : hip_fail(e, "fl_convect_apply launch");
}

size_t fl_rk_workspace_bytes(const fl_mesh *m, int scheme, int S) {
    if (!m || S < 1 || S > FL_MAX_SCALARS || (scheme != FL_EULER && scheme != FL_SSPRK3)) return 0;
    size_t b = 2 * align256((size_t)m->h.nc * S * sizeof(double));
    if (m->path == FL_PATH_FACE_CELL) b += align256((size_t)m->h.nf * S * sizeof(double));
    return b + slot_velocity_bytes(m);
}

fl_status fl_rk_steps(const fl_mesh *m, int lim, int scheme, double dt, int S, int64_t n_steps,
                      double *theta, const double *u, void *work, void *stream) {
    fl_status s = check_compute(m, lim, S);
    if (s != FL_OK) return s;
    if (scheme != FL_EULER && scheme != FL_SSPRK3) return fail(FL_E_INVALID, "unknown scheme");
    if (!theta || !u || !work) return fail(FL_E_INVALID, "NULL device pointer");
    if (misaligned(theta) || misaligned(u) || ((uintptr_t)work & 255u))
        return fail(FL_E_INVALID, "theta/u must be 8-byte and work 256-byte aligned");
    if (n_steps < 0) return fail(FL_E_INVALID, "n_steps must be >= 0");
    if (!(dt == dt)) return fail(FL_E_INVALID, "dt is NaN");
    DeviceGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    s = finite_inputs(m, {{theta, m->h.nc * S}, {u, m->h.nf}}, dt, st);
    if (s != FL_OK) return s;
    Work w = carve(m, S, work);
    Plan vs;
    hipError_t e = prepare_rates(m, u, S, n_steps, w, st, &vs);
    if (scheme == FL_EULER) {
        if (m->path == FL_PATH_FACE_CELL) {
            for (int64_t i = 0; i < n_steps && e == hipSuccess; ++i)
                e = stage(m, lim, S, dt, 0.0, 1.0, MODE_EULER, theta, theta, u, theta, w.phi, st);
        } else {
            // the fused kernel gathers its input, so it cannot write in place: ping-pong
            double *src = theta, *dst = w.t1;
            for (int64_t i = 0; i < n_steps && e == hipSuccess; ++i) {
                e = stage(m, lim, S, dt, 0.0, 1.0, MODE_EULER, src, src, u, dst, w.phi, st, 1.0, vs);
                std::swap(src, dst);
            }
            if (e == hipSuccess && src != theta)
                e = hipMemcpyAsync(theta, src, m->h.nc * S * sizeof(double),
                                   hipMemcpyDeviceToDevice, st);
        }
    } else {
        for (int64_t i = 0; i < n_steps && e == hipSuccess; ++i) {
            e = stage(m, lim, S, dt, kRk3A[0], kRk3B[0], MODE_EULER, theta, theta, u, w.t1, w.phi, st, 1.0, vs);
            if (e == hipSuccess)
                e = stage(m, lim, S, dt, kRk3A[1], kRk3B[1], MODE_RK, w.t1, theta, u, w.t2, w.phi, st, 1.0, vs);
            if (e == hipSuccess)
                e = stage(m, lim, S, dt, kRk3A[2], kRk3B[2], MODE_RK, w.t2, theta, u, theta, w.phi, st, 1.0, vs);
        }
    }
    return e == hipSuccess ? FL_OK : hip_fail(e, "fl_rk_step launch");
}

fl_status fl_rk_steps_scaled(const fl_mesh *m, int lim, int scheme, double dt, int S,
                             int64_t n_steps, double *theta, const double *u,
                             const double *u_scale, void *work, void *stream) {
    fl_status s = check_compute(m, lim, S);
    if (s != FL_OK) return s;
    if (scheme != FL_EULER && scheme != FL_SSPRK3) return fail(FL_E_INVALID, "unknown scheme");
    if (!theta || !u || !work || (n_steps > 0 && !u_scale))
        return fail(FL_E_INVALID, "NULL pointer");
    if (misaligned(theta) || misaligned(u) || ((uintptr_t)work & 255u))
        return fail(FL_E_INVALID, "theta/u must be 8-byte and work 256-byte aligned");
    if (n_steps < 0) return fail(FL_E_INVALID, "n_steps must be >= 0");
    DeviceGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    if (check_finite_enabled()) {
        const int64_t ns = n_steps * (scheme == FL_EULER ? 1 : 3);
        for (int64_t i = 0; i < ns; ++i)
            if (!std::isfinite(u_scale[i])) return fail(FL_E_NONFINITE, "u_scale is not finite");
    }
    s = finite_inputs(m, {{theta, m->h.nc * S}, {u, m->h.nf}}, dt, st);
    if (s != FL_OK) return s;
    Work w = carve(m, S, work);
    Plan vs;
    hipError_t e = prepare_rates(m, u, S, n_steps, w, st, &vs);
    const double *sc = u_scale;
    if (scheme == FL_EULER) {
        double *src = theta, *dst = w.t1;
        for (int64_t i = 0; i < n_steps && e == hipSuccess; ++i) {
            if (m->path == FL_PATH_FACE_CELL) {
                e = stage(m, lim, S, dt, 0.0, 1.0, MODE_EULER, theta, theta, u, theta, w.phi, st, sc[i]);
            } else {
                e = stage(m, lim, S, dt, 0.0, 1.0, MODE_EULER, src, src, u, dst, w.phi, st, sc[i], vs);
                std::swap(src, dst);
            }
        }
        if (e == hipSuccess && src != theta)
            e = hipMemcpyAsync(theta, src, m->h.nc * S * sizeof(double), hipMemcpyDeviceToDevice, st);
    } else {
        for (int64_t i = 0; i < n_steps && e == hipSuccess; ++i) {
            const double *si = sc + 3 * i;
            e = stage(m, lim, S, dt, kRk3A[0], kRk3B[0], MODE_EULER, theta, theta, u, w.t1, w.phi, st, si[0], vs);
            if (e == hipSuccess)
                e = stage(m, lim, S, dt, kRk3A[1], kRk3B[1], MODE_RK, w.t1, theta, u, w.t2, w.phi, st, si[1], vs);
            if (e == hipSuccess)
                e = stage(m, lim, S, dt, kRk3A[2], kRk3B[2], MODE_RK, w.t2, theta, u, theta, w.phi, st, si[2], vs);
        }
    }
    return e == hipSuccess ? FL_OK : hip_fail(e, "fl_rk_steps_scaled launch");
}

fl_status fl_rk_step(const fl_mesh *m, int lim, int scheme, double dt, int S, double *theta,
                     const double *u, void *work, void *stream) {
    return fl_rk_steps(m, lim, scheme, dt, S, 1, theta, u, work, stream);
}

// ------------------------------------------------------------------------------------------
// Adjoint
// ------------------------------------------------------------------------------------------
// General cells (side lists: projected faces, boundary faces, face distances) run the
// two-kernel adjoint, whose face terms need a buffer; the paired kernels gather everything they
// need.
static bool general_adjoint(const fl_mesh *m) { return m->h.general != 0; }

size_t fl_adjoint_workspace_bytes(const fl_mesh *m, int S) {
    if (!m || S < 1 || S > FL_MAX_SCALARS || !general_adjoint(m)) return 0;
    return align256(adjoint_general_term_bytes(m, S));
}

static fl_status check_adjoint(const fl_mesh *m, int lim, int S) {
    fl_status s = check_compute(m, lim, S);
    if (s != FL_OK) return s;
    if (m->h.pairs == 0 && !m->h.general)
        return fail(FL_E_UNSUPPORTED,
                    "the adjoint needs cells whose faces form opposite pairs, or side lists");
    return FL_OK;
}

fl_status fl_convect_adjoint(const fl_mesh *m, int lim, int S, const double *theta,
                             const double *u, const double *rhs_bar, double *theta_bar,
                             double *u_bar, void *work, void *stream) {
    fl_status s = check_adjoint(m, lim, S);
    if (s != FL_OK) return s;
    if (!theta || !u || !rhs_bar || !theta_bar) return fail(FL_E_INVALID, "NULL device pointer");
    if (misaligned(theta) || misaligned(u) || misaligned(rhs_bar) || misaligned(theta_bar) ||
        misaligned(u_bar))
        return fail(FL_E_INVALID, "device pointers must be 8-byte aligned");
    if (theta_bar == rhs_bar || theta_bar == theta)
        return fail(FL_E_INVALID, "theta_bar must not alias theta or rhs_bar");
    DeviceGuard g(m->device);
    s = finite_inputs(m, {{theta, m->h.nc * S}, {u, m->h.nf}, {rhs_bar, m->h.nc * S}}, 0.0,
                      (hipStream_t)stream);
    if (s != FL_OK) return s;
    hipError_t e;
    if (general_adjoint(m)) {
        if (!work || ((uintptr_t)work & 255u))
            return fail(FL_E_INVALID, "general cells need a 256-byte aligned work buffer of "
                                      "fl_adjoint_workspace_bytes bytes");
        e = launch_adjoint_general(m, lim, S, u, theta, rhs_bar, 0.0, 1.0, 0.0, ADJ_APPLY,
                                   theta_bar, nullptr, u_bar, (double *)work, (hipStream_t)stream);
    } else {
        e = launch_adjoint(m, lim, S, u, theta, rhs_bar, 0.0, 1.0, 0.0, ADJ_APPLY, theta_bar,
                           nullptr, u_bar, (hipStream_t)stream);
    }
    return e == hipSuccess ? FL_OK : hip_fail(e, "fl_convect_adjoint launch");
}

size_t fl_rk_adjoint_workspace_bytes(const fl_mesh *m, int scheme, int S) {
    if (!m || S < 1 || S > FL_MAX_SCALARS || (scheme != FL_EULER && scheme != FL_SSPRK3)) return 0;
    // cell buffers (Euler: 1, SSP-RK3: 3), then the general cells' face terms
    return (scheme == FL_EULER ? 1 : 3) * align256((size_t)m->h.nc * S * sizeof(double)) +
           fl_adjoint_workspace_bytes(m, S);
}

fl_status fl_rk_step_store(const fl_mesh *m, int lim, int scheme, double dt, int S,
                           double *theta, const double *u, double *stages, void *work,
                           void *stream) {
    fl_status s = check_compute(m, lim, S);
    if (s != FL_OK) return s;
    if (scheme != FL_EULER && scheme != FL_SSPRK3) return fail(FL_E_INVALID, "unknown scheme");
    if (!theta || !u || !stages || !work) return fail(FL_E_INVALID, "NULL device pointer");
    if (misaligned(theta) || misaligned(u) || misaligned(stages) || ((uintptr_t)work & 255u))
        return fail(FL_E_INVALID, "theta/u/stages must be 8-byte and work 256-byte aligned");
    DeviceGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t cell = (size_t)m->h.nc * S;
    s = finite_inputs(m, {{theta, (int64_t)cell}, {u, m->h.nf}}, dt, st);
    if (s != FL_OK) return s;
    Work w = carve(m, S, work);
    hipError_t e = hipMemcpyAsync(stages, theta, cell * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) {
        if (scheme == FL_EULER) {
            // stage input is theta^n itself (already stored); out of place, then back
            e = stage(m, lim, S, dt, 0.0, 1.0, MODE_EULER, stages, stages, u, theta, w.phi, st);
        } else {
            double *t1 = stages + cell, *t2 = stages + 2 * cell;
            e = stage(m, lim, S, dt, kRk3A[0], kRk3B[0], MODE_EULER, theta, theta, u, t1, w.phi, st);
            if (e == hipSuccess)
                e = stage(m, lim, S, dt, kRk3A[1], kRk3B[1], MODE_RK, t1, theta, u, t2, w.phi, st);
            if (e == hipSuccess)
                e = stage(m, lim, S, dt, kRk3A[2], kRk3B[2], MODE_RK, t2, theta, u, theta, w.phi, st);
        }
    }
    return e == hipSuccess ? FL_OK : hip_fail(e, "fl_rk_step_store launch");
}

fl_status fl_rk_steps_store(const fl_mesh *m, int lim, int scheme, double dt, int S,
                            int64_t n_steps, double *theta, const double *u, double *stages,
                            void *work, void *stream) {
    fl_status s = check_compute(m, lim, S);
    if (s != FL_OK) return s;
    if (scheme != FL_EULER && scheme != FL_SSPRK3) return fail(FL_E_INVALID, "unknown scheme");
    if (!theta || !u || !stages || !work) return fail(FL_E_INVALID, "NULL device pointer");
    if (misaligned(theta) || misaligned(u) || misaligned(stages) || ((uintptr_t)work & 255u))
        return fail(FL_E_INVALID, "theta/u/stages must be 8-byte and work 256-byte aligned");
    if (n_steps < 0) return fail(FL_E_INVALID, "n_steps must be >= 0");
    if (n_steps == 0) return FL_OK;
    DeviceGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t cell = (size_t)m->h.nc * S;
    const size_t per_step = cell * (scheme == FL_EULER ? 1 : 3);
    s = finite_inputs(m, {{theta, (int64_t)cell}, {u, m->h.nf}}, dt, st);
    if (s != FL_OK) return s;
    Work w = carve(m, S, work);
    Plan vs;
    hipError_t e = prepare_rates(m, u, S, n_steps, w, st, &vs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stages, theta, cell * sizeof(double), hipMemcpyDeviceToDevice, st);
    // each step's last stage writes the next step's stored input directly (the last: theta)
    for (int64_t i = 0; i < n_steps && e == hipSuccess; ++i) {
        double *tn = stages + i * per_step;
        double *next = (i + 1 < n_steps) ? tn + per_step : theta;
        if (scheme == FL_EULER) {
            e = stage(m, lim, S, dt, 0.0, 1.0, MODE_EULER, tn, tn, u, next, w.phi, st, 1.0, vs);
        } else {
            double *t1 = tn + cell, *t2 = tn + 2 * cell;
            e = stage(m, lim, S, dt, kRk3A[0], kRk3B[0], MODE_EULER, tn, tn, u, t1, w.phi, st, 1.0, vs);
            if (e == hipSuccess)
                e = stage(m, lim, S, dt, kRk3A[1], kRk3B[1], MODE_RK, t1, tn, u, t2, w.phi, st, 1.0, vs);
            if (e == hipSuccess)
                e = stage(m, lim, S, dt, kRk3A[2], kRk3B[2], MODE_RK, t2, tn, u, next, w.phi, st, 1.0, vs);
        }
    }
    return e == hipSuccess ? FL_OK : hip_fail(e, "fl_rk_steps_store launch");
}

fl_status fl_rk_step_adjoint(const fl_mesh *m, int lim, int scheme, double dt, int S,
                             const double *stages, const double *u, double *lambda,
                             double *u_bar, void *work, void *stream) {
    fl_status s = check_adjoint(m, lim, S);
    if (s != FL_OK) return s;
    if (scheme != FL_EULER && scheme != FL_SSPRK3) return fail(FL_E_INVALID, "unknown scheme");
    if (!stages || !u || !lambda || !work) return fail(FL_E_INVALID, "NULL device pointer");
    if (misaligned(stages) || misaligned(u) || misaligned(lambda) || misaligned(u_bar) ||
        ((uintptr_t)work & 255u))
        return fail(FL_E_INVALID, "pointers must be 8-byte and work 256-byte aligned");
    DeviceGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t cell = (size_t)m->h.nc * S;
    s = finite_inputs(m, {{stages, (int64_t)cell * (scheme == FL_EULER ? 1 : 3)}, {u, m->h.nf},
                          {lambda, (int64_t)cell}}, dt, st);
    if (s != FL_OK) return s;
    const size_t slab = align256(cell * sizeof(double));
    double *w1 = (double *)work;
    double *w2 = (double *)((char *)work + slab);
    double *w3 = (double *)((char *)work + 2 * slab);
    double *term = (double *)((char *)work + (scheme == FL_EULER ? 1 : 3) * slab);  // general
    auto adj = [&](const double *th, const double *lam, double a, double b, int mode,
                   double *out, double *acc) {
        return general_adjoint(m)
                   ? launch_adjoint_general(m, lim, S, u, th, lam, a, b, dt, mode, out, acc,
                                            u_bar, term, st)
                   : launch_adjoint(m, lim, S, u, th, lam, a, b, dt, mode, out, acc, u_bar, st);
    };
    hipError_t e;
    // Each reverse stage gathers its input cotangent, so it writes a different buffer.
    if (scheme == FL_EULER) {
        e = adj(stages, lambda, 0.0, 1.0, ADJ_EULER, w1, nullptr);
        if (e == hipSuccess)
            e = hipMemcpyAsync(lambda, w1, cell * sizeof(double), hipMemcpyDeviceToDevice, st);
    } else {
        // lambda -> w1 (stage 3), w1 -> w3 (stage 2), w3 -> lambda (stage 1); w2 accumulates
        // the theta^n cotangent
        e = adj(stages + 2 * cell, lambda, kRk3A[2], kRk3B[2], ADJ_LAST, w1, w2);
        if (e == hipSuccess) e = adj(stages + cell, w1, kRk3A[1], kRk3B[1], ADJ_MID, w3, w2);
        if (e == hipSuccess) e = adj(stages, w3, kRk3A[0], kRk3B[0], ADJ_FIRST, lambda, w2);
    }
    return e == hipSuccess ? FL_OK : hip_fail(e, "fl_rk_step_adjoint launch");
}

// ------------------------------------------------------------------------------------------
// Multi-step reverse sweep
// ------------------------------------------------------------------------------------------
static fl_status check_steps_adjoint(const fl_mesh *m, int lim, int S) {
    fl_status s = check_adjoint(m, lim, S);
    if (s != FL_OK) return s;
    if (m->path != FL_PATH_FUSED || !m->h.forward_slots || !m->d_adj_fr)
        return fail(FL_E_UNSUPPORTED,
                    "the multi-step reverse sweep needs a fused-path mesh with forward face slots");
    return FL_OK;
}

size_t fl_adjoint_uacc_bytes(const fl_mesh *m) {
    if (!m || m->path != FL_PATH_FUSED || !m->h.forward_slots) return 0;
    return (size_t)m->h.pairs * m->h.nc * sizeof(double);
}

// On meshes with aligned slots the reverse stages read one rate per face (the forward rates);
// otherwise two per-slot planes.
bool adjoint_fwd_rates(const fl_mesh *m) { return m->h.aligned_slots && g_fwd_rates; }

size_t fl_adjoint_rates_bytes(const fl_mesh *m) {
    if (!m || m->path != FL_PATH_FUSED) return 0;
    return (size_t)2 * m->h.pairs * m->h.nc * kAdjRateBytes;
}

fl_status fl_adjoint_rates(const fl_mesh *m, const double *u, void *rates, void *stream) {
    fl_status s = check_steps_adjoint(m, 0, 1);
    if (s != FL_OK) return s;
    if (!u || !rates) return fail(FL_E_INVALID, "NULL device pointer");
    if (misaligned(u) || ((uintptr_t)rates & 15u))
        return fail(FL_E_INVALID, "u must be 8-byte and rates 16-byte aligned");
    DeviceGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    s = finite_inputs(m, {{u, m->h.nf}}, 0.0, st);
    if (s != FL_OK) return s;
    // the form follows the mesh and FL_OPT_FWD_RATES (a table written under one setting of the
    // option is read under the same setting)
    const bool fwd = adjoint_fwd_rates(m);
    hipError_t e = fwd ? launch_adjoint_fwd_rates(m, u, static_cast<double *>(rates), st)
                       : launch_adjoint_rates(m, u, rates, st);
    return e == hipSuccess ? FL_OK : hip_fail(e, "fl_adjoint_rates launch");
}

size_t fl_rk_steps_adjoint_workspace_bytes(const fl_mesh *m, int scheme, int S) {
    if (!m || S < 1 || S > FL_MAX_SCALARS || (scheme != FL_EULER && scheme != FL_SSPRK3) ||
        m->path != FL_PATH_FUSED)
        return 0;
    return 2 * align256((size_t)m->h.nc * S * sizeof(double));
}

fl_status fl_rk_steps_adjoint(const fl_mesh *m, int lim, int scheme, double dt, int S,
                              int64_t n_steps, const double *stages, const void *rates,
                              double *lambda, double *u_acc, void *work, void *stream) {
    fl_status s = check_steps_adjoint(m, lim, S);
    if (s != FL_OK) return s;
    if (scheme != FL_EULER && scheme != FL_SSPRK3) return fail(FL_E_INVALID, "unknown scheme");
    if (n_steps < 0) return fail(FL_E_INVALID, "n_steps must be >= 0");
    if ((n_steps > 0 && !stages) || !rates || !lambda || !work)
        return fail(FL_E_INVALID, "NULL device pointer");
    if (misaligned(stages) || ((uintptr_t)rates & 15u) || misaligned(lambda) ||
        misaligned(u_acc) || ((uintptr_t)work & 255u))
        return fail(FL_E_INVALID,
                    "stages/lambda/u_acc must be 8-byte, rates 16-byte and work 256-byte aligned");
    if (n_steps == 0) return FL_OK;
    DeviceGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t cell = (size_t)m->h.nc * S;
    const int ns = scheme == FL_EULER ? 1 : 3;
    s = finite_inputs(m, {{stages, (int64_t)(cell * ns * n_steps)}, {lambda, (int64_t)cell}}, dt,
                      st);
    if (s != FL_OK) return s;
    const void *wr = rates;
    const bool fwd = adjoint_fwd_rates(m);
    auto rstage = [&](const double *th, const double *lm, double a, double b, double a3, int mode,
                      const double *lin, const double *l3, double *out) {
        return fwd ? launch_adjoint_fwd_stage(m, lim, S, static_cast<const double *>(wr), th, lm,
                                              a, b, a3, dt, mode, lin, l3, out, u_acc, st)
                   : launch_adjoint_rate_stage(m, lim, S, wr, th, lm, a, b, a3, dt, mode, lin, l3,
                                               out, u_acc, st);
    };
    double *w1 = (double *)work;
    double *w3 = (double *)((char *)work + align256(cell * sizeof(double)));
    hipError_t e = hipSuccess;
    double *lam = lambda;  // holds the current step's input cotangent
    for (int64_t i = n_steps - 1; i >= 0 && e == hipSuccess; --i) {
        const double *tn = stages + (size_t)i * ns * cell;
        if (scheme == FL_EULER) {
            double *dst = (lam == lambda) ? w1 : lambda;
            e = rstage(tn, lam, 0.0, 1.0, 0.0, ADJ_EULER, nullptr, nullptr, dst);
            lam = dst;
        } else {
            // stage 3 (theta2): lam -> w1; stage 2 (theta1): w1 -> w3; stage 1 (theta^n):
            // w3 -> lam, completed with the theta^n terms of stages 3 and 2
            e = rstage(tn + 2 * cell, lam, kRk3A[2], kRk3B[2], 0.0, ADJ_LAST, nullptr, nullptr, w1);
            if (e == hipSuccess)
                e = rstage(tn + cell, w1, kRk3A[1], kRk3B[1], 0.0, ADJ_MID, nullptr, nullptr, w3);
            if (e == hipSuccess)
                e = rstage(tn, w3, kRk3A[1], kRk3B[0], kRk3A[2], ADJ_FIRST, lam, w1, lam);
        }
    }
    if (e == hipSuccess && lam != lambda)
        e = hipMemcpyAsync(lambda, lam, cell * sizeof(double), hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? FL_OK : hip_fail(e, "fl_rk_steps_adjoint launch");
}

fl_status fl_adjoint_uacc_scatter(const fl_mesh *m, const double *u_acc, double *u_bar,
                                  void *stream) {
    fl_status s = check_steps_adjoint(m, 0, 1);
    if (s != FL_OK) return s;
    if (!u_acc || !u_bar) return fail(FL_E_INVALID, "NULL device pointer");
    if (misaligned(u_acc) || misaligned(u_bar))
        return fail(FL_E_INVALID, "device pointers must be 8-byte aligned");
    DeviceGuard g(m->device);
    hipError_t e = launch_adjoint_uacc_scatter(m, u_acc, u_bar, (hipStream_t)stream);
    return e == hipSuccess ? FL_OK : hip_fail(e, "fl_adjoint_uacc_scatter launch");
}

fl_status fl_debug_select(const fl_mesh *m, const double *u, int32_t *cdu, void *stream) {
    fl_status s = check_compute(m, 0, 1);
    if (s != FL_OK) return s;
    if (!u || !cdu) return fail(FL_E_INVALID, "NULL pointer");
    DeviceGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    int32_t *d = nullptr;
    hipError_t e = hipMalloc((void **)&d, m->h.nf * 3 * sizeof(int32_t));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    e = launch_select(m, u, d, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(cdu, d, m->h.nf * 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    return e == hipSuccess ? FL_OK : hip_fail(e, "fl_debug_select");
}

}  // extern "C"
