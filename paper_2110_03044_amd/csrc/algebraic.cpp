// Algebraic form of the operator (Algorithms 3 and 4): builds the paper's sparse matrices from a
// mesh's tables and runs the SpMV + pointwise-kernel chain.  Host C++; kernels in
// fl_algebraic.hip.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <sstream>

#include "fl_algebraic.h"
#include "fl_kernels.h"

namespace fl {
namespace {

fl_status alg_hip_fail(hipError_t e, const char *what) {
    std::ostringstream os;
    os << what << ": " << hipGetErrorString(e);
    return fail(e == hipErrorOutOfMemory ? FL_E_NOMEM : FL_E_HIP, os.str());
}

// Small per-row accumulator of (column, coefficient) pairs in first-seen order.
struct Row {
    std::vector<int32_t> col;
    std::vector<double> val;
    void add(int32_t c, double v) {
        for (size_t i = 0; i < col.size(); ++i)
            if (col[i] == c) {
                val[i] += v;
                return;
            }
        col.push_back(c);
        val.push_back(v);
    }
    void clear() {
        col.clear();
        val.clear();
    }
};

// Fills an ELLPACK matrix row by row: storage for `cap` entries per row, trimmed at the end to
// the widest row (the planes are column-major, so trimming drops trailing planes).  Short rows
// are padded with zero coefficients on their first column.
struct EllFill {
    Ell &A;
    int32_t cap;
    EllFill(Ell &m, int64_t rows, int32_t cap_) : A(m), cap(cap_) {
        A.rows = rows;
        A.width = 0;
        A.val.assign((size_t)cap * rows, 0.0);
        A.col.assign((size_t)cap * rows, 0);
    }
    void set(int64_t i, const Row &r) {
        const int32_t n = (int32_t)r.col.size();
        A.width = std::max(A.width, n);
        for (int32_t k = 0; k < cap; ++k) {
            A.col[(size_t)k * A.rows + i] = k < n ? r.col[k] : (n ? r.col[0] : 0);
            A.val[(size_t)k * A.rows + i] = k < n ? r.val[k] : 0.0;
        }
    }
    void finish() {
        A.val.resize((size_t)A.width * A.rows);
        A.col.resize((size_t)A.width * A.rows);
        A.val.shrink_to_fit();
        A.col.shrink_to_fit();
    }
};

// The matrices of Section 2 / Section 3 for face f with own a and nbr b (unit normal a -> b):
//   E[f][a] = -1, E[f][b] = +1 (oriented incidence), B = |E|, W = diag(B 1) = 2 on interior faces;
//   A_FF[f][j] = (B B^T - W)[f][j] = 1 for the faces j != f sharing a cell with f;
//   A^D_FF[f][j] = E[f][shared cell of f and j] (-1 behind the face, +1 ahead);
//   T[f][:] = (1/2) sum_j (n_f . n_j) A_FF[f][j] E[j][:], S likewise with A^D_FF;
//   UUD = T, OUD = -S, Pi[f][a] = Pi[f][b] = 1/2, M[c][f] = E[f][c] a_f / V_c.
// A row of T or S holds a, b and the far cell of every face adjacent to f: at most
// deg(a) + deg(b) columns (2k on a k-regular mesh).
void build(const HostTables &h, Ell m[5]) {
    const int64_t nf = h.nf, nc = h.nc;
    const int32_t *fc = h.fc.data();
    const double *nrm = h.nrm.data();
    const int32_t kmax = std::max<int32_t>(h.max_degree, 1);
    EllFill D(m[FL_ALG_D], nf, 2), T(m[FL_ALG_UUD], nf, 2 * kmax), O(m[FL_ALG_OUD], nf, 2 * kmax),
        P(m[FL_ALG_PI], nf, 2);
    Row d, t, o, pi;
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t a = fc[2 * f], b = fc[2 * f + 1];
        d.clear();
        pi.clear();
        t.clear();
        o.clear();
        d.add(a, -1.0);
        d.add(b, 1.0);
        pi.add(a, 0.5);
        pi.add(b, 0.5);
        t.add(a, 0.0);
        t.add(b, 0.0);
        o.add(a, 0.0);
        o.add(b, 0.0);
        for (int side = 0; side < 2; ++side) {
            const int32_t cell = side == 0 ? a : b;
            const double sigma = side == 0 ? -1.0 : 1.0;  // A^D: shared cell a (behind) or b
            for (int64_t p = h.cf_ptr[cell]; p < h.cf_ptr[cell + 1]; ++p) {
                const int32_t e = h.cf_idx[p];
                const int32_t j = e >= 0 ? e : ~e;
                if (j == f) continue;
                const double nn = nrm[3 * f] * nrm[3 * j] + nrm[3 * f + 1] * nrm[3 * j + 1] +
                                  nrm[3 * f + 2] * nrm[3 * j + 2];
                const double c = 0.5 * nn;
                const int32_t oj = fc[2 * j], bj = fc[2 * j + 1];
                // T += c E[j]; OUD = -S -= sigma c E[j]
                t.add(oj, -c);
                t.add(bj, c);
                o.add(oj, sigma * c);
                o.add(bj, -sigma * c);
            }
        }
        D.set(f, d);
        P.set(f, pi);
        T.set(f, t);
        O.set(f, o);
    }
    D.finish();
    P.finish();
    T.finish();
    O.finish();
    EllFill M(m[FL_ALG_M], nc, kmax);
    Row r;
    for (int64_t c = 0; c < nc; ++c) {
        r.clear();
        const double V = h.vol.empty() ? h.vol0 : h.vol[c];
        for (int64_t p = h.cf_ptr[c]; p < h.cf_ptr[c + 1]; ++p) {
            const int32_t e = h.cf_idx[p];
            const int32_t f = e >= 0 ? e : ~e;
            const double af = h.area.empty() ? h.area0 : h.area[f];
            r.add(f, (e >= 0 ? 1.0 : -1.0) * af / V);
        }
        M.set(c, r);
    }
    M.finish();
}

template <class T>
fl_status to_device(const std::vector<T> &src, T **dst, int64_t &bytes) {
    *dst = nullptr;
    if (src.empty()) return FL_OK;
    hipError_t e = hipMalloc((void **)dst, src.size() * sizeof(T));
    if (e != hipSuccess) {
        *dst = nullptr;
        return alg_hip_fail(e, "hipMalloc of an ELLPACK array");
    }
    bytes += (int64_t)(src.size() * sizeof(T));
    e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    return e == hipSuccess ? FL_OK : alg_hip_fail(e, "copy of an ELLPACK array");
}

void release(fl_algebraic *g) {
    for (Ell &A : g->m) {
        if (A.d_val) (void)hipFree(A.d_val);
        if (A.d_col) (void)hipFree(A.d_col);
        A.d_val = nullptr;
        A.d_col = nullptr;
    }
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct AlgWork {
    double *d = nullptr, *r = nullptr, *tf = nullptr, *rhs = nullptr, *t1 = nullptr,
           *t2 = nullptr;
};

AlgWork carve(const fl_algebraic *g, void *work) {
    const size_t F = a256((size_t)g->mesh->h.nf * sizeof(double));
    const size_t C = a256((size_t)g->mesh->h.nc * sizeof(double));
    char *p = (char *)work;
    AlgWork w;
    w.d = (double *)p;
    w.r = (double *)(p + F);
    w.tf = (double *)(p + 2 * F);
    w.rhs = (double *)(p + 3 * F);
    w.t1 = (double *)(p + 3 * F + C);
    w.t2 = (double *)(p + 3 * F + 2 * C);
    return w;
}

// theta_f = Pi theta + F(r) o d_u (Section 3.1): the face interpolation of Section 2's shift
// plus the limited correction along the flow, from the two velocity-oriented differences
//   d_U = (Q UUD + OUD) theta   (the simplified upstream-difference equation; w.r)
//   d_u = Q D theta             (the face-difference equation; w.d)
// and r = d_U / d_u (the gradient-ratio equation), each product by the diagonal Q or by a
// pointwise function one kbin launch.  Every term is one sparse product or one pointwise pass
// over a face vector, so the chain is the eight launches of Algorithm 3 in the order its data
// dependencies allow.
hipError_t face_values(const fl_algebraic *g, int lim, const double *th, const double *u,
                       const AlgWork &w, double *tf, hipStream_t st) {
    const int64_t nf = g->mesh->h.nf;
    auto spmv = [&](int which, double *out, int accumulate) {
        return launch_ell_spmv(g->m[which], th, out, accumulate, st);
    };
    auto kbin = [&](int op, const double *x, const double *y, double *out) {
        return launch_kbin(op, lim, nf, x, y, out, st);
    };
    hipError_t e = spmv(FL_ALG_UUD, w.r, 0);
    if (e == hipSuccess) e = kbin(KBIN_SIGNXTY, u, w.r, w.r);
    if (e == hipSuccess) e = spmv(FL_ALG_OUD, w.r, 1);
    if (e == hipSuccess) e = spmv(FL_ALG_D, w.d, 0);
    if (e == hipSuccess) e = kbin(KBIN_SIGNXTY, u, w.d, w.d);
    if (e == hipSuccess) e = kbin(KBIN_AXDY, w.d, w.r, w.r);
    if (e == hipSuccess) e = kbin(KBIN_LIMXTY, w.r, w.d, tf);
    if (e == hipSuccess) e = spmv(FL_ALG_PI, tf, 1);
    return e;
}

// rhs = M U(u) theta_f(ts), then the stage combination into out.
hipError_t stage(const fl_algebraic *g, int lim, const double *ts, const double *tn,
                 const double *u, double a, double b, double dt, int mode, double *out,
                 const AlgWork &w, hipStream_t st) {
    hipError_t e = face_values(g, lim, ts, u, w, w.tf, st);
    if (e == hipSuccess) e = launch_kbin(KBIN_UXTY, lim, g->mesh->h.nf, u, w.tf, w.r, st);
    if (e == hipSuccess) e = launch_ell_spmv(g->m[FL_ALG_M], w.r, w.rhs, 0, st);
    if (e == hipSuccess) e = launch_combine(g->mesh->h.nc, ts, tn, w.rhs, a, b, dt, mode, out, st);
    return e;
}

constexpr double kA[3] = {0.0, 0.75, 1.0 / 3.0};
constexpr double kB[3] = {1.0, 0.25, 2.0 / 3.0};

struct Guard {
    int prev = -1;
    bool changed = false;
    explicit Guard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = hipSetDevice(dev) == hipSuccess;
    }
    ~Guard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

fl_status check_run(const fl_algebraic *g, int lim, const void *a, const void *b, const void *work) {
    if (!g) return fail(FL_E_INVALID, "NULL algebraic object");
    if (g->device < 0) return fail(FL_E_NODEVICE, "the algebraic object is host-only");
    if (lim < FL_UPWIND || lim > FL_CENTRAL) return fail(FL_E_INVALID, "unknown limiter");
    if (!a || !b || !work) return fail(FL_E_INVALID, "NULL device pointer");
    if (((uintptr_t)a & 7u) || ((uintptr_t)b & 7u) || ((uintptr_t)work & 255u))
        return fail(FL_E_INVALID, "vectors must be 8-byte and work 256-byte aligned");
    return FL_OK;
}

}  // namespace
}  // namespace fl

using namespace fl;

extern "C" {

fl_status fl_algebraic_create(const fl_mesh *mesh, fl_algebraic **out) {
    if (!out) return fail(FL_E_INVALID, "NULL output pointer");
    *out = nullptr;
    if (!mesh) return fail(FL_E_INVALID, "NULL mesh");
    if (mesh->h.n_boundary > 0 || mesh->h.dist_weighted)
        return fail(FL_E_UNSUPPORTED,
                    "the algebraic chain covers closed meshes without face distances");
    fl_algebraic *g = new (std::nothrow) fl_algebraic();
    if (!g) return fail(FL_E_NOMEM, "host allocation failed");
    g->mesh = mesh;
    g->device = mesh->device;
    try {
        build(mesh->h, g->m);
    } catch (const std::bad_alloc &) {
        delete g;
        return fail(FL_E_NOMEM, "host allocation of the matrices failed");
    }
    if (g->device >= 0) {
        Guard gd(g->device);
        for (Ell &A : g->m) {
            fl_status st = to_device(A.val, &A.d_val, g->device_bytes);
            if (st == FL_OK) st = to_device(A.col, &A.d_col, g->device_bytes);
            if (st != FL_OK) {
                release(g);
                delete g;
                return st;
            }
        }
    }
    *out = g;
    return FL_OK;
}

fl_status fl_algebraic_destroy(fl_algebraic *g) {
    if (!g) return FL_OK;
    if (g->device >= 0) {
        Guard gd(g->device);
        release(g);
    }
    delete g;
    return FL_OK;
}

fl_status fl_algebraic_info(const fl_algebraic *g, fl_algebraic_info_t *info) {
    if (!g || !info) return fail(FL_E_INVALID, "NULL argument");
    for (int i = 0; i < 5; ++i) {
        info->rows[i] = g->m[i].rows;
        info->width[i] = g->m[i].width;
    }
    info->device_bytes = g->device_bytes;
    return FL_OK;
}

fl_status fl_algebraic_export(const fl_algebraic *g, int which, double *val, int32_t *col) {
    if (!g) return fail(FL_E_INVALID, "NULL algebraic object");
    if (which < 0 || which > 4) return fail(FL_E_INVALID, "unknown matrix");
    const Ell &A = g->m[which];
    if (val && !A.val.empty()) std::memcpy(val, A.val.data(), A.val.size() * sizeof(double));
    if (col && !A.col.empty()) std::memcpy(col, A.col.data(), A.col.size() * sizeof(int32_t));
    return FL_OK;
}

size_t fl_algebraic_workspace_bytes(const fl_algebraic *g) {
    if (!g) return 0;
    return 3 * a256((size_t)g->mesh->h.nf * sizeof(double)) +
           3 * a256((size_t)g->mesh->h.nc * sizeof(double));
}

fl_status fl_algebraic_face_values(const fl_algebraic *g, int lim, const double *theta,
                                   const double *u, double *theta_f, void *work, void *stream) {
    fl_status s = check_run(g, lim, theta, u, work);
    if (s != FL_OK) return s;
    if (!theta_f || ((uintptr_t)theta_f & 7u)) return fail(FL_E_INVALID, "bad theta_f pointer");
    Guard gd(g->device);
    AlgWork w = carve(g, work);
    hipError_t e = face_values(g, lim, theta, u, w, theta_f, (hipStream_t)stream);
    return e == hipSuccess ? FL_OK : alg_hip_fail(e, "fl_algebraic_face_values launch");
}

fl_status fl_algebraic_rk_steps(const fl_algebraic *g, int lim, int scheme, double dt,
                                int64_t n_steps, double *theta, const double *u, void *work,
                                void *stream) {
    fl_status s = check_run(g, lim, theta, u, work);
    if (s != FL_OK) return s;
    if (scheme != FL_EULER && scheme != FL_SSPRK3) return fail(FL_E_INVALID, "unknown scheme");
    if (n_steps < 0) return fail(FL_E_INVALID, "n_steps must be >= 0");
    Guard gd(g->device);
    hipStream_t st = (hipStream_t)stream;
    AlgWork w = carve(g, work);
    hipError_t e = hipSuccess;
    for (int64_t i = 0; i < n_steps && e == hipSuccess; ++i) {
        if (scheme == FL_EULER) {
            // theta_f is formed before the combination overwrites theta, so in place is safe
            e = stage(g, lim, theta, theta, u, 0.0, 1.0, dt, MODE_EULER, theta, w, st);
        } else {
            e = stage(g, lim, theta, theta, u, kA[0], kB[0], dt, MODE_EULER, w.t1, w, st);
            if (e == hipSuccess) e = stage(g, lim, w.t1, theta, u, kA[1], kB[1], dt, MODE_RK, w.t2, w, st);
            if (e == hipSuccess) e = stage(g, lim, w.t2, theta, u, kA[2], kB[2], dt, MODE_RK, theta, w, st);
        }
    }
    return e == hipSuccess ? FL_OK : alg_hip_fail(e, "fl_algebraic_rk_steps launch");
}

}  // extern "C"
