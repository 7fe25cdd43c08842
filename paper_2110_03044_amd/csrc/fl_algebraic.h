// Internal declarations of the algebraic (SpMV + pointwise kernel) form of the operator.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <vector>

#include "fl_internal.h"

namespace fl {

// ELLPACK matrix: every row stores `width` (coefficient, column) entries, column-major
// [width][rows] so that consecutive rows (threads) read consecutive addresses.
struct Ell {
    int64_t rows = 0;
    int32_t width = 0;
    std::vector<double> val;   // host copy
    std::vector<int32_t> col;
    double *d_val = nullptr;   // device copy (null for host-only objects)
    int32_t *d_col = nullptr;
};

// y = A x, or y = y + A x (accumulate).
hipError_t launch_ell_spmv(const Ell &A, const double *x, double *y, int accumulate,
                           hipStream_t st);

// Pointwise kernels (kbin) of Algorithms 3 and 4, one thread per element.
enum KbinOp {
    KBIN_SIGNXTY = 0,  // y = y * (u > 0 ? +1 : -1)
    KBIN_AXDY = 1,     // y = (d == 0) ? 0 : y / d          (x = d)
    KBIN_LIMXTY = 2,   // out = (d == 0) ? 0 : (psi(r) - 1) / 2 * d   (x = r, y = d)
    KBIN_UXTY = 3,     // out = u * y
};
hipError_t launch_kbin(int op, int lim, int64_t n, const double *x, const double *y, double *out,
                       hipStream_t st);
// out = a tn + b (ts + dt rhs) (mode MODE_RK) or ts + dt rhs (MODE_EULER), one thread per cell.
hipError_t launch_combine(int64_t n, const double *ts, const double *tn, const double *rhs,
                          double a, double b, double dt, int mode, double *out, hipStream_t st);

}  // namespace fl

struct fl_algebraic {
    const fl_mesh *mesh = nullptr;
    int device = -1;
    fl::Ell m[5];  // D, UUD, OUD, Pi, M
    int64_t device_bytes = 0;
};
