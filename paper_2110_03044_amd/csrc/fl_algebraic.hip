// Kernels of the algebraic form of the operator (Algorithms 3 and 4): ELLPACK sparse
// matrix-vector products and the pointwise "kbin" kernels, for gfx950, FP64.
//
// This is the paper's own implementation strategy, kept to compare with the fused stage kernel:
// every step is a separate memory pass with unit-stride access except the SpMV input vector.
#include <hip/hip_runtime.h>

#include "fl_algebraic.h"
#include "fl_device.h"

namespace fl {
namespace alg {

constexpr int kBlock = 256;

// One thread per row; W > 0 unrolls a known width, W == 0 loops over `width`.  The row's
// products are summed in column-slot order, then added to y when accumulating.
template <int W>
__global__ __launch_bounds__(kBlock) void ell_spmv_kernel(int64_t rows, int width,
                                                          const double *__restrict__ val,
                                                          const int32_t *__restrict__ col,
                                                          const double *__restrict__ x, double *y,
                                                          int accumulate) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= rows) return;
    double s = 0.0;
    if constexpr (W > 0) {
#pragma unroll
        for (int k = 0; k < W; ++k) s += val[(int64_t)k * rows + i] * x[col[(int64_t)k * rows + i]];
    } else {
        for (int k = 0; k < width; ++k) s += val[(int64_t)k * rows + i] * x[col[(int64_t)k * rows + i]];
    }
    y[i] = accumulate ? y[i] + s : s;
}

// Called in place (out == y, or out == y with x another vector): every thread reads its
// elements before writing its own, so the pointers may alias (no __restrict__).
template <int OP>
__global__ __launch_bounds__(kBlock) void kbin_kernel(int64_t n, int lim, const double *x,
                                                      const double *y, double *out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if constexpr (OP == KBIN_SIGNXTY) {
        out[i] = y[i] * (x[i] > 0.0 ? 1.0 : -1.0);  // x = u_f (Table 1 signxty)
    } else if constexpr (OP == KBIN_AXDY) {
        const double d = x[i];
        out[i] = d == 0.0 ? 0.0 : y[i] / d;
    } else if constexpr (OP == KBIN_LIMXTY) {
        const double d = y[i];
        out[i] = d == 0.0 ? 0.0 : d * (0.5 * (dev::psi(lim, x[i]) - 1.0));
    } else {
        out[i] = x[i] * y[i];
    }
}

// out may alias ts and tn (forward Euler in place).
__global__ __launch_bounds__(kBlock) void combine_kernel(int64_t n, const double *ts,
                                                         const double *tn, const double *rhs,
                                                         double a, double b, double dt, int mode,
                                                         double *out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (mode == MODE_EULER) out[i] = ts[i] + dt * rhs[i];
    else out[i] = a * tn[i] + b * (ts[i] + dt * rhs[i]);
}

unsigned blocks(int64_t n) {
    const int64_t nb = (n + kBlock - 1) / kBlock;
    return (unsigned)(nb < 1 ? 1 : nb);
}

}  // namespace alg

hipError_t launch_ell_spmv(const Ell &A, const double *x, double *y, int accumulate,
                           hipStream_t st) {
    const unsigned nb = alg::blocks(A.rows);
    switch (A.width) {
#define FL_ELL(W)                                                                             \
    case W:                                                                                   \
        alg::ell_spmv_kernel<W><<<nb, alg::kBlock, 0, st>>>(A.rows, W, A.d_val, A.d_col, x, y, \
                                                             accumulate);                     \
        break;
        FL_ELL(2)
        FL_ELL(4)
        FL_ELL(6)
        FL_ELL(8)
        FL_ELL(12)
#undef FL_ELL
        default:
            alg::ell_spmv_kernel<0><<<nb, alg::kBlock, 0, st>>>(A.rows, A.width, A.d_val, A.d_col,
                                                                 x, y, accumulate);
    }
    return hipGetLastError();
}

hipError_t launch_kbin(int op, int lim, int64_t n, const double *x, const double *y, double *out,
                       hipStream_t st) {
    const unsigned nb = alg::blocks(n);
    switch (op) {
        case KBIN_SIGNXTY: alg::kbin_kernel<KBIN_SIGNXTY><<<nb, alg::kBlock, 0, st>>>(n, lim, x, y, out); break;
        case KBIN_AXDY: alg::kbin_kernel<KBIN_AXDY><<<nb, alg::kBlock, 0, st>>>(n, lim, x, y, out); break;
        case KBIN_LIMXTY: alg::kbin_kernel<KBIN_LIMXTY><<<nb, alg::kBlock, 0, st>>>(n, lim, x, y, out); break;
        case KBIN_UXTY: alg::kbin_kernel<KBIN_UXTY><<<nb, alg::kBlock, 0, st>>>(n, lim, x, y, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_combine(int64_t n, const double *ts, const double *tn, const double *rhs,
                          double a, double b, double dt, int mode, double *out, hipStream_t st) {
    alg::combine_kernel<<<alg::blocks(n), alg::kBlock, 0, st>>>(n, ts, tn, rhs, a, b, dt, mode,
                                                                 out);
    return hipGetLastError();
}

}  // namespace fl
