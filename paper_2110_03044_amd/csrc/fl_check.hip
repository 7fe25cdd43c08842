// Opt-in check that the floating-point inputs of a call are finite (FL_OPT_CHECK_FINITE).
//
// With the option on, the compute entry points scan their device inputs before enqueuing any
// work and return FL_E_NONFINITE if a NaN or an infinity is found.  The scan synchronises the
// caller's stream (its answer decides the return status), so a call with the check on cannot be
// captured into a graph; with the option off (the default) nothing here runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "fl_internal.h"
#include "fl_kernels.h"

namespace fl {
namespace {

// One flag per device: set to 1 by any lane that sees a non-finite value.
__device__ __align__(256) unsigned int g_nonfinite_flag;

__global__ __launch_bounds__(256) void clear_flag_kernel(unsigned int *flag) {
    if (threadIdx.x == 0) *flag = 0u;
}

__global__ __launch_bounds__(256) void nonfinite_kernel(const double *__restrict__ a, int64_t n,
                                                        unsigned int *flag) {
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(a[i]);
    if (bad) atomicOr(flag, 1u);
}

std::mutex g_mu;                 // the flag is shared by all calls on a device
std::vector<unsigned int *> g_flag;  // device address of the flag, per device
int g_check_finite = 0;

}  // namespace

void set_check_finite(int on) { g_check_finite = on; }
bool check_finite_enabled() { return g_check_finite != 0; }

fl_status check_finite(int device, const FiniteSpan *spans, int n_spans, hipStream_t st) {
    std::lock_guard<std::mutex> lock(g_mu);
    if ((int)g_flag.size() <= device) g_flag.resize(device + 1, nullptr);
    if (!g_flag[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_nonfinite_flag));
        if (e != hipSuccess) return fail(FL_E_HIP, "hipGetSymbolAddress of the finite-check flag");
        g_flag[device] = static_cast<unsigned int *>(p);
    }
    unsigned int *flag = g_flag[device];
    clear_flag_kernel<<<1, 64, 0, st>>>(flag);
    for (int i = 0; i < n_spans; ++i) {
        if (!spans[i].p || spans[i].n <= 0) continue;
        const int64_t blocks = std::min<int64_t>((spans[i].n + 255) / 256, 4096);
        nonfinite_kernel<<<(unsigned)blocks, 256, 0, st>>>(spans[i].p, spans[i].n, flag);
    }
    unsigned int h = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(FL_E_HIP, std::string("finite check: ") + hipGetErrorString(e));
    return h ? fail(FL_E_NONFINITE, "an input holds a NaN or an infinity") : FL_OK;
}

}  // namespace fl
