// fl_rk_steps_noalloc: fl_rk_steps with its workspace in a fixed device array instead of a
// caller-provided buffer, for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The workspace (stage buffers theta1 / theta2, the face fluxes of the face path, and the
// per-call slot rates or records of multi-step calls) lives in `scratch`, a file-scope device
// array of kNoAllocScratchBytes bytes.  Each GPU the library runs on holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in, not a device address, so its
// device address is looked up once per device (hipGetSymbolAddress, with that device current) on
// the first call there and kept; only that address is ever passed to kernels.
//
// Every call on a GPU shares that GPU's array: calls that may overlap on one GPU (different
// streams, different threads) race on it and must be serialised by the caller.  No part of the
// workspace needs to start at zero (every buffer is written before it is read in each call), so
// nothing is cleared and the contents left by the last call do not matter.
#include <hip/hip_runtime.h>

#include <mutex>
#include <sstream>
#include <vector>

#include "fl_internal.h"
#include "fl_kernels.h"

namespace {

__device__ __align__(256) unsigned char scratch[FL_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
std::vector<void *> g_scratch;  // device address of `scratch`, per device (null: not looked up)

// The device address of `scratch` on `device` (looked up with that device current).
fl_status scratch_on(int device, void **out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if ((int)g_scratch.size() <= device) g_scratch.resize(device + 1, nullptr);
    if (!g_scratch[device]) {
        int prev = -1;
        hipError_t e = hipGetDevice(&prev);
        if (e == hipSuccess && prev != device) e = hipSetDevice(device);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess || !p)
            return fl::fail(FL_E_HIP, std::string("hipGetSymbolAddress of the scratch array: ") +
                                          hipGetErrorString(e));
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return FL_OK;
}

}  // namespace

extern "C" {

fl_status fl_rk_steps_noalloc(const fl_mesh *m, int lim, int scheme, double dt, int S,
                              int64_t n_steps, double *theta, const double *u, void *stream) {
    if (!m) return fl::fail(FL_E_INVALID, "mesh is NULL");
    if (m->device < 0) return fl::fail(FL_E_NODEVICE, "the mesh was created host-only (device = -1)");
    const size_t need = fl_rk_workspace_bytes(m, scheme, S);
    if (need == 0) return fl::fail(FL_E_INVALID, "bad scheme or n_scalars");
    if (need > (size_t)FL_NOALLOC_SCRATCH_BYTES) {
        std::ostringstream os;
        os << "fl_rk_steps_noalloc: this mesh and scalar count need " << need
           << " bytes of workspace, more than the fixed " << (size_t)FL_NOALLOC_SCRATCH_BYTES
           << " bytes; use fl_rk_steps with a caller-provided workspace";
        return fl::fail(FL_E_INVALID, os.str());
    }
    void *work = nullptr;
    fl_status s = scratch_on(m->device, &work);
    if (s != FL_OK) return s;
    return fl_rk_steps(m, lim, scheme, dt, S, n_steps, theta, u, work, stream);
}

}  // extern "C"
