// rve_static.hip -- rve_solve_batch_static: the batched RVE solve with its
// workspace in a static device array, for callers that cannot allocate.
//
// The persistent solver needs device memory beyond its inputs and outputs: the
// queue counter of the persistent workgroups and one workspace slot per
// workgroup (Newton vectors, element matrices, factor panels, update matrices).
// rve_solve_batch uses the slots that rve_batch_create allocated; this entry
// point uses `scratch` below instead and calls no allocating routine.  Each
// device holds its own copy of the array from the first call on that device
// until the process ends.  The kernels are the same; only the number of
// persistent workgroups is limited to the slots that fit.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/rve.h"

int rve_internal_set_error(int code, const std::string& msg);  // rve_abi.cpp
int rve_internal_solve_ext(rve_batch b, const double* F, double* P, double* A, double* w_state, int32_t* status,
                           int32_t* iters, const rve_opts* opts, void* hip_stream, void* ext_ws, size_t ext_bytes,
                           int device);  // rve_abi.cpp

namespace {

constexpr size_t kScratchBytes = (size_t)RVE_STATIC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

// queue counter (first 256 bytes), then the workspace slots
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // device address of `scratch` per device

// the device address of this device's copy of `scratch`, looked up once per
// device with that device current (the array's name is only a host stand-in)
int scratch_ptr(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices)
        return rve_internal_set_error(RVE_EUNSUPPORTED, "rve_solve_batch_static: device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return rve_internal_set_error(RVE_EHIP, std::string("rve_solve_batch_static: hipGetSymbolAddress: ") +
                                                        hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return RVE_OK;
}

}  // namespace

extern "C" int rve_solve_batch_static(rve_batch b, const double* F, double* P, double* A, double* w_state,
                                      int32_t* status, int32_t* iters, const rve_opts* opts, void* hip_stream) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return rve_internal_set_error(RVE_EHIP, std::string("rve_solve_batch_static: hipGetDevice: ") +
                                                    hipGetErrorString(e));
    void* ptr = nullptr;
    int st = scratch_ptr(dev, &ptr);
    if (st) return st;
    return rve_internal_solve_ext(b, F, P, A, w_state, status, iters, opts, hip_stream, ptr, kScratchBytes, dev);
}
