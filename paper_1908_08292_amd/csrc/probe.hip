// probe.hip -- measured ceilings of this chip, next to which the roofline
// fractions of the solver are read: dense FP64 and FP32 MFMA issue rates and
// the HBM copy bandwidth (include/rve.h: rve_probe_peaks).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/rve.h"

int rve_internal_set_error(int code, const std::string& msg);  // rve_abi.cpp

namespace {

typedef double pd4 __attribute__((ext_vector_type(4)));
typedef float pf4 __attribute__((ext_vector_type(4)));

constexpr int kAcc = 8;  // independent accumulators per wave (hides the MFMA latency)

// every wave issues iters * kAcc independent 16x16x4 MFMAs (2048 flop each)
__global__ __launch_bounds__(256) void probe_mfma_f64(int iters, double seed, double* out) {
    pd4 acc[kAcc];
#pragma unroll
    for (int k = 0; k < kAcc; ++k) acc[k] = pd4{seed * k, 0.0, 0.0, 0.0};
    const double a = seed + 1e-9 * threadIdx.x, b = seed - 1e-9 * threadIdx.x;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < kAcc; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kAcc; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void probe_mfma_f32(int iters, float seed, double* out) {
    pf4 acc[kAcc];
#pragma unroll
    for (int k = 0; k < kAcc; ++k) acc[k] = pf4{seed * k, 0.f, 0.f, 0.f};
    const float a = seed + 1e-6f * threadIdx.x, b = seed - 1e-6f * threadIdx.x;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < kAcc; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kAcc; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// plain copy, 16 bytes per thread and step, grid-stride
__global__ __launch_bounds__(256) void probe_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                                  size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

#define PR_HIP(expr)                                                                                        \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess) {                                                                             \
            err = rve_internal_set_error(RVE_EHIP, std::string("rve_probe_peaks: ") + #expr + ": " +        \
                                                       hipGetErrorString(e_));                              \
            goto done;                                                                                      \
        }                                                                                                   \
    } while (0)

extern "C" int rve_probe_peaks(double* fp64_mfma_tflops, double* fp32_mfma_tflops, double* hbm_copy_gbs,
                               void* hip_stream) {
    if (!fp64_mfma_tflops || !fp32_mfma_tflops || !hbm_copy_gbs)
        return rve_internal_set_error(RVE_EINVAL, "rve_probe_peaks: NULL output");
    hipStream_t s = (hipStream_t)hip_stream;
    int err = RVE_OK;
    int dev = 0, ncu = 0;
    const int iters = 4000, per_cu = 8;
    size_t n2 = 0;
    int grid = 0;
    double* out = nullptr;
    double2 *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float best[3] = {1e30f, 1e30f, 1e30f};
    PR_HIP(hipGetDevice(&dev));
    PR_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    grid = ncu * per_cu;
    n2 = (size_t)1 << 26;  // 64 Mi double2 = 1 GiB per buffer
    PR_HIP(hipMalloc((void**)&out, sizeof(double) * (size_t)grid * 256));
    PR_HIP(hipMalloc((void**)&a, sizeof(double2) * n2));
    PR_HIP(hipMalloc((void**)&b, sizeof(double2) * n2));
    PR_HIP(hipMemsetAsync(a, 0, sizeof(double2) * n2, s));
    PR_HIP(hipEventCreate(&e0));
    PR_HIP(hipEventCreate(&e1));
    for (int rep = 0; rep < 4; ++rep) {  // the first repetition warms up
        for (int which = 0; which < 3; ++which) {
            PR_HIP(hipEventRecord(e0, s));
            if (which == 0)
                hipLaunchKernelGGL(probe_mfma_f64, dim3(grid), dim3(256), 0, s, iters, 1.0 + rep, out);
            else if (which == 1)
                hipLaunchKernelGGL(probe_mfma_f32, dim3(grid), dim3(256), 0, s, iters, 1.0f + rep, out);
            else
                hipLaunchKernelGGL(probe_copy, dim3(ncu * 16), dim3(256), 0, s, a, b, n2);
            PR_HIP(hipGetLastError());
            PR_HIP(hipEventRecord(e1, s));
            PR_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            PR_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) best[which] = std::min(best[which], ms);
        }
    }
    {
        const double flop = (double)grid * 4 /* waves */ * iters * kAcc * 2048.0;
        *fp64_mfma_tflops = flop / (best[0] * 1e-3) / 1e12;
        *fp32_mfma_tflops = flop / (best[1] * 1e-3) / 1e12;
        *hbm_copy_gbs = 2.0 * sizeof(double2) * (double)n2 / (best[2] * 1e-3) / 1e9;
    }
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    (void)hipFree(a);
    (void)hipFree(b);
    return err;
}
