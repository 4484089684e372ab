// Measured peaks of the device, for the rooflines the contraction is held to:
// the FP64 matrix-core rate (v_mfma_f64_16x16x4f64 chains held in registers),
// the FP64 vector FMA rate, and the rate of a streaming device copy.  The
// kernels touch no memory but their one output value per thread (the copy
// aside), so they time the units themselves.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int kMfmaPerTrip = 128;   // 4 independent chains x 32 steps
constexpr int kFmaChains = 8;

// Each wave runs 4 independent 16x16x4 FP64 MFMA chains: 2 * 16 * 16 * 4 =
// 2048 FLOP per instruction, 32 steps of each chain per loop trip (the
// compiler moves the accumulators out of the matrix-core registers and back
// once per trip: 64 moves per 128 MFMAs).  The chains start from different
// values so that none can be merged with another.
__global__ void __launch_bounds__(256) mfma_f64_loop_kernel(int trips, double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const double a = 1.0 + 1e-3 * lane, b = 1.0 - 1e-3 * lane;
    d4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {1e-3, 0.0, 0.0, 0.0};
    d4 c2 = {2e-3, 0.0, 0.0, 0.0}, c3 = {3e-3, 0.0, 0.0, 0.0};
    for (int i = 0; i < trips; ++i) {
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c1, 0, 0, 0);
            c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c2, 0, 0, 0);
            c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c3, 0, 0, 0);
        }
    }
    const d4 t = c0 + c1 + c2 + c3;
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = t[0] + t[1] + t[2] + t[3];
}

// kFmaChains independent FP64 FMA chains per thread, 2 FLOP each.
__global__ void __launch_bounds__(256) fma_f64_loop_kernel(int iters, double* __restrict__ out) {
    double x[kFmaChains];
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) x[k] = 1e-9 * (threadIdx.x + k);
    const double m = 0.999999, c = 1e-7;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kFmaChains; ++k) x[k] = fma(x[k], m, c);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) s += x[k];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// dst[i] = src[i] over n 16-byte elements, grid-stride.
__global__ void __launch_bounds__(256) copy_kernel(const d2* __restrict__ src, d2* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Milliseconds of the fastest of `reps` launches of f on s.
template <class F>
hipError_t best_ms(F f, int reps, hipStream_t s, float* ms) {
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    float best = 1e30f;
    f();  // warm-up
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) f();
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e == hipSuccess) best = std::min(best, t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = best;
    return e;
}

}  // namespace

extern "C" esmf_status esmf_probe_peaks(int64_t copy_bytes, void* hip_stream, esmf_peaks* out) {
    esmf::clear_error();
    if (!out) return esmf::fail(ESMF_ERR_INVALID_ARG, "out is NULL");
    if (copy_bytes < (1 << 20) || copy_bytes > ((int64_t)64 << 30))
        return esmf::fail(ESMF_ERR_INVALID_ARG, "copy_bytes must be in 1 MiB .. 64 GiB");
    hipStream_t s = (hipStream_t)hip_stream;
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return esmf::device_fail(e, "device properties");
    const int cus = prop.multiProcessorCount;
    // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    const int grid = 8 * cus, block = 256;
    double* res = nullptr;
    if (hipMalloc((void**)&res, sizeof(double) * (size_t)grid * block) != hipSuccess) {
        (void)hipGetLastError();
        return esmf::fail(ESMF_ERR_OUT_OF_MEMORY, "probe output");
    }
    const int mfma_trips = 625, fma_iters = 100000;
    float t_mfma = 0.0f, t_fma = 0.0f, t_copy = 0.0f;
    e = best_ms([&] { mfma_f64_loop_kernel<<<grid, block, 0, s>>>(mfma_trips, res); }, 3, s, &t_mfma);
    if (e == hipSuccess)
        e = best_ms([&] { fma_f64_loop_kernel<<<grid, block, 0, s>>>(fma_iters, res); }, 3, s, &t_fma);
    const int64_t n = copy_bytes / 16;
    d2 *src = nullptr, *dst = nullptr;
    if (e == hipSuccess) {
        if (hipMalloc((void**)&src, 16 * (size_t)n) != hipSuccess || hipMalloc((void**)&dst, 16 * (size_t)n) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(src);
            (void)hipFree(res);
            return esmf::fail(ESMF_ERR_OUT_OF_MEMORY, "probe copy buffers");
        }
        e = hipMemsetAsync(src, 0, 16 * (size_t)n, s);
        if (e == hipSuccess)
            e = best_ms([&] { copy_kernel<<<(int)std::min<int64_t>((n + block - 1) / block, 64 * cus), block, 0, s>>>(src, dst, n); },
                        10, s, &t_copy);
    }
    (void)hipFree(src);
    (void)hipFree(dst);
    (void)hipFree(res);
    if (e != hipSuccess) return esmf::device_fail(e, "peak probe");
    const double waves = (double)grid * (block / 64);
    out->fp64_mfma_tflops = waves * mfma_trips * kMfmaPerTrip * 2048.0 / (t_mfma * 1e-3) / 1e12;
    out->fp64_fma_tflops = (double)grid * block * fma_iters * kFmaChains * 2.0 / (t_fma * 1e-3) / 1e12;
    out->copy_tbps = 2.0 * 16.0 * (double)n / (t_copy * 1e-3) / 1e12;
    out->compute_units = cus;
    out->clock_mhz = prop.clockRate / 1000;
    return ESMF_OK;
}
