// ceilings.hip -- what this chip actually delivers on the units the hot path
// uses, measured beside the spec-sheet peaks the rooflines are quoted
// against: device copy bandwidth (HBM), bf16 and FP32 matrix-core rates,
// FP32 and FP64 vector FMA rates (this build has packed FP32 switched off,
// so the FP32 vector figure is the unpacked one), and the rate of the
// hardware exp2 (the transcendental the ESS log-likelihood spends one of per
// element).  Each compute kernel keeps independent accumulators per wave so
// that the unit, not the dependency chain, sets the rate; results are
// written out so nothing is optimised away.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fsmmc_host.h"

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8c __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Four 16-byte loads in flight per thread, then their four stores; n is a
// multiple of 4 * the grid's thread count (the host sizes it so).
__global__ __launch_bounds__(256) void ceil_copy_kernel(const f32x4* __restrict__ src, f32x4* __restrict__ dst,
                                                        size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += 4 * stride) {
        f32x4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = src[i + k * stride];
#pragma unroll
        for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(v[k], &dst[i + k * stride]);
    }
}

__global__ __launch_bounds__(256) void ceil_mfma_bf16_kernel(int iters, float* out)
{
    const int lane = threadIdx.x & 63;
    bf16x8c a, b;
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(0.001f * (float)(lane + i));
        b[i] = (__bf16)(0.002f * (float)(lane - i));
    }
    f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
    for (int it = 0; it < iters; ++it) {
        c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c3, 0, 0, 0);
    }
    float s = 0.0f;
    for (int i = 0; i < 16; ++i) s += c0[i] + c1[i] + c2[i] + c3[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void ceil_mfma_f32_kernel(int iters, float* out)
{
    const int lane = threadIdx.x & 63;
    const float a = 0.001f * (float)lane, b = 0.002f * (float)(lane + 1);
    f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
    for (int it = 0; it < iters; ++it) {
        c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c3, 0, 0, 0);
    }
    float s = 0.0f;
    for (int i = 0; i < 16; ++i) s += c0[i] + c1[i] + c2[i] + c3[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void ceil_fma_kernel(int iters, T m, T k, T* out)
{
    T v[8];
    for (int i = 0; i < 8; ++i) v[i] = (T)(threadIdx.x + i);
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = fma(v[i], m, k);
    T s = 0;
    for (int i = 0; i < 8; ++i) s += v[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void ceil_exp_kernel(int iters, float* out)
{
    float v[8];
    for (int i = 0; i < 8; ++i) v[i] = 0.01f * (float)(threadIdx.x + i);
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = __builtin_amdgcn_exp2f(-v[i]);  // stays in (0, 1]
    float s = 0.0f;
    for (int i = 0; i < 8; ++i) s += v[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Best of `reps` timed launches (after one untimed), in milliseconds.
template <typename F>
hipError_t best_ms(F&& launch, int reps, double* ms)
{
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    double best = 1e300;
    if (e == hipSuccess) {
        launch();
        e = hipGetLastError();
    }
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        e = hipEventRecord(a, 0);
        if (e == hipSuccess) {
            launch();
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(b, 0);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        if (e == hipSuccess) best = std::min(best, (double)t);
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    *ms = best;
    return e;
}

}  // namespace

extern "C" fsmmc_status fsmmc_measure_ceilings(int device, size_t copy_bytes, fsmmc_ceilings* out)
{
    using namespace fsmmc;
    if (!out) return fail(FSMMC_EINVAL, "out is NULL");
    if (copy_bytes < (64u << 20) || copy_bytes % 16) return fail(FSMMC_EINVAL, "copy_bytes must be >= 64 MiB, a multiple of 16");
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t p;
    HIP_TRY(hipGetDeviceProperties(&p, device));
    *out = fsmmc_ceilings{};
    out->cus = p.multiProcessorCount;
    out->clock_mhz = p.clockRate / 1000;
    const int blocks = p.multiProcessorCount * 8, threads = 256;  // 8 waves per SIMD
    const double waves = (double)blocks * threads / 64.0;
    void *src = nullptr, *dst = nullptr, *res = nullptr;
    hipError_t e = hipMalloc(&src, copy_bytes);
    if (e == hipSuccess) e = hipMalloc(&dst, copy_bytes);
    if (e == hipSuccess) e = hipMalloc(&res, (size_t)blocks * threads * sizeof(double));
    if (e == hipSuccess) e = hipMemset(src, 0, copy_bytes);
    double ms = 0.0;
    if (e == hipSuccess) {
        const unsigned cgrid = (unsigned)p.multiProcessorCount * 16;
        const size_t quantum = (size_t)cgrid * 256 * 4;  // 16-byte units per round of the grid
        const size_t n4 = copy_bytes / 16 / quantum * quantum;
        e = best_ms([&] { hipLaunchKernelGGL(ceil_copy_kernel, dim3(cgrid), dim3(256), 0, 0,
                                             (const f32x4*)src, (f32x4*)dst, n4); }, 5, &ms);
        out->hbm_copy_gbps = 2.0 * (double)n4 * 16 / (ms * 1e-3) / 1e9;
    }
    if (e == hipSuccess) {
        const int it = 4000;
        e = best_ms([&] { hipLaunchKernelGGL(ceil_mfma_bf16_kernel, dim3(blocks), dim3(threads), 0, 0, it,
                                             (float*)res); }, 3, &ms);
        out->mfma_bf16_tflops = waves * it * 4 * (32.0 * 32 * 16 * 2) / (ms * 1e-3) / 1e12;
    }
    if (e == hipSuccess) {
        const int it = 2000;
        e = best_ms([&] { hipLaunchKernelGGL(ceil_mfma_f32_kernel, dim3(blocks), dim3(threads), 0, 0, it,
                                             (float*)res); }, 3, &ms);
        out->mfma_f32_tflops = waves * it * 4 * (32.0 * 32 * 2 * 2) / (ms * 1e-3) / 1e12;
    }
    if (e == hipSuccess) {
        const int it = 8000;
        e = best_ms([&] { hipLaunchKernelGGL(ceil_fma_kernel<float>, dim3(blocks), dim3(threads), 0, 0, it,
                                             0.999999f, 1e-6f, (float*)res); }, 3, &ms);
        out->valu_f32_tflops = (double)blocks * threads * it * 8 * 2 / (ms * 1e-3) / 1e12;
    }
    if (e == hipSuccess) {
        const int it = 4000;
        e = best_ms([&] { hipLaunchKernelGGL(ceil_fma_kernel<double>, dim3(blocks), dim3(threads), 0, 0, it,
                                             0.999999, 1e-6, (double*)res); }, 3, &ms);
        out->valu_f64_tflops = (double)blocks * threads * it * 8 * 2 / (ms * 1e-3) / 1e12;
    }
    if (e == hipSuccess) {
        const int it = 2000;
        e = best_ms([&] { hipLaunchKernelGGL(ceil_exp_kernel, dim3(blocks), dim3(threads), 0, 0, it,
                                             (float*)res); }, 3, &ms);
        out->exp_f32_gops = (double)blocks * threads * it * 8 / (ms * 1e-3) / 1e9;
    }
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    if (res) (void)hipFree(res);
    if (e != hipSuccess) return hip_fail(e, "ceiling kernels");
    return FSMMC_OK;
}
