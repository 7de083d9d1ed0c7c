// ess.hip -- elliptical slice sampling (Murray, Adams, MacKay 2010) as an FSM
// (Sec. 3.1: states INIT, SHRINK, DONE; Appendix, Alg. "Transition kernel for
// elliptical slice sampler"), for latent Gaussian-process targets.
//
// Kernels:
//   * nu_gemm_mfma_kernel: ellipse directions nu = L z for a window of
//     (chain, draw) columns; z is drawn inside the kernel from the Philox
//     stream of its (chain, draw), L is the triangular prior factor; the
//     product runs on FP32 MFMA (32x32x2) for Dp <= 256 and, above, on the
//     bf16 MFMA (32x32x16) from exact three-piece bf16 splits of z and L (six
//     piece products per FP32 product), FP32 accumulation in both.
//   * nu_gemm_simple_kernel: the same product in plain FMA (FP64 jobs).
//   * ess_fsm_kernel: one wavefront per chain; the chain steps through its
//     FSM for every draw of its window without waiting for any other chain.
//     Every step is the bundled, amortized step of the Appendix (cheap states
//     back to back, then one fused proposal + log-likelihood evaluation).
//   * ess_sync_kernel / ess_pad_kernel: the synchronized baseline -- one
//     draw of every chain per launch; the padding kernel then runs the loop
//     bodies a batched while loop executes for chains that already exited.
//   * *_full_kernel: the same kernels for D == 64 x elements per lane, where
//     the element range masks drop out (same operations on the same values).
//
// Both runtimes call the same __device__ functions in the same order for a
// chain, so their draws agree bit for bit.
#include "ess_device.h"

namespace fsmmc {

template <int RT>
__global__ __launch_bounds__(512) void nu_gemm_mfma_kernel(NuK<float> a)
{
    nu_gemm_block<RT>(a, blockIdx.x * 64);
}

// One column per block: draw z into LDS, then row-wise triangular dot products.
template <typename T>
__global__ __launch_bounds__(256) void nu_gemm_simple_kernel(NuK<T> a)
{
    extern __shared__ unsigned char smem_raw[];
    T* zs = reinterpret_cast<T*>(smem_raw);
    const int g = blockIdx.x;
    const int ch = g / a.W, w = g - ch * a.W;
    const uint32_t draw = a.draw_fixed >= 0 ? (uint32_t)a.draw_fixed : a.t[ch] + a.tadd + (uint32_t)w;
    const bool valid = a.draw_fixed >= 0 || draw < (uint32_t)a.n;
    for (int b = threadIdx.x; b < (a.Dp >> 2); b += blockDim.x) {
        T z[4] = {T(0), T(0), T(0), T(0)};
        if (valid && 4 * b < a.D) {
            normals4<T>(a.seed, (uint32_t)ch, draw, a.role, 0, (uint32_t)b, z);
            for (int i = 0; i < 4; ++i)
                if (4 * b + i >= a.D) z[i] = T(0);
        }
        for (int i = 0; i < 4; ++i) zs[4 * b + i] = z[i];
    }
    __syncthreads();
    T* o = a.out + ((size_t)ch * a.W + w) * a.Dp;
    for (int row = threadIdx.x; row < a.Dp; row += blockDim.x) {
        const T* Lr = a.L + (size_t)row * a.Dp;
        T s = T(0);
        for (int k = 0; k <= row; ++k) s = M<T>::fma_(Lr[k], zs[k], s);
        o[row] = s;
    }
}

// ------------------------------------------------------------ FSM kernel
// One wave = one chain, for one window of draws (ess_window).
// FULL (D == 64 EPL) drops the element masks; it is a kernel of its own so
// that each instantiation holds only one form of the loop (registers).
template <typename T, int EPL, bool FULL>
__device__ __forceinline__ void ess_fsm_body(const EssK<T>& a)
{
    __shared__ unsigned long long s_sum;
    const int lane = threadIdx.x & 63;
    const int j = uni((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    EssTally tl;
    if (j < a.m) {
        if (a.target == FSMMC_GP_GAUSS)
            (void)ess_window_run<T, EPL, FULL, FSMMC_GP_GAUSS>(a, j, lane, tl);
        else
            (void)ess_window_run<T, EPL, FULL, FSMMC_GP_LOGISTIC>(a, j, lane, tl);
    }
    // one atomic per block and counter
    const unsigned long long steps = block_sum_u64(tl.steps, &s_sum);
    if (threadIdx.x == 0 && steps) atomicAdd(&a.ctr[0], steps);
    const unsigned long long guards = block_sum_u64(tl.guards, &s_sum);
    if (threadIdx.x == 0 && guards) atomicAdd(&a.ctr[2], guards);
    const unsigned long long live = block_sum_u64(tl.live, &s_sum);
    if (threadIdx.x == 0 && live) atomicAdd(&a.ctr[4], live);
    const unsigned long long left = block_sum_u64(tl.budget_left, &s_sum);
    if (threadIdx.x == 0 && left) atomicAdd(&a.ctr[3], left);
}

template <typename T, int EPL>
__global__ __launch_bounds__(256) void ess_fsm_kernel(EssK<T> a)
{
    ess_fsm_body<T, EPL, false>(a);
}

template <typename T, int EPL>
__global__ __launch_bounds__(256) void ess_fsm_full_kernel(EssK<T> a)
{
    ess_fsm_body<T, EPL, true>(a);
}

// ------------------------------------------------------------ synchronized
// One draw of every chain (all chains at `draw`, at a draw boundary).
// Chain j's draw `draw` (one wave); returns its evaluations, sets *rejected.
template <typename T, int EPL, bool FULL>
__device__ __forceinline__ int ess_sync_run(const EssK<T>& a, int j, int lane, uint32_t draw, uint32_t slot,
                                            bool* rejected)
{
    T x[EPL], nu[EPL], xp[EPL], yv[EPL];
    const T* xj = a.x + (size_t)j * a.Dp;
    const T* nj = a.nu + ((size_t)j * a.W + slot) * a.Dp;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        x[e] = xj[e * 64 + lane];
        yv[e] = a.y[e * 64 + lane];
        nu[e] = nj[e * 64 + lane];
    }
    const EssLin L = ess_lin_of<T, EPL, FULL>(x, nu, yv, lane, a.D, a.target);
    T lx = uni(a.lx[j]), logu, theta, tmin, tmax;
    ess_begin<T>(a.seed, (uint32_t)j, draw, logu, theta, tmin, tmax);
    int evals = 0;
    T lp;
    for (;;) {
        lp = uni(ess_propose_eval<T, EPL, FULL>(x, nu, xp, yv, theta, lane, a.D, a.target, a.inv2v, L));
        ++evals;
        if (lp - lx > logu || evals >= kEssMaxEvals) break;
        ess_shrink<T>(a.seed, (uint32_t)j, draw, evals, theta, tmin, tmax);
    }
    const bool accept = lp - lx > logu;
    if (accept) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) x[e] = xp[e];
        lx = lp;
    }
    ess_emit<T, EPL>(a, j, draw, x, evals, lane);
    T* xo = a.x + (size_t)j * a.Dp;
#pragma unroll
    for (int e = 0; e < EPL; ++e) xo[e * 64 + lane] = x[e];
    if (lane == 0) {
        a.lx[j] = lx;
        a.t[j] = draw + 1;
    }
    *rejected = !accept;
    return evals;
}

template <typename T, int EPL, bool FULL>
__device__ __forceinline__ void ess_sync_body(const EssK<T>& a, uint32_t draw, uint32_t slot)
{
    __shared__ unsigned long long s_sum;
    __shared__ int s_max;
    const int lane = threadIdx.x & 63;
    const int j = uni((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    int evals = 0;
    bool rejected = false;
    if (j < a.m) evals = ess_sync_run<T, EPL, FULL>(a, j, lane, draw, slot, &rejected);
    // one atomic per block and counter
    const unsigned long long steps = block_sum_u64((unsigned long long)evals, &s_sum);
    if (threadIdx.x == 0 && steps) atomicAdd(&a.ctr[0], steps);
    const unsigned long long rej = block_sum_u64(rejected ? 1ull : 0ull, &s_sum);
    if (threadIdx.x == 0 && rej) atomicAdd(&a.ctr[2], rej);
    const int mx = block_max_i32(evals, &s_max);
    if (threadIdx.x == 0) atomicMax(&a.maxN[draw], mx);
}

template <typename T, int EPL>
__global__ __launch_bounds__(256) void ess_sync_kernel(EssK<T> a, uint32_t draw, uint32_t slot)
{
    ess_sync_body<T, EPL, false>(a, draw, slot);
}

template <typename T, int EPL>
__global__ __launch_bounds__(256) void ess_sync_full_kernel(EssK<T> a, uint32_t draw, uint32_t slot)
{
    ess_sync_body<T, EPL, true>(a, draw, slot);
}

// The loop bodies a batched while loop runs for chain j after its own exit:
// max_j N_j - N_j more proposals and log-likelihood evaluations, discarded.
template <typename T, int EPL, bool FULL>
__device__ __forceinline__ int ess_pad_run(const EssK<T>& a, int j, int lane, uint32_t draw, uint32_t slot)
{
    const int nj_evals = uni(a.counts[(size_t)j * a.n + draw]);
    const int extra = uni(a.maxN[draw]) - nj_evals;
    if (extra <= 0) return 0;
    T x[EPL], nu[EPL], xp[EPL], yv[EPL];
    const T* xj = a.x + (size_t)j * a.Dp;
    const T* nj = a.nu + ((size_t)j * a.W + slot) * a.Dp;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        x[e] = xj[e * 64 + lane];
        yv[e] = a.y[e * 64 + lane];
        nu[e] = nj[e * 64 + lane];
    }
    const EssLin L = ess_lin_of<T, EPL, FULL>(x, nu, yv, lane, a.D, a.target);
    T sum = T(0);
    for (int i = 0; i < extra; ++i) {
        const T theta = Pi<T>::two_pi * uniform<T>(a.seed, (uint32_t)j, draw, ROLE_ANGLE,
                                                    (uint32_t)(nj_evals + i));
        sum += ess_propose_eval<T, EPL, FULL>(x, nu, xp, yv, theta, lane, a.D, a.target, a.inv2v, L);
    }
    if (lane == 0) a.sink[j] = sum;
    return extra;
}

template <typename T, int EPL, bool FULL>
__device__ __forceinline__ void ess_pad_body(const EssK<T>& a, uint32_t draw, uint32_t slot)
{
    __shared__ unsigned long long s_sum;
    const int lane = threadIdx.x & 63;
    const int j = uni((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    int extra = 0;
    if (j < a.m) extra = ess_pad_run<T, EPL, FULL>(a, j, lane, draw, slot);
    const unsigned long long tot = block_sum_u64((unsigned long long)extra, &s_sum);
    if (threadIdx.x == 0 && tot) atomicAdd(&a.ctr[1], tot);
}

template <typename T, int EPL>
__global__ __launch_bounds__(256) void ess_pad_kernel(EssK<T> a, uint32_t draw, uint32_t slot)
{
    ess_pad_body<T, EPL, false>(a, draw, slot);
}

template <typename T, int EPL>
__global__ __launch_bounds__(256) void ess_pad_full_kernel(EssK<T> a, uint32_t draw, uint32_t slot)
{
    ess_pad_body<T, EPL, true>(a, draw, slot);
}

// ------------------------------------------------------------ host side
int ess_supported_epl(int D, int dtype)
{
    const int need = (D + 63) / 64;
    static const int f32[] = {1, 2, 4, 6, 8, 12, 16};
    static const int f64[] = {1, 2, 4};
    if (dtype == FSMMC_F32) {
        for (int e : f32)
            if (e >= need) return e;
    } else {
        for (int e : f64)
            if (e >= need) return e;
    }
    return 0;
}

template <typename T>
static hipError_t launch_nu(const JobDev& j, NuK<T> a, int ncols, hipStream_t s);

template <>
hipError_t launch_nu<float>(const JobDev& j, NuK<float> a, int ncols, hipStream_t s)
{
    const dim3 grid((ncols + 63) / 64), block(512);
    switch (ess_gemm_rt(a.Dp)) {
    case 1: hipLaunchKernelGGL(nu_gemm_mfma_kernel<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(nu_gemm_mfma_kernel<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(nu_gemm_mfma_kernel<3>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(nu_gemm_mfma_kernel<4>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <>
hipError_t launch_nu<double>(const JobDev& j, NuK<double> a, int ncols, hipStream_t s)
{
    hipLaunchKernelGGL(nu_gemm_simple_kernel<double>, dim3(ncols), dim3(256),
                       (size_t)a.Dp * sizeof(double), s, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t prior_draw_t(const JobDev& j, hipStream_t s)
{
    NuK<T> a;
    a.m = j.m;
    a.n = j.n;
    a.D = j.D;
    a.Dp = j.Dp;
    a.W = 1;
    a.seed = j.seed;
    a.role = ROLE_INIT;
    a.draw_fixed = 0;
    a.tadd = 0;
    a.t = j.t;
    a.L = (const T*)j.L;
    a.Lp = (const uint16_t*)j.Lp;
    a.out = (T*)j.x;
    return launch_nu<T>(j, a, j.m, s);
}

template <typename T>
static hipError_t fill_window_t(const JobDev& j, hipStream_t s)
{
    return launch_nu<T>(j, ess_window_view<T>(j, j.nu_cur), j.m * j.W, s);
}

template <typename T>
static hipError_t fill_next_window_t(const JobDev& j, int buf, hipStream_t s)
{
    return launch_nu<T>(j, ess_window_view<T>(j, buf, j.tsnap, (uint32_t)j.W), j.m * j.W, s);
}

__global__ void copy_u32_kernel(uint32_t* dst, const uint32_t* src, int n)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) dst[i] = src[i];
}

hipError_t copy_u32(uint32_t* dst, const uint32_t* src, int n, hipStream_t s)
{
    hipLaunchKernelGGL(copy_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

// log L(x) of every chain's current state (wave per chain).
template <typename T, int EPL>
__global__ __launch_bounds__(256) void ess_loglik_kernel(EssK<T> a)
{
    const int lane = threadIdx.x & 63;
    const int j = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (j >= a.m) return;
    const T* xj = a.x + (size_t)j * a.Dp;
    T xr[EPL], yv[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        xr[e] = xj[e * 64 + lane];
        yv[e] = a.y[e * 64 + lane];
    }
    T acc = ess_lane_loglik<T, EPL>(xr, yv, lane, a.D, a.target, a.inv2v);
    acc = wave_sum(acc);
    if (lane == 0) a.lx[j] = acc;
}

#define FSMMC_EPL_CASE_F32(T, E, KERNEL, ...)                   \
    case E:                                                     \
        if constexpr (sizeof(T) == 4) {                         \
            hipLaunchKernelGGL((KERNEL<T, E>), __VA_ARGS__);    \
        } else {                                                \
            return hipErrorInvalidValue;                        \
        }                                                       \
        break;

// Launch KERNEL<T, EPL> for the job's elements-per-lane (FP64 jobs support
// EPL <= 4 only; other values are rejected at job creation).
#define FSMMC_EPL_DISPATCH(T, EPL_, KERNEL, ...)                \
    switch (EPL_) {                                             \
    case 1: hipLaunchKernelGGL((KERNEL<T, 1>), __VA_ARGS__); break; \
    case 2: hipLaunchKernelGGL((KERNEL<T, 2>), __VA_ARGS__); break; \
    case 4: hipLaunchKernelGGL((KERNEL<T, 4>), __VA_ARGS__); break; \
    FSMMC_EPL_CASE_F32(T, 6, KERNEL, __VA_ARGS__)               \
    FSMMC_EPL_CASE_F32(T, 8, KERNEL, __VA_ARGS__)               \
    FSMMC_EPL_CASE_F32(T, 12, KERNEL, __VA_ARGS__)              \
    FSMMC_EPL_CASE_F32(T, 16, KERNEL, __VA_ARGS__)              \
    default: return hipErrorInvalidValue;                       \
    }

template <typename T>
static hipError_t loglik_t(const JobDev& j, hipStream_t s)
{
    EssK<T> a = ess_view<T>(j);
    const dim3 grid((j.m + 3) / 4), block(256);
    FSMMC_EPL_DISPATCH(T, j.EPL, ess_loglik_kernel, grid, block, 0, s, a)
    return hipGetLastError();
}

template <typename T>
static hipError_t fsm_round_t(const JobDev& j, hipStream_t s)
{
    EssK<T> a = ess_view<T>(j);
    const dim3 grid((j.m + 3) / 4), block(256);
    if (j.D == 64 * j.EPL) {
        FSMMC_EPL_DISPATCH(T, j.EPL, ess_fsm_full_kernel, grid, block, 0, s, a)
    } else {
        FSMMC_EPL_DISPATCH(T, j.EPL, ess_fsm_kernel, grid, block, 0, s, a)
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t sync_draw_t(const JobDev& j, uint32_t draw, uint32_t slot, hipStream_t s)
{
    EssK<T> a = ess_view<T>(j);
    const dim3 grid((j.m + 3) / 4), block(256);
    if (j.D == 64 * j.EPL) {
        FSMMC_EPL_DISPATCH(T, j.EPL, ess_sync_full_kernel, grid, block, 0, s, a, draw, slot)
    } else {
        FSMMC_EPL_DISPATCH(T, j.EPL, ess_sync_kernel, grid, block, 0, s, a, draw, slot)
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t pad_draw_t(const JobDev& j, uint32_t draw, uint32_t slot, hipStream_t s)
{
    EssK<T> a = ess_view<T>(j);
    const dim3 grid((j.m + 3) / 4), block(256);
    if (j.D == 64 * j.EPL) {
        FSMMC_EPL_DISPATCH(T, j.EPL, ess_pad_full_kernel, grid, block, 0, s, a, draw, slot)
    } else {
        FSMMC_EPL_DISPATCH(T, j.EPL, ess_pad_kernel, grid, block, 0, s, a, draw, slot)
    }
    return hipGetLastError();
}

hipError_t ess_prior_draw(const JobDev& j, const void* x0, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (!x0) e = (j.dtype == FSMMC_F32) ? prior_draw_t<float>(j, s) : prior_draw_t<double>(j, s);
    if (e != hipSuccess) return e;
    return (j.dtype == FSMMC_F32) ? loglik_t<float>(j, s) : loglik_t<double>(j, s);
}

hipError_t ess_fill_window(const JobDev& j, hipStream_t s)
{
    return (j.dtype == FSMMC_F32) ? fill_window_t<float>(j, s) : fill_window_t<double>(j, s);
}

hipError_t ess_fill_next_window(const JobDev& j, int buf, hipStream_t s)
{
    return (j.dtype == FSMMC_F32) ? fill_next_window_t<float>(j, buf, s) : fill_next_window_t<double>(j, buf, s);
}

hipError_t ess_fsm_round(const JobDev& j, hipStream_t s)
{
    return (j.dtype == FSMMC_F32) ? fsm_round_t<float>(j, s) : fsm_round_t<double>(j, s);
}

hipError_t ess_sync_draw(const JobDev& j, uint32_t draw, uint32_t slot, hipStream_t s)
{
    return (j.dtype == FSMMC_F32) ? sync_draw_t<float>(j, draw, slot, s) : sync_draw_t<double>(j, draw, slot, s);
}

hipError_t ess_pad_draw(const JobDev& j, uint32_t draw, uint32_t slot, hipStream_t s)
{
    return (j.dtype == FSMMC_F32) ? pad_draw_t<float>(j, draw, slot, s) : pad_draw_t<double>(j, draw, slot, s);
}

}  // namespace fsmmc
