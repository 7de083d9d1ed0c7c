// ess.hip -- elliptical slice sampling (Murray, Adams, MacKay 2010) as an FSM
// (Sec. 3.1: states INIT, SHRINK, DONE; Appendix, Alg. "Transition kernel for
// elliptical slice sampler"), for latent Gaussian-process targets.
//
// Kernels:
//   * nu_gemm_mfma_kernel: ellipse directions nu = L z for a window of
//     (chain, draw) columns; z is drawn inside the kernel from the Philox
//     stream of its (chain, draw), L is the triangular prior factor, the
//     product runs on FP32 MFMA (32x32x2) with FP32 accumulation.
//   * nu_gemm_simple_kernel: the same product in plain FMA (FP64 jobs).
//   * ess_fsm_kernel: one wavefront per chain; the chain steps through its
//     FSM for every draw of its window without waiting for any other chain.
//     Every step is the bundled, amortized step of the Appendix (cheap states
//     back to back, then one fused proposal + log-likelihood evaluation).
//   * ess_sync_kernel / ess_pad_kernel: the synchronized baseline -- one
//     draw of every chain per launch; the padding kernel then runs the loop
//     bodies a batched while loop executes for chains that already exited.
//
// Both runtimes call the same __device__ functions in the same order for a
// chain, so their draws agree bit for bit.
#include "fsmmc_device.h"
#include "fsmmc_internal.h"

namespace fsmmc {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------ kernel views
template <typename T>
struct NuK {
    int m, n, D, Dp, W;
    uint64_t seed;
    uint32_t role;
    int draw_fixed;     // >= 0: every column uses this draw; < 0: draw = t[chain] + w
    const uint32_t* t;  // chain draw counters
    const T* L;         // Dp x Dp lower factor, zero padded
    T* out;             // column (chain, w) -> out[(chain * W + w) * Dp + row]
};

template <typename T>
struct EssK {
    int m, n, D, Dp, W, target;
    uint64_t seed;
    T inv2v;
    const T* y;
    const T* nu;
    int32_t* k;
    uint32_t* t;
    int32_t* evals;
    int64_t* budget;
    T *theta, *tmin, *tmax, *logy, *lx, *x, *out;
    int32_t* counts;
    unsigned long long* ctr;
    int32_t* maxN;
    T* sink;
};

// ------------------------------------------------------------ ellipse GEMM
// Block: 8 waves, 64 columns, all Dp rows.  Wave w owns RT row tiles of 32
// rows in "snake" order (w, 15-w, 16+w, 31-w, ...) so the triangular work is
// balanced across waves.  Per K chunk of 32: the block draws its 32 x 64
// normals into LDS (one Philox block per thread), then every wave multiplies
// its L rows (read as float4 along k from L2) by them.  The MFMA computes
// nu^T = z^T L^T so each output register row is 32 consecutive nu entries
// of one column (128-byte coalesced stores).
template <int RT>
__global__ __launch_bounds__(512) void nu_gemm_mfma_kernel(NuK<float> a)
{
    __shared__ float Zs[32][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int ncols = a.m * a.W;
    const int col0 = blockIdx.x * 64;

    const int zc = tid & 63, zb = tid >> 6;
    const int gcol = col0 + zc;
    bool zvalid = gcol < ncols;
    int zchain = 0;
    uint32_t zdraw = 0;
    if (zvalid) {
        zchain = gcol / a.W;
        const int zw = gcol - zchain * a.W;
        zdraw = a.draw_fixed >= 0 ? (uint32_t)a.draw_fixed : a.t[zchain] + (uint32_t)zw;
        zvalid = a.draw_fixed >= 0 || zdraw < (uint32_t)a.n;
    }

    const int ntiles = a.Dp >> 5;
    int tiles[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const int idx = (r & 1) ? r * 8 + 7 - wave : r * 8 + wave;
        tiles[r] = idx < ntiles ? idx : -1;
    }
    floatx16 acc[RT][2];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[r][c][q] = 0.0f;

    for (int kc = 0; kc < a.Dp; kc += 32) {
        float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        const int kb = kc + 4 * zb;
        if (zvalid && kb < a.D) {
            normals4<float>(a.seed, (uint32_t)zchain, zdraw, a.role, 0, (uint32_t)(kb >> 2), z);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (kb + i >= a.D) z[i] = 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) Zs[4 * zb + i][zc] = z[i];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const int ti = tiles[r];
            if (ti < 0 || 32 * ti + 31 < kc) continue;
            const float4* Lr =
                reinterpret_cast<const float4*>(a.L + (size_t)(32 * ti + l32) * a.Dp + kc + 16 * h);
            float lr[16];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float4 q4 = Lr[v];
                lr[4 * v + 0] = q4.x;
                lr[4 * v + 1] = q4.y;
                lr[4 * v + 2] = q4.z;
                lr[4 * v + 3] = q4.w;
            }
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const float av = Zs[16 * h + kk][c * 32 + l32];
                    acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, lr[kk], acc[r][c], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const int ti = tiles[r];
        if (ti < 0) continue;
        const int row = 32 * ti + l32;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int col = c * 32 + 8 * (q >> 2) + 4 * h + (q & 3);
                const int g = col0 + col;
                if (g < ncols) {
                    const int ch = g / a.W, w = g - ch * a.W;
                    a.out[((size_t)ch * a.W + w) * a.Dp + row] = acc[r][c][q];
                }
            }
        }
    }
}

// One column per block: draw z into LDS, then row-wise triangular dot products.
template <typename T>
__global__ __launch_bounds__(256) void nu_gemm_simple_kernel(NuK<T> a)
{
    extern __shared__ unsigned char smem_raw[];
    T* zs = reinterpret_cast<T*>(smem_raw);
    const int g = blockIdx.x;
    const int ch = g / a.W, w = g - ch * a.W;
    const uint32_t draw = a.draw_fixed >= 0 ? (uint32_t)a.draw_fixed : a.t[ch] + (uint32_t)w;
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

// ------------------------------------------------------------ ESS blocks
template <typename T>
__device__ __forceinline__ T ess_term(T f, T yv, int target, T inv2v)
{
    if (target == FSMMC_GP_GAUSS) {
        const T r = yv - f;
        return -(r * r) * inv2v;
    }
    return yv * f - M<T>::softplus(f);
}

// x' = x cos(theta) + nu sin(theta) and log L(x'), summed in a fixed order
// (lane-local over e, then a wave butterfly); the result is wave-uniform.
template <typename T, int EPL>
__device__ __forceinline__ T ess_propose_eval(const T (&x)[EPL], const T (&nu)[EPL], T (&xp)[EPL],
                                              const T (&yv)[EPL], T theta, int lane, int D, int target,
                                              T inv2v)
{
    T s, c;
    M<T>::sincos_(theta, &s, &c);
    T acc = T(0);
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        const T f = M<T>::fma_(x[e], c, nu[e] * s);
        xp[e] = f;
        const T term = ess_term(f, yv[e], target, inv2v);
        acc += (e * 64 + lane < D) ? term : T(0);
    }
    return wave_sum(acc);
}

// INIT: threshold log y = log L(x) + log u and the initial bracket.
template <typename T>
__device__ __forceinline__ void ess_begin(uint64_t seed, uint32_t chain, uint32_t draw, T lx, T& logy,
                                          T& theta, T& tmin, T& tmax)
{
    logy = lx + M<T>::log_(uniform<T>(seed, chain, draw, ROLE_THRESH, 0));
    theta = Pi<T>::two_pi * uniform<T>(seed, chain, draw, ROLE_ANGLE, 0);
    tmin = theta - Pi<T>::two_pi;
    tmax = theta;
}

// SHRINK: move the bracket end on theta's side to theta, draw a new angle.
template <typename T>
__device__ __forceinline__ void ess_shrink(uint64_t seed, uint32_t chain, uint32_t draw, int evals,
                                           T& theta, T& tmin, T& tmax)
{
    if (theta < T(0))
        tmin = theta;
    else
        tmax = theta;
    theta = tmin + (tmax - tmin) * uniform<T>(seed, chain, draw, ROLE_ANGLE, (uint32_t)evals);
}

template <typename T, int EPL>
__device__ __forceinline__ void ess_emit(const EssK<T>& a, int j, uint32_t t, const T (&x)[EPL], int evals,
                                         int lane)
{
    T* o = a.out + ((size_t)j * a.n + t) * a.D;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        const int d = e * 64 + lane;
        if (d < a.D) o[d] = x[e];
    }
    if (lane == 0) a.counts[(size_t)j * a.n + t] = evals;
}

// ------------------------------------------------------------ FSM kernel
// One wave = one chain.  Runs FSM steps until the chain has used the ellipse
// window [t0, t0 + W), reached n draws, or spent its step budget.
template <typename T, int EPL>
__global__ __launch_bounds__(256) void ess_fsm_kernel(EssK<T> a)
{
    const int lane = threadIdx.x & 63;
    const int j = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (j >= a.m) return;
    uint32_t t = a.t[j];
    if (t >= (uint32_t)a.n) return;
    const uint32_t t0 = t;
    const uint32_t wend = min(t0 + (uint32_t)a.W, (uint32_t)a.n);
    int k = a.k[j], evals = a.evals[j];
    T theta = a.theta[j], tmin = a.tmin[j], tmax = a.tmax[j], logy = a.logy[j], lx = a.lx[j];
    int64_t budget = a.budget[j];

    T x[EPL], nu[EPL], xp[EPL], yv[EPL];
    const T* xj = a.x + (size_t)j * a.Dp;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        x[e] = xj[e * 64 + lane];
        yv[e] = a.y[e * 64 + lane];
    }
    unsigned long long steps = 0;
    int guards = 0;
    bool have_nu = false;
    while (t < wend && budget > 0) {
        if (!have_nu) {
            const T* nj = a.nu + ((size_t)j * a.W + (t - t0)) * a.Dp;
#pragma unroll
            for (int e = 0; e < EPL; ++e) nu[e] = nj[e * 64 + lane];
            have_nu = true;
        }
        if (k == 1) {
            ess_begin<T>(a.seed, (uint32_t)j, t, lx, logy, theta, tmin, tmax);
            evals = 0;
        } else {
            ess_shrink<T>(a.seed, (uint32_t)j, t, evals, theta, tmin, tmax);
        }
        const T lp = ess_propose_eval<T, EPL>(x, nu, xp, yv, theta, lane, a.D, a.target, a.inv2v);
        ++evals;
        ++steps;
        --budget;
        const bool accept = lp > logy;
        if (accept || evals >= kEssMaxEvals) {
            if (accept) {
#pragma unroll
                for (int e = 0; e < EPL; ++e) x[e] = xp[e];
                lx = lp;
            } else {
                ++guards;
            }
            ess_emit<T, EPL>(a, j, t, x, evals, lane);
            ++t;
            k = 1;
            have_nu = false;
        } else {
            k = 2;
        }
    }
    T* xo = a.x + (size_t)j * a.Dp;
#pragma unroll
    for (int e = 0; e < EPL; ++e) xo[e * 64 + lane] = x[e];
    if (lane == 0) {
        a.t[j] = t;
        a.k[j] = k;
        a.evals[j] = evals;
        a.theta[j] = theta;
        a.tmin[j] = tmin;
        a.tmax[j] = tmax;
        a.logy[j] = logy;
        a.lx[j] = lx;
        a.budget[j] = budget;
        atomicAdd(&a.ctr[0], steps);
        if (guards) atomicAdd(&a.ctr[2], (unsigned long long)guards);
        if (t < (uint32_t)a.n) {
            atomicAdd(&a.ctr[4], 1ull);
            if (budget > 0) atomicAdd(&a.ctr[3], 1ull);
        }
    }
}

// ------------------------------------------------------------ synchronized
// One draw of every chain (all chains at `draw`, at a draw boundary).
template <typename T, int EPL>
__global__ __launch_bounds__(256) void ess_sync_kernel(EssK<T> a, uint32_t draw, uint32_t slot)
{
    const int lane = threadIdx.x & 63;
    const int j = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (j >= a.m) return;
    T x[EPL], nu[EPL], xp[EPL], yv[EPL];
    const T* xj = a.x + (size_t)j * a.Dp;
    const T* nj = a.nu + ((size_t)j * a.W + slot) * a.Dp;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        x[e] = xj[e * 64 + lane];
        yv[e] = a.y[e * 64 + lane];
        nu[e] = nj[e * 64 + lane];
    }
    T lx = a.lx[j], logy, theta, tmin, tmax;
    ess_begin<T>(a.seed, (uint32_t)j, draw, lx, logy, theta, tmin, tmax);
    int evals = 0;
    T lp;
    for (;;) {
        lp = ess_propose_eval<T, EPL>(x, nu, xp, yv, theta, lane, a.D, a.target, a.inv2v);
        ++evals;
        if (lp > logy || evals >= kEssMaxEvals) break;
        ess_shrink<T>(a.seed, (uint32_t)j, draw, evals, theta, tmin, tmax);
    }
    const bool accept = lp > logy;
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
        atomicAdd(&a.ctr[0], (unsigned long long)evals);
        if (!accept) atomicAdd(&a.ctr[2], 1ull);
        atomicMax(&a.maxN[draw], evals);
    }
}

// The loop bodies a batched while loop runs for chain j after its own exit:
// max_j N_j - N_j more proposals and log-likelihood evaluations, discarded.
template <typename T, int EPL>
__global__ __launch_bounds__(256) void ess_pad_kernel(EssK<T> a, uint32_t draw, uint32_t slot)
{
    const int lane = threadIdx.x & 63;
    const int j = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (j >= a.m) return;
    const int nj_evals = a.counts[(size_t)j * a.n + draw];
    const int extra = a.maxN[draw] - nj_evals;
    if (extra <= 0) return;
    T x[EPL], nu[EPL], xp[EPL], yv[EPL];
    const T* xj = a.x + (size_t)j * a.Dp;
    const T* nj = a.nu + ((size_t)j * a.W + slot) * a.Dp;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        x[e] = xj[e * 64 + lane];
        yv[e] = a.y[e * 64 + lane];
        nu[e] = nj[e * 64 + lane];
    }
    T sum = T(0);
    for (int i = 0; i < extra; ++i) {
        const T theta = Pi<T>::two_pi * uniform<T>(a.seed, (uint32_t)j, draw, ROLE_ANGLE,
                                                    (uint32_t)(nj_evals + i));
        sum += ess_propose_eval<T, EPL>(x, nu, xp, yv, theta, lane, a.D, a.target, a.inv2v);
    }
    if (lane == 0) {
        a.sink[j] = sum;
        atomicAdd(&a.ctr[1], (unsigned long long)extra);
    }
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
static EssK<T> ess_view(const JobDev& j)
{
    EssK<T> a;
    a.m = j.m;
    a.n = j.n;
    a.D = j.D;
    a.Dp = j.Dp;
    a.W = j.W;
    a.target = j.target;
    a.seed = j.seed;
    a.inv2v = (j.target == FSMMC_GP_GAUSS) ? (T)(1.0 / (2.0 * j.noise_sd * j.noise_sd)) : T(0);
    a.y = (const T*)j.y;
    a.nu = (const T*)j.nu;
    a.k = j.k;
    a.t = j.t;
    a.evals = j.evals;
    a.budget = j.budget;
    a.theta = (T*)j.theta;
    a.tmin = (T*)j.tmin;
    a.tmax = (T*)j.tmax;
    a.logy = (T*)j.logy;
    a.lx = (T*)j.lx;
    a.x = (T*)j.x;
    a.out = (T*)j.out;
    a.counts = j.counts;
    a.ctr = j.ctr;
    a.maxN = j.maxN;
    a.sink = (T*)j.sink;
    return a;
}

template <typename T>
static hipError_t launch_nu(const JobDev& j, NuK<T> a, int ncols, hipStream_t s);

template <>
hipError_t launch_nu<float>(const JobDev& j, NuK<float> a, int ncols, hipStream_t s)
{
    const int ntiles = a.Dp / 32;
    const int rt = (ntiles + 7) / 8;
    const dim3 grid((ncols + 63) / 64), block(512);
    switch (rt) {
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
    a.t = j.t;
    a.L = (const T*)j.L;
    a.out = (T*)j.x;
    return launch_nu<T>(j, a, j.m, s);
}

template <typename T>
static hipError_t fill_window_t(const JobDev& j, hipStream_t s)
{
    NuK<T> a;
    a.m = j.m;
    a.n = j.n;
    a.D = j.D;
    a.Dp = j.Dp;
    a.W = j.W;
    a.seed = j.seed;
    a.role = ROLE_NU;
    a.draw_fixed = -1;
    a.t = j.t;
    a.L = (const T*)j.L;
    a.out = (T*)j.nu;
    return launch_nu<T>(j, a, j.m * j.W, s);
}

// log L(x) of every chain's current state (wave per chain).
template <typename T, int EPL>
__global__ __launch_bounds__(256) void ess_loglik_kernel(EssK<T> a)
{
    const int lane = threadIdx.x & 63;
    const int j = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (j >= a.m) return;
    const T* xj = a.x + (size_t)j * a.Dp;
    T acc = T(0);
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        const int d = e * 64 + lane;
        const T term = ess_term(xj[d], a.y[d], a.target, a.inv2v);
        acc += (d < a.D) ? term : T(0);
    }
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
    FSMMC_EPL_DISPATCH(T, j.EPL, ess_fsm_kernel, grid, block, 0, s, a)
    return hipGetLastError();
}

template <typename T>
static hipError_t sync_draw_t(const JobDev& j, uint32_t draw, uint32_t slot, hipStream_t s)
{
    EssK<T> a = ess_view<T>(j);
    const dim3 grid((j.m + 3) / 4), block(256);
    FSMMC_EPL_DISPATCH(T, j.EPL, ess_sync_kernel, grid, block, 0, s, a, draw, slot)
    return hipGetLastError();
}

template <typename T>
static hipError_t pad_draw_t(const JobDev& j, uint32_t draw, uint32_t slot, hipStream_t s)
{
    EssK<T> a = ess_view<T>(j);
    const dim3 grid((j.m + 3) / 4), block(256);
    FSMMC_EPL_DISPATCH(T, j.EPL, ess_pad_kernel, grid, block, 0, s, a, draw, slot)
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
