// mog.hip -- the no-U-turn sampler on a mixture of Gaussians sharing one
// covariance (Sec. 7.3: a 100-dimensional correlated mixture whose modes lie
// along the principal direction; the loop counts are heavy-tailed, so the
// per-draw barrier of a vmapped sampler waits for rare 1000-leapfrog draws).
//
//   pi(x) ∝ sum_k w_k exp(-q_k / 2),  q_k = (x - mu_k)^T P (x - mu_k)
//   U = -log pi,  grad U = P x - sum_k r_k P mu_k,  r_k = w_k e^(-q_k/2) / sum.
//
// The gradient is a matrix-vector product per chain (2 D^2 flop), cheap next
// to the FSM bookkeeping, so it is computed by the chain's own wavefront
// inside the step instead of by a separate batched launch: the NUTS FSM step
// (nuts_chain_body, shared with the logistic-regression path) runs with a
// gradient policy that evaluates
//   y = P x (P staged in LDS, x broadcast lane by lane from registers),
//   s_0 = x . y,  s_k = (P mu_k) . x,
//   a_k = (log w_k - mu_k^T P mu_k / 2) - s_0 / 2 + s_k,
//   U = -logsumexp_k a_k,  grad U = y - sum_k e^(a_k + U) P mu_k.
// P mu_k and the constants are formed once per job (mog_setup_kernel).
// Precision: inputs, state and outputs are FP32, but these sums are carried
// in FP64.  A strongly correlated covariance makes P badly conditioned (at
// rho = 0.99, D = 100 its eigenvalues are 100 and 0.0101), and P x along the
// principal direction is a small difference of large entries: an FP32 sum
// loses about four digits there (gradient errors ~1e-3 relative, enough to
// move a 1000-leapfrog trajectory by more than 1e-4).  Every product of two
// FP32 numbers is exact in FP64, so only the FP64 sums round.
//
// nuts_mog_kernel is persistent: every wavefront takes chains from a device
// ticket counter and runs each one through its FSM steps until the chain has
// its draws (or its step budget is spent) -- no chain ever waits for another
// (Sec. 3.2, Alg. "FSM MCMC algorithm").  The synchronized runtime launches
// it once per draw (tstop = draw + 1), so every chain finishes draw i before
// any starts draw i + 1; in vmap mode nuts_mog_pad_kernel then evaluates, for
// every chain, the max_j N_j - N_j gradients a batched while loop would
// compute and discard.
#include "nuts_device.h"

namespace fsmmc {

constexpr int kMogMaxK = 8;

struct MogK {
    const float* P;   // Dp x Dp, zero padded, symmetric
    const double* B;  // K x Dp: P mu_k
    const double* C;  // K: log w_k - mu_k^T P mu_k / 2
    int D, Dp, K;
};

// LDS image (in floats): rows k < D of P interleaved per lane ([k][lane][e],
// so a lane reads its EPL entries of row k in one access), then B [K][Dp]
// and C [K] as doubles (the P part has an even number of floats).
template <int EPL>
__host__ __device__ inline size_t mog_lds_floats(int D, int Dp, int K)
{
    return (size_t)D * 64 * EPL + 2 * ((size_t)K * Dp + (size_t)K);
}

template <int EPL>
__device__ __forceinline__ void mog_stage(const MogK& mk, float* sm)
{
    const int nP = mk.D * 64 * EPL;
    for (int i = threadIdx.x; i < nP; i += blockDim.x) {
        const int k = i / (64 * EPL), r = i - k * 64 * EPL, l = r / EPL, e = r - l * EPL;
        sm[i] = mk.P[(size_t)k * mk.Dp + e * 64 + l];
    }
    double* Bs = reinterpret_cast<double*>(sm + nP);
    for (int i = threadIdx.x; i < mk.K * mk.Dp; i += blockDim.x) Bs[i] = mk.B[i];
    double* Cs = Bs + mk.K * mk.Dp;
    for (int i = threadIdx.x; i < mk.K; i += blockDim.x) Cs[i] = mk.C[i];
    __syncthreads();
}

// Gradient policy of the NUTS step: U and grad U at th, from the LDS image.
struct MogGrad {
    const float* P;
    const double* B;
    const double* C;
    int D, Dp, K;

    template <int EPL>
    __device__ __forceinline__ void operator()(int, const WaveVec<EPL>& th, int lane, WaveVec<EPL>& g,
                                               float& U) const
    {
        double y[EPL];
#pragma unroll
        for (int e = 0; e < EPL; ++e) y[e] = 0.0;
        // y = P th: row k of P times th_k, k ascending; th_k read from lane k & 63
        // of register e = k / 64 (a scalar broadcast, no LDS traffic)
#pragma unroll
        for (int es = 0; es < EPL; ++es) {
            const int k0 = es * 64;
            const int kn = min(64, D - k0);
            const int thv = __float_as_int(th.r[es]);
            const float* pr = P + ((size_t)k0 * 64 + lane) * EPL;
#pragma unroll 4
            for (int l = 0; l < kn; ++l) {
                const double tk = (double)__int_as_float(__builtin_amdgcn_readlane(thv, l));
                const float* q = pr + (size_t)l * 64 * EPL;
#pragma unroll
                for (int e = 0; e < EPL; ++e) y[e] = fma((double)q[e], tk, y[e]);
            }
        }
        // s_0 = th . y and s_k = b_k . th, lane-local then one butterfly each
        double p0 = 0.0, pk[kMogMaxK];
#pragma unroll
        for (int e = 0; e < EPL; ++e) p0 += (double)th.r[e] * y[e];
#pragma unroll
        for (int kc = 0; kc < kMogMaxK; ++kc) {
            pk[kc] = 0.0;
            if (kc < K) {
#pragma unroll
                for (int e = 0; e < EPL; ++e) pk[kc] += B[kc * Dp + e * 64 + lane] * (double)th.r[e];
            }
        }
        const double s0 = uni(wave_sum(p0));
        double ak[kMogMaxK];
        double amax = -INFINITY;
#pragma unroll
        for (int kc = 0; kc < kMogMaxK; ++kc) {
            if (kc < K) {
                const double sk = uni(wave_sum(pk[kc]));
                ak[kc] = (C[kc] - 0.5 * s0) + sk;
                amax = fmax(amax, ak[kc]);
            }
        }
        double z = 0.0;
#pragma unroll
        for (int kc = 0; kc < kMogMaxK; ++kc)
            if (kc < K) z += exp(ak[kc] - amax);
        const double lse = amax + log(z);
        U = (float)(-lse);
#pragma unroll
        for (int kc = 0; kc < kMogMaxK; ++kc) {
            if (kc < K) {
                const double r = exp(ak[kc] - lse);
#pragma unroll
                for (int e = 0; e < EPL; ++e) y[e] -= r * B[kc * Dp + e * 64 + lane];
            }
        }
#pragma unroll
        for (int e = 0; e < EPL; ++e) g.r[e] = (float)y[e];
    }
};

template <int EPL>
__device__ __forceinline__ MogGrad mog_policy(const MogK& mk, const float* sm)
{
    const double* Bs = reinterpret_cast<const double*>(sm + (size_t)mk.D * 64 * EPL);
    return MogGrad{sm, Bs, Bs + (size_t)mk.K * mk.Dp, mk.D, mk.Dp, mk.K};
}

// Next chain of a persistent kernel: tickets count up across launches; this
// launch's tickets start at base (the host advances base by m + the launch's
// wavefronts after each launch: every wave takes one ticket past the end).
// Returns m when the tickets are used up.
__device__ __forceinline__ int mog_next_chain(unsigned long long* q, unsigned long long base, int m, int lane)
{
    unsigned long long tk = 0;
    if (lane == 0) tk = atomicAdd(q, 1ull);
    // every lane of the wave is active here: the first active lane is lane 0
    const unsigned long long off = (unsigned long long)uni((int64_t)tk) - base;
    return off < (unsigned long long)m ? (int)off : m;
}

// Persistent FSM kernel.  sync != 0: the launch is one draw of the
// synchronized runtime (a.tstop = draw + 1) and the draw's largest leapfrog
// count goes to maxN[draw].
template <int EPL>
__global__ __launch_bounds__(512) void nuts_mog_kernel(NutsK a, MogK mk, unsigned long long* q,
                                                      unsigned long long base, int sync)
{
    extern __shared__ float sm[];
    mog_stage<EPL>(mk, sm);
    const MogGrad G = mog_policy<EPL>(mk, sm);
    const int lane = threadIdx.x & 63;
    unsigned long long steps = 0;
    for (;;) {
        const int c = mog_next_chain(q, base, a.m, lane);
        if (c >= a.m) break;
        const uint32_t t = uni(a.t[c]);
        if (t >= a.tstop) continue;
        NutsScal S = nuts_load(a, c, t);
        int bits;
        do {
            bits = nuts_chain_body<EPL>(a, G, c, lane, S);
            steps += (bits & NC_REQ) ? 1ull : 0ull;
        } while (bits & NC_REQ);
        nuts_store(a, c, S, 0, lane);
        if (sync && lane == 0 && S.t > t) atomicMax(&a.maxN[t], S.nleap);
    }
    if (lane == 0 && steps) atomicAdd(&a.ctr[0], steps);
}

// vmap padding of draw `draw`: chain c evaluates maxN[draw] - N_c more
// gradients at its position and discards them (into sink).
template <int EPL>
__global__ __launch_bounds__(512) void nuts_mog_pad_kernel(NutsK a, MogK mk, unsigned long long* q,
                                                          unsigned long long base, uint32_t draw, float* sink)
{
    extern __shared__ float sm[];
    mog_stage<EPL>(mk, sm);
    const MogGrad G = mog_policy<EPL>(mk, sm);
    const int lane = threadIdx.x & 63;
    const int mx = a.maxN[draw];
    unsigned long long padded = 0;
    for (;;) {
        const int c = mog_next_chain(q, base, a.m, lane);
        if (c >= a.m) break;
        const int reps = mx - uni(a.counts[(size_t)c * a.n + draw]);
        if (reps <= 0) continue;
        WaveVec<EPL> th, g;
        th.load(a.V + ((size_t)c * a.nvec + V_THP) * a.Dp, lane);
        float acc = 0.0f;
        for (int r = 0; r < reps; ++r) {
            float U;
            G(c, th, lane, g, U);
            acc += g.r[0] + U;
        }
        if (lane == 0) sink[c] = acc;
        padded += (unsigned long long)reps;
    }
    if (lane == 0 && padded) atomicAdd(&a.ctr[1], padded);
}

// U and grad U at n points (wave per point): pts row stride ldp, G row
// stride ldg with the first gcols entries written, U stride ldu.
template <int EPL>
__global__ __launch_bounds__(512) void mog_eval_kernel(MogK mk, const float* pts, int ldp, int n, float* Gout,
                                                      int ldg, int gcols, float* Uout, int ldu)
{
    extern __shared__ float sm[];
    mog_stage<EPL>(mk, sm);
    const MogGrad G = mog_policy<EPL>(mk, sm);
    const int lane = threadIdx.x & 63;
    const int nw = (int)(gridDim.x * (blockDim.x >> 6));
    for (int i = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); i < n; i += nw) {
        WaveVec<EPL> th, g;
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            const int d = e * 64 + lane;
            th.r[e] = d < mk.D ? pts[(size_t)i * ldp + d] : 0.0f;
        }
        float U;
        G(i, th, lane, g, U);
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            const int d = e * 64 + lane;
            if (Gout && d < gcols) Gout[(size_t)i * ldg + d] = g.r[e];
        }
        if (lane == 0) Uout[(size_t)i * ldu] = U;
    }
}

// P mu_k and log w_k - mu_k^T P mu_k / 2 in FP64, one wave per component (k ascending).
__global__ void mog_setup_kernel(const float* P, const float* means, const float* logw, int D, int Dp, int K,
                                 double* B, double* C)
{
    const int kc = blockIdx.x, lane = threadIdx.x;
    if (kc >= K || lane >= 64) return;
    const float* mu = means + (size_t)kc * D;
    double part = 0.0;
    for (int d = lane; d < Dp; d += 64) {
        double s = 0.0;
        for (int k = 0; k < D; ++k) s = fma((double)P[(size_t)k * Dp + d], (double)mu[k], s);
        B[(size_t)kc * Dp + d] = s;
        if (d < D) part += s * (double)mu[d];
    }
    const double q = wave_sum(part);
    if (lane == 0) C[kc] = (double)logw[kc] - 0.5 * q;
}

// Default start theta0 ~ N(0, I) from the INIT stream.
__global__ void mog_normal_init_kernel(float* thp, int vstride, int m, int D, int Dp, uint64_t seed)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)m * Dp) return;
    const int c = (int)(i / Dp), d = (int)(i % Dp);
    thp[(size_t)c * vstride + d] = d < D ? normal_at<float>(seed, (uint32_t)c, 0, ROLE_INIT, 0, (uint32_t)d) : 0.0f;
}

// ------------------------------------------------------------ host side
static MogK mog_view(const JobDev& j)
{
    MogK mk;
    mk.P = (const float*)j.prec;
    mk.B = (const double*)j.mogB;
    mk.C = (const double*)j.mogC;
    mk.D = j.D;
    mk.Dp = j.Dp;
    mk.K = j.K;
    return mk;
}

static size_t mog_lds_bytes(const JobDev& j)
{
    return 4 * (j.EPL == 1 ? mog_lds_floats<1>(j.D, j.Dp, j.K) : mog_lds_floats<2>(j.D, j.Dp, j.K));
}

// Launch shape of the persistent kernels: waves per block grow with the
// chain count (one wave per block for small jobs, so chains spread over the
// CUs; 8 per block when the chip is full), blocks capped at what the chip
// holds at once (LDS bound).
static void mog_shape(JobDev& j)
{
    const int w = std::min(8, std::max(1, (j.m + 511) / 512));
    const int need = (j.m + w - 1) / w;
    const size_t lds = mog_lds_bytes(j);
    int per_cu = (int)std::min<size_t>(8, (160 * 1024) / std::max<size_t>(lds, 1));
    per_cu = std::max(per_cu, 1);
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    j.pwpb = w;
    j.pblocks = std::max(1, std::min(need, cus * per_cu));
}

hipError_t mog_setup(JobDev& j, hipStream_t s)
{
    mog_shape(j);
    const size_t lds = mog_lds_bytes(j);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)nuts_mog_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)nuts_mog_pad_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)mog_eval_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(mog_setup_kernel, dim3(j.K), dim3(64), 0, s, (const float*)j.prec, (const float*)j.X,
                       (const float*)j.y, j.D, j.Dp, j.K, (double*)j.mogB, (double*)j.mogC);
    return hipGetLastError();
}

hipError_t mog_eval(const JobDev& j, int n, const float* pts, int ldp, float* G, int ldg, int gcols, float* U,
                    int ldu, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const MogK mk = mog_view(j);
    const int blocks = std::min((n + 7) / 8, 2048);
    const size_t lds = mog_lds_bytes(j);
    if (j.EPL == 1)
        hipLaunchKernelGGL(mog_eval_kernel<1>, dim3(blocks), dim3(512), lds, s, mk, pts, ldp, n, G, ldg, gcols, U, ldu);
    else
        hipLaunchKernelGGL(mog_eval_kernel<2>, dim3(blocks), dim3(512), lds, s, mk, pts, ldp, n, G, ldg, gcols, U, ldu);
    return hipGetLastError();
}

hipError_t mog_eval(const JobDev& j, int n, const float* pts, float* G, float* U, hipStream_t s)
{
    return mog_eval(j, n, pts, j.D, G, j.D, j.D, U, 1, s);
}

hipError_t mog_init_state(const JobDev& j, const void* x0, hipStream_t s)
{
    float* thp = (float*)j.V + (size_t)V_THP * j.Dp;
    const int vstride = j.nvec * j.Dp;
    hipError_t e;
    if (x0) {
        e = hipMemcpy2DAsync(thp, (size_t)vstride * 4, x0, (size_t)j.D * 4, (size_t)j.D * 4, j.m,
                             hipMemcpyDeviceToDevice, s);
    } else {
        const size_t tot = (size_t)j.m * j.Dp;
        hipLaunchKernelGGL(mog_normal_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, thp, vstride,
                           j.m, j.D, j.Dp, j.seed);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    // U and grad U at the start, straight into the proposal slots (gP, UP)
    float* gp = (float*)j.V + (size_t)V_GP * j.Dp;
    return mog_eval(j, j.m, thp, vstride, gp, vstride, j.Dp, (float*)j.lx, 1, s);
}

hipError_t mog_run(const JobDev& j, int sync, uint32_t draw, unsigned long long* ticket, hipStream_t s)
{
    NutsK a = nuts_view(j, 0, 0);
    if (sync) a.tstop = draw + 1;
    const MogK mk = mog_view(j);
    const int wpb = j.pwpb, blocks = j.pblocks;
    const size_t lds = mog_lds_bytes(j);
    unsigned long long* q = (unsigned long long*)j.queue;
    if (j.EPL == 1)
        hipLaunchKernelGGL(nuts_mog_kernel<1>, dim3(blocks), dim3(64 * wpb), lds, s, a, mk, q, *ticket, sync);
    else
        hipLaunchKernelGGL(nuts_mog_kernel<2>, dim3(blocks), dim3(64 * wpb), lds, s, a, mk, q, *ticket, sync);
    *ticket += (unsigned long long)j.m + (unsigned long long)blocks * wpb;
    return hipGetLastError();
}

hipError_t mog_pad(const JobDev& j, uint32_t draw, unsigned long long* ticket, hipStream_t s)
{
    NutsK a = nuts_view(j, 0, 0);
    const MogK mk = mog_view(j);
    const int wpb = j.pwpb, blocks = j.pblocks;
    const size_t lds = mog_lds_bytes(j);
    unsigned long long* q = (unsigned long long*)j.queue;
    if (j.EPL == 1)
        hipLaunchKernelGGL(nuts_mog_pad_kernel<1>, dim3(blocks), dim3(64 * wpb), lds, s, a, mk, q, *ticket, draw,
                           (float*)j.sink);
    else
        hipLaunchKernelGGL(nuts_mog_pad_kernel<2>, dim3(blocks), dim3(64 * wpb), lds, s, a, mk, q, *ticket, draw,
                           (float*)j.sink);
    *ticket += (unsigned long long)j.m + (unsigned long long)blocks * wpb;
    return hipGetLastError();
}

}  // namespace fsmmc
