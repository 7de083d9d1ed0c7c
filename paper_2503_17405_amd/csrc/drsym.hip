// drsym.hip -- symmetric delayed rejection (Mira 2001; Sec. 7.1): up to M
// tries per draw, each proposal re-centred on the previous rejected one,
//   y_0 = x + sigma z_0,  y_s = y_{s-1} + sigma z_s,
// accepted with probability
//   alpha_s = min(1, max(0, pi(y_s) - pi*_s) / (pi(x) - pi*_s)),
//   pi*_s = max_{j<s} pi(y_j)  (pi*_0 = 0: alpha_0 is the Metropolis ratio);
// after M rejections x is kept.  Densities enter relative to pi(x)
// (l = log pi): alpha_s = (e^(ly - lx) - e^(l* - lx)) / (-expm1(l* - lx)),
// so nothing is exponentiated but differences.
//
// One lane per chain; the chain's x, the current centre c, the pending
// proposal y and their log densities live in registers; state in HBM is
// [field][d][chain].  Two FSMs of the same sampler (Sec. 7.1's ablation):
//   * condensed (fsm_states = 1): INIT and DONE are empty, so the whole loop
//     body -- propose, evaluate, test, re-centre or finish -- is one state;
//     one FSM step = one try;
//   * split (fsm_states = 4): the loop body as four states PROPOSE, EVAL,
//     TEST, NEXT, one per FSM step.  Lanes of a wave sit in different states,
//     so a wave runs each present state's code with the other lanes masked:
//     the cost of not bundling (Sec. 5.1).
// Both run the same device functions in the same order for each chain, so
// they, and the synchronized runtime, give the same bits.
#include "dr_device.h"

namespace fsmmc {

struct DrsK {
    DrK pd;  // density parameters only (target, D, prec)
    int m, n, D, M, split;
    uint32_t tstop;
    uint64_t seed;
    float sigma;
    float *x, *c, *y;          // [d][chain]
    float *lx, *lstar, *ly;    // [chain]
    int32_t *s, *sub, *acc;    // tries so far in the draw, sub-state (split), test outcome
    uint32_t* t;
    int64_t* budget;
    float* out;
    int32_t* counts;
    unsigned long long* ctr;
    int32_t* maxN;
    float* sink;
};

template <int NM>
struct DrsLane {
    float x[NM], c[NM], y[NM];
    float lx, lstar, ly;
    int s, sub, acc;
    uint32_t t;
};

template <int NM>
__device__ __forceinline__ void drs_load(const DrsK& a, int c, DrsLane<NM>& L)
{
#pragma unroll
    for (int d = 0; d < NM; ++d) {
        const bool in = d < a.D;
        L.x[d] = in ? a.x[(size_t)d * a.m + c] : 0.0f;
        L.c[d] = in ? a.c[(size_t)d * a.m + c] : 0.0f;
        L.y[d] = in ? a.y[(size_t)d * a.m + c] : 0.0f;
    }
    L.lx = a.lx[c];
    L.lstar = a.lstar[c];
    L.ly = a.ly[c];
    L.s = a.s[c];
    L.sub = a.sub[c];
    L.acc = a.acc[c];
    L.t = a.t[c];
}

template <int NM>
__device__ __forceinline__ void drs_store(const DrsK& a, int c, const DrsLane<NM>& L)
{
#pragma unroll
    for (int d = 0; d < NM; ++d) {
        if (d < a.D) {
            a.x[(size_t)d * a.m + c] = L.x[d];
            a.c[(size_t)d * a.m + c] = L.c[d];
            a.y[(size_t)d * a.m + c] = L.y[d];
        }
    }
    a.lx[c] = L.lx;
    a.lstar[c] = L.lstar;
    a.ly[c] = L.ly;
    a.s[c] = L.s;
    a.sub[c] = L.sub;
    a.acc[c] = L.acc;
    a.t[c] = L.t;
}

// alpha_s from log pi(x), log pi(y_s), log pi*_s.  Every rejected proposal
// lies below x (alpha < 1 needs pi(y) < pi(x)), so l* < lx; l* = lx can only
// come from rounding and then alpha is 1 above x and 0 otherwise.  The
// numerator e^(ly - lx) - e^(l* - lx) is formed as e^(l* - lx) expm1(ly - l*)
// when the two are within a factor e (no cancellation), else as the plain
// difference (no overflow of expm1, no 0 * inf when e^(l* - lx) underflows).
__device__ __forceinline__ float drs_alpha(float lx, float ly, float lstar)
{
    if (!(ly > lstar)) return 0.0f;
    const float dm = lstar - lx;
    if (dm == -INFINITY) return fminf(1.0f, expf(ly - lx));
    if (!(dm < 0.0f)) return 1.0f;
    const float gap = ly - lstar;
    const float num = gap < 1.0f ? expf(dm) * expm1f(gap) : expf(ly - lx) - expf(dm);
    return fminf(num / (-expm1f(dm)), 1.0f);
}

// PROPOSE: y = c + sigma z(PROP, s)
template <int NM>
__device__ __forceinline__ void drs_propose(const DrsK& a, int c, DrsLane<NM>& L)
{
#pragma unroll
    for (int b = 0; b < NM / 4; ++b) {
        float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (4 * b < a.D) normals4<float>(a.seed, (uint32_t)c, L.t, ROLE_PROP, (uint32_t)L.s, (uint32_t)b, z);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int d = 4 * b + i;
            L.y[d] = d < a.D ? L.c[d] + a.sigma * z[i] : 0.0f;
        }
    }
}

// EVAL: log pi(y)
template <int NM>
__device__ __forceinline__ void drs_eval(const DrsK& a, DrsLane<NM>& L)
{
    L.ly = dr_logpdf<NM>(a.pd, L.y);
}

// TEST: u(ACC, s) < alpha_s
template <int NM>
__device__ __forceinline__ void drs_test(const DrsK& a, int c, DrsLane<NM>& L)
{
    const float u = uniform<float>(a.seed, (uint32_t)c, L.t, ROLE_ACC, (uint32_t)L.s);
    L.acc = u < drs_alpha(L.lx, L.ly, L.lstar) ? 1 : 0;
}

// NEXT: accept and finish, finish after the M-th rejection, or re-centre on
// y.  A finished draw is emitted (DONE) and the next one set up (INIT).
// Returns 1 when the draw ended.
template <int NM>
__device__ __forceinline__ int drs_next(const DrsK& a, int c, DrsLane<NM>& L)
{
    const bool acc = L.acc != 0;
    L.s += 1;
    const bool end = acc || L.s >= a.M;
#pragma unroll
    for (int d = 0; d < NM; ++d) L.x[d] = acc ? L.y[d] : L.x[d];
    L.lx = acc ? L.ly : L.lx;
    L.lstar = end ? -INFINITY : fmaxf(L.lstar, L.ly);
#pragma unroll
    for (int d = 0; d < NM; ++d) L.c[d] = end ? L.x[d] : L.y[d];
    if (end) {
        float* o = a.out + ((size_t)c * a.n + L.t) * a.D;
#pragma unroll
        for (int d = 0; d < NM; ++d)
            if (d < a.D) o[d] = L.x[d];
        a.counts[(size_t)c * a.n + L.t] = L.s;
        L.t += 1;
        L.s = 0;
    }
    L.acc = 0;
    return end ? 1 : 0;
}

// One FSM step of the lane's chain.  Returns 1 when it ended a draw.
template <int NM, bool SPLIT>
__device__ __forceinline__ int drs_step(const DrsK& a, int c, DrsLane<NM>& L)
{
    if (!SPLIT) {
        drs_propose<NM>(a, c, L);
        drs_eval<NM>(a, L);
        drs_test<NM>(a, c, L);
        return drs_next<NM>(a, c, L);
    }
    const int k = L.sub;
    L.sub = (k + 1) & 3;
    if (k == 0) {
        drs_propose<NM>(a, c, L);
    } else if (k == 1) {
        drs_eval<NM>(a, L);
    } else if (k == 2) {
        drs_test<NM>(a, c, L);
    } else {
        return drs_next<NM>(a, c, L);
    }
    return 0;
}

// FSM runtime: every lane runs its chain to tstop or through its budget;
// lane occupancy counted as for the other lane-per-chain kernels.
template <int NM, bool SPLIT>
__global__ __launch_bounds__(256) void drs_fsm_kernel(DrsK a)
{
    __shared__ unsigned long long s_sum;
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    uint32_t steps = 0, live = 0;
    if (c < a.m) {
        DrsLane<NM> L;
        drs_load<NM>(a, c, L);
        int64_t budget = a.budget[c];
        const uint32_t stop = min(a.tstop, (uint32_t)a.n);
        while (L.t < stop && budget > 0) {
            (void)drs_step<NM, SPLIT>(a, c, L);
            ++steps;
            --budget;
        }
        drs_store<NM>(a, c, L);
        a.budget[c] = budget;
        live = L.t < (uint32_t)a.n ? 1u : 0u;
    }
    const unsigned long long st = block_sum_u64(wave_sum_u64(steps), &s_sum);
    if (threadIdx.x == 0 && st) atomicAdd(&a.ctr[0], st);
    const unsigned long long lv = block_sum_u64(wave_sum_u64(live), &s_sum);
    if (threadIdx.x == 0 && lv) atomicAdd(&a.ctr[4], lv);
    dr_count_lanes(a.pd, steps, steps, &s_sum);
}

// Synchronized runtime: draw `draw` of every chain (condensed body); the
// draw's largest try count goes to maxN[draw].
template <int NM>
__global__ __launch_bounds__(256) void drs_sync_kernel(DrsK a, uint32_t draw)
{
    __shared__ unsigned long long s_sum;
    __shared__ int s_max;
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    uint32_t steps = 0;
    if (c < a.m) {
        DrsLane<NM> L;
        drs_load<NM>(a, c, L);
        while (L.t <= draw) {
            (void)drs_step<NM, false>(a, c, L);
            ++steps;  // one try per step: the loop runs exactly the draw's tries
        }
        drs_store<NM>(a, c, L);
    }
    const int tries = (int)steps;
    const int mx = block_max_i32(wave_max_i32(tries), &s_max);
    if (threadIdx.x == 0) atomicMax(&a.maxN[draw], mx);
    const unsigned long long st = block_sum_u64(wave_sum_u64(steps), &s_sum);
    if (threadIdx.x == 0 && st) atomicAdd(&a.ctr[0], st);
    dr_count_lanes(a.pd, steps, steps, &s_sum);
}

// vmap padding of draw `draw`: the max_j N_j - N_j try bodies (propose,
// evaluate, test) a batched while loop runs after chain c has finished,
// computed and discarded.
template <int NM>
__global__ __launch_bounds__(256) void drs_pad_kernel(DrsK a, uint32_t draw)
{
    __shared__ unsigned long long s_sum;
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    int extra = 0;
    if (c < a.m) {
        const int done = a.counts[(size_t)c * a.n + draw];
        extra = a.maxN[draw] - done;
        if (extra > 0) {
            DrsLane<NM> L;
            drs_load<NM>(a, c, L);
            L.t = draw;
            float sink = 0.0f;
            for (int i = 0; i < extra; ++i) {
                L.s = done + i;
                drs_propose<NM>(a, c, L);
                drs_eval<NM>(a, L);
                drs_test<NM>(a, c, L);
                sink += L.ly + (float)L.acc;
            }
            a.sink[c] = sink;
        }
    }
    const unsigned long long tot = block_sum_u64(wave_sum_u64((unsigned long long)max(extra, 0)), &s_sum);
    if (threadIdx.x == 0 && tot) atomicAdd(&a.ctr[1], tot);
    dr_count_lanes(a.pd, 0u, (uint32_t)max(extra, 0), &s_sum);
}

// Starts: x (already [d][chain], from x0 or the default draw of dr_init_state)
// -> centre c = x, log pi*, sub-state, test outcome.
__global__ void drs_init_kernel(DrsK a)
{
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= a.m) return;
    for (int d = 0; d < a.D; ++d) a.c[(size_t)d * a.m + c] = a.x[(size_t)d * a.m + c];
    a.lstar[c] = -INFINITY;
    a.s[c] = 0;
    a.sub[c] = 0;
    a.acc[c] = 0;
}

// ------------------------------------------------------------ host side
static DrsK drs_view(const JobDev& j)
{
    DrsK a;
    a.pd = dr_view(j);
    a.m = j.m;
    a.n = j.n;
    a.D = j.D;
    a.M = j.n_stages;
    a.split = j.fsm_states == 4 ? 1 : 0;
    a.tstop = j.tstop;
    a.seed = j.seed;
    a.sigma = (float)j.scales[0];
    a.x = (float*)j.x;
    a.c = (float*)j.V;
    a.y = (float*)j.V + (size_t)j.m * j.D;
    a.lx = (float*)j.lx;
    a.lstar = (float*)j.H0;
    a.ly = (float*)j.Wsum;
    a.s = j.evals;
    a.sub = j.k;
    a.acc = j.flags;
    a.t = j.t;
    a.budget = j.budget;
    a.out = (float*)j.out;
    a.counts = j.counts;
    a.ctr = j.ctr;
    a.maxN = j.maxN;
    a.sink = (float*)j.sink;
    return a;
}

hipError_t drs_init_state(const JobDev& j, const void* x0, hipStream_t s)
{
    hipError_t e = dr_init_state(j, x0, s);  // x in [d][chain] and log pi(x)
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(drs_init_kernel, dim3((j.m + 255) / 256), dim3(256), 0, s, drs_view(j));
    return hipGetLastError();
}

#define FSMMC_DRS_DISPATCH(KERNEL, D_, ...)                                          \
    if ((D_) <= 4)                                                                 \
        hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__);                                \
    else if ((D_) <= 8)                                                            \
        hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__);                                \
    else if ((D_) <= 12)                                                           \
        hipLaunchKernelGGL(KERNEL<12>, __VA_ARGS__);                               \
    else                                                                           \
        hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__);

template <int NM>
static void drs_fsm_launch(const DrsK& a, hipStream_t s)
{
    const dim3 grid((a.m + 255) / 256), block(256);
    if (a.split)
        hipLaunchKernelGGL((drs_fsm_kernel<NM, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((drs_fsm_kernel<NM, false>), grid, block, 0, s, a);
}

hipError_t drs_fsm_round(const JobDev& j, hipStream_t s)
{
    const DrsK a = drs_view(j);
    if (j.D <= 4)
        drs_fsm_launch<4>(a, s);
    else if (j.D <= 8)
        drs_fsm_launch<8>(a, s);
    else if (j.D <= 12)
        drs_fsm_launch<12>(a, s);
    else
        drs_fsm_launch<16>(a, s);
    return hipGetLastError();
}

hipError_t drs_sync_draw(const JobDev& j, uint32_t draw, hipStream_t s)
{
    const DrsK a = drs_view(j);
    FSMMC_DRS_DISPATCH(drs_sync_kernel, j.D, dim3((j.m + 255) / 256), dim3(256), 0, s, a, draw)
    return hipGetLastError();
}

hipError_t drs_pad_draw(const JobDev& j, uint32_t draw, hipStream_t s)
{
    const DrsK a = drs_view(j);
    FSMMC_DRS_DISPATCH(drs_pad_kernel, j.D, dim3((j.m + 255) / 256), dim3(256), 0, s, a, draw)
    return hipGetLastError();
}

}  // namespace fsmmc
