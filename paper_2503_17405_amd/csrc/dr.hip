// dr.hip -- delayed-rejection Metropolis-Hastings with up to three proposal
// stages (Tierney & Mira 1999; Mira 2001) as an FSM (Sec. 3.1, Fig. "Finite
// state machines ...", delayed-rejection panel: INIT, PROPOSE, DONE; Sec. 7.1:
// INIT and DONE are nearly empty, so one bundled state per step).
//
// One lane per chain: the chain's state (x, the rejected proposals y1, y2 and
// their log densities) lives in registers for the whole launch.
//   * dr_fsm_kernel: every lane runs its own FSM; one step = one proposal
//     stage (draw y_s = x + scale_s z_s, log pi(y_s), alpha_s, accept / next
//     stage / reject) with DONE and the next INIT bundled into the step that
//     ends a draw.  Lanes of a wave are at different draws and stages; the
//     wave keeps going while any lane has work.
//   * dr_sync_kernel: one draw of every chain per launch (the draw barrier);
//     dr_pad_kernel adds, in vmap mode, the max_j N_j - N_j stage bodies of a
//     batched while loop.
// Reading: every stage centred at the current state x; log alpha in log space
// with the reverse-path factors; a zero factor of the reverse path gives
// alpha_3 = 0 before the bounded factor 1 - alpha_2(y3, y2, y1) is formed.
#include "dr_device.h"

namespace fsmmc {

// Counters are summed per wave and block: one atomic per block and counter.
template <int NM>
__global__ __launch_bounds__(256) void dr_fsm_kernel(DrK a)
{
    __shared__ unsigned long long s_sum;
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    uint32_t steps = 0, live = 0;
    if (c < a.m) (void)dr_run<NM>(a, c, a.tstop, &steps, &live);
    const unsigned long long st = block_sum_u64(wave_sum_u64(steps), &s_sum);
    if (threadIdx.x == 0 && st) atomicAdd(&a.ctr[0], st);
    const unsigned long long lv = block_sum_u64(wave_sum_u64(live), &s_sum);
    if (threadIdx.x == 0 && lv) atomicAdd(&a.ctr[4], lv);
    dr_count_lanes(a, steps, steps, &s_sum);
}

template <int NM>
__device__ __forceinline__ int dr_sync_one(const DrK& a, int c, uint32_t draw, int* stages)
{
    DrLane<NM> L;
    dr_load<NM>(a, c, L);
    int steps = 0;
    for (;;) {
        const int end = dr_stage<NM>(a, c, L);
        ++steps;
        if (end) break;
    }
    *stages = L.s;
    dr_emit<NM>(a, c, L);
    dr_store<NM>(a, c, L);
    return steps;
}

template <int NM>
__global__ __launch_bounds__(256) void dr_sync_kernel(DrK a, uint32_t draw)
{
    __shared__ unsigned long long s_sum;
    __shared__ int s_max;
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    int steps = 0, stages = 0;
    if (c < a.m) steps = dr_sync_one<NM>(a, c, draw, &stages);
    const int mx = block_max_i32(wave_max_i32(stages), &s_max);
    if (threadIdx.x == 0) atomicMax(&a.maxN[draw], mx);
    const unsigned long long st = block_sum_u64(wave_sum_u64((unsigned long long)steps), &s_sum);
    if (threadIdx.x == 0 && st) atomicAdd(&a.ctr[0], st);
    dr_count_lanes(a, (uint32_t)steps, (uint32_t)steps, &s_sum);
}

// The stage bodies a batched while loop runs after chain c has finished
// draw `draw`: proposal, density and acceptance, discarded.
template <int NM>
__device__ __forceinline__ int dr_pad_one(const DrK& a, int c, uint32_t draw)
{
    const int done = a.counts[(size_t)c * a.n + draw];
    const int extra = a.maxN[draw] - done;
    if (extra <= 0) return 0;
    DrLane<NM> L;
    dr_load<NM>(a, c, L);
    L.t = draw;
    float acc = 0.0f;
    for (int i = 0; i < extra; ++i) {
        L.s = min(done + i, a.n_stages - 1);
        float y[NM];
        dr_propose<NM>(a, c, L, y);
        acc += dr_logpdf<NM>(a, y) + logf(uniform<float>(a.seed, (uint32_t)c, draw, ROLE_ACC, (uint32_t)L.s));
    }
    a.sink[c] = acc;
    return extra;
}

template <int NM>
__global__ __launch_bounds__(256) void dr_pad_kernel(DrK a, uint32_t draw)
{
    __shared__ unsigned long long s_sum;
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    int extra = 0;
    if (c < a.m) extra = dr_pad_one<NM>(a, c, draw);
    const unsigned long long tot = block_sum_u64(wave_sum_u64((unsigned long long)extra), &s_sum);
    if (threadIdx.x == 0 && tot) atomicAdd(&a.ctr[1], tot);
    dr_count_lanes(a, 0u, (uint32_t)extra, &s_sum);  // discarded bodies: slots, no useful lanes
}

// Default starts: an exact funnel draw (v = 3 z0, x_i = e^{v/2} z_i) or N(0, I).
__global__ void dr_init_kernel(DrK a, int has_x0)
{
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= a.m) return;
    float v[kDrMaxDim];
    for (int d = 0; d < kDrMaxDim; ++d) v[d] = 0.0f;
    if (has_x0) {
        for (int d = 0; d < a.D; ++d) v[d] = a.x[(size_t)d * a.m + c];
    } else {
        for (int d = 0; d < a.D; ++d) v[d] = normal_at<float>(a.seed, (uint32_t)c, 0, ROLE_INIT, 0, (uint32_t)d);
        if (a.target == FSMMC_FUNNEL) {
            v[0] = 3.0f * v[0];
            const float s = expf(0.5f * v[0]);
            for (int d = 1; d < a.D; ++d) v[d] = s * v[d];
        }
        for (int d = 0; d < a.D; ++d) a.x[(size_t)d * a.m + c] = v[d];
    }
    a.lx[c] = dr_logpdf<kDrMaxDim>(a, v);
}

// x0 given chain-major (m x D) -> [d][chain].
__global__ void dr_transpose_kernel(const float* x0, float* x, int m, int D)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= m * D) return;
    const int c = i / D, d = i - c * D;
    x[(size_t)d * m + c] = x0[i];
}

// ------------------------------------------------------------ host side
int dr_max_dim() { return kDrMaxDim; }

hipError_t dr_init_state(const JobDev& j, const void* x0, hipStream_t s)
{
    DrK a = dr_view(j);
    const dim3 grid((j.m + 255) / 256), block(256);
    if (x0) {
        hipLaunchKernelGGL(dr_transpose_kernel, dim3((j.m * j.D + 255) / 256), block, 0, s, (const float*)x0,
                           (float*)j.x, j.m, j.D);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(dr_init_kernel, grid, block, 0, s, a, x0 ? 1 : 0);
    return hipGetLastError();
}

// Kernels are instantiated for dimension bounds 4, 8, 12 and 16 so the lane
// state stays in registers.
#define FSMMC_DR_DISPATCH(KERNEL, D_, ...)                                           \
    if ((D_) <= 4)                                                                 \
        hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__);                                \
    else if ((D_) <= 8)                                                            \
        hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__);                                \
    else if ((D_) <= 12)                                                           \
        hipLaunchKernelGGL(KERNEL<12>, __VA_ARGS__);                               \
    else                                                                           \
        hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__);

hipError_t dr_fsm_round(const JobDev& j, hipStream_t s)
{
    DrK a = dr_view(j);
    FSMMC_DR_DISPATCH(dr_fsm_kernel, j.D, dim3((j.m + 255) / 256), dim3(256), 0, s, a)
    return hipGetLastError();
}

hipError_t dr_sync_draw(const JobDev& j, uint32_t draw, hipStream_t s)
{
    DrK a = dr_view(j);
    FSMMC_DR_DISPATCH(dr_sync_kernel, j.D, dim3((j.m + 255) / 256), dim3(256), 0, s, a, draw)
    return hipGetLastError();
}

hipError_t dr_pad_draw(const JobDev& j, uint32_t draw, hipStream_t s)
{
    DrK a = dr_view(j);
    FSMMC_DR_DISPATCH(dr_pad_kernel, j.D, dim3((j.m + 255) / 256), dim3(256), 0, s, a, draw)
    return hipGetLastError();
}

}  // namespace fsmmc
