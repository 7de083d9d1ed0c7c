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
#include "fsmmc_device.h"
#include "fsmmc_internal.h"

namespace fsmmc {

constexpr int kDrMaxDim = 16;

struct DrK {
    int m, n, D, target, n_stages;
    uint32_t tstop;
    uint64_t seed;
    float sc[3];
    const float* prec;  // GAUSS_DIAG precisions (D)
    // state, [field][d][chain] / [chain]
    float *x, *y1, *y2, *lx, *l1, *l2;
    int32_t* s;
    uint32_t* t;
    int64_t* budget;
    float* out;
    int32_t* counts;
    unsigned long long* ctr;
    int32_t* maxN;
    float* sink;
};

// log pi (up to a constant).  Entries d >= D of every lane vector are zero.
template <int NM>
__device__ __forceinline__ float dr_logpdf(const DrK& a, const float* v)
{
    if (a.target == FSMMC_FUNNEL) {
        float ss = 0.0f;
#pragma unroll
        for (int d = 1; d < NM; ++d) ss += v[d] * v[d];
        const float u = v[0];
        return -(u * u) / 18.0f - 0.5f * (float)(a.D - 1) * u - 0.5f * expf(-u) * ss;
    }
    float s = 0.0f;
#pragma unroll
    for (int d = 0; d < NM; ++d) s += (d < a.D ? a.prec[d] : 0.0f) * v[d] * v[d];
    return -0.5f * s;
}

// log(1 - e^a), a <= 0 (Maechler 2012).
__device__ __forceinline__ float log1mexp_f(float a)
{
    return a > -0.69314718f ? logf(-expm1f(a)) : log1pf(-expf(a));
}

// log min(1, e^d); NaN stays NaN (never accepts).
__device__ __forceinline__ float log_min1(float d) { return d >= 0.0f ? 0.0f : d; }

template <int NM>
__device__ __forceinline__ float lq(const float* a, const float* b, int D, float sc)
{
    float s = 0.0f;
#pragma unroll
    for (int d = 0; d < NM; ++d) {
        const float r = b[d] - a[d];
        s += r * r;
    }
    return -s / (2.0f * sc * sc);
}

// log alpha_2(a, b, c): from a, b rejected at stage 1, c proposed at stage 2.
__device__ __forceinline__ float dr_la2(float la, float lb, float lc, float lq1_ab, float lq1_cb)
{
    const float num = lc + lq1_cb + log1mexp_f(log_min1(lb - lc));
    const float den = la + lq1_ab + log1mexp_f(log_min1(lb - la));
    return log_min1(num - den);
}

// log alpha of stage s (0-based) for x -> y_s given the earlier rejections.
template <int NM>
__device__ __forceinline__ float dr_log_alpha(const DrK& a, int s, const float* x, const float* y1, const float* y2,
                                              const float* y3, float lx, float l1, float l2, float l3)
{
    const int D = a.D;
    if (s == 0) return log_min1(l1 - lx);
    if (s == 1) return dr_la2(lx, l1, l2, lq<NM>(x, y1, D, a.sc[0]), lq<NM>(y2, y1, D, a.sc[0]));
    const float q0 = lq<NM>(x, y1, D, a.sc[0]);   // q1(x -> y1)
    const float q1 = lq<NM>(y2, y1, D, a.sc[0]);  // q1(y2 -> y1)
    const float q2 = lq<NM>(x, y2, D, a.sc[1]);   // q2(x -> y2)
    const float q3 = lq<NM>(y3, y2, D, a.sc[0]);  // q1(y3 -> y2)
    const float q4 = lq<NM>(y3, y1, D, a.sc[1]);  // q2(y3 -> y1)
    const float q5 = lq<NM>(y1, y2, D, a.sc[0]);  // q1(y1 -> y2)
    const float la1_x1 = log_min1(l1 - lx);
    const float la2_x12 = dr_la2(lx, l1, l2, q0, q1);
    const float la1_32 = log_min1(l2 - l3);
    const float part = q3 + q4 + log1mexp_f(la1_32);
    if (part == -INFINITY) return -INFINITY;
    const float la2_321 = dr_la2(l3, l2, l1, q3, q5);
    const float num = l3 + part + log1mexp_f(la2_321);
    const float den = lx + q0 + q2 + log1mexp_f(la1_x1) + log1mexp_f(la2_x12);
    return log_min1(num - den);
}

template <int NM>
struct DrLane {
    float x[NM], y1[NM], y2[NM];
    float lx, l1, l2;
    int s;
    uint32_t t;
};

template <int NM>
__device__ __forceinline__ void dr_load(const DrK& a, int c, DrLane<NM>& L)
{
#pragma unroll
    for (int d = 0; d < NM; ++d) {
        const bool in = d < a.D;
        L.x[d] = in ? a.x[(size_t)d * a.m + c] : 0.0f;
        L.y1[d] = in ? a.y1[(size_t)d * a.m + c] : 0.0f;
        L.y2[d] = in ? a.y2[(size_t)d * a.m + c] : 0.0f;
    }
    L.lx = a.lx[c];
    L.l1 = a.l1[c];
    L.l2 = a.l2[c];
    L.s = a.s[c];
    L.t = a.t[c];
}

template <int NM>
__device__ __forceinline__ void dr_store(const DrK& a, int c, const DrLane<NM>& L)
{
#pragma unroll
    for (int d = 0; d < NM; ++d) {
        if (d < a.D) {
            a.x[(size_t)d * a.m + c] = L.x[d];
            a.y1[(size_t)d * a.m + c] = L.y1[d];
            a.y2[(size_t)d * a.m + c] = L.y2[d];
        }
    }
    a.lx[c] = L.lx;
    a.l1[c] = L.l1;
    a.l2[c] = L.l2;
    a.s[c] = L.s;
    a.t[c] = L.t;
}

// Draw y_s = x + scale_s z_s into y.
template <int NM>
__device__ __forceinline__ void dr_propose(const DrK& a, int c, const DrLane<NM>& L, float* y)
{
    const int s = L.s;
    const float sc = s == 0 ? a.sc[0] : (s == 1 ? a.sc[1] : a.sc[2]);
#pragma unroll
    for (int b = 0; b < NM / 4; ++b) {
        float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (4 * b < a.D) normals4<float>(a.seed, (uint32_t)c, L.t, ROLE_PROP, (uint32_t)s, (uint32_t)b, z);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int d = 4 * b + i;
            y[d] = d < a.D ? L.x[d] + sc * z[i] : 0.0f;
        }
    }
}

// One PROPOSE stage.  Returns 1 when the draw ends (accepted or last stage).
template <int NM>
__device__ __forceinline__ int dr_stage(const DrK& a, int c, DrLane<NM>& L)
{
    float y[NM];
    dr_propose<NM>(a, c, L, y);
    const float ly = dr_logpdf<NM>(a, y);
    const int s = L.s;
    float la;
    if (s == 0) {
        la = log_min1(ly - L.lx);
    } else if (s == 1) {
        la = dr_la2(L.lx, L.l1, ly, lq<NM>(L.x, L.y1, a.D, a.sc[0]), lq<NM>(y, L.y1, a.D, a.sc[0]));
    } else {
        la = dr_log_alpha<NM>(a, 2, L.x, L.y1, L.y2, y, L.lx, L.l1, L.l2, ly);
    }
    const float u = uniform<float>(a.seed, (uint32_t)c, L.t, ROLE_ACC, (uint32_t)s);
    // value selects (no branches around the array writes keep them in registers)
    const bool acc = logf(u) < la;
    const bool to1 = !acc && s == 0, to2 = !acc && s == 1;
#pragma unroll
    for (int d = 0; d < NM; ++d) {
        L.x[d] = acc ? y[d] : L.x[d];
        L.y1[d] = to1 ? y[d] : L.y1[d];
        L.y2[d] = to2 ? y[d] : L.y2[d];
    }
    L.lx = acc ? ly : L.lx;
    L.l1 = to1 ? ly : L.l1;
    L.l2 = to2 ? ly : L.l2;
    L.s = s + 1;
    return acc || L.s >= a.n_stages;
}

// DONE: emit x as draw t; the stage count is the draw's loop count.
template <int NM>
__device__ __forceinline__ void dr_emit(const DrK& a, int c, DrLane<NM>& L)
{
    float* o = a.out + ((size_t)c * a.n + L.t) * a.D;
#pragma unroll
    for (int d = 0; d < NM; ++d)
        if (d < a.D) o[d] = L.x[d];
    a.counts[(size_t)c * a.n + L.t] = L.s;
    L.t += 1;
    L.s = 0;
}

template <int NM>
__global__ __launch_bounds__(256) void dr_fsm_kernel(DrK a)
{
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= a.m) return;
    DrLane<NM> L;
    dr_load<NM>(a, c, L);
    int64_t budget = a.budget[c];
    unsigned long long steps = 0;
    while (L.t < a.tstop && budget > 0) {
        const int end = dr_stage<NM>(a, c, L);
        ++steps;
        --budget;
        if (end) dr_emit<NM>(a, c, L);
    }
    dr_store<NM>(a, c, L);
    a.budget[c] = budget;
    atomicAdd(&a.ctr[0], steps);
    if (L.t < a.tstop) atomicAdd(&a.ctr[4], 1ull);
}

template <int NM>
__global__ __launch_bounds__(256) void dr_sync_kernel(DrK a, uint32_t draw)
{
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= a.m) return;
    DrLane<NM> L;
    dr_load<NM>(a, c, L);
    int steps = 0;
    for (;;) {
        const int end = dr_stage<NM>(a, c, L);
        ++steps;
        if (end) break;
    }
    atomicMax(&a.maxN[draw], L.s);
    dr_emit<NM>(a, c, L);
    dr_store<NM>(a, c, L);
    atomicAdd(&a.ctr[0], (unsigned long long)steps);
}

// The stage bodies a batched while loop runs after chain c has finished
// draw `draw`: proposal, density and acceptance, discarded.
template <int NM>
__global__ __launch_bounds__(256) void dr_pad_kernel(DrK a, uint32_t draw)
{
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= a.m) return;
    const int done = a.counts[(size_t)c * a.n + draw];
    const int extra = a.maxN[draw] - done;
    if (extra <= 0) return;
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
    atomicAdd(&a.ctr[1], (unsigned long long)extra);
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
static DrK dr_view(const JobDev& j)
{
    DrK a;
    a.m = j.m;
    a.n = j.n;
    a.D = j.D;
    a.target = j.target;
    a.n_stages = j.n_stages;
    a.tstop = j.tstop;
    a.seed = j.seed;
    for (int i = 0; i < 3; ++i) a.sc[i] = (float)j.scales[i];
    a.prec = (const float*)j.prec;
    a.x = (float*)j.x;
    a.y1 = (float*)j.V;
    a.y2 = (float*)j.V + (size_t)j.m * j.D;
    a.lx = (float*)j.lx;
    a.l1 = (float*)j.H0;
    a.l2 = (float*)j.Wsum;
    a.s = j.evals;
    a.t = j.t;
    a.budget = j.budget;
    a.out = (float*)j.out;
    a.counts = j.counts;
    a.ctr = j.ctr;
    a.maxN = j.maxN;
    a.sink = (float*)j.sink;
    return a;
}

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
