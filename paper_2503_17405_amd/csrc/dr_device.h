// dr_device.h -- delayed-rejection Metropolis-Hastings (Tierney & Mira 1999;
// Mira 2001) building blocks shared by the single-job kernels (dr.hip) and
// the grouped multi-job kernels (batch.hip).  Sec. 3.1, Fig. "Finite state
// machines ...", delayed-rejection panel; Sec. 7.1.
//
// One lane per chain: x, the rejected proposals y1, y2 and their log
// densities stay in registers; state is stored [field][d][chain].
#pragma once
#include "fsmmc_device.h"
#include "fsmmc_internal.h"

namespace fsmmc {

constexpr int kDrMaxDim = 16;

struct DrK {
    int m, n, D, target, n_stages;
    uint32_t tstop;
    uint64_t seed;
    float sc0, sc1, sc2;  // proposal standard deviations of stages 1..3
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
    if (s == 1) return dr_la2(lx, l1, l2, lq<NM>(x, y1, D, a.sc0), lq<NM>(y2, y1, D, a.sc0));
    const float q0 = lq<NM>(x, y1, D, a.sc0);   // q1(x -> y1)
    const float q1 = lq<NM>(y2, y1, D, a.sc0);  // q1(y2 -> y1)
    const float q2 = lq<NM>(x, y2, D, a.sc1);   // q2(x -> y2)
    const float q3 = lq<NM>(y3, y2, D, a.sc0);  // q1(y3 -> y2)
    const float q4 = lq<NM>(y3, y1, D, a.sc1);  // q2(y3 -> y1)
    const float q5 = lq<NM>(y1, y2, D, a.sc0);  // q1(y1 -> y2)
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
    const float sc = s == 0 ? a.sc0 : (s == 1 ? a.sc1 : a.sc2);
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
        la = dr_la2(L.lx, L.l1, ly, lq<NM>(L.x, L.y1, a.D, a.sc0), lq<NM>(y, L.y1, a.D, a.sc0));
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

// One lane runs chain c through PROPOSE steps until it reaches draw `stop`
// (or n) or spends its budget.  Returns the draws it emitted; *steps gets the
// steps taken and *live whether the chain is still short of n (the caller
// adds them to the job counters [0] and [4]).
template <int NM>
__device__ __forceinline__ uint32_t dr_run(const DrK& a, int c, uint32_t stop, uint32_t* steps_out, uint32_t* live)
{
    DrLane<NM> L;
    dr_load<NM>(a, c, L);
    const uint32_t t0 = L.t;
    stop = min(stop, (uint32_t)a.n);
    int64_t budget = a.budget[c];
    uint32_t steps = 0;
    while (L.t < stop && budget > 0) {
        const int end = dr_stage<NM>(a, c, L);
        ++steps;
        --budget;
        if (end) dr_emit<NM>(a, c, L);
    }
    dr_store<NM>(a, c, L);
    a.budget[c] = budget;
    *steps_out = steps;
    *live = L.t < (uint32_t)a.n ? 1u : 0u;
    return L.t - t0;
}

// Lane occupancy of a lane-per-chain loop (every thread of the block calls
// it): a wave runs its loop body as often as its busiest lane, so it spends
// 64 * max(iters) lane slots, of which sum(useful) did a chain's work.
// ctr[5] += useful lane-iterations, ctr[6] += lane slots; one atomic per block.
__device__ __forceinline__ void dr_count_lanes(const DrK& a, uint32_t useful, uint32_t iters,
                                               unsigned long long* s_slot)
{
    const unsigned long long act = block_sum_u64(wave_sum_u64((unsigned long long)useful), s_slot);
    if (threadIdx.x == 0 && act) atomicAdd(&a.ctr[5], act);
    const unsigned long long slots =
        block_sum_u64(64ull * (unsigned long long)wave_max_i32((int)iters), s_slot);
    if (threadIdx.x == 0 && slots) atomicAdd(&a.ctr[6], slots);
}

inline DrK dr_view(const JobDev& j)
{
    DrK a;
    a.m = j.m;
    a.n = j.n;
    a.D = j.D;
    a.target = j.target;
    a.n_stages = j.n_stages;
    a.tstop = j.tstop;
    a.seed = j.seed;
    a.sc0 = (float)j.scales[0];
    a.sc1 = (float)j.scales[1];
    a.sc2 = (float)j.scales[2];
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

// Register bound of the lane state for dimension D (instantiated 4, 8, 12, 16).
inline int dr_nm(int D) { return D <= 4 ? 4 : (D <= 8 ? 8 : (D <= 12 ? 12 : 16)); }

}  // namespace fsmmc
