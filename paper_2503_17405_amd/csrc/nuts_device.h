// nuts_device.h -- the no-U-turn sampler's FSM step (Hoffman & Gelman 2014;
// Sec. 3.1, Fig. "Finite state machines ...", HMC-NUTS panel; Sec. 7.3) and
// the request compaction, shared by the single-job kernels (nuts.hip) and the
// grouped multi-job kernels (batch.hip).
#pragma once
#include "fsmmc_device.h"
#include "fsmmc_internal.h"

namespace fsmmc {


enum NutsState : int32_t { NS_INIT = 1, NS_DOUBLE = 2, NS_INTEGRATE = 3, NS_CHECK = 4, NS_DONE = 5, NS_WAIT = 6 };
enum NutsFlag : int32_t { NF_INVALID = 1, NF_STOP = 2, NF_DIVERGED = 4, NF_TURNED = 8, NF_PENDING = 16 };

constexpr float kDeltaMax = 1000.0f;

__device__ __forceinline__ float logaddexp_f(float a, float b)
{
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    const float mx = fmaxf(a, b);
    return mx + log1pf(expf(-fabsf(a - b)));
}

struct NutsK {
    int m, n, D, Dp, J, nvec, ckp0, ckr0, mode;
    uint32_t step, tstop;
    uint64_t seed;
    float eps;
    int32_t *k, *jd, *v, *nn, *flags, *nleap;
    uint32_t* t;
    int64_t* budget;
    float *H0, *W, *Ws, *UP, *US;
    float* V;  // [chain][nvec][Dp]
    float* Thq;
    const float* Gpart;  // gradient row-slice partials: [slice][chain][Dp]
    const float* Upart;  // log-likelihood row-slice partials: [slice][chain]
    int nslices;
    int32_t* req;
    float* out;
    int32_t* counts;
    unsigned long long* ctr;
    uint32_t* wctr;
    float* acc;       // per chain: sum over its leapfrogs of min(1, e^(H0 - H))
    int32_t* maxN;    // per draw: largest leapfrog count over chains (synchronized inline runtime)
    int32_t* queue;   // persistent inline kernel: next chain to take
};

enum { V_THL = 0, V_PL, V_GL, V_THR, V_PR, V_GR, V_THP, V_GP, V_THS, V_GS, V_RHO, V_RHOS, V_PH, V_FIXED };

// One runtime step of a chain (one wavefront): finish the leapfrog whose
// gradient has arrived, then run the cheap states back to back until the
// chain requests its next gradient (Appendix, Alg. "bundled step as input to
// amortized step").
// NC_REQ: the step ended with a gradient request (the leapfrog is pending).
enum NutsChainBits { NC_ALIVE = 1, NC_INDRAW = 2, NC_REQ = 4 };

// Scalar state of one chain, wave-uniform, held in registers while the
// chain is stepped.
struct NutsScal {
    uint32_t t;
    int k, j, v, nn, fl, nleap;
    int64_t budget;
    float H0, W, Ws, UP, US, acc;
};

__device__ __forceinline__ NutsScal nuts_load(const NutsK& a, int c, uint32_t t)
{
    NutsScal s;
    s.t = t;
    s.k = uni(a.k[c]);
    s.j = uni(a.jd[c]);
    s.v = uni(a.v[c]);
    s.nn = uni(a.nn[c]);
    s.fl = uni(a.flags[c]);
    s.nleap = uni(a.nleap[c]);
    s.budget = uni((int64_t)a.budget[c]);
    s.H0 = uni(a.H0[c]);
    s.W = uni(a.W[c]);
    s.Ws = uni(a.Ws[c]);
    s.UP = uni(a.UP[c]);
    s.US = uni(a.US[c]);
    s.acc = uni(a.acc[c]);
    return s;
}

__device__ __forceinline__ void nuts_store(const NutsK& a, int c, const NutsScal& s, int req, int lane)
{
    if (lane == 0) {
        a.t[c] = s.t;
        a.k[c] = s.k;
        a.jd[c] = s.j;
        a.v[c] = s.v;
        a.nn[c] = s.nn;
        a.flags[c] = s.fl;
        a.nleap[c] = s.nleap;
        a.budget[c] = s.budget;
        a.H0[c] = s.H0;
        a.W[c] = s.W;
        a.Ws[c] = s.Ws;
        a.UP[c] = s.UP;
        a.US[c] = s.US;
        a.acc[c] = s.acc;
        a.req[c] = req;
    }
}

// Logistic regression: the gradient of the pending leapfrog arrives as
// row-slice partials, added in slice order:
//   grad U = theta - sum_s X_s^T r_s,  U = |theta|^2 / 2 - sum_s loglik_s.
// The slice sums sum_s X_s^T r_s (into gs) and sum_s loglik_s (returned).
template <int EPL>
__device__ __forceinline__ float slice_sums(const NutsK& a, int c, int lane, WaveVec<EPL>& gs)
{
    float ll = 0.0f;
#pragma unroll
    for (int e = 0; e < EPL; ++e) gs.r[e] = 0.0f;
    // unrolled so that the loads of several slices are in flight at once
    // (the additions keep their order)
#pragma unroll 8
    for (int s = 0; s < a.nslices; ++s) {
        const float* gp = a.Gpart + ((size_t)s * a.m + c) * a.Dp;
#pragma unroll
        for (int e = 0; e < EPL; ++e) gs.r[e] += gp[e * 64 + lane];
        ll += a.Upart[(size_t)s * a.m + c];
    }
    return ll;
}

template <int EPL>
__device__ __forceinline__ void slice_finish(const WaveVec<EPL>& th, const WaveVec<EPL>& gs, float ll,
                                             WaveVec<EPL>& g, float& U)
{
#pragma unroll
    for (int e = 0; e < EPL; ++e) g.r[e] = th.r[e] - gs.r[e];
    U = uni(0.5f * wdot(th, th) - ll);
}

struct SliceGrad {
    const NutsK& a;
    template <int EPL>
    __device__ __forceinline__ void operator()(int c, const WaveVec<EPL>& th, int lane, WaveVec<EPL>& g,
                                               float& U) const
    {
        WaveVec<EPL> gs;
        const float ll = slice_sums<EPL>(a, c, lane, gs);
        slice_finish<EPL>(th, gs, ll, g, U);
    }
};

// The same with the slice sums formed ahead (one chain's).
template <int EPL>
struct PreSliceGrad {
    const WaveVec<EPL>& gs;
    float ll;
    __device__ __forceinline__ void operator()(int, const WaveVec<EPL>& th, int, WaveVec<EPL>& g, float& U) const
    {
        slice_finish<EPL>(th, gs, ll, g, U);
    }
};

// Acceptance statistic of one leaf: min(1, e^w), w = H0 - H; a divergent or
// undefined energy counts 0.
__device__ __forceinline__ float nuts_leaf_accept(float w)
{
    if (w >= 0.0f) return 1.0f;
    return w > -INFINITY ? expf(w) : 0.0f;
}

// The step on a chain's registers: finish the pending leapfrog with the
// gradient `grad` supplies at its new position, then run the cheap states
// until the next request.  Returns NutsChainBits.
// The vectors a pending leapfrog reads (half-step momentum, new position,
// rho of the subtree), loaded before the chain's scalars arrive: in the FSM
// runtime a live chain has a leapfrog pending at every step but its first.
template <int EPL>
struct NutsPre {
    WaveVec<EPL> ph, th, rs;
};

template <int EPL, class Grad, bool PRE = false>
__device__ __forceinline__ int nuts_chain_body(const NutsK& a, const Grad& grad, int c, int lane, NutsScal& S,
                                               const NutsPre<EPL>* pre = nullptr)
{
    float* Vc = a.V + (size_t)c * a.nvec * a.Dp;
    auto vec = [&](int i) { return Vc + (size_t)i * a.Dp; };
    uint32_t t = S.t;
    int k = S.k, j = S.j, v = S.v, nn = S.nn, fl = S.fl, nleap = S.nleap;
    int64_t budget = S.budget;
    float H0 = S.H0, W = S.W, Ws = S.Ws, UP = S.UP, US = S.US, acc = S.acc;
    const bool release = a.mode != 0 && uni(a.wctr[(a.step + 2) % 3]) == 0u;
    const float he = 0.5f * a.eps;
    int req = 0;

    // Edge vectors (theta, p, grad U) of the side(s) in `cside` held in registers
    // (bit 1: left edge, bit 2: right edge), so INTEGRATE need not reload what
    // this invocation has just computed or read.
    WaveVec<EPL> cth, cp, cg;
    int cside = 0;

    // 1) the leapfrog whose gradient has arrived
    if (fl & NF_PENDING) {
        const int eth = v > 0 ? V_THR : V_THL, ep = v > 0 ? V_PR : V_PL, eg = v > 0 ? V_GR : V_GL;
        const float vhe = (float)v * he;
        // independent loads issued together: half-step momentum, new edge position, rho_sub
        WaveVec<EPL> g, p, ph, th, rs;
        if constexpr (PRE) {
            ph = pre->ph;
            th = pre->th;  // the request buffer holds the new edge position too
            rs = pre->rs;
        } else {
            ph.load(vec(V_PH), lane);
            th.load(vec(eth), lane);
            rs.load(vec(V_RHOS), lane);
        }
        float Un;
        grad(c, th, lane, g, Un);
#pragma unroll
        for (int e = 0; e < EPL; ++e) p.r[e] = ph.r[e] - vhe * g.r[e];
        ++nleap;
        const float w = H0 - (Un + 0.5f * wdot(p, p));
        acc += nuts_leaf_accept(w);
        p.store(vec(ep), lane);
        g.store(vec(eg), lane);
        if (!(-w <= kDeltaMax)) {
            fl |= NF_INVALID | NF_DIVERGED;
        } else {
            const float Wn = logaddexp_f(Ws, w);
            if (logf(uniform<float>(a.seed, (uint32_t)c, t, ROLE_LEAF, ((uint32_t)j << 16) | (uint32_t)nn)) <
                w - Wn) {
                th.store(vec(V_THS), lane);
                g.store(vec(V_GS), lane);
                US = Un;
            }
            Ws = Wn;
#pragma unroll
            for (int e = 0; e < EPL; ++e) rs.r[e] += p.r[e];
            rs.store(vec(V_RHOS), lane);
            for (int lev = 1; lev <= j; ++lev) {
                if ((nn & ((1 << lev) - 1)) == 0) {
                    WaveVec<EPL> ck;
#pragma unroll
                    for (int e = 0; e < EPL; ++e) ck.r[e] = rs.r[e] - p.r[e];
                    p.store(vec(a.ckp0 + lev), lane);
                    ck.store(vec(a.ckr0 + lev), lane);
                }
            }
            for (int lev = 1; lev <= j; ++lev) {
                if (((nn + 1) & ((1 << lev) - 1)) == 0) {
                    WaveVec<EPL> ckp, span;
                    ckp.load(vec(a.ckp0 + lev), lane);
                    span.load(vec(a.ckr0 + lev), lane);
#pragma unroll
                    for (int e = 0; e < EPL; ++e) span.r[e] = rs.r[e] - span.r[e];
                    if (wdot(ckp, span) <= 0.0f || wdot(p, span) <= 0.0f) fl |= NF_INVALID | NF_TURNED;
                }
            }
            if (!(fl & NF_INVALID)) ++nn;
        }
        cth = th;
        cp = p;
        cg = g;
        cside = v > 0 ? 2 : 1;
        fl &= ~NF_PENDING;
        k = (!(fl & NF_INVALID) && nn < (1 << j)) ? NS_INTEGRATE : NS_CHECK;
    }

    // 2) cheap states back to back until the next gradient request
    for (int guard = 0; guard < 8; ++guard) {
        if (k == NS_WAIT) {
            if (!release) break;
            k = NS_INIT;
        }
        if (k == NS_INIT) {
            WaveVec<EPL> p0, th, g;
            th.load(vec(V_THP), lane);
            g.load(vec(V_GP), lane);
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const int d = e * 64 + lane;
                p0.r[e] = d < a.D ? normal_at<float>(a.seed, (uint32_t)c, t, ROLE_MOM, 0, (uint32_t)d) : 0.0f;
            }
            H0 = UP + 0.5f * wdot(p0, p0);
            p0.store(vec(V_PL), lane);
            p0.store(vec(V_PR), lane);
            p0.store(vec(V_RHO), lane);
            th.store(vec(V_THL), lane);
            th.store(vec(V_THR), lane);
            g.store(vec(V_GL), lane);
            g.store(vec(V_GR), lane);
            cth = th;
            cp = p0;
            cg = g;
            cside = 3;
            W = 0.0f;
            j = 0;
            fl = 0;
            nleap = 0;
            k = (j < a.J) ? NS_DOUBLE : NS_DONE;
            continue;
        }
        if (k == NS_DOUBLE) {
            v = uniform<float>(a.seed, (uint32_t)c, t, ROLE_DIR, (uint32_t)j) < 0.5f ? 1 : -1;
            Ws = -INFINITY;
            WaveVec<EPL> z;
#pragma unroll
            for (int e = 0; e < EPL; ++e) z.r[e] = 0.0f;
            z.store(vec(V_RHOS), lane);
            nn = 0;
            fl &= ~NF_INVALID;
            k = NS_INTEGRATE;
            continue;
        }
        if (k == NS_INTEGRATE) {
            if (budget <= 0) break;
            const int eth = v > 0 ? V_THR : V_THL, ep = v > 0 ? V_PR : V_PL, eg = v > 0 ? V_GR : V_GL;
            const float vhe = (float)v * he, veps = (float)v * a.eps;
            WaveVec<EPL> th, p, g, ph;
            if (cside & (v > 0 ? 2 : 1)) {
                th = cth;
                p = cp;
                g = cg;
            } else {
                th.load(vec(eth), lane);
                p.load(vec(ep), lane);
                g.load(vec(eg), lane);
            }
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                ph.r[e] = p.r[e] - vhe * g.r[e];
                th.r[e] = th.r[e] + veps * ph.r[e];
            }
            ph.store(vec(V_PH), lane);
            th.store(vec(eth), lane);
            th.store(a.Thq + (size_t)c * a.Dp, lane);
            fl |= NF_PENDING;
            req = 1;
            --budget;
            break;
        }
        if (k == NS_CHECK) {
            if (fl & NF_INVALID) {
                fl |= NF_STOP;
            } else {
                if (logf(uniform<float>(a.seed, (uint32_t)c, t, ROLE_MERGE, (uint32_t)j)) < Ws - W) {
                    WaveVec<EPL> th, g;
                    th.load(vec(V_THS), lane);
                    g.load(vec(V_GS), lane);
                    th.store(vec(V_THP), lane);
                    g.store(vec(V_GP), lane);
                    UP = US;
                }
                W = logaddexp_f(W, Ws);
                WaveVec<EPL> rho, rs, pl, pr;
                rho.load(vec(V_RHO), lane);
                rs.load(vec(V_RHOS), lane);
#pragma unroll
                for (int e = 0; e < EPL; ++e) rho.r[e] += rs.r[e];
                rho.store(vec(V_RHO), lane);
                if (cside & 1)
                    pl = cp;
                else
                    pl.load(vec(V_PL), lane);
                if (cside & 2)
                    pr = cp;
                else
                    pr.load(vec(V_PR), lane);
                if (wdot(pl, rho) <= 0.0f || wdot(pr, rho) <= 0.0f) fl |= NF_STOP | NF_TURNED;
            }
            ++j;
            k = (!(fl & NF_STOP) && j < a.J) ? NS_DOUBLE : NS_DONE;
            continue;
        }
        if (k == NS_DONE) {
            WaveVec<EPL> th;
            th.load(vec(V_THP), lane);
            float* o = a.out + ((size_t)c * a.n + t) * a.D;
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const int d = e * 64 + lane;
                if (d < a.D) o[d] = th.r[e];
            }
            if (lane == 0) a.counts[(size_t)c * a.n + t] = nleap;
            ++t;
            k = NS_INIT;
            if (t >= a.tstop) break;
            if (a.mode != 0) {
                k = NS_WAIT;
                break;
            }
            continue;
        }
        break;
    }
    S.t = t;
    S.k = k;
    S.j = j;
    S.v = v;
    S.nn = nn;
    S.fl = fl;
    S.nleap = nleap;
    S.budget = budget;
    S.H0 = H0;
    S.W = W;
    S.Ws = Ws;
    S.UP = UP;
    S.US = US;
    S.acc = acc;
    const int rq = req ? NC_REQ : 0;
    if (t >= a.tstop) return rq;
    return rq | NC_ALIVE | ((a.mode != 0 && k != NS_WAIT) ? NC_INDRAW : 0);
}

// One runtime step of chain c (one wavefront) with its state in memory:
// load, step, store.  Returns NC_ALIVE if the chain is short of tstop
// afterwards, plus NC_INDRAW if it is also still inside its draw
// (synchronized runtimes).  Gradient requests (the steps) are counted by the
// compaction.
template <int EPL, class Grad>
__device__ __forceinline__ int nuts_chain_step(const NutsK& a, const Grad& grad, int c, int lane)
{
    c = uni(c);
    // the draw counter and the rest of the chain's scalars in one round of
    // loads (a finished chain reads them for nothing; they are only a few words)
    NutsScal S = nuts_load(a, c, uni(a.t[c]));
    if (S.t >= a.tstop) {
        if (lane == 0) a.req[c] = 0;
        return 0;
    }
    const int bits = nuts_chain_body<EPL>(a, grad, c, lane, S);
    nuts_store(a, c, S, (bits & NC_REQ) ? 1 : 0, lane);
    return bits & (NC_ALIVE | NC_INDRAW);
}

// Logistic regression (gradient from the row-slice partials).  FSM runtime:
// the pending leapfrog's vectors and slice sums are loaded in the same round
// as the chain's scalars (a chain that turns out finished or not pending
// read them for nothing; the synchronized runtimes, whose waiting chains are
// not pending, load after the scalars).
template <int EPL>
__device__ __forceinline__ int nuts_chain_step(const NutsK& a, int c, int lane)
{
    if (a.mode != 0) return nuts_chain_step<EPL>(a, SliceGrad{a}, c, lane);
    c = uni(c);
    const float* Vc = a.V + (size_t)c * a.nvec * a.Dp;
    NutsPre<EPL> P;
    P.ph.load(Vc + (size_t)V_PH * a.Dp, lane);
    P.th.load(a.Thq + (size_t)c * a.Dp, lane);
    P.rs.load(Vc + (size_t)V_RHOS * a.Dp, lane);
    WaveVec<EPL> gs;
    const float ll = slice_sums<EPL>(a, c, lane, gs);
    NutsScal S = nuts_load(a, c, uni(a.t[c]));
    if (S.t >= a.tstop) {
        if (lane == 0) a.req[c] = 0;
        return 0;
    }
    const int bits = nuts_chain_body<EPL, PreSliceGrad<EPL>, true>(a, PreSliceGrad<EPL>{gs, ll}, c, lane, S, &P);
    nuts_store(a, c, S, (bits & NC_REQ) ? 1 : 0, lane);
    return bits & (NC_ALIVE | NC_INDRAW);
}

// Chains of one job that asked for a gradient, in chain order (one block of
// NT threads).  The flags are read in coalesced rounds of NT chains; within a
// round a wave places its requesters by ballot and bit count, and the waves'
// offsets come from their counts in LDS.  In vmap mode a gradient phase that
// anyone needs covers every chain.
template <int NT>
__device__ __forceinline__ void nuts_compact_block(const int32_t* req, int m, int vmap, int32_t* list,
                                                   int32_t* count, unsigned long long* ctr)
{
    constexpr int NW = NT / 64;
    __shared__ int wsum[NW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long below_mask = (1ull << lane) - 1ull;
    int total = 0;  // requesters in the rounds before this one (the same in every thread)
    for (int r0 = 0; r0 < m; r0 += NT) {
        const int i = r0 + tid;
        const bool f = i < m && req[i] != 0;
        const unsigned long long bal = __ballot(f);
        if (lane == 0) wsum[wave] = __popcll(bal);
        __syncthreads();
        int woff = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int v = wsum[w];
            woff += w < wave ? v : 0;
            tot += v;
        }
        if (f && !vmap) list[total + woff + __popcll(bal & below_mask)] = i;
        total += tot;
        __syncthreads();  // wsum is rewritten by the next round
    }
    if (vmap) {
        if (tid == 0) {
            *count = total > 0 ? m : 0;
            if (total > 0) {
                atomicAdd(&ctr[0], (unsigned long long)total);
                atomicAdd(&ctr[1], (unsigned long long)(m - total));
            }
        }
        if (total > 0)
            for (int i = tid; i < m; i += NT) list[i] = i;
        return;
    }
    if (tid == 0) {
        *count = total;
        if (total > 0) atomicAdd(&ctr[0], (unsigned long long)total);
    }
}

inline NutsK nuts_view(const JobDev& j, int mode, uint32_t step)
{
    NutsK a;
    a.m = j.m;
    a.n = j.n;
    a.D = j.D;
    a.Dp = j.Dp;
    a.J = j.max_depth;
    a.nvec = j.nvec;
    a.ckp0 = V_FIXED - 1;  // level lev in [1, J] lives at ckp0 + lev
    a.ckr0 = V_FIXED - 1 + j.max_depth;
    a.mode = mode;
    a.step = step;
    a.tstop = j.tstop;
    a.seed = j.seed;
    a.eps = (float)j.step_size;
    a.k = j.k;
    a.jd = j.jd;
    a.v = j.vdir;
    a.nn = j.nn;
    a.flags = j.flags;
    a.nleap = j.evals;
    a.t = j.t;
    a.budget = j.budget;
    a.H0 = (float*)j.H0;
    a.W = (float*)j.Wsum;
    a.Ws = (float*)j.Wsub;
    a.UP = (float*)j.lx;
    a.US = (float*)j.US;
    a.V = (float*)j.V;
    a.Thq = (float*)j.Thq;
    a.Gpart = (const float*)j.Gpart;
    a.Upart = (const float*)j.Upart;
    a.nslices = j.nslices;
    a.req = j.req;
    a.out = (float*)j.out;
    a.counts = j.counts;
    a.ctr = j.ctr;
    a.wctr = j.wctr;
    a.acc = (float*)j.acc;
    a.maxN = j.maxN;
    a.queue = j.queue;
    return a;
}

}  // namespace fsmmc
