// nuts.hip -- the no-U-turn sampler (Hoffman & Gelman 2014) as an FSM
// (Sec. 3.1, Fig. "Finite state machines ...", HMC-NUTS panel: INIT, DOUBLE,
// INTEGRATE, CHECK, DONE; Sec. 7.3: iterative form, an outer doubling loop
// and an inner integration loop), for Bayesian logistic regression.
//
// One runtime step for every chain:
//   1. nuts_step_kernel (one wavefront per chain): finish the leapfrog whose
//      gradient just arrived (second half-kick, multinomial leaf choice,
//      U-turn checkpoints), then run the cheap states back to back (CHECK,
//      DONE, INIT, DOUBLE) until the chain needs the next gradient, and
//      issue the first half of that leapfrog (Appendix, Alg. "bundled step
//      as input to amortized step").
//   2. nuts_compact_kernel: list of chains that asked for a gradient, in
//      chain order.
//   3. logreg_grad_kernel: eta = X Theta, r = y - sigmoid(eta), X^T r and
//      the log-likelihood, fused on FP32 MFMA for a tile of 64 listed chains
//      and a slice of rows; eta never leaves registers.
//   4. logreg_reduce_kernel: sums the row-slice partials in a fixed order:
//      grad U = theta - X^T r, U = |theta|^2 / 2 - loglik.
// The synchronized runtime uses the same kernels; a chain that finishes a
// draw waits until every chain has finished it (device-side barrier), and in
// vmap mode the gradient phase then covers every chain.
// Readings: multinomial leaf sampling inside a subtree, biased progressive
// merge of subtrees, generalized U-turn criterion on every aligned sub-span,
// divergence when H - H0 > 1000, identity mass.
#include "fsmmc_device.h"
#include "fsmmc_internal.h"

namespace fsmmc {

typedef float floatx16 __attribute__((ext_vector_type(16)));

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
    const float* Gres;
    const float* Ures;
    int32_t* req;
    float* out;
    int32_t* counts;
    unsigned long long* ctr;
    uint32_t* wctr;
};

template <int EPL>
struct WaveVec {
    float r[EPL];
    __device__ __forceinline__ void load(const float* p, int lane)
    {
#pragma unroll
        for (int e = 0; e < EPL; ++e) r[e] = p[e * 64 + lane];
    }
    __device__ __forceinline__ void store(float* p, int lane) const
    {
#pragma unroll
        for (int e = 0; e < EPL; ++e) p[e * 64 + lane] = r[e];
    }
};

template <int EPL>
__device__ __forceinline__ float wdot(const WaveVec<EPL>& a, const WaveVec<EPL>& b)
{
    float s = 0.0f;
#pragma unroll
    for (int e = 0; e < EPL; ++e) s += a.r[e] * b.r[e];
    return wave_sum(s);
}

enum { V_THL = 0, V_PL, V_GL, V_THR, V_PR, V_GR, V_THP, V_GP, V_THS, V_GS, V_RHO, V_RHOS, V_PH, V_FIXED };

template <int EPL>
__global__ __launch_bounds__(256) void nuts_step_kernel(NutsK a)
{
    const int lane = threadIdx.x & 63;
    const int c = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.wctr[(a.step + 1) % 3] = 0u;
        a.wctr[3 + (a.step + 1) % 3] = 0u;
    }
    if (c >= a.m) return;
    uint32_t t = a.t[c];
    if (t >= a.tstop) {
        if (lane == 0) a.req[c] = 0;
        return;
    }
    float* Vc = a.V + (size_t)c * a.nvec * a.Dp;
    auto vec = [&](int i) { return Vc + (size_t)i * a.Dp; };
    int k = a.k[c], j = a.jd[c], v = a.v[c], nn = a.nn[c], fl = a.flags[c], nleap = a.nleap[c];
    int64_t budget = a.budget[c];
    float H0 = a.H0[c], W = a.W[c], Ws = a.Ws[c], UP = a.UP[c], US = a.US[c];
    const bool release = a.mode != 0 && a.wctr[(a.step + 2) % 3] == 0u;
    const float he = 0.5f * a.eps;
    int req = 0;
    unsigned long long steps = 0;

    // 1) the leapfrog whose gradient has arrived
    if (fl & NF_PENDING) {
        const int eth = v > 0 ? V_THR : V_THL, ep = v > 0 ? V_PR : V_PL, eg = v > 0 ? V_GR : V_GL;
        const float vhe = (float)v * he;
        WaveVec<EPL> g, p, ph;
        g.load(a.Gres + (size_t)c * a.Dp, lane);
        ph.load(vec(V_PH), lane);
#pragma unroll
        for (int e = 0; e < EPL; ++e) p.r[e] = ph.r[e] - vhe * g.r[e];
        const float Un = a.Ures[c];
        ++nleap;
        const float w = H0 - (Un + 0.5f * wdot(p, p));
        p.store(vec(ep), lane);
        g.store(vec(eg), lane);
        if (!(-w <= kDeltaMax)) {
            fl |= NF_INVALID | NF_DIVERGED;
        } else {
            const float Wn = logaddexp_f(Ws, w);
            if (logf(uniform<float>(a.seed, (uint32_t)c, t, ROLE_LEAF, ((uint32_t)j << 16) | (uint32_t)nn)) <
                w - Wn) {
                WaveVec<EPL> th;
                th.load(vec(eth), lane);
                th.store(vec(V_THS), lane);
                g.store(vec(V_GS), lane);
                US = Un;
            }
            Ws = Wn;
            WaveVec<EPL> rs;
            rs.load(vec(V_RHOS), lane);
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
            WaveVec<EPL> p0;
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const int d = e * 64 + lane;
                p0.r[e] = d < a.D ? normal_at<float>(a.seed, (uint32_t)c, t, ROLE_MOM, 0, (uint32_t)d) : 0.0f;
            }
            H0 = UP + 0.5f * wdot(p0, p0);
            p0.store(vec(V_PL), lane);
            p0.store(vec(V_PR), lane);
            p0.store(vec(V_RHO), lane);
            WaveVec<EPL> th, g;
            th.load(vec(V_THP), lane);
            g.load(vec(V_GP), lane);
            th.store(vec(V_THL), lane);
            th.store(vec(V_THR), lane);
            g.store(vec(V_GL), lane);
            g.store(vec(V_GR), lane);
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
            th.load(vec(eth), lane);
            p.load(vec(ep), lane);
            g.load(vec(eg), lane);
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
            ++steps;
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
                pl.load(vec(V_PL), lane);
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
    if (lane == 0) {
        a.t[c] = t;
        a.k[c] = k;
        a.jd[c] = j;
        a.v[c] = v;
        a.nn[c] = nn;
        a.flags[c] = fl;
        a.nleap[c] = nleap;
        a.budget[c] = budget;
        a.H0[c] = H0;
        a.W[c] = W;
        a.Ws[c] = Ws;
        a.UP[c] = UP;
        a.US[c] = US;
        a.req[c] = req;
        if (steps) atomicAdd(&a.ctr[0], steps);
        if (t < a.tstop) {
            atomicAdd(&a.wctr[3 + a.step % 3], 1u);
            if (a.mode != 0 && k != NS_WAIT) atomicAdd(&a.wctr[a.step % 3], 1u);
        }
    }
}

// Chains that asked for a gradient, in chain order (one block).  In vmap mode
// a gradient phase that anyone needs covers every chain.
__global__ __launch_bounds__(1024) void nuts_compact_kernel(const int32_t* req, int m, int vmap, int32_t* list,
                                                            int32_t* count, unsigned long long* ctr)
{
    __shared__ int part[1024];
    const int tid = threadIdx.x;
    const int per = (m + 1023) / 1024;
    const int b = tid * per, e = min(m, b + per);
    int local = 0;
    for (int i = b; i < e; ++i) local += req[i] != 0;
    part[tid] = local;
    __syncthreads();
    // inclusive scan (Hillis-Steele)
    for (int o = 1; o < 1024; o <<= 1) {
        const int add = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    const int total = part[1023];
    if (vmap) {
        if (tid == 0) {
            *count = total > 0 ? m : 0;
            if (total > 0) atomicAdd(&ctr[1], (unsigned long long)(m - total));
        }
        if (total > 0)
            for (int i = tid; i < m; i += 1024) list[i] = i;
        return;
    }
    int pos = part[tid] - local;
    for (int i = b; i < e; ++i)
        if (req[i]) list[pos++] = i;
    if (tid == 0) *count = total;
}

struct GradK {
    int m, N, Dp, slice_rows, nslices, dense;  // dense > 0: columns are chains 0 .. dense-1
    const float* X;  // Np x Dp
    const float* y;  // Np
    const float* Th; // m x Dp, indexed by chain
    const int32_t* list;
    const int32_t* count;
    float* Gpart;    // nslices x m x Dp
    float* Upart;    // nslices x m
};

// Block: 4 waves, 64 listed chains, one slice of rows.  Each wave walks row
// chunks of 32: eta (32 x 64) = X_chunk Theta^T on MFMA, r = y - sigmoid(eta)
// in place, then X_chunk^T r accumulated into DT x 2 tiles of 32 x 32.  The
// second product takes its B operand straight from the first product's
// accumulator registers: at k-step s a lane contributes the row its own
// register s holds.  The four waves' partials are added in LDS in wave order.
template <int DT>
__global__ __launch_bounds__(256) void logreg_grad_kernel(GradK a)
{
    constexpr int DP = 32 * DT;
    __shared__ float Ths[64 * (DP + 1)];
    __shared__ float Ured[64];
    __shared__ int cols[64];
    const int ncols = a.dense > 0 ? a.dense : *a.count;
    const int ct = blockIdx.x, sl = blockIdx.y;
    if (ct * 64 >= ncols) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, l32 = lane & 31;
    if (tid < 64) {
        const int g = ct * 64 + tid;
        cols[tid] = g < ncols ? (a.dense > 0 ? g : a.list[g]) : -1;
        Ured[tid] = 0.0f;
    }
    __syncthreads();
    for (int i = tid; i < 64 * DP; i += 256) {
        const int col = i / DP, d = i - col * DP;
        const int ch = cols[col];
        Ths[col * (DP + 1) + d] = ch >= 0 ? a.Th[(size_t)ch * DP + d] : 0.0f;
    }
    __syncthreads();

    floatx16 accg[DT][2];
#pragma unroll
    for (int dt = 0; dt < DT; ++dt)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int q = 0; q < 16; ++q) accg[dt][c][q] = 0.0f;
    float uacc[2] = {0.0f, 0.0f};

    const int rb = sl * a.slice_rows, re = min(rb + a.slice_rows, a.N);
    for (int r0 = rb + wave * 32; r0 < re; r0 += 128) {
        floatx16 eta[2];
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int q = 0; q < 16; ++q) eta[c][q] = 0.0f;
        const float* xr = a.X + (size_t)(r0 + l32) * DP + h * (DP / 2);
#pragma unroll 4
        for (int kb = 0; kb < DP / 2; kb += 4) {
            const float4 xv = *reinterpret_cast<const float4*>(xr + kb);
            const float xa[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int d = h * (DP / 2) + kb + i;
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    eta[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[i], Ths[(c * 32 + l32) * (DP + 1) + d],
                                                                 eta[c], 0, 0, 0);
            }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int row = r0 + 8 * (q >> 2) + 4 * h + (q & 3);
                const float e = eta[c][q];
                const bool ok = row < a.N;
                const float yv = a.y[row];
                const float ex = expf(-fabsf(e));
                const float sig = e >= 0.0f ? 1.0f / (1.0f + ex) : ex / (1.0f + ex);
                const float sp = fmaxf(e, 0.0f) + log1pf(ex);
                uacc[c] += ok ? (yv * e - sp) : 0.0f;
                eta[c][q] = ok ? (yv - sig) : 0.0f;
            }
        }
#pragma unroll
        for (int dt = 0; dt < DT; ++dt) {
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int row = r0 + 8 * (s >> 2) + 4 * h + (s & 3);
                const float xa = a.X[(size_t)row * DP + dt * 32 + l32];
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    accg[dt][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(xa, eta[c][s], accg[dt][c], 0, 0, 0);
            }
        }
    }
    // per-column log-likelihood of this wave: both lane halves hold half the rows
#pragma unroll
    for (int c = 0; c < 2; ++c) uacc[c] += __shfl_xor(uacc[c], 32, 64);
    __syncthreads();
    float* Red = Ths;  // DP x 64, reused
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int dt = 0; dt < DT; ++dt)
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int d = dt * 32 + 8 * (q >> 2) + 4 * h + (q & 3);
                        const int col = c * 32 + l32;
                        float* cell = &Red[d * 64 + col];
                        *cell = (w == 0) ? accg[dt][c][q] : *cell + accg[dt][c][q];
                    }
            if (h == 0) {
#pragma unroll
                for (int c = 0; c < 2; ++c) Ured[c * 32 + l32] += uacc[c];
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < 64 * DP; i += 256) {
        const int col = i / DP, d = i - col * DP;
        const int ch = cols[col];
        if (ch >= 0) a.Gpart[((size_t)sl * a.m + ch) * DP + d] = Red[d * 64 + col];
    }
    if (tid < 64 && cols[tid] >= 0) a.Upart[(size_t)sl * a.m + cols[tid]] = Ured[tid];
}

struct ReduceK {
    int m, Dp, nslices, dense;  // dense > 0: columns are chains 0 .. dense-1
    const float* Th;
    const int32_t* list;
    const int32_t* count;
    const float* Gpart;
    const float* Upart;
    float* G;  // chain-indexed outputs, row stride gstride
    float* U;
    int gstride;
};

// grad U = theta - sum_s partial_s, U = |theta|^2/2 - sum_s loglik_s (slice order).
template <int EPL>
__global__ __launch_bounds__(256) void logreg_reduce_kernel(ReduceK a)
{
    const int lane = threadIdx.x & 63;
    const int p = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int ncols = a.dense > 0 ? a.dense : *a.count;
    if (p >= ncols) return;
    const int c = a.dense > 0 ? p : a.list[p];
    WaveVec<EPL> th, g;
    th.load(a.Th + (size_t)c * a.Dp, lane);
#pragma unroll
    for (int e = 0; e < EPL; ++e) g.r[e] = 0.0f;
    for (int s = 0; s < a.nslices; ++s) {
        const float* gp = a.Gpart + ((size_t)s * a.m + c) * a.Dp;
#pragma unroll
        for (int e = 0; e < EPL; ++e) g.r[e] += gp[e * 64 + lane];
    }
#pragma unroll
    for (int e = 0; e < EPL; ++e) g.r[e] = th.r[e] - g.r[e];
    g.store(a.G + (size_t)c * a.gstride, lane);
    float ll = 0.0f;
    for (int s = 0; s < a.nslices; ++s) ll += a.Upart[(size_t)s * a.m + c];
    const float U = 0.5f * wdot(th, th) - ll;
    if (lane == 0) a.U[c] = U;
}

// Default start: theta0 ~ N(0, I) from the INIT stream (into both buffers).
__global__ void nuts_normal_init_kernel(float* thp, int vstride, float* thq, int m, int D, int Dp, uint64_t seed)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)m * Dp) return;
    const int c = (int)(i / Dp), d = (int)(i % Dp);
    const float z = d < D ? normal_at<float>(seed, (uint32_t)c, 0, ROLE_INIT, 0, (uint32_t)d) : 0.0f;
    thp[(size_t)c * vstride + d] = z;
    thq[(size_t)c * Dp + d] = z;
}

// ------------------------------------------------------------ host side
static NutsK nuts_view(const JobDev& j, int mode, uint32_t step)
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
    a.Gres = (const float*)j.Gres;
    a.Ures = (const float*)j.Ures;
    a.req = j.req;
    a.out = (float*)j.out;
    a.counts = j.counts;
    a.ctr = j.ctr;
    a.wctr = j.wctr;
    return a;
}

int nuts_nvec(int max_depth) { return V_FIXED + 2 * max_depth; }

static hipError_t grad_launch(const JobDev& j, int dense, float* Gout, float* Uout, int gstride, hipStream_t s)
{
    GradK g;
    g.m = j.m;
    g.N = j.N;
    g.Dp = j.Dp;
    g.slice_rows = j.slice_rows;
    g.nslices = j.nslices;
    g.dense = dense;
    g.X = (const float*)j.X;
    g.y = (const float*)j.y;
    g.Th = (const float*)j.Thq;
    g.list = j.list;
    g.count = j.count;
    g.Gpart = (float*)j.Gpart;
    g.Upart = (float*)j.Upart;
    const dim3 grid((j.m + 63) / 64, j.nslices), block(256);
    switch (j.Dp / 32) {
    case 1: hipLaunchKernelGGL(logreg_grad_kernel<1>, grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL(logreg_grad_kernel<2>, grid, block, 0, s, g); break;
    case 4: hipLaunchKernelGGL(logreg_grad_kernel<4>, grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ReduceK r;
    r.m = j.m;
    r.Dp = j.Dp;
    r.nslices = j.nslices;
    r.dense = dense;
    r.Th = (const float*)j.Thq;
    r.list = j.list;
    r.count = j.count;
    r.Gpart = (const float*)j.Gpart;
    r.Upart = (const float*)j.Upart;
    r.G = Gout;
    r.U = Uout;
    r.gstride = gstride;
    const dim3 rg((j.m + 3) / 4);
    if (j.Dp <= 64)
        hipLaunchKernelGGL(logreg_reduce_kernel<1>, rg, dim3(256), 0, s, r);
    else
        hipLaunchKernelGGL(logreg_reduce_kernel<2>, rg, dim3(256), 0, s, r);
    return hipGetLastError();
}

hipError_t nuts_init_state(const JobDev& j, const void* x0, hipStream_t s)
{
    float* thp = (float*)j.V + (size_t)V_THP * j.Dp;
    const int vstride = j.nvec * j.Dp;
    if (x0) {
        hipError_t e = hipMemcpy2DAsync(thp, (size_t)vstride * 4, x0, (size_t)j.D * 4, (size_t)j.D * 4, j.m,
                                        hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpy2DAsync(j.Thq, (size_t)j.Dp * 4, x0, (size_t)j.D * 4, (size_t)j.D * 4, j.m,
                             hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    } else {
        const size_t tot = (size_t)j.m * j.Dp;
        hipLaunchKernelGGL(nuts_normal_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, thp,
                           vstride, (float*)j.Thq, j.m, j.D, j.Dp, j.seed);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // grad U and U at the start, straight into the proposal slots (gP, UP)
    float* gp = (float*)j.V + (size_t)V_GP * j.Dp;
    return grad_launch(j, j.m, gp, (float*)j.lx, vstride, s);
}

hipError_t nuts_transition(const JobDev& j, int mode, uint32_t step, hipStream_t s)
{
    NutsK a = nuts_view(j, mode, step);
    const dim3 grid((j.m + 3) / 4), block(256);
    if (j.Dp <= 64)
        hipLaunchKernelGGL(nuts_step_kernel<1>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(nuts_step_kernel<2>, grid, block, 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(nuts_compact_kernel, dim3(1), dim3(1024), 0, s, j.req, j.m, mode == 1 ? 1 : 0, j.list, j.count,
                       j.ctr);
    return hipGetLastError();
}

hipError_t nuts_gradient(const JobDev& j, hipStream_t s)
{
    return grad_launch(j, 0, (float*)j.Gres, (float*)j.Ures, j.Dp, s);
}

}  // namespace fsmmc

namespace fsmmc {
hipError_t nuts_gradient_dense(const JobDev& j, int ncols, float* Gout, float* Uout, int gstride, hipStream_t s)
{
    return grad_launch(j, ncols, Gout, Uout, gstride, s);
}
}  // namespace fsmmc
