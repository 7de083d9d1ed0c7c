// gph.hip -- elliptical slice sampling of GP-regression hyperparameters
// (Sec. 7.2): theta = (tau, lambda, sigma) with the N(0, I) prior, and the
// marginal likelihood
//   y ~ N(0, C),  C = tau^2 exp(-lambda^2 |x_i - x_k|^2) + (sigma^2 + jitter) I,
//   log L = -y^T C^-1 y / 2 - log det C / 2,
// an O(n^3) Cholesky factorisation inside every loop iteration: the regime
// where the log-density dominates each transition and the FSM gain tracks R(m).
//
// Persistent kernel, one wavefront per block and per chain at a time: the
// wave takes chains from a device ticket counter and runs each one's ESS FSM
// (INIT, SHRINK, DONE; every step = one proposal and one likelihood) to its
// draw budget, so no chain waits for another.  The likelihood is computed by
// the wave in FP64 (kernel matrices of smooth kernels are badly
// conditioned; the 3-D chain state is FP64 too):
//   * C's lower triangle is built in LDS (packed rows, n(n+1)/2 doubles) from
//     the inputs staged in LDS;
//   * right-looking Cholesky, column by column: the column below the
//     diagonal is scaled (lane i mod 64 holds rows i) into registers and an
//     LDS column buffer, the forward solve L z = y runs alongside (y in
//     registers), and each lane applies the rank-1 update to its own rows of
//     the trailing triangle, four columns at a time; a block barrier (one
//     wave) orders the LDS updates;
//   * log L = -|z|^2 / 2 - sum_j log L_jj; -inf when a pivot is not positive.
// More than 96 observations (the paper's data set has 414): one block of
// four waves per chain (gph_big_kernel), C in a global slot of the block
// (n rounded up to 32, identity padding), blocked right-looking Cholesky
// with 32-column panels:
//   * wave 0 factors the panel's diagonal block in LDS (lane per row) and
//     solves its part of L z = y;
//   * the rows below are solved against it (thread per row, right-looking
//     inside the row) into an LDS copy of the panel, and their y entries
//     take the panel's part of the forward solve;
//   * each wave updates 32 x 32 tiles of the trailing triangle in the slot,
//     a 4 x 4 block per lane, with the panel's columns read from LDS.
// The library builds with contraction off, so the updates are written as
// explicit FMAs (one instruction and one rounding per term).
// The synchronized runtime launches the kernel once per draw (tstop =
// draw + 1); in vmap mode a second launch evaluates the max_j N_j - N_j
// likelihoods a batched while loop would compute and discard.
#include "fsmmc_device.h"
#include "fsmmc_internal.h"

namespace fsmmc {

constexpr int kGphMaxN = 96;      // observations, in-wave likelihood: up to two rows per lane
constexpr int kGphBigMaxN = 512;  // observations, block likelihood (LDS holds a 32-column panel)
constexpr int kGphBigWaves = 4;   // waves per block of the block likelihood
constexpr int kGphMaxP = 16;      // input dimension

struct GphK {
    int m, n, N, p;
    uint32_t tstop;
    uint64_t seed;
    double jitter;
    const double* X;  // N x p inputs
    const double* y;  // N outputs
    double *th, *nu;  // [chain][3]
    double *lx, *phi, *pmin, *pmax, *logu;
    int32_t *k, *evals;
    uint32_t* t;
    int64_t* budget;
    double* out;  // m x n x 3
    int32_t* counts;
    unsigned long long* ctr;
    int32_t* maxN;
    double* sink;
    double* slots;  // block likelihood: ld x ld doubles per block
    int ld;         // N rounded up to 32
};

__device__ __forceinline__ int gph_next_chain(unsigned long long* q, unsigned long long base, int m, int lane)
{
    unsigned long long tk = 0;
    if (lane == 0) tk = atomicAdd(q, 1ull);
    const unsigned long long off = (unsigned long long)uni((int64_t)tk) - base;
    return off < (unsigned long long)m ? (int)off : m;
}

__device__ __forceinline__ double rl(double v, int l)
{
    const int64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// log L(th) by the wave; A: n(n+1)/2 doubles of LDS (packed rows), cb: n
// doubles of LDS (the current column), Xs: the inputs in LDS.  Lane l owns
// rows l and l + 64.  Column j: the lanes scale their entries of column j
// (registers and cb), then every lane updates its own rows' entries k of the
// trailing triangle, four consecutive k at a time with L_kj read from cb (one
// broadcast per k): n^2 / 8 independent iteration groups instead of a
// latency-bound sweep.
__device__ double gph_loglik(const GphK& a, const double* th, double* A, double* cb, const double* Xs, int lane)
{
    const int n = a.N, p = a.p;
    const double tau2 = th[0] * th[0], lam2 = th[1] * th[1], s2 = th[2] * th[2] + a.jitter;
    for (int i = 0; i < n; ++i) {
        const int base = i * (i + 1) / 2;
        for (int k = lane; k <= i; k += 64) {
            double r2 = 0.0;
            for (int d = 0; d < p; ++d) {
                const double e = Xs[i * p + d] - Xs[k * p + d];
                r2 = fma(e, e, r2);
            }
            A[base + k] = tau2 * exp(-lam2 * r2) + (i == k ? s2 : 0.0);
        }
    }
    double yv[2];
    int rb[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int i = lane + 64 * r;
        yv[r] = i < n ? a.y[i] : 0.0;
        rb[r] = i * (i + 1) / 2;
    }
    __syncthreads();
    double quad = 0.0, ld = 0.0;
    for (int j = 0; j < n; ++j) {
        const double ajj = A[j * (j + 1) / 2 + j];
        if (!(ajj > 0.0)) return -INFINITY;  // wave-uniform
        const double ljj = sqrt(ajj);
        ld += log(ljj);
        // column j below the diagonal: registers and cb
        double col[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int i = lane + 64 * r;
            const bool own = i > j && i < n;
            col[r] = own ? A[rb[r] + j] / ljj : 0.0;
            if (own) cb[i] = col[r];
        }
        // forward solve alongside: z_j = y_j / L_jj, y_i -= L_ij z_j
        const double zj = (j < 64 ? rl(yv[0], j) : rl(yv[1], j - 64)) / ljj;
        quad += zj * zj;
#pragma unroll
        for (int r = 0; r < 2; ++r) yv[r] = fma(-col[r], zj, yv[r]);
        __syncthreads();  // cb complete
        // trailing triangle: A_ik -= L_ij L_kj for j < k <= i, k in groups of four
        for (int k0 = j + 1; k0 < n; k0 += 4) {
            double lk[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) lk[q] = k0 + q < n ? cb[k0 + q] : 0.0;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int i = lane + 64 * r;
                if (i >= k0 && i < n) {
                    double* ar = A + rb[r] + k0;
                    double v[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = k0 + q <= i ? ar[q] : 0.0;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (k0 + q <= i) ar[q] = fma(-col[r], lk[q], v[q]);
                }
            }
        }
        __syncthreads();  // the trailing triangle is updated; cb may be rewritten
    }
    return -0.5 * quad - ld;
}

// One FSM step of chain c (ESS: INIT or SHRINK, then the proposal and its
// likelihood, accept -> DONE).  Returns 1 when the step ended a draw.
struct GphState {
    double th[3], nu[3], lx, phi, pmin, pmax, logu;
    int k, evals;
    uint32_t t;
};

template <typename LL>
__device__ __forceinline__ int gph_step(const GphK& a, int c, GphState& S, LL loglik, int lane, uint32_t* guard)
{
    if (S.k == 1) {  // INIT: direction, threshold, first angle and bracket
#pragma unroll
        for (int d = 0; d < 3; ++d) S.nu[d] = normal_at<double>(a.seed, (uint32_t)c, S.t, ROLE_NU, 0, (uint32_t)d);
        S.logu = log(uniform<double>(a.seed, (uint32_t)c, S.t, ROLE_THRESH, 0));
        S.phi = 2.0 * 3.14159265358979323846 * uniform<double>(a.seed, (uint32_t)c, S.t, ROLE_ANGLE, 0);
        S.pmin = S.phi - 2.0 * 3.14159265358979323846;
        S.pmax = S.phi;
        S.evals = 0;
    } else {  // SHRINK: the bracket moves to the rejected angle, draw again
        if (S.phi < 0.0)
            S.pmin = S.phi;
        else
            S.pmax = S.phi;
        S.phi = S.pmin + (S.pmax - S.pmin) * uniform<double>(a.seed, (uint32_t)c, S.t, ROLE_ANGLE, (uint32_t)S.evals);
    }
    const double cs = cos(S.phi), sn = sin(S.phi);
    double tp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) tp[d] = S.th[d] * cs + S.nu[d] * sn;
    const double lp = loglik(tp);
    S.evals += 1;
    const bool acc = lp - S.lx > S.logu;
    const bool stop = !acc && S.evals >= kEssMaxEvals;
    if (!acc && !stop) {
        S.k = 2;
        return 0;
    }
    if (acc) {
#pragma unroll
        for (int d = 0; d < 3; ++d) S.th[d] = tp[d];
        S.lx = lp;
    } else {
        *guard += 1;
    }
    // DONE: emit, then INIT of the next draw
    if (lane < 3) a.out[((size_t)c * a.n + S.t) * 3 + lane] = lane == 0 ? S.th[0] : (lane == 1 ? S.th[1] : S.th[2]);
    if (lane == 0) a.counts[(size_t)c * a.n + S.t] = S.evals;
    S.t += 1;
    S.k = 1;
    return 1;
}

__device__ __forceinline__ void gph_load(const GphK& a, int c, GphState& S)
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        S.th[d] = uni(a.th[(size_t)c * 3 + d]);
        S.nu[d] = uni(a.nu[(size_t)c * 3 + d]);
    }
    S.lx = uni(a.lx[c]);
    S.phi = uni(a.phi[c]);
    S.pmin = uni(a.pmin[c]);
    S.pmax = uni(a.pmax[c]);
    S.logu = uni(a.logu[c]);
    S.k = uni(a.k[c]);
    S.evals = uni(a.evals[c]);
    S.t = uni(a.t[c]);
}

__device__ __forceinline__ void gph_store(const GphK& a, int c, const GphState& S, int lane)
{
    if (lane == 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            a.th[(size_t)c * 3 + d] = S.th[d];
            a.nu[(size_t)c * 3 + d] = S.nu[d];
        }
        a.lx[c] = S.lx;
        a.phi[c] = S.phi;
        a.pmin[c] = S.pmin;
        a.pmax[c] = S.pmax;
        a.logu[c] = S.logu;
        a.k[c] = S.k;
        a.evals[c] = S.evals;
        a.t[c] = S.t;
    }
}

__device__ __forceinline__ void gph_stage(const GphK& a, double* Xs)
{
    for (int i = threadIdx.x; i < a.N * a.p; i += blockDim.x) Xs[i] = a.X[i];
    __syncthreads();
}

// mode 0: FSM (to tstop or through the budget); mode 1: one draw of the
// synchronized runtime (tstop = draw + 1), recording its largest count;
// mode 2: vmap padding of draw `draw`.
__global__ __launch_bounds__(64) void gph_kernel(GphK a, unsigned long long* q, unsigned long long base, int mode,
                                                 uint32_t draw)
{
    extern __shared__ double gsm[];
    double* Xs = gsm;
    double* A = gsm + ((a.N * a.p + 1) & ~1);
    double* cb = A + a.N * (a.N + 1) / 2;
    gph_stage(a, Xs);
    const int lane = threadIdx.x;
    unsigned long long steps = 0, padded = 0;
    uint32_t guard = 0;
    for (;;) {
        const int c = gph_next_chain(q, base, a.m, lane);
        if (c >= a.m) break;
        if (mode == 2) {
            const int reps = a.maxN[draw] - uni(a.counts[(size_t)c * a.n + draw]);
            double th[3], acc = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) th[d] = uni(a.th[(size_t)c * 3 + d]);
            for (int r = 0; r < reps; ++r) acc += gph_loglik(a, th, A, cb, Xs, lane);
            if (reps > 0 && lane == 0) a.sink[c] = acc;
            padded += (unsigned long long)max(reps, 0);
            continue;
        }
        GphState S;
        gph_load(a, c, S);
        const uint32_t stop = mode == 1 ? draw + 1 : a.tstop;
        if (S.t >= stop) continue;
        const uint32_t t0 = S.t;
        int64_t budget = uni((int64_t)a.budget[c]);
        while (S.t < stop && budget > 0) {
            (void)gph_step(a, c, S, [&](const double* tp) { return gph_loglik(a, tp, A, cb, Xs, lane); }, lane,
                           &guard);
            ++steps;
            --budget;
        }
        gph_store(a, c, S, lane);
        if (lane == 0) a.budget[c] = budget;
        if (mode == 1 && lane == 0 && S.t > t0) atomicMax(&a.maxN[t0], a.counts[(size_t)c * a.n + t0]);
    }
    if (lane == 0) {
        if (steps) atomicAdd(&a.ctr[0], steps);
        if (padded) atomicAdd(&a.ctr[1], padded);
        if (guard) atomicAdd(&a.ctr[2], (unsigned long long)guard);
    }
}

// Starting state: theta (from x0 or a prior draw N(0, I) on the INIT stream)
// and its log-likelihood, one wave per chain.
__global__ __launch_bounds__(64) void gph_init_kernel(GphK a, int has_x0)
{
    extern __shared__ double gsm[];
    double* Xs = gsm;
    double* A = gsm + ((a.N * a.p + 1) & ~1);
    double* cb = A + a.N * (a.N + 1) / 2;
    gph_stage(a, Xs);
    const int lane = threadIdx.x;
    for (int c = blockIdx.x; c < a.m; c += gridDim.x) {
        double th[3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            th[d] = has_x0 ? uni(a.th[(size_t)c * 3 + d]) : normal_at<double>(a.seed, (uint32_t)c, 0, ROLE_INIT, 0, (uint32_t)d);
        const double lx = gph_loglik(a, th, A, cb, Xs, lane);
        if (lane == 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) a.th[(size_t)c * 3 + d] = th[d];
            a.lx[c] = lx;
            a.k[c] = 1;
        }
    }
}

// ------------------------------------------------------------ n > 96
// LDS of the block likelihood, in doubles: the panel below the diagonal block
// [32][ld - 32] (column t, row r), the diagonal block [32][33], the
// reciprocal pivots [32], y [ld], and 8 scalars.
__host__ __device__ constexpr size_t gph_big_lds_doubles(int ld) { return 32 * (size_t)(ld - 32) + 32 * 33 + 32 + ld + 8; }

// log L(th) by the block (kGphBigWaves waves) with C in `slot` (ld x ld, row-major,
// lower triangle).  The result is the same in every thread.
__device__ double gph_loglik_big(const GphK& a, const double* th, double* slot, double* sm)
{
    const int ld = a.ld, n = a.N, p = a.p;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int pr = ld - 32;  // panel row pitch
    double* Lp = sm;
    double* Ds = Lp + 32 * (size_t)pr;
    double* rinv = Ds + 32 * 33;
    double* yv = rinv + 32;
    double* red = yv + ld;  // [0] sum log L_jj, [1] |z|^2, [2] a pivot was not positive
    const double tau2 = th[0] * th[0], lam2 = th[1] * th[1], s2 = th[2] * th[2] + a.jitter;
    // C's lower triangle; rows and columns past n are the identity's.  Lane
    // k of a 64-column chunk keeps x_k in registers; the row's x_i is the
    // same for the whole wave.
    for (int k0c = 0; k0c < ld; k0c += 64) {
        const int k = k0c + lane;
        double xk[kGphMaxP];
#pragma unroll
        for (int d = 0; d < kGphMaxP; ++d) xk[d] = (d < p && k < n) ? a.X[k * p + d] : 0.0;
        for (int i = k0c + wave; i < ld; i += kGphBigWaves) {
            if (k > i) continue;
            double v;
            if (i < n && k < n) {
                double r2 = 0.0;
#pragma unroll
                for (int d = 0; d < kGphMaxP; ++d) {
                    if (d < p) {
                        const double e = a.X[i * p + d] - xk[d];
                        r2 = fma(e, e, r2);
                    }
                }
                v = tau2 * exp(-lam2 * r2) + (i == k ? s2 : 0.0);
            } else {
                v = i == k ? 1.0 : 0.0;
            }
            slot[(size_t)i * ld + k] = v;
        }
    }
    for (int i = tid; i < ld; i += blockDim.x) yv[i] = i < n ? a.y[i] : 0.0;
    if (tid < 3) red[tid] = 0.0;
    __syncthreads();
    for (int k0 = 0; k0 < ld; k0 += 32) {
        const int m = ld - k0 - 32;  // rows below the panel's diagonal block
        // (a) the diagonal block by wave 0, in registers: lane r < 32 holds
        //     row r; column entries of other rows come by lane broadcast
        if (wave == 0) {
            double dr[32];
#pragma unroll
            for (int c = 0; c < 32; ++c)
                dr[c] = (lane < 32 && c <= lane) ? slot[(size_t)(k0 + lane) * ld + k0 + c] : 0.0;
            double ld_acc = 0.0, yr = lane < 32 ? yv[k0 + lane] : 0.0, q = 0.0;
            bool bad = false;
#pragma unroll
            for (int j = 0; j < 32; ++j) {
                const double djj = rl(dr[j], j);
                bad = bad || !(djj > 0.0);
                const double ljj = sqrt(djj), r = 1.0 / ljj;
                ld_acc += log(ljj);
                const double zj = rl(yr, j) * r;  // forward solve inside the block
                q += zj * zj;
                dr[j] = lane > j ? dr[j] * r : (lane == j ? ljj : dr[j]);  // L_rj
                if (lane > j) yr = fma(-dr[j], zj, yr);
#pragma unroll
                for (int c = j + 1; c < 32; ++c) {
                    const double lcj = rl(dr[j], c);
                    if (lane >= c) dr[c] = fma(-dr[j], lcj, dr[c]);
                }
                if (lane == j) {
                    rinv[j] = r;
                    yv[k0 + j] = zj;  // z_j, read by the rows below
                }
            }
            if (lane < 32) {
#pragma unroll
                for (int c = 0; c < 32; ++c) Ds[lane * 33 + c] = dr[c];
            }
            if (lane == 0) {
                red[0] += ld_acc;
                red[1] += q;
                if (bad) red[2] = 1.0;
            }
        }
        __syncthreads();
        if (red[2] != 0.0) return -INFINITY;  // block-uniform
        // (b) the rows below: L_it = (C_it - sum_{s<t} L_is L_ts) / L_tt, right-looking
        //     within the row; y_i -= sum_t L_it z_t
        for (int r = tid; r < m; r += blockDim.x) {
            const int i = k0 + 32 + r;
            double v[32];
            const double* src = slot + (size_t)i * ld + k0;
#pragma unroll
            for (int t = 0; t < 32; ++t) v[t] = src[t];
            double yi = yv[i];
#pragma unroll
            for (int t = 0; t < 32; ++t) {
                v[t] *= rinv[t];
#pragma unroll
                for (int u = t + 1; u < 32; ++u) v[u] = fma(-v[t], Ds[u * 33 + t], v[u]);
                yi = fma(-v[t], yv[k0 + t], yi);
                Lp[(size_t)t * pr + r] = v[t];
            }
            yv[i] = yi;
        }
        __syncthreads();
        // (c) trailing triangle, 32 x 32 tiles (bi >= bj), a 4 x 4 block per lane
        const int nb = m / 32, ntile = nb * (nb + 1) / 2;
        const int a4 = 4 * (lane >> 3), b4 = 4 * (lane & 7);
        for (int tI = wave; tI < ntile; tI += kGphBigWaves) {
            int bi = (int)((sqrt(8.0 * tI + 1.0) - 1.0) * 0.5);
            while ((bi + 1) * (bi + 2) / 2 <= tI) ++bi;
            while (bi * (bi + 1) / 2 > tI) --bi;
            const int bj = tI - bi * (bi + 1) / 2;
            const int r0 = 32 * bi + a4, c0 = 32 * bj + b4;
            if (bi == bj && c0 > r0 + 3) continue;  // wholly above the diagonal
            double acc[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int w = 0; w < 4; ++w) acc[u][w] = slot[(size_t)(k0 + 32 + r0 + u) * ld + k0 + 32 + c0 + w];
#pragma unroll 4
            for (int t = 0; t < 32; ++t) {
                const double* lt = Lp + (size_t)t * pr;
                double li[4], lj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    li[u] = lt[r0 + u];
                    lj[u] = lt[c0 + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int w = 0; w < 4; ++w) acc[u][w] = fma(-li[u], lj[w], acc[u][w]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    if (c0 + w <= r0 + u) slot[(size_t)(k0 + 32 + r0 + u) * ld + k0 + 32 + c0 + w] = acc[u][w];
        }
        __syncthreads();
    }
    return -0.5 * red[1] - red[0];
}

__device__ __forceinline__ int gph_block_next_chain(unsigned long long* q, unsigned long long base, int m, int* sh)
{
    __syncthreads();  // the previous chain's reads of *sh are done
    if (threadIdx.x == 0) {
        const unsigned long long off = atomicAdd(q, 1ull) - base;
        *sh = off < (unsigned long long)m ? (int)off : m;
    }
    __syncthreads();
    return *sh;
}

// The block forms of gph_kernel and gph_init_kernel (n > 96).
__global__ __launch_bounds__(64 * kGphBigWaves) void gph_big_kernel(GphK a, unsigned long long* q, unsigned long long base, int mode,
                                                      uint32_t draw)
{
    extern __shared__ double gsm[];
    __shared__ int s_chain;
    double* slot = a.slots + (size_t)blockIdx.x * a.ld * a.ld;
    const int tid = threadIdx.x;
    auto ll = [&](const double* tp) { return gph_loglik_big(a, tp, slot, gsm); };
    unsigned long long steps = 0, padded = 0;
    uint32_t guard = 0;
    for (;;) {
        const int c = gph_block_next_chain(q, base, a.m, &s_chain);
        if (c >= a.m) break;
        if (mode == 2) {
            const int reps = a.maxN[draw] - a.counts[(size_t)c * a.n + draw];
            double th[3], acc = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) th[d] = a.th[(size_t)c * 3 + d];
            for (int r = 0; r < reps; ++r) acc += ll(th);
            if (reps > 0 && tid == 0) a.sink[c] = acc;
            padded += (unsigned long long)max(reps, 0);
            continue;
        }
        GphState S;
        gph_load(a, c, S);
        const uint32_t stop = mode == 1 ? draw + 1 : a.tstop;
        if (S.t >= stop) continue;
        const uint32_t t0 = S.t;
        int64_t budget = a.budget[c];
        while (S.t < stop && budget > 0) {
            (void)gph_step(a, c, S, ll, tid, &guard);
            ++steps;
            --budget;
        }
        __syncthreads();  // every thread has read the chain's state before it is stored
        gph_store(a, c, S, tid);
        if (tid == 0) a.budget[c] = budget;
        if (mode == 1 && tid == 0 && S.t > t0) atomicMax(&a.maxN[t0], a.counts[(size_t)c * a.n + t0]);
    }
    if (tid == 0) {
        if (steps) atomicAdd(&a.ctr[0], steps);
        if (padded) atomicAdd(&a.ctr[1], padded);
        if (guard) atomicAdd(&a.ctr[2], (unsigned long long)guard);
    }
}

__global__ __launch_bounds__(64 * kGphBigWaves) void gph_big_init_kernel(GphK a, int has_x0)
{
    extern __shared__ double gsm[];
    double* slot = a.slots + (size_t)blockIdx.x * a.ld * a.ld;
    for (int c = blockIdx.x; c < a.m; c += gridDim.x) {
        double th[3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            th[d] = has_x0 ? a.th[(size_t)c * 3 + d] : normal_at<double>(a.seed, (uint32_t)c, 0, ROLE_INIT, 0, (uint32_t)d);
        const double lx = gph_loglik_big(a, th, slot, gsm);
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) a.th[(size_t)c * 3 + d] = th[d];
            a.lx[c] = lx;
            a.k[c] = 1;
        }
    }
}

// ------------------------------------------------------------ host side
static GphK gph_view(const JobDev& j)
{
    GphK a;
    a.m = j.m;
    a.n = j.n;
    a.N = j.N;
    a.p = j.pdim;
    a.tstop = j.tstop;
    a.seed = j.seed;
    a.jitter = j.noise_sd;
    a.X = (const double*)j.X;
    a.y = (const double*)j.y;
    a.th = (double*)j.x;
    a.nu = (double*)j.V;
    a.lx = (double*)j.lx;
    a.phi = (double*)j.theta;
    a.pmin = (double*)j.tmin;
    a.pmax = (double*)j.tmax;
    a.logu = (double*)j.logu;
    a.k = j.k;
    a.evals = j.evals;
    a.t = j.t;
    a.budget = j.budget;
    a.out = (double*)j.out;
    a.counts = j.counts;
    a.ctr = j.ctr;
    a.maxN = j.maxN;
    a.sink = (double*)j.sink;
    a.slots = (double*)j.gslot;
    a.ld = (j.N + 31) / 32 * 32;
    return a;
}

static bool gph_big(const JobDev& j) { return j.N > kGphMaxN; }

int gph_max_obs() { return kGphBigMaxN; }
int gph_max_inputs() { return kGphMaxP; }

static size_t gph_lds_bytes(const JobDev& j)
{
    if (gph_big(j)) return 8 * gph_big_lds_doubles((j.N + 31) / 32 * 32);
    return 8 * ((size_t)((j.N * j.pdim + 1) & ~1) + (size_t)j.N * (j.N + 1) / 2 + (size_t)j.N);
}

static int gph_cus()
{
    int cus = 256, dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
        cus = v;
    return cus;
}

static int gph_blocks(const JobDev& j)
{
    const size_t lds = gph_lds_bytes(j);
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(16, (160 * 1024) / std::max<size_t>(lds, 1)));
    return std::max(1, std::min(j.m, gph_cus() * per_cu));
}

size_t gph_slot_bytes(const JobDev& j)
{
    if (!gph_big(j)) return 0;
    const size_t ld = (size_t)(j.N + 31) / 32 * 32;
    return (size_t)gph_blocks(j) * ld * ld * 8;
}

hipError_t gph_setup(JobDev& j)
{
    const size_t lds = gph_lds_bytes(j);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
        const void* k0 = gph_big(j) ? (const void*)gph_big_kernel : (const void*)gph_kernel;
        const void* k1 = gph_big(j) ? (const void*)gph_big_init_kernel : (const void*)gph_init_kernel;
        hipError_t e = hipFuncSetAttribute(k0, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e == hipSuccess) e = hipFuncSetAttribute(k1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    j.pblocks = gph_blocks(j);
    j.pwpb = gph_big(j) ? kGphBigWaves : 1;
    return hipSuccess;
}

hipError_t gph_init_state(const JobDev& j, const void* x0, hipStream_t s)
{
    if (x0) {
        hipError_t e = hipMemcpyAsync(j.x, x0, (size_t)j.m * 3 * 8, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    if (gph_big(j))
        hipLaunchKernelGGL(gph_big_init_kernel, dim3(j.pblocks), dim3(64 * kGphBigWaves), gph_lds_bytes(j), s, gph_view(j), x0 ? 1 : 0);
    else
        hipLaunchKernelGGL(gph_init_kernel, dim3(j.pblocks), dim3(64), gph_lds_bytes(j), s, gph_view(j), x0 ? 1 : 0);
    return hipGetLastError();
}

hipError_t gph_run(const JobDev& j, int mode, uint32_t draw, unsigned long long* ticket, hipStream_t s)
{
    if (gph_big(j))
        hipLaunchKernelGGL(gph_big_kernel, dim3(j.pblocks), dim3(64 * kGphBigWaves), gph_lds_bytes(j), s, gph_view(j),
                           (unsigned long long*)j.queue, *ticket, mode, draw);
    else
        hipLaunchKernelGGL(gph_kernel, dim3(j.pblocks), dim3(64), gph_lds_bytes(j), s, gph_view(j),
                           (unsigned long long*)j.queue, *ticket, mode, draw);
    *ticket += (unsigned long long)j.m + (unsigned long long)j.pblocks;
    return hipGetLastError();
}

}  // namespace fsmmc
