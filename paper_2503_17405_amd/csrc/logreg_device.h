// logreg_device.h -- batched potential and gradient of Bayesian logistic
// regression (the NUTS g), shared by the single-job kernels (logreg.hip) and
// the grouped multi-job kernels (batch.hip).  Layout and tiling are described
// in logreg.hip.
#pragma once
#include "fsmmc_device.h"
#include "fsmmc_internal.h"

namespace fsmmc {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

struct GradK {
    int m, N, D, Dp, slice_rows, nslices, dense;  // dense > 0: columns are chains 0 .. dense-1
    const float* X;   // Np x Dp, zero padded
    const float* y;   // Np
    const float* Th;  // m x Dp, indexed by chain
    const int32_t* list;
    const int32_t* count;
    float* Gpart;  // nslices x m x Dp (indexed by chain)
    float* Upart;  // nslices x m
};

// One block (4 waves): listed chains 64 ct .. 64 ct + 63, row slice sl.
// NK8 > 0: the dimension rounded up to 8 is 8 NK8 (compile-time trip counts,
// fully unrolled); NK8 = 0: any dimension up to 32 DT (run-time trip counts).
template <int DT, int NK8 = 0>
__device__ __forceinline__ void logreg_grad_tile(const GradK& a, int ct, int sl)
{
    static_assert(NK8 >= 0 && 8 * NK8 <= 32 * DT, "dimension class exceeds the tile");
    constexpr int DP = 32 * DT;  // padded dimension (row pitch of X and Theta in HBM)
    constexpr int TP = DP + 4;   // LDS row pitch of Theta and X chunks (conflict-free eta reads)
    constexpr int RP = 64 + 16;  // LDS row pitch of r (conflict-free gradient reads)
    constexpr int NT = DP / 16;  // gradient d tiles of 16 (at most)
    __shared__ float Ths[64 * TP];
    __shared__ float Xs[2][32 * TP];
    __shared__ float Rs[32 * RP];
    __shared__ float Ured[4][64];
    __shared__ int cols[64];

    const int ncols = a.dense > 0 ? a.dense : *a.count;
    if (ct * 64 >= ncols) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, q4 = lane >> 4;
    // K steps of 4 for eta, 16-row tiles of the gradient
    const int nk4 = NK8 > 0 ? 2 * NK8 : (a.D + 3) >> 2;
    const int nt16 = NK8 > 0 ? (NK8 + 1) / 2 : (a.D + 15) >> 4;

    if (tid < 64) {
        const int g = ct * 64 + tid;
        cols[tid] = g < ncols ? (a.dense > 0 ? g : a.list[g]) : -1;
    }
    __syncthreads();
    for (int i = tid; i < 64 * DP; i += 256) {
        const int col = i / DP, d = i - col * DP;
        const int ch = cols[col];
        Ths[col * TP + d] = ch >= 0 ? a.Th[(size_t)ch * DP + d] : 0.0f;
    }
    // roles: eta rows 16 rt .. +15 x chain tiles et0, et0 + 1; gradient: chain tile `wave`, every d tile
    const int rt = wave & 1;
    const int et0 = 2 * (wave >> 1);
    floatx4 accg[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) accg[t][q] = 0.0f;
    float uacc[2] = {0.0f, 0.0f};

    const int rb = sl * a.slice_rows;
    const int re = min(rb + a.slice_rows, a.N);
    const int nchunk = (re - rb + 31) / 32;
    constexpr int V4 = 32 * DP / 4 / 256;
    floatx4 stage[V4];
    if (nchunk > 0) {
        const floatx4* src = reinterpret_cast<const floatx4*>(a.X + (size_t)rb * DP);
#pragma unroll
        for (int v = 0; v < V4; ++v) {
            const int f = tid + 256 * v, row = f / (DP / 4), c4 = f - row * (DP / 4);
            *reinterpret_cast<floatx4*>(&Xs[0][row * TP + 4 * c4]) = src[f];
        }
    }
    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunk) {
            const floatx4* src = reinterpret_cast<const floatx4*>(a.X + (size_t)(rb + 32 * (ch + 1)) * DP);
#pragma unroll
            for (int v = 0; v < V4; ++v) stage[v] = src[tid + 256 * v];
        }
        __syncthreads();  // chunk ch in Xs[buf]; previous chunk's Rs and Xs[buf ^ 1] no longer read
        const float* X = Xs[buf];
        // 1. eta tiles (16 rows x 16 chains), K = D rounded up to 4
        floatx4 e0 = {0.0f, 0.0f, 0.0f, 0.0f}, e1 = {0.0f, 0.0f, 0.0f, 0.0f};
        // operands of step kk + 1 are read from LDS while the MFMAs of step kk run
        // (the read after the last step stays inside the row: k <= DP + 3 < TP)
        const float* xrow = X + (16 * rt + l16) * TP + q4;
        const float* b0row = Ths + (16 * et0 + l16) * TP + q4;
        const float* b1row = Ths + (16 * (et0 + 1) + l16) * TP + q4;
        float xa = xrow[0], b0 = b0row[0], b1 = b1row[0];
#pragma unroll 8
        for (int kk = 0; kk < nk4; ++kk) {
            const float xn = xrow[4 * kk + 4], b0n = b0row[4 * kk + 4], b1n = b1row[4 * kk + 4];
            __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the MFMAs
            e0 = __builtin_amdgcn_mfma_f32_16x16x4f32(xa, b0, e0, 0, 0, 0);
            e1 = __builtin_amdgcn_mfma_f32_16x16x4f32(xa, b1, e1, 0, 0, 0);
            xa = xn;
            b0 = b0n;
            b1 = b1n;
        }
        // 2. r = y - sigmoid(eta) into LDS, and the log-likelihood: sum [y eta - max(eta, 0)]
        //    minus one log of the product of the four factors 1 + e^-|eta| (each in (1, 2])
        const int r0 = rb + 32 * ch;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const floatx4 e = t ? e1 : e0;
            const int col = 16 * (et0 + t) + l16;
            float lin = 0.0f, prod = 1.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int lr = 16 * rt + 4 * q4 + i;
                const int row = r0 + lr;
                const bool ok = row < re;
                const float v = e[i];
                const float yv = a.y[row];
                const float ex = __expf(-fabsf(v));
                const float inv = __builtin_amdgcn_rcpf(1.0f + ex);  // hardware reciprocal, 1 ulp
                const float sig = v >= 0.0f ? inv : ex * inv;
                lin += ok ? (yv * v - fmaxf(v, 0.0f)) : 0.0f;
                prod *= ok ? 1.0f + ex : 1.0f;
                Rs[lr * RP + col] = ok ? (yv - sig) : 0.0f;
            }
            uacc[t] += lin - __logf(prod);
        }
        __syncthreads();  // r complete
        // 3. X_chunk^T r: 16 d x 16 chains tiles, K = 32 rows in steps of 4
        float rv[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) rv[kk] = Rs[(4 * kk + q4) * RP + 16 * wave + l16];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t < nt16) {
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) {
                    const float xa = X[(4 * kk + q4) * TP + 16 * t + l16];
                    accg[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa, rv[kk], accg[t], 0, 0, 0);
                }
            }
        }
        if (ch + 1 < nchunk) {
#pragma unroll
            for (int v = 0; v < V4; ++v) {
                const int f = tid + 256 * v, row = f / (DP / 4), c4 = f - row * (DP / 4);
                *reinterpret_cast<floatx4*>(&Xs[buf ^ 1][row * TP + 4 * c4]) = stage[v];
            }
        }
    }
    // log-likelihood per chain: lanes of one column hold different rows
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        uacc[t] += __shfl_xor(uacc[t], 16, 64);
        uacc[t] += __shfl_xor(uacc[t], 32, 64);
    }
    __syncthreads();
    if (q4 == 0) {
        Ured[wave][16 * et0 + l16] = uacc[0];
        Ured[wave][16 * (et0 + 1) + l16] = uacc[1];
    }
    // gradient tiles -> LDS [chain][d] (reusing Ths) for coalesced stores
    float* Red = Ths;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int d = 16 * t + 4 * q4 + q;
            Red[(16 * wave + l16) * TP + d] = t < nt16 ? accg[t][q] : 0.0f;
        }
    __syncthreads();
    for (int i = tid; i < 64 * DP; i += 256) {
        const int col = i / DP, d = i - col * DP;
        const int chn = cols[col];
        if (chn >= 0) a.Gpart[((size_t)sl * a.m + chn) * DP + d] = Red[col * TP + d];
    }
    if (tid < 64 && cols[tid] >= 0) {
        // waves 2k and 2k+1 cover the two row tiles of chains 32k .. 32k+31
        const int w0 = (tid >> 5) * 2;
        a.Upart[(size_t)sl * a.m + cols[tid]] = Ured[w0][tid] + Ured[w0 + 1][tid];
    }
}

// v2: eta on 16x16x4 with K = ceil(D/4)*4; X^T r on 16x16x4 tiles of 16 d; one log per 4 rows

struct ReduceK {
    int m, Dp, nslices, dense;
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
__device__ __forceinline__ void logreg_reduce_one(const ReduceK& a, int p, int lane)
{

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

// Views of a NUTS job's gradient buffers.  dense > 0: the columns are chains
// 0 .. dense-1 instead of the compacted request list.
inline GradK grad_view(const JobDev& j, int dense)
{
    GradK g;
    g.m = j.m;
    g.N = j.N;
    g.D = j.D;
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
    return g;
}

inline ReduceK reduce_view(const JobDev& j, int dense, float* Gout, float* Uout, int gstride)
{
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
    return r;
}

}  // namespace fsmmc
