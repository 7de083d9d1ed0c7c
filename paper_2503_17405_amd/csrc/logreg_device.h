// logreg_device.h -- batched potential and gradient of Bayesian logistic
// regression (the NUTS g), shared by the single-job kernels (logreg.hip) and
// the grouped multi-job kernels (batch.hip), so a job's gradients are the
// same bits in either.  Layout and tiling are described in logreg.hip.
#pragma once
#include "fsmmc_device.h"
#include "fsmmc_internal.h"

namespace fsmmc {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

struct GradK {
    int m, N, D, Dp, slice_rows, nslices, dense;  // dense > 0: columns are chains 0 .. dense-1
    const float* X;   // Np x Dp, zero padded
    const uint16_t* Xb;  // X split into three bf16 pieces, two layouts per 32-row chunk (logreg.hip)
    const float* y;   // Np
    const float* Th;  // m x Dp, indexed by chain
    const int32_t* list;
    const int32_t* count;
    float* Gpart;  // nslices x m x Dp (indexed by chain)
    float* Upart;  // nslices x m
};

template <int DT>
struct GradB {
    static constexpr int DP = 32 * DT;          // padded dimension
    static constexpr int PR = 2 * DP + 16;      // LDS bytes per row of a row-major piece
    static constexpr int PD = 80;               // LDS bytes per column of a d-major piece (32 rows + pad)
    static constexpr int XR = 3 * 32 * PR;      // row-major pieces of one chunk
    static constexpr int XBUF = XR + 3 * DP * PD;  // + d-major pieces
    static constexpr int RS = 3 * 128 * PD;     // r pieces, chain-major
    static constexpr int LDS = 2 * XBUF + RS + 8 * 32 * 4 + 128 * 4;
    static constexpr int CHUNK = 384 * DP;      // HBM bytes of one 32-row chunk (both layouts)
    static constexpr int NV = CHUNK / 16 / 512; // 16-byte loads per thread per chunk
    static_assert(CHUNK % (16 * 512) == 0, "chunk loads do not tile the block");
    static_assert(128 * (DP + 4) * 4 <= 2 * XBUF, "gradient staging exceeds the X buffers");
};

// LDS byte offset of the 16-byte unit f of a chunk (HBM order: row-major
// pieces [p][row][d], then d-major pieces [p][d][row]).
template <int DT>
__device__ __forceinline__ int gradb_lds_off(int f)
{
    using S = GradB<DT>;
    constexpr int DP = S::DP;
    if (f < 12 * DP) {
        const int p = f / (4 * DP), r = f - p * 4 * DP;
        const int row = r / (DP / 8), c = r - row * (DP / 8);
        return p * 32 * S::PR + row * S::PR + 16 * c;
    }
    const int g = f - 12 * DP;
    const int p = g / (4 * DP), r = g - p * 4 * DP;
    return S::XR + p * DP * S::PD + (r >> 2) * S::PD + 16 * (r & 3);
}

__device__ __forceinline__ uint4 pack_bf16x8(const uint32_t (&v)[8])
{
    return make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16), v[6] | (v[7] << 16));
}

// acc += A B for FP32 A, B given as three bf16 pieces each (the six leading
// piece products, small terms first).
__device__ __forceinline__ floatx4 mfma_bf16x6(const uint4 (&A)[3], const uint4 (&B)[3], floatx4 acc)
{
    const bf16x8 ah = __builtin_bit_cast(bf16x8, A[0]), am = __builtin_bit_cast(bf16x8, A[1]),
                 al = __builtin_bit_cast(bf16x8, A[2]);
    const bf16x8 bh = __builtin_bit_cast(bf16x8, B[0]), bm = __builtin_bit_cast(bf16x8, B[1]),
                 bl = __builtin_bit_cast(bf16x8, B[2]);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
    return acc;
}

// One block of 8 waves (GradB<DT>::LDS bytes of dynamic LDS at lds): listed
// chains 128 ct .. 128 ct + 127, row slice sl.  NK8 > 0: the dimension rounded
// up to 8 is 8 NK8 (compile-time trip counts); NK8 = 0: any dimension up to
// 32 DT (run-time trip counts over the same unrolled steps, so both forms
// give the same bits).
template <int DT, int NK8 = 0>
__device__ __forceinline__ void logreg_grad_tile(const GradK& a, int ct, int sl, unsigned char* lds)
{
    using S = GradB<DT>;
    constexpr int DP = S::DP, PR = S::PR, PD = S::PD;
    constexpr int NK32 = NK8 > 0 ? (NK8 + 3) / 4 : DT;  // eta k steps of 32 (d), at most
    constexpr int NT = NK8 > 0 ? (NK8 + 1) / 2 : 2 * DT;  // gradient d tiles of 16 that can be nonzero
    constexpr int NTW = (NT + 1) / 2;                   // d tiles per wave (at most)
    static_assert(NK8 >= 0 && 32 * NK32 <= DP, "dimension class exceeds the tile");
    const int nk32 = NK8 > 0 ? NK32 : (a.D + 31) >> 5;
    const int nt = NK8 > 0 ? NT : (a.D + 15) >> 4;
    unsigned char* Rs = lds + 2 * S::XBUF;
    float* Ured = reinterpret_cast<float*>(Rs + S::RS);  // [wave][32 chains]
    int* cols = reinterpret_cast<int*>(Ured + 8 * 32);

    const int ncols = a.dense > 0 ? a.dense : *a.count;
    if (ct * 128 >= ncols) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, q4 = lane >> 4;
    if (tid < 128) {
        const int g = ct * 128 + tid;
        cols[tid] = g < ncols ? (a.dense > 0 ? g : a.list[g]) : -1;
    }
    const int rb = sl * a.slice_rows;
    const int re = min(rb + a.slice_rows, a.N);
    const int nchunk = (re - rb + 31) / 32;
    const uint4* xsrc = reinterpret_cast<const uint4*>(a.Xb) + (size_t)(rb / 32) * (S::CHUNK / 16);
    // a chunk's share of this thread (named registers: an array here ends up in scratch)
    static_assert(S::NV == 3 || S::NV == 6, "chunk share");
    uint4 s0, s1, s2, s3, s4, s5;
    auto load_chunk = [&](const uint4* src) {
        s0 = src[tid];
        s1 = src[tid + 512];
        s2 = src[tid + 1024];
        if (S::NV == 6) {
            s3 = src[tid + 1536];
            s4 = src[tid + 2048];
            s5 = src[tid + 2560];
        }
    };
    auto store_chunk = [&](unsigned char* dst) {
        *reinterpret_cast<uint4*>(dst + gradb_lds_off<DT>(tid)) = s0;
        *reinterpret_cast<uint4*>(dst + gradb_lds_off<DT>(tid + 512)) = s1;
        *reinterpret_cast<uint4*>(dst + gradb_lds_off<DT>(tid + 1024)) = s2;
        if (S::NV == 6) {
            *reinterpret_cast<uint4*>(dst + gradb_lds_off<DT>(tid + 1536)) = s3;
            *reinterpret_cast<uint4*>(dst + gradb_lds_off<DT>(tid + 2048)) = s4;
            *reinterpret_cast<uint4*>(dst + gradb_lds_off<DT>(tid + 2560)) = s5;
        }
    };
    if (nchunk > 0) load_chunk(xsrc);
    __syncthreads();  // cols

    // eta roles and the Theta pieces of this wave's two chain tiles (B operand:
    // lane holds Theta[chain 16 t + l16][32 kk + 8 q4 .. + 7])
    const int rt = wave & 1, ep = wave >> 1;
    uint4 thb[2][NK32][3];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int ch = cols[32 * ep + 16 * t + l16];
#pragma unroll
        for (int kk = 0; kk < NK32; ++kk) {
            float4 u0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), u1 = u0;
            if (ch >= 0 && kk < nk32) {
                const float4* p = reinterpret_cast<const float4*>(a.Th + (size_t)ch * DP + 32 * kk + 8 * q4);
                u0 = p[0];
                u1 = p[1];
            }
            const float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
            uint32_t h[8], m[8], l[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) split_bf16x3(v[e], h[e], m[e], l[e]);
            thb[t][kk][0] = pack_bf16x8(h);
            thb[t][kk][1] = pack_bf16x8(m);
            thb[t][kk][2] = pack_bf16x8(l);
        }
    }
    if (nchunk > 0) store_chunk(lds);

    // gradient roles: chain tiles 2 cp, 2 cp + 1; d tiles h, h + 2, ...
    const int cp = wave & 3, hh = wave >> 2;
    floatx4 accg[NTW][2];
#pragma unroll
    for (int j = 0; j < NTW; ++j)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) accg[j][u][q] = 0.0f;
    float uacc[2] = {0.0f, 0.0f};

    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        // the next chunk (the last chunk again on the last pass: its copy into
        // the idle buffer is never read)
        load_chunk(xsrc + (size_t)min(ch + 1, nchunk - 1) * (S::CHUNK / 16));
        __syncthreads();  // chunk ch in buffer buf; the previous chunk's r and buffer buf ^ 1 no longer read
        const unsigned char* XB = lds + buf * S::XBUF;
        // 1. eta: A = X rows (lane: row 16 rt + l16, d 32 kk + 8 q4 .. + 7), B = Theta pieces
        floatx4 e0 = {0.0f, 0.0f, 0.0f, 0.0f}, e1 = e0;
        const unsigned char* xr = XB + (16 * rt + l16) * PR + 16 * q4;
#pragma unroll
        for (int kk = 0; kk < NK32; ++kk) {
            if (kk >= nk32) break;
            const uint4 xa[3] = {*reinterpret_cast<const uint4*>(xr + 64 * kk),
                                 *reinterpret_cast<const uint4*>(xr + 32 * PR + 64 * kk),
                                 *reinterpret_cast<const uint4*>(xr + 64 * PR + 64 * kk)};
            e0 = mfma_bf16x6(xa, thb[0][kk], e0);
            e1 = mfma_bf16x6(xa, thb[1][kk], e1);
        }
        // 2. r = y - sigmoid(eta), split into pieces, to LDS; log-likelihood:
        //    sum [y eta - max(eta, 0)] minus one log of the product of the four
        //    factors 1 + e^-|eta| (each in (1, 2])
        const int r0 = rb + 32 * ch;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const floatx4 e = t ? e1 : e0;
            const int col = 32 * ep + 16 * t + l16;
            float lin = 0.0f, prod = 1.0f;
            uint32_t ph[4], pm[4], pl[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = r0 + 16 * rt + 4 * q4 + i;
                const bool ok = row < re;
                const float v = e[i];
                const float yv = a.y[row];
                const float ex = __expf(-fabsf(v));
                const float inv = __builtin_amdgcn_rcpf(1.0f + ex);  // hardware reciprocal, 1 ulp
                const float sig = v >= 0.0f ? inv : ex * inv;
                lin += ok ? (yv * v - fmaxf(v, 0.0f)) : 0.0f;
                prod *= ok ? 1.0f + ex : 1.0f;
                split_bf16x3(ok ? (yv - sig) : 0.0f, ph[i], pm[i], pl[i]);
            }
            uacc[t] += lin - __logf(prod);
            unsigned char* rp = Rs + col * PD + 2 * (16 * rt + 4 * q4);
            *reinterpret_cast<uint2*>(rp) = make_uint2(ph[0] | (ph[1] << 16), ph[2] | (ph[3] << 16));
            *reinterpret_cast<uint2*>(rp + 128 * PD) = make_uint2(pm[0] | (pm[1] << 16), pm[2] | (pm[3] << 16));
            *reinterpret_cast<uint2*>(rp + 256 * PD) = make_uint2(pl[0] | (pl[1] << 16), pl[2] | (pl[3] << 16));
        }
        __syncthreads();  // r complete
        // 3. X_chunk^T r: A = X columns (lane: d 16 t + l16, rows 8 q4 .. + 7), B = r pieces
        uint4 rpc[2][3];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const unsigned char* rp = Rs + (32 * cp + 16 * u + l16) * PD + 16 * q4;
#pragma unroll
            for (int p = 0; p < 3; ++p) rpc[u][p] = *reinterpret_cast<const uint4*>(rp + p * 128 * PD);
        }
        const unsigned char* XD = XB + S::XR;
#pragma unroll
        for (int j = 0; j < NTW; ++j) {
            const int t = hh + 2 * j;
            if (t < nt) {
                const unsigned char* xp = XD + (16 * t + l16) * PD + 16 * q4;
                const uint4 xa[3] = {*reinterpret_cast<const uint4*>(xp),
                                     *reinterpret_cast<const uint4*>(xp + DP * PD),
                                     *reinterpret_cast<const uint4*>(xp + 2 * DP * PD)};
                accg[j][0] = mfma_bf16x6(xa, rpc[0], accg[j][0]);
                accg[j][1] = mfma_bf16x6(xa, rpc[1], accg[j][1]);
            }
        }
        store_chunk(lds + (buf ^ 1) * S::XBUF);
    }
    // log-likelihood per chain: lanes of one column hold different rows
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        uacc[t] += __shfl_xor(uacc[t], 16, 64);
        uacc[t] += __shfl_xor(uacc[t], 32, 64);
    }
    __syncthreads();  // X buffers free
    if (q4 == 0) {
        Ured[wave * 32 + l16] = uacc[0];
        Ured[wave * 32 + 16 + l16] = uacc[1];
    }
    // gradient tiles -> LDS [chain][d] over the X buffers, for coalesced stores
    constexpr int TP = DP + 4;
    float* Red = reinterpret_cast<float*>(lds);
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
        const int t = hh + 2 * j;
        if (t < nt) {
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    Red[(32 * cp + 16 * u + l16) * TP + 16 * t + 4 * q4 + q] = accg[j][u][q];
        }
    }
    const int DZ = DP - 16 * nt;  // d past the last tile: zero
    if (DZ > 0) {
        for (int i = tid; i < 128 * DZ; i += 512) {
            const int col = i / DZ;
            Red[col * TP + 16 * nt + (i - col * DZ)] = 0.0f;
        }
    }
    __syncthreads();
    for (int i = tid; i < 128 * DP; i += 512) {
        const int col = i / DP, d = i - col * DP;
        const int chn = cols[col];
        if (chn >= 0) a.Gpart[((size_t)sl * a.m + chn) * DP + d] = Red[col * TP + d];
    }
    if (tid < 128 && cols[tid] >= 0) {
        // waves 2k (rows 0..15 of each chunk) and 2k+1 (rows 16..31) cover chains 32k .. 32k+31
        const int w0 = 2 * (tid >> 5), i = tid & 31;
        a.Upart[(size_t)sl * a.m + cols[tid]] = Ured[w0 * 32 + i] + Ured[(w0 + 1) * 32 + i];
    }
}

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
    g.Xb = (const uint16_t*)j.Xb;
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
