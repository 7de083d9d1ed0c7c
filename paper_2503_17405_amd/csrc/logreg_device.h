// logreg_device.h -- batched potential and gradient of Bayesian logistic
// regression (the NUTS g), shared by the single-job kernels (logreg.hip) and
// the grouped multi-job kernels (batch.hip), so a job's gradients are the
// same bits in either.  Layout and tiling are described in logreg.hip.
#pragma once
#include "fsmmc_device.h"
#include "fsmmc_internal.h"
#include <type_traits>

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

// LDS images of X chunks and of r, unpadded, with 16-byte units permuted
// (XOR swizzles) so that the operand reads (16-byte reads: four passes of 16
// lanes, lanes 0-7 with 16-23, 8-15 with 24-31, ...) touch 64 distinct banks
// per pass.
template <int DT>
struct GradB {
    static constexpr int DP = 32 * DT;      // padded dimension
    static constexpr int PR = 2 * DP;       // LDS bytes per row of a row-major piece
    static constexpr int XRB = 3 * 32 * PR; // row-major pieces of one chunk
    static constexpr int XDB = 3 * DP * 64; // d-major pieces of one chunk (64 bytes = 32 rows per column)
    static constexpr int RSB = 3 * 128 * 64; // r pieces of one chunk, chain-major
    static constexpr int XD0 = 2 * XRB, RS0 = XD0 + 2 * XDB, AUX0 = RS0 + 2 * RSB;
    static constexpr int LDS = AUX0 + 8 * 32 * 4 + 128 * 4;
    static constexpr int CHUNK = 384 * DP;  // HBM bytes of one 32-row chunk: row-major pieces, then d-major
    static constexpr int NU = XRB / 16;     // 16-byte units per layout per chunk
    static_assert(XRB == XDB, "chunk layouts");
    static_assert(128 * (DP + 4) * 4 <= AUX0, "gradient staging exceeds the buffers");
    // unit permutation of a row-major row: rows 8k .. 8k+7 map the eight lanes
    // of a read pass to eight distinct unit pairs
    static __device__ __forceinline__ int rowswz(int row)
    {
        return DT == 4 ? 2 * (4 * (row & 1) + ((row >> 1) & 3)) : 2 * ((row >> 1) & 3);
    }
    // unit permutation of a 64-byte column (d-major X, r)
    static __device__ __forceinline__ int colswz(int col) { return (col >> 1) & 3; }
};

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
//
// The waves split the work by role, so that one wave's vector work overlaps
// the other's matrix-core work on each SIMD:
//   * waves 0-3 (E): wave e owns chains 32 e .. +31 (two 16-chain tiles) and
//     both 16-row tiles of every 32-row chunk: eta on the matrix cores with
//     the Theta pieces in registers, then r = y - sigmoid(eta), split into
//     pieces, into LDS, and the log-likelihood;
//   * waves 4-7 (X): wave 4 + x owns chains 32 x .. +31 and every d tile of
//     X_chunk^T r.
// Software pipeline over the slice's chunks, one barrier per pass: pass c
// (c = -2 .. nchunk - 1) has the E waves compute eta of chunk c + 2 with the
// residuals of chunk c + 1 (from the eta they computed in pass c - 1)
// placed between its MFMA groups, and the X waves X^T r of chunk c.  The
// row-major half of chunk c + 3 (E waves) and the d-major half of chunk
// c + 1 (X waves) are loaded into registers at the top of the pass and
// written to the idle LDS buffers at its end.
template <int DT, int NK8 = 0>
__device__ __forceinline__ void logreg_grad_tile(const GradK& a, int ct, int sl, unsigned char* lds)
{
    using S = GradB<DT>;
    constexpr int DP = S::DP, PR = S::PR;
    constexpr float kLn2 = 0.693147180559945309f;
    constexpr int NK32 = NK8 > 0 ? (NK8 + 3) / 4 : DT;  // eta k steps of 32 (d), at most
    constexpr int NT = NK8 > 0 ? (NK8 + 1) / 2 : 2 * DT;  // gradient d tiles of 16 that can be nonzero
    static_assert(NK8 >= 0 && 32 * NK32 <= DP, "dimension class exceeds the tile");
    const int nk32 = NK8 > 0 ? NK32 : (a.D + 31) >> 5;
    const int nt = NK8 > 0 ? NT : (a.D + 15) >> 4;
    float* Ured = reinterpret_cast<float*>(lds + S::AUX0);  // [E wave][2 chain tiles][16]
    int* cols = reinterpret_cast<int*>(Ured + 8 * 32);

    const int ncols = a.dense > 0 ? a.dense : *a.count;
    if (ct * 128 >= ncols) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, q4 = lane >> 4;
    const bool ewave = wave < 4;
    const int w4 = wave & 3;  // E: chains 32 w4 ..; X: chains 32 w4 ..
    if (tid < 128) {
        const int g = ct * 128 + tid;
        cols[tid] = g < ncols ? (a.dense > 0 ? g : a.list[g]) : -1;
    }
    const int rb = sl * a.slice_rows;
    const int re = min(rb + a.slice_rows, a.N);
    const int nchunk = (re - rb + 31) / 32;
    const unsigned char* xsrc = reinterpret_cast<const unsigned char*>(a.Xb) + (size_t)(rb / 32) * S::CHUNK;

    // Staging: the E waves (threads 0-255) move row-major halves, the X waves
    // (threads 256-511) d-major halves, HBM -> registers -> LDS.  LDS unit L of
    // the row-major image holds (piece, row, unit L ^ rowswz(row)) of the
    // chunk; of the d-major image, (piece, d, unit L ^ colswz(d)).  Named
    // registers: an array here ends up in scratch.
    constexpr int NU = S::NU;                  // 16-byte units per half chunk
    constexpr int NS = (NU + 255) / 256;       // per thread of a role (at most)
    static_assert(NS <= 6, "half-chunk share");
    const int rtid = tid & 255;
    auto off_of = [&](int f) {
        if (ewave) {
            const int row = (f / (DP / 8)) & 31, u = f % (DP / 8);
            return 16 * (f - u + (u ^ S::rowswz(row)));
        }
        const int d = (f >> 2) & (DP - 1), u = f & 3;
        return 16 * (f - u + (u ^ S::colswz(d)));
    };
    int so[6];
#pragma unroll
    for (int v = 0; v < 6; ++v) so[v] = off_of(rtid + 256 * v);
    uint4 st0, st1, st2, st3, st4, st5;
    auto stage_load = [&](const unsigned char* src) {
        const uint4* s4 = reinterpret_cast<const uint4*>(src);
        if (NS > 0 && rtid < NU) st0 = s4[rtid];
        if (NS > 1 && rtid + 256 < NU) st1 = s4[rtid + 256];
        if (NS > 2 && rtid + 512 < NU) st2 = s4[rtid + 512];
        if (NS > 3 && rtid + 768 < NU) st3 = s4[rtid + 768];
        if (NS > 4 && rtid + 1024 < NU) st4 = s4[rtid + 1024];
        if (NS > 5 && rtid + 1280 < NU) st5 = s4[rtid + 1280];
    };
    auto stage_store = [&](unsigned char* dst) {
        if (NS > 0 && rtid < NU) *reinterpret_cast<uint4*>(dst + so[0]) = st0;
        if (NS > 1 && rtid + 256 < NU) *reinterpret_cast<uint4*>(dst + so[1]) = st1;
        if (NS > 2 && rtid + 512 < NU) *reinterpret_cast<uint4*>(dst + so[2]) = st2;
        if (NS > 3 && rtid + 768 < NU) *reinterpret_cast<uint4*>(dst + so[3]) = st3;
        if (NS > 4 && rtid + 1024 < NU) *reinterpret_cast<uint4*>(dst + so[4]) = st4;
        if (NS > 5 && rtid + 1280 < NU) *reinterpret_cast<uint4*>(dst + so[5]) = st5;
    };
    auto rows_src = [&](int c) { return xsrc + (size_t)c * S::CHUNK; };
    auto cols_src = [&](int c) { return xsrc + (size_t)c * S::CHUNK + S::XRB; };
    auto rows_buf = [&](int c) { return lds + (c & 1) * S::XRB; };
    auto cols_buf = [&](int c) { return lds + S::XD0 + (c & 1) * S::XDB; };
    auto r_buf = [&](int c) { return lds + S::RS0 + (c & 1) * S::RSB; };
    if (ewave && nchunk > 0) {
        stage_load(rows_src(0));
        stage_store(rows_buf(0));
    }
    __syncthreads();  // cols, and the row-major half of chunk 0

    float uacc[2] = {0.0f, 0.0f};
    if (ewave) {
        // ---------------------------------------------------------------- E waves
        // Theta pieces of chain tiles 2 w4, 2 w4 + 1 (B operand: lane holds
        // Theta[chain 16 t + l16][32 kk + 8 q4 .. + 7])
        uint4 thb[2][NK32][3];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int ch = cols[32 * w4 + 16 * t + l16];
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
        int xsw[2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) xsw[rt] = S::rowswz(16 * rt + l16);
        // eta tiles [row tile][chain tile] of the chunk computed last pass
        floatx4 ec[2][2], en[2][2];
        // X row pieces of row tile rt at k step kk of chunk c (A operand)
        auto load_x = [&](int c, int rt, int kk, uint4 (&xa)[3]) {
            const unsigned char* xr = rows_buf(c) + (16 * rt + l16) * PR + 16 * ((4 * kk + q4) ^ xsw[rt]);
            xa[0] = *reinterpret_cast<const uint4*>(xr);
            xa[1] = *reinterpret_cast<const uint4*>(xr + 32 * PR);
            xa[2] = *reinterpret_cast<const uint4*>(xr + 64 * PR);
        };
        // residual value j of chunk c: row tile j >> 3, chain tile (j >> 2) & 1,
        // row 4 q4 + (j & 3) of the tile; rows past the data are zero rows of X
        // and y (eta = 0): they leave the gradient and the linear term unchanged,
        // and their factor 2 is taken back once at the end of the slice
        float rr[16], lin[2] = {0.0f, 0.0f}, prod[2][2] = {{1.0f, 1.0f}, {1.0f, 1.0f}};
        float yv[2][4];
        auto res_value = [&](int j) {
            const int rt = j >> 3, t = (j >> 2) & 1, i = j & 3;
            const float v = ec[rt][t][i];
            const float y = yv[rt][i];
            const bool pos = v >= 0.0f;
            const float ex = __expf(-fabsf(v));
            const float inv = __builtin_amdgcn_rcpf(1.0f + ex);  // hardware reciprocal, 1 ulp
            const float sig = pos ? inv : ex * inv;
            lin[t] = fmaf(pos ? y - 1.0f : y, v, lin[t]);  // y v - max(v, 0)
            prod[rt][t] *= 1.0f + ex;
            rr[j] = y - sig;
        };
        auto res_finish = [&](int c) {
            unsigned char* Rs = r_buf(c);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                // the four factors of each row tile lie in (1, 2]: their product in [1, 16]
                uacc[t] += lin[t] - kLn2 * (__builtin_amdgcn_logf(prod[0][t]) + __builtin_amdgcn_logf(prod[1][t]));
                lin[t] = 0.0f;
                prod[0][t] = prod[1][t] = 1.0f;
                const int col = 32 * w4 + 16 * t + l16;
#pragma unroll
                for (int rt = 0; rt < 2; ++rt) {
                    uint32_t ph[4], pm[4], pl[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) split_bf16x3(rr[8 * rt + 4 * t + i], ph[i], pm[i], pl[i]);
                    // rows 16 rt + 4 q4 .. + 3: 8 bytes in unit 2 rt + q4 / 2 of the column
                    unsigned char* rp = Rs + col * 64 + 16 * ((2 * rt + (q4 >> 1)) ^ S::colswz(col)) + 8 * (q4 & 1);
                    *reinterpret_cast<uint2*>(rp) = make_uint2(ph[0] | (ph[1] << 16), ph[2] | (ph[3] << 16));
                    *reinterpret_cast<uint2*>(rp + 128 * 64) = make_uint2(pm[0] | (pm[1] << 16), pm[2] | (pm[3] << 16));
                    *reinterpret_cast<uint2*>(rp + 256 * 64) = make_uint2(pl[0] | (pl[1] << 16), pl[2] | (pl[3] << 16));
                }
            }
        };
        auto load_y = [&](int c) {
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                const float4 y4 = *reinterpret_cast<const float4*>(a.y + rb + 32 * c + 16 * rt + 4 * q4);
                yv[rt][0] = y4.x;
                yv[rt][1] = y4.y;
                yv[rt][2] = y4.z;
                yv[rt][3] = y4.w;
            }
        };
        // eta of chunk ce into en (DE), with the residuals of chunk cr (from
        // ec, DR) between its MFMA groups: 4 NK32 groups of six MFMAs (tile
        // (rt, t) at step kk), a residual value after each; each row tile's X
        // pieces are read one group pair ahead.  The fences keep the vector
        // work spread over the matrix-core work.
        auto eta_res = [&](auto de, auto dr, int ce, int cr) {
            constexpr bool DE = decltype(de)::value, DR = decltype(dr)::value;
            if constexpr (DE) {
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int t = 0; t < 2; ++t) en[rt][t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            }
            uint4 xa[2][3];
            if constexpr (DE) load_x(ce, 0, 0, xa[0]);
            int j = 0;
#pragma unroll
            for (int kk = 0; kk < NK32; ++kk) {
                if (kk >= nk32) break;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int rt = g >> 1, t = g & 1;
                    if constexpr (DE) {
                        if (g == 0) load_x(ce, 1, kk, xa[1]);
                        if (g == 2 && kk + 1 < NK32 && kk + 1 < nk32) load_x(ce, 0, kk + 1, xa[0]);
                        en[rt][t] = mfma_bf16x6(xa[rt], thb[t][kk], en[rt][t]);
                    }
                    if constexpr (DR) {
                        if (j < 16) res_value(j);
                    }
                    ++j;
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            if constexpr (DR) {
                for (; j < 16; ++j) res_value(j);
                res_finish(cr);
            }
        };
        using T1 = std::integral_constant<bool, true>;
        using F0 = std::integral_constant<bool, false>;
        for (int c = -2; c < nchunk; ++c) {
            const bool doe = c + 2 < nchunk, dor = c + 1 >= 0 && c + 1 < nchunk;
            if (c + 3 < nchunk) stage_load(rows_src(c + 3));
            if (dor) load_y(c + 1);
            if (doe && dor)
                eta_res(T1{}, T1{}, c + 2, c + 1);
            else if (doe)
                eta_res(T1{}, F0{}, c + 2, -1);
            else if (dor)
                eta_res(F0{}, T1{}, -1, c + 1);
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int t = 0; t < 2; ++t) ec[rt][t] = en[rt][t];
            if (c + 3 < nchunk) stage_store(rows_buf(c + 3));
            __syncthreads();
        }
        // ln 2 per padding row of this lane's rows (only the slice's last chunk
        // can hold any), then the lanes of one column (they hold different rows)
        if (nchunk > 0) {
            float npad = 0.0f;
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                const int rowl = rb + 32 * (nchunk - 1) + 16 * rt + 4 * q4;
                npad += (float)min(4, max(0, rowl + 4 - re));
            }
            uacc[0] += npad * kLn2;
            uacc[1] += npad * kLn2;
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            uacc[t] += __shfl_xor(uacc[t], 16, 64);
            uacc[t] += __shfl_xor(uacc[t], 32, 64);
        }
    } else {
        // ---------------------------------------------------------------- X waves
        floatx4 accg[NT][2];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) accg[t][u][q] = 0.0f;
        const int csw = 16 * (q4 ^ S::colswz(l16));  // this lane's unit in a 64-byte column
        // X_chunk^T r of chunk c: A = X columns (lane: d 16 t + l16, rows 8 q4 .. + 7),
        // B = r pieces of chain tiles 2 w4, 2 w4 + 1
        auto xtr = [&](int c) {
            const unsigned char* Rs = r_buf(c);
            uint4 rpc[2][3];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const unsigned char* rp = Rs + (32 * w4 + 16 * u + l16) * 64 + csw;
#pragma unroll
                for (int p = 0; p < 3; ++p) rpc[u][p] = *reinterpret_cast<const uint4*>(rp + p * 128 * 64);
            }
            const unsigned char* XD = cols_buf(c) + l16 * 64 + csw;
            uint4 xb[2][3];  // ping-pong by tile parity (static indices once unrolled)
            auto ld = [&](int t, uint4 (&x)[3]) {
                const unsigned char* xp = XD + 16 * t * 64;
                x[0] = *reinterpret_cast<const uint4*>(xp);
                x[1] = *reinterpret_cast<const uint4*>(xp + DP * 64);
                x[2] = *reinterpret_cast<const uint4*>(xp + 2 * DP * 64);
            };
            ld(0, xb[0]);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (t + 1 < NT && t + 1 < nt) ld(t + 1, xb[(t + 1) & 1]);
                if (t < nt) {
                    accg[t][0] = mfma_bf16x6(xb[t & 1], rpc[0], accg[t][0]);
                    accg[t][1] = mfma_bf16x6(xb[t & 1], rpc[1], accg[t][1]);
                }
            }
        };
        for (int c = -2; c < nchunk; ++c) {
            if (c + 1 >= 0 && c + 1 < nchunk) stage_load(cols_src(c + 1));
            if (c >= 0) xtr(c);
            if (c + 1 >= 0 && c + 1 < nchunk) stage_store(cols_buf(c + 1));
            __syncthreads();
        }
        __syncthreads();  // matches the E waves' barrier below (X and r buffers free)
        // gradient tiles -> LDS [chain][d] over the X buffers, for coalesced stores
        constexpr int TP = DP + 4;
        float* Red = reinterpret_cast<float*>(lds);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t < nt) {
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        Red[(32 * w4 + 16 * u + l16) * TP + 16 * t + 4 * q4 + q] = accg[t][u][q];
            }
        }
        const int DZ = DP - 16 * nt;  // d past the last tile: zero
        if (DZ > 0) {
            for (int i = tid - 256; i < 128 * DZ; i += 256) {
                const int col = i / DZ;
                Red[col * TP + 16 * nt + (i - col * DZ)] = 0.0f;
            }
        }
    }
    if (ewave) {
        __syncthreads();  // matches the X waves' barrier above
        if (q4 == 0) {
            Ured[w4 * 32 + l16] = uacc[0];
            Ured[w4 * 32 + 16 + l16] = uacc[1];
        }
    }
    __syncthreads();
    constexpr int TP = DP + 4;
    const float* Red = reinterpret_cast<const float*>(lds);
    for (int i = tid; i < 128 * DP; i += 512) {
        const int col = i / DP, d = i - col * DP;
        const int chn = cols[col];
        if (chn >= 0) a.Gpart[((size_t)sl * a.m + chn) * DP + d] = Red[col * TP + d];
    }
    if (tid < 128 && cols[tid] >= 0) a.Upart[(size_t)sl * a.m + cols[tid]] = Ured[tid];
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
