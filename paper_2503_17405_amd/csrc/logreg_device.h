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
    static constexpr int NVH = (NU + 511) / 512;  // of which one thread of the block moves (at most)
    static_assert(XRB == XDB && NVH <= 3, "chunk layouts");
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
// Software pipeline over the slice's 32-row chunks, one barrier per chunk:
// pass i computes eta of chunk i + 1 (and its r, into the other r buffer)
// and X^T r of chunk i, while the row-major half of chunk i + 2 and the
// d-major half of chunk i + 1 stream into the idle X buffers, so the
// sigmoid's vector work and the loads overlap the matrix-core work.
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
    float* Ured = reinterpret_cast<float*>(lds + S::AUX0);  // [wave][32 chains]
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
    const unsigned char* xsrc = reinterpret_cast<const unsigned char*>(a.Xb) + (size_t)(rb / 32) * S::CHUNK;

    // One layout of a chunk moves HBM -> registers (coalesced 16-byte loads,
    // issued at the top of a pass) -> LDS (at its end).  LDS unit L of the
    // row-major image holds (piece, row, unit L ^ rowswz(row)) of the chunk;
    // of the d-major image, (piece, d, unit L ^ colswz(d)).  Named registers:
    // an array here ends up in scratch.
    auto rows_off = [&](int f) {
        const int row = (f / (DP / 8)) & 31, u = f % (DP / 8);
        return 16 * (f - u + (u ^ S::rowswz(row)));
    };
    auto cols_off = [&](int f) {
        const int d = (f >> 2) & (DP - 1), u = f & 3;
        return 16 * (f - u + (u ^ S::colswz(d)));
    };
    // this thread's units of each layout: f = tid, tid + 512, tid + 1024 (when < NU)
    const bool has1 = S::NVH > 1 && tid + 512 < S::NU, has2 = S::NVH > 2 && tid + 1024 < S::NU;
    const int ro0 = rows_off(tid), ro1 = rows_off(tid + 512), ro2 = rows_off(tid + 1024);
    const int co0 = cols_off(tid), co1 = cols_off(tid + 512), co2 = cols_off(tid + 1024);
    uint4 sr0, sr1, sr2;  // row-major half in flight
    auto stage_rows = [&](const unsigned char* src) {
        const uint4* s4 = reinterpret_cast<const uint4*>(src);
        sr0 = s4[tid];
        if (has1) sr1 = s4[tid + 512];
        if (has2) sr2 = s4[tid + 1024];
    };
    auto store_rows = [&](unsigned char* dst) {
        *reinterpret_cast<uint4*>(dst + ro0) = sr0;
        if (has1) *reinterpret_cast<uint4*>(dst + ro1) = sr1;
        if (has2) *reinterpret_cast<uint4*>(dst + ro2) = sr2;
    };
    uint4 sd0, sd1, sd2;  // d-major half in flight
    auto stage_cols = [&](const unsigned char* src) {
        const uint4* s4 = reinterpret_cast<const uint4*>(src);
        sd0 = s4[tid];
        if (has1) sd1 = s4[tid + 512];
        if (has2) sd2 = s4[tid + 1024];
    };
    auto store_cols = [&](unsigned char* dst) {
        *reinterpret_cast<uint4*>(dst + co0) = sd0;
        if (has1) *reinterpret_cast<uint4*>(dst + co1) = sd1;
        if (has2) *reinterpret_cast<uint4*>(dst + co2) = sd2;
    };
    auto rows_src = [&](int c) { return xsrc + (size_t)c * S::CHUNK; };
    auto cols_src = [&](int c) { return xsrc + (size_t)c * S::CHUNK + S::XRB; };
    if (nchunk > 0) {
        stage_rows(rows_src(0));
        store_rows(lds);
    }
    __syncthreads();  // cols, and the row-major half of chunk 0

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

    // gradient roles: chain tile `wave` (chains 16 wave .. + 15), every d tile
    floatx4 accg[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) accg[t][q] = 0.0f;
    float uacc[2] = {0.0f, 0.0f};

    // 1. eta of chunk c (32 rows x 128 chains): A = X rows (lane: row 16 rt + l16,
    //    d 32 kk + 8 q4 .. + 7), B = Theta pieces
    const int xsw = S::rowswz(16 * rt + l16);
    auto eta = [&](int c, floatx4& e0, floatx4& e1) {
        const unsigned char* xr = lds + (c & 1) * S::XRB + (16 * rt + l16) * PR;
        e0 = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        e1 = e0;
#pragma unroll
        for (int kk = 0; kk < NK32; ++kk) {
            if (kk >= nk32) break;
            const int o = 16 * ((4 * kk + q4) ^ xsw);
            const uint4 xa[3] = {*reinterpret_cast<const uint4*>(xr + o),
                                 *reinterpret_cast<const uint4*>(xr + 32 * PR + o),
                                 *reinterpret_cast<const uint4*>(xr + 64 * PR + o)};
            e0 = mfma_bf16x6(xa, thb[0][kk], e0);
            e1 = mfma_bf16x6(xa, thb[1][kk], e1);
        }
    };
    // 2. r = y - sigmoid(eta) of chunk c, split into pieces, into r buffer c & 1;
    //    log-likelihood: sum [y eta - max(eta, 0)] minus one log of the product
    //    of the four factors 1 + e^-|eta| (each in (1, 2], so the product is a
    //    normal number in [1, 16] and the hardware log2 is accurate).  Rows
    //    past the data are zero rows of X and y, so eta = 0 there: they leave
    //    the gradient and the linear term unchanged, and their factor 2 is
    //    taken back (ln 2 each) once at the end of the slice.
    //    Value j: column tile j / 4, row j % 4 of the lane's four.
    struct Resid {
        float r[8];
        float lin[2], prod[2];
    };
    auto resid_value = [&](int j, const floatx4& e0, const floatx4& e1, const float4& yv4, Resid& R) {
        const int i = j & 3, t = j >> 2;
        const float v = t ? e1[i] : e0[i];
        const float yv = i == 0 ? yv4.x : i == 1 ? yv4.y : i == 2 ? yv4.z : yv4.w;
        const bool pos = v >= 0.0f;
        const float ex = __expf(-fabsf(v));
        const float inv = __builtin_amdgcn_rcpf(1.0f + ex);  // hardware reciprocal, 1 ulp
        const float sig = pos ? inv : ex * inv;
        R.lin[t] = fmaf(pos ? yv - 1.0f : yv, v, R.lin[t]);  // y v - max(v, 0)
        R.prod[t] *= 1.0f + ex;
        R.r[j] = yv - sig;
    };
    auto resid_finish = [&](int c, Resid& R) {
        unsigned char* Rs = lds + S::RS0 + (c & 1) * S::RSB;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            uacc[t] += R.lin[t] - kLn2 * __builtin_amdgcn_logf(R.prod[t]);  // hardware log2
            uint32_t ph[4], pm[4], pl[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) split_bf16x3(R.r[4 * t + i], ph[i], pm[i], pl[i]);
            // rows 16 rt + 4 q4 .. + 3: 8 bytes in unit 2 rt + q4 / 2 of the column
            const int col = 32 * ep + 16 * t + l16;
            unsigned char* rp = Rs + col * 64 + 16 * ((2 * rt + (q4 >> 1)) ^ S::colswz(col)) + 8 * (q4 & 1);
            *reinterpret_cast<uint2*>(rp) = make_uint2(ph[0] | (ph[1] << 16), ph[2] | (ph[3] << 16));
            *reinterpret_cast<uint2*>(rp + 128 * 64) = make_uint2(pm[0] | (pm[1] << 16), pm[2] | (pm[3] << 16));
            *reinterpret_cast<uint2*>(rp + 256 * 64) = make_uint2(pl[0] | (pl[1] << 16), pl[2] | (pl[3] << 16));
        }
    };
    auto resid = [&](int c, const floatx4& e0, const floatx4& e1, const float4& yv4) {
        Resid R = {{}, {0.0f, 0.0f}, {1.0f, 1.0f}};
#pragma unroll
        for (int j = 0; j < 8; ++j) resid_value(j, e0, e1, yv4, R);
        resid_finish(c, R);
    };
    // 3. X^T r of chunk c: A = X columns (lane: d 16 t + l16, rows 8 q4 .. + 7),
    //    B = r pieces.  Fused form: the residual values of chunk cr ride
    //    between the d tiles' MFMAs (one per tile, fenced so that the
    //    scheduler keeps them there and the vector work overlaps the matrix
    //    cores); cr < 0: none.
    const int csw = 16 * (q4 ^ S::colswz(l16));  // this lane's unit in a 64-byte column
    auto xtr_resid = [&](int c, int cr, const floatx4& e0, const floatx4& e1, const float4& yv4) {
        const unsigned char* Rs = lds + S::RS0 + (c & 1) * S::RSB;
        uint4 rpc[3];
        const unsigned char* rp = Rs + (16 * wave + l16) * 64 + csw;
#pragma unroll
        for (int p = 0; p < 3; ++p) rpc[p] = *reinterpret_cast<const uint4*>(rp + p * 128 * 64);
        const unsigned char* XD = lds + S::XD0 + (c & 1) * S::XDB + l16 * 64 + csw;
        Resid R = {{}, {0.0f, 0.0f}, {1.0f, 1.0f}};
        // d tile t's pieces are read one group ahead of its MFMAs
        auto ld = [&](int t, uint4 (&x)[3]) {
            const unsigned char* xp = XD + 16 * t * 64;
            x[0] = *reinterpret_cast<const uint4*>(xp);
            x[1] = *reinterpret_cast<const uint4*>(xp + DP * 64);
            x[2] = *reinterpret_cast<const uint4*>(xp + 2 * DP * 64);
        };
        uint4 xb[2][3];  // ping-pong by tile parity (static indices once unrolled)
        ld(0, xb[0]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t + 1 < NT && t + 1 < nt) ld(t + 1, xb[(t + 1) & 1]);
            if (t < nt) accg[t] = mfma_bf16x6(xb[t & 1], rpc, accg[t]);
            if (cr >= 0 && t < 8) resid_value(t, e0, e1, yv4, R);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (cr >= 0) {
#pragma unroll
            for (int j = NT; j < 8; ++j) resid_value(j, e0, e1, yv4, R);
            resid_finish(cr, R);
        }
    };
    // y of this lane's four rows of chunk c (16-byte aligned; rows past the
    // data are read from the zero padding and masked)
    auto yload = [&](int c) {
        return *reinterpret_cast<const float4*>(a.y + rb + 32 * c + 16 * rt + 4 * q4);
    };

    // Pass c (c = -1 .. nchunk - 2) reads the row-major half of chunk c + 1,
    // the d-major half of chunk c and r of chunk c, all in place since the
    // barrier that ended pass c - 1, and fills buffers whose readers finished
    // before that barrier: the row-major half of chunk c + 2 goes where chunk
    // c's was, the d-major half of c + 1 where c - 1's was, r of c + 1 where
    // r of c - 1 was.
    if (nchunk > 0) {
        stage_cols(cols_src(0));
        if (nchunk > 1) stage_rows(rows_src(1));
        floatx4 e0, e1;
        eta(0, e0, e1);
        resid(0, e0, e1, yload(0));
        float4 yv = yload(min(1, nchunk - 1));  // y one pass ahead: in registers when the pass starts
        store_cols(lds + S::XD0);
        if (nchunk > 1) store_rows(lds + S::XRB);
        __syncthreads();
        for (int c = 0; c + 1 < nchunk; ++c) {
            const bool more = c + 2 < nchunk;
            if (more) stage_rows(rows_src(c + 2));
            stage_cols(cols_src(c + 1));
            const float4 ycur = yv;
            yv = yload(min(c + 2, nchunk - 1));
            eta(c + 1, e0, e1);
            xtr_resid(c, c + 1, e0, e1, ycur);
            if (more) store_rows(lds + (c & 1) * S::XRB);
            store_cols(lds + S::XD0 + ((c + 1) & 1) * S::XDB);
            __syncthreads();
        }
        xtr_resid(nchunk - 1, -1, e0, e1, yv);
    }
    // log-likelihood per chain: take back ln 2 per padding row of this lane
    // (only the slice's last chunk can hold any), then add up the lanes of one
    // column (they hold different rows)
    if (nchunk > 0) {
        const int rowl = rb + 32 * (nchunk - 1) + 16 * rt + 4 * q4;
        const float npad = (float)(min(4, max(0, rowl + 4 - re)));
        uacc[0] += npad * kLn2;
        uacc[1] += npad * kLn2;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        uacc[t] += __shfl_xor(uacc[t], 16, 64);
        uacc[t] += __shfl_xor(uacc[t], 32, 64);
    }
    __syncthreads();  // X and r buffers free
    if (q4 == 0) {
        Ured[wave * 32 + l16] = uacc[0];
        Ured[wave * 32 + 16 + l16] = uacc[1];
    }
    // gradient tiles -> LDS [chain][d] over the X buffers, for coalesced stores
    constexpr int TP = DP + 4;
    float* Red = reinterpret_cast<float*>(lds);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (t < nt) {
#pragma unroll
            for (int q = 0; q < 4; ++q) Red[(16 * wave + l16) * TP + 16 * t + 4 * q4 + q] = accg[t][q];
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
