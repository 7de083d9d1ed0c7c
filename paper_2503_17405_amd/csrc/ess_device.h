// ess_device.h -- elliptical slice sampling (Murray, Adams, MacKay 2010)
// building blocks shared by the single-job kernels (ess.hip) and the grouped
// multi-job kernels (batch.hip).  Sec. 3.1: states INIT, SHRINK, DONE;
// Appendix, Alg. "Transition kernel for elliptical slice sampler".
//
// Every kernel that advances an ESS chain calls these functions in the same
// order, so a chain's draws are the same bits whichever kernel runs it.
#pragma once
#include "fsmmc_device.h"
#include "fsmmc_internal.h"

namespace fsmmc {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Ellipse-direction product nu = L z for the columns (chain, w) of a window.
template <typename T>
struct NuK {
    int m, n, D, Dp, W;
    uint64_t seed;
    uint32_t role;
    int draw_fixed;     // >= 0: every column uses this draw; < 0: draw = t[chain] + tadd + w
    uint32_t tadd;      // offset of the window from t (the next window while this one runs)
    const uint32_t* t;  // chain draw counters (or a snapshot of them)
    const T* L;         // Dp x Dp lower factor, zero padded
    T* out;             // column (chain, w) -> out[(chain * W + w) * Dp + row]
    const uint16_t* Lp; // FP32 with Dp > 256: L = hi + mid + lo in bf16, packed by (row tile, chunk)
};

template <typename T>
struct EssK {
    int m, n, D, Dp, W, target;
    uint64_t seed;
    T inv2v;
    const T* y;
    const T* nu;
    int32_t* k;
    uint32_t* t;
    int32_t* evals;
    int64_t* budget;
    T *theta, *tmin, *tmax, *logu, *lx, *x, *out;
    int32_t* counts;
    unsigned long long* ctr;
    int32_t* maxN;
    T* sink;
};

// ------------------------------------------------------------ ellipse GEMM
// One row tile per wave (Dp <= 256): one block of 8 waves computes NC = 32 CT
// columns (col0 ..) over all Dp rows.
// Wave w owns RT row tiles of 32 rows in "snake" order (w, 15-w, 16+w, 31-w,
// ...) so the triangular work is balanced across waves.  The K dimension is
// walked in chunks of 32, software-pipelined: while the MFMAs of chunk k run
// (v_mfma_f32_32x32x2f32, FP32 accumulation, from the LDS tile of chunk k and
// L rows read as float4 along k), each thread draws its normals of chunk k+1
// (one Philox block per thread and 64 columns) into registers and stores them
// into the other LDS buffer afterwards -- one barrier per chunk.  The MFMA
// computes nu^T = z^T L^T so each output register row is 32 consecutive nu
// entries of one column (128-byte coalesced stores).  The products and their
// order per output element do not depend on the pipelining.  A block whose
// columns are all past their chain's last draw exits at once.  The directions
// go out with nontemporal stores (the next window's kernel reads them once).
template <int RT, int CT = 2>
__device__ __forceinline__ void nu_gemm_block_flat(const NuK<float>& a, int col0)
{
    static_assert(CT == 2 || CT == 4, "64 or 128 columns per block");
    constexpr int NC = 32 * CT, ZC = CT / 2;
    __shared__ float Zs[2][32][NC];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int ncols = a.m * a.W;

    const int zc = tid & 63, zb = tid >> 6;
    bool zvalid[ZC];
    int zchain[ZC];
    uint32_t zdraw[ZC];
    int any = 0;
#pragma unroll
    for (int cc = 0; cc < ZC; ++cc) {
        const int gcol = col0 + zc + 64 * cc;
        zvalid[cc] = gcol < ncols;
        zchain[cc] = 0;
        zdraw[cc] = 0;
        if (zvalid[cc]) {
            zchain[cc] = gcol / a.W;
            const int zw = gcol - zchain[cc] * a.W;
            zdraw[cc] = a.draw_fixed >= 0 ? (uint32_t)a.draw_fixed : a.t[zchain[cc]] + a.tadd + (uint32_t)zw;
            zvalid[cc] = a.draw_fixed >= 0 || zdraw[cc] < (uint32_t)a.n;
        }
        any |= zvalid[cc] ? 1 : 0;
    }
    if (!__syncthreads_or(any)) return;

    // this thread's 4 normals (rows 4 zb .. 4 zb + 3 of chunk kc) per column group
    auto draw = [&](int kc, float (&z)[ZC][4]) {
        const int kb = kc + 4 * zb;
#pragma unroll
        for (int cc = 0; cc < ZC; ++cc) {
#pragma unroll
            for (int i = 0; i < 4; ++i) z[cc][i] = 0.0f;
            if (zvalid[cc] && kb < a.D) {
                normals4<float>(a.seed, (uint32_t)zchain[cc], zdraw[cc], a.role, 0, (uint32_t)(kb >> 2), z[cc]);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (kb + i >= a.D) z[cc][i] = 0.0f;
            }
        }
    };
    auto put = [&](int buf, const float (&z)[ZC][4]) {
#pragma unroll
        for (int cc = 0; cc < ZC; ++cc)
#pragma unroll
            for (int i = 0; i < 4; ++i) Zs[buf][4 * zb + i][zc + 64 * cc] = z[cc][i];
    };

    const int ntiles = a.Dp >> 5;
    int tiles[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const int idx = (r & 1) ? r * 8 + 7 - wave : r * 8 + wave;
        tiles[r] = idx < ntiles ? idx : -1;
    }
    floatx16 acc[RT][CT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[r][c][q] = 0.0f;

    {
        float z0[ZC][4];
        draw(0, z0);
        put(0, z0);
    }
    __syncthreads();
    int buf = 0;
    for (int kc = 0; kc < a.Dp; kc += 32) {
        float zn[ZC][4];
        const bool more = kc + 32 < a.Dp;
        if (more) draw(kc + 32, zn);
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const int ti = tiles[r];
            if (ti < 0 || 32 * ti + 31 < kc) continue;
            const float4* Lr =
                reinterpret_cast<const float4*>(a.L + (size_t)(32 * ti + l32) * a.Dp + kc + 16 * h);
            float lr[16];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float4 q4 = Lr[v];
                lr[4 * v + 0] = q4.x;
                lr[4 * v + 1] = q4.y;
                lr[4 * v + 2] = q4.z;
                lr[4 * v + 3] = q4.w;
            }
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    const float av = Zs[buf][16 * h + kk][c * 32 + l32];
                    acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, lr[kk], acc[r][c], 0, 0, 0);
                }
            }
        }
        if (more) put(buf ^ 1, zn);
        __syncthreads();
        buf ^= 1;
    }
    // column g = chain * W + w is stored at out[g * Dp + row]
#pragma unroll
    for (int c = 0; c < CT; ++c) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int g = col0 + c * 32 + 8 * (q >> 2) + 4 * h + (q & 3);
            if (g >= ncols) continue;
            float* o = a.out + (size_t)g * a.Dp + l32;
#pragma unroll
            for (int r = 0; r < RT; ++r)
                if (tiles[r] >= 0) __builtin_nontemporal_store(acc[r][c][q], o + 32 * tiles[r]);
        }
    }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The 2- to 4-tile shapes (Dp > 256) on the bf16 matrix cores.  z and L are split
// exactly into three bf16 pieces each, and every 16-k block of a 32 x 32 tile
// takes the six piece products down to relative order 2^-16 (lo*hi, mid*mid,
// hi*lo, mid*hi, hi*mid, hi*hi; v_mfma_f32_32x32x16_bf16, FP32 accumulation):
// the dropped ones are below 2^-23 of the product, so the result has FP32
// accuracy at 6 bf16 products per FP32 product (the bf16 cores run 16 times
// the FP32 MFMA rate).
// One block of 8 waves computes 64 columns (col0 ..) over all Dp rows; wave w
// owns RT row tiles in snake order (visited from the last one down, so the
// tiles that reach K chunk k are a prefix).  The z pieces of 4 chunks of 32 k
// sit in one of two LDS buffers ([piece][column][k], rows padded to 136
// halfwords so the 16-byte reads do not conflict), so the block meets at a
// barrier once per 128 k.  Per chunk: the thread draws its 4 normals of the
// same chunk of the next 128 and stores their pieces in the other buffer, and
// the (tile, k-block) pairs run in order with the next pair's L pieces in
// flight -- the last pair loads the next chunk's first one.  L's pieces are packed so that
// one pair's are contiguous: for row tile ti, chunk c <= ti, k-block kb and
// piece p, the 32 x 16 block L[32 ti + r][32 c + 16 kb + kk] is the 512
// halfwords [r][kk] of block ((ti (ti + 1) / 2 + c) 2 + kb) 3 + p, so each
// load fills whole lines.  The products and their order per output element
// do not depend on this scheduling.  A block whose columns are all past their
// chain's last draw exits at once.  The directions are written with
// nontemporal stores (they are read once, by the next window's kernel), which
// keeps L's pieces in L2.
// The four normals of a direction block with the hardware transcendentals
// (log2, square root, and sine / cosine of 2 pi u, which the hardware takes
// in revolutions): the same Philox words and Box-Muller pairs as normals4,
// about 1e-6 absolute error per normal instead of the library functions'
// correct rounding, for a fraction of the vector instructions.  Only the
// large-D direction product uses them (its z generation competes with the
// matrix cores for issue); every kernel that computes those directions calls
// this function, so all runtimes see the same bits.
__device__ __forceinline__ void normals4_hw(uint64_t seed, uint32_t chain, uint32_t draw, uint32_t role,
                                            uint32_t b, float z[4])
{
    const Ctr4 w = stream_block(seed, chain, draw, role, 0, b);
    const uint32_t wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const float u1 = u01<float>(wv[2 * p]), u2 = u01<float>(wv[2 * p + 1]);
        const float r = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u1));  // -2 ln u1
        z[2 * p] = r * __builtin_amdgcn_cosf(u2);
        z[2 * p + 1] = r * __builtin_amdgcn_sinf(u2);
    }
}

template <int RT, int CT = 2>
__device__ __forceinline__ void nu_gemm_block_bf16(const NuK<float>& a, int col0)
{
    static_assert(CT == 2, "64 columns per block");
    constexpr int NC = 32 * CT, SUB = 4, KS = 32 * SUB, KR = KS + 8;
    __shared__ uint16_t Zs[2][3][NC][KR];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int ncols = a.m * a.W;

    const int zc = tid & 63, zb = tid >> 6;
    bool zvalid = false;
    int zchain = 0;
    uint32_t zdraw = 0;
    {
        const int gcol = col0 + zc;
        zvalid = gcol < ncols;
        if (zvalid) {
            zchain = gcol / a.W;
            const int zw = gcol - zchain * a.W;
            zdraw = a.draw_fixed >= 0 ? (uint32_t)a.draw_fixed : a.t[zchain] + a.tadd + (uint32_t)zw;
            zvalid = a.draw_fixed >= 0 || zdraw < (uint32_t)a.n;
        }
    }
    if (!__syncthreads_or(zvalid ? 1 : 0)) return;

    // this thread's 4 normals (rows kc + 4 zb .. + 3 of column zc; 0 past D or
    // for a missing column), split, as 4 consecutive k (from koff) in each
    // piece plane of buffer buf
    auto draw_put = [&](int kc, int buf, int koff) {
        const int kb = kc + 4 * zb;
        float z[4];
        normals4_hw(a.seed, (uint32_t)zchain, zdraw, a.role, (uint32_t)(kb >> 2), z);
#pragma unroll
        for (int i = 0; i < 4; i += 2) {
            uint32_t pc[2][3];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint32_t keep = (zvalid && kb + i + j < a.D) ? 0xFFFFFFFFu : 0u;
                uint32_t bits;
                asm("v_and_b32 %0, %1, %2" : "=v"(bits) : "v"(__float_as_uint(z[i + j])), "v"(keep));
                split_bf16x3(__uint_as_float(bits), pc[j][0], pc[j][1], pc[j][2]);
            }
#pragma unroll
            for (int q = 0; q < 3; ++q)
                *reinterpret_cast<uint32_t*>(&Zs[buf][q][zc][koff + 4 * zb + i]) = pc[0][q] | (pc[1][q] << 16);
        }
    };

    // the wave's row tiles, last first; missing ones (-1) at the end
    const int ntiles = a.Dp >> 5;
    int tiles[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) tiles[r] = -1;
    int nt = 0;
#pragma unroll
    for (int rr = RT - 1; rr >= 0; --rr) {
        const int idx = (rr & 1) ? rr * 8 + 7 - wave : rr * 8 + wave;
        if (idx < ntiles) {
#pragma unroll
            for (int p = 0; p < RT; ++p)
                if (p == nt) tiles[p] = idx;
            ++nt;
        }
    }
#pragma unroll
    for (int r = 0; r < RT; ++r) tiles[r] = uni(tiles[r]);
    floatx16 acc[RT][CT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[r][c][q] = 0.0f;

    // pieces of L[32 ti + l32][k0 + 8 h .. + 7] (k0 a multiple of 16; a chunk
    // past the diagonal, only ever prefetched and unused, reads the diagonal's)
    auto load_l = [&](u32x4 (&lr)[3], int ti, int k0) {
        const int c = min(k0 >> 5, ti), kb = (k0 >> 4) & 1;
        const uint16_t* base = a.Lp + (size_t)(((ti * (ti + 1) / 2 + c) * 2 + kb) * 3) * 512 + 16 * l32 + 8 * h;
#pragma unroll
        for (int p = 0; p < 3; ++p) lr[p] = *reinterpret_cast<const u32x4*>(base + 512 * p);
    };

#pragma unroll
    for (int p = 0; p < SUB; ++p)
        if (32 * p < a.Dp) draw_put(32 * p, 0, 32 * p);
    const int t0row = tiles[0] >= 0 ? tiles[0] : 0;  // a valid row tile for the address
    u32x4 lb[2][3];
    load_l(lb[0], t0row, 0);
    __syncthreads();
    int buf = 0;
    for (int kc = 0; kc < a.Dp; kc += 32) {
        const bool more = kc + 32 < a.Dp;
        const int sub = (kc >> 5) & (SUB - 1);  // the chunk's place in its 128 k
        int na = 0;  // tiles that reach this chunk: tiles[0 .. na-1]
#pragma unroll
        for (int r = 0; r < RT; ++r) na += (tiles[r] >= 0 && 32 * tiles[r] + 31 >= kc) ? 1 : 0;
        na = uni(na);
        if (kc + KS < a.Dp) draw_put(kc + KS, buf ^ 1, 32 * sub);
        // za[kb][c][p]: piece p of z rows kc + 16 kb + 8 h .. + 7, column 32 c + l32
        u32x4 za[2][CT][3];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int p = 0; p < 3; ++p)
                    za[kb][c][p] = *reinterpret_cast<const u32x4*>(&Zs[buf][p][32 * c + l32][32 * sub + 16 * kb + 8 * h]);
        // pair q = (tile q / 2, k-block q % 2) uses lb[q % 2] and loads pair q + 1
#pragma unroll
        for (int q = 0; q < 2 * RT; ++q) {
            const int r = q >> 1, kb = q & 1;
            if (r >= na) break;
            u32x4(&cur)[3] = lb[q & 1];
            u32x4(&nxt)[3] = lb[(q + 1) & 1];
            if (q + 1 < 2 * na)
                load_l(nxt, tiles[(q + 1) >> 1], kc + 16 * ((q + 1) & 1));
            else
                load_l(nxt, t0row, more ? kc + 32 : kc);
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const bf16x8 zh = __builtin_bit_cast(bf16x8, za[kb][c][0]);
                const bf16x8 zm = __builtin_bit_cast(bf16x8, za[kb][c][1]);
                const bf16x8 zl = __builtin_bit_cast(bf16x8, za[kb][c][2]);
                const bf16x8 Lh = __builtin_bit_cast(bf16x8, cur[0]);
                const bf16x8 Lm = __builtin_bit_cast(bf16x8, cur[1]);
                const bf16x8 Ll = __builtin_bit_cast(bf16x8, cur[2]);
                floatx16 t = acc[r][c];
                t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(zl, Lh, t, 0, 0, 0);
                t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(zm, Lm, t, 0, 0, 0);
                t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(zh, Ll, t, 0, 0, 0);
                t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(zm, Lh, t, 0, 0, 0);
                t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(zh, Lm, t, 0, 0, 0);
                t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(zh, Lh, t, 0, 0, 0);
                acc[r][c] = t;
            }
        }
        if (sub == SUB - 1 || !more) {  // the other buffer holds the next 128 k
            __syncthreads();
            buf ^= 1;
        }
    }
    // column g = chain * W + w is stored at out[g * Dp + row]
#pragma unroll
    for (int c = 0; c < CT; ++c) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int g = col0 + c * 32 + 8 * (q >> 2) + 4 * h + (q & 3);
            if (g >= ncols) continue;
            float* o = a.out + (size_t)g * a.Dp + l32;
#pragma unroll
            for (int r = 0; r < RT; ++r)
                if (tiles[r] >= 0) __builtin_nontemporal_store(acc[r][c][q], o + 32 * tiles[r]);
        }
    }
}

// Ellipse-direction product for the columns col0 .. col0 + 32 CT - 1 of a window:
// FP32 MFMA for one row tile per wave (Dp <= 256), the bf16 matrix cores with
// exact three-piece splits above.  A job's padded dimension fixes the variant,
// so every kernel that computes its directions gives the same bits.
template <int RT, int CT = 2>
__device__ __forceinline__ void nu_gemm_block(const NuK<float>& a, int col0)
{
    if constexpr (RT >= 2)
        nu_gemm_block_bf16<RT, CT>(a, col0);
    else
        nu_gemm_block_flat<RT, CT>(a, col0);
}

// ------------------------------------------------------------ ESS blocks
// FP32 logistic likelihood along an ellipse.  x' = x cos(theta) + nu sin(theta)
// is linear in (x, nu), so the lane sums of y x' and of x' are
// cos (sum y x, sum x) + sin (sum y nu, sum nu): EssLin holds the four sums,
// formed once per (x, nu) -- per draw -- instead of once per evaluation.
// With max(f, 0) = (f + |f|) / 2 the evaluation then spends, per element,
// two instructions on x', one on the sum of |x'| and one FMA on the product
// of the factors 1 + e^-|x'| (p + p e^-|x'|): each lies in (1, 2], so the
// product of at most 16 stays in [1, 2^16], where the hardware log2 is
// accurate, and one log replaces EPL of them (the vector units bound this
// loop, so it is written for few instructions per element).
struct EssLin {
    float yx, yn, sx, sn;
};

template <int EPL, bool FULL>
__device__ __forceinline__ EssLin ess_lin(const float (&x)[EPL], const float (&nu)[EPL], const float (&yv)[EPL],
                                          int lane, int D)
{
    EssLin L{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        const bool in = FULL || e * 64 + lane < D;
        const float xe = in ? x[e] : 0.0f, ne = in ? nu[e] : 0.0f;
        L.yx = fmaf(yv[e], xe, L.yx);
        L.yn = fmaf(yv[e], ne, L.yn);
        L.sx += xe;
        L.sn += ne;
    }
    return L;
}

// Lane part of log L(x') for the FP32 logistic likelihood, x' into xp.
template <int EPL, bool FULL>
__device__ __forceinline__ float ess_lane_logistic_lin(const float (&x)[EPL], const float (&nu)[EPL],
                                                       float (&xp)[EPL], float c, float s, const EssLin& L,
                                                       int lane, int D)
{
    static_assert(EPL <= 16, "the factor product must stay below 2^16");
    float asum = 0.0f, prod = 1.0f;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        const bool in = FULL || e * 64 + lane < D;
        const float f = fmaf(x[e], c, nu[e] * s);
        xp[e] = f;
        const float af = in ? fabsf(f) : 0.0f;
        asum = e == 0 ? af : asum + af;
        prod = fmaf(prod, in ? __expf(-fabsf(f)) : 0.0f, prod);
    }
    const float yf = fmaf(c, L.yx, s * L.yn), sf = fmaf(c, L.sx, s * L.sn);
    return yf - 0.5f * (sf + asum) - 0.693147180559945309f * __builtin_amdgcn_logf(prod);
}

// log L(x) of a state (FP32 logistic): the same arithmetic at theta = 0.
template <int EPL, bool FULL>
__device__ __forceinline__ float ess_lane_logistic_at(const float (&x)[EPL], const float (&yv)[EPL], int lane, int D)
{
    float xp[EPL];
    return ess_lane_logistic_lin<EPL, FULL>(x, x, xp, 1.0f, 0.0f, ess_lin<EPL, FULL>(x, x, yv, lane, D), lane, D);
}

// Lane-local part of log L(f) over the lane's elements d = e * 64 + lane < D.
//   Gaussian:  -sum (y - f)^2 / (2 sd^2)
//   logistic:  sum y f - softplus(f), softplus(f) = max(f, 0) + log(1 + e^-|f|).
// FP32 logistic: the arithmetic of the evaluations along an ellipse
// (ess_lane_logistic_at).
// FULL: D == 64 EPL, every lane element exists and the masks drop out (the
// same operations on the same values as the masked form).
template <typename T, int EPL, bool FULL = false>
__device__ __forceinline__ T ess_lane_loglik(const T (&f)[EPL], const T (&yv)[EPL], int lane, int D, int target,
                                             T inv2v)
{
    T acc = T(0);
    if (target == FSMMC_GP_GAUSS) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            const T r = yv[e] - f[e];
            const T term = -(r * r) * inv2v;
            acc += (FULL || e * 64 + lane < D) ? term : T(0);
        }
        return acc;
    }
    if constexpr (sizeof(T) == 4) {
        return ess_lane_logistic_at<EPL, FULL>(f, yv, lane, D);
    } else {
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            const T term = yv[e] * f[e] - M<T>::softplus(f[e]);
            acc += (FULL || e * 64 + lane < D) ? term : T(0);
        }
        return acc;
    }
}

// x' = x cos(theta) + nu sin(theta) and log L(x'), summed in a fixed order
// (lane-local, then a wave butterfly); the result is wave-uniform.  L: the
// sums of (x, nu) for the FP32 logistic likelihood (unused otherwise).
template <typename T, int EPL, bool FULL = false>
__device__ __forceinline__ T ess_propose_eval(const T (&x)[EPL], const T (&nu)[EPL], T (&xp)[EPL],
                                              const T (&yv)[EPL], T theta, int lane, int D, int target,
                                              T inv2v, const EssLin& L)
{
    T s, c;
    M<T>::sincos_(theta, &s, &c);
    if constexpr (sizeof(T) == 4)
        if (target == FSMMC_GP_LOGISTIC) return wave_sum(ess_lane_logistic_lin<EPL, FULL>(x, nu, xp, c, s, L, lane, D));
#pragma unroll
    for (int e = 0; e < EPL; ++e) xp[e] = M<T>::fma_(x[e], c, nu[e] * s);
    return wave_sum(ess_lane_loglik<T, EPL, FULL>(xp, yv, lane, D, target, inv2v));
}

// EssLin of (x, nu) when the job's likelihood uses it (FP32 logistic).
template <typename T, int EPL, bool FULL>
__device__ __forceinline__ EssLin ess_lin_of(const T (&x)[EPL], const T (&nu)[EPL], const T (&yv)[EPL], int lane,
                                             int D, int target)
{
    if constexpr (sizeof(T) == 4)
        if (target == FSMMC_GP_LOGISTIC) return ess_lin<EPL, FULL>(x, nu, yv, lane, D);
    return EssLin{0.0f, 0.0f, 0.0f, 0.0f};
}

// INIT: the slice level log y = log L(x) + log u, kept as log u, and the
// initial bracket.  A proposal is accepted when log L(x') - log L(x) > log u,
// which is log L(x') > log y in exact arithmetic; in floating point it still
// accepts x' == x (the limit of a collapsing bracket), whereas log L(x) + log u
// rounds to log L(x) when |log u| is below the rounding of log L(x) and then
// no proposal near x would ever pass.
template <typename T>
__device__ __forceinline__ void ess_begin(uint64_t seed, uint32_t chain, uint32_t draw, T& logu, T& theta,
                                          T& tmin, T& tmax)
{
    logu = M<T>::log_(uniform<T>(seed, chain, draw, ROLE_THRESH, 0));
    theta = Pi<T>::two_pi * uniform<T>(seed, chain, draw, ROLE_ANGLE, 0);
    tmin = theta - Pi<T>::two_pi;
    tmax = theta;
}

// SHRINK: move the bracket end on theta's side to theta, draw a new angle.
template <typename T>
__device__ __forceinline__ void ess_shrink(uint64_t seed, uint32_t chain, uint32_t draw, int evals,
                                           T& theta, T& tmin, T& tmax)
{
    if (theta < T(0))
        tmin = theta;
    else
        tmax = theta;
    theta = tmin + (tmax - tmin) * uniform<T>(seed, chain, draw, ROLE_ANGLE, (uint32_t)evals);
}

template <typename T, int EPL>
__device__ __forceinline__ void ess_emit(const EssK<T>& a, int j, uint32_t t, const T (&x)[EPL], int evals,
                                         int lane)
{
    T* o = a.out + ((size_t)j * a.n + t) * a.D;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        const int d = e * 64 + lane;
        if (d < a.D) o[d] = x[e];
    }
    if (lane == 0) a.counts[(size_t)j * a.n + t] = evals;
}

// What one chain's window adds to the job counters: [0] steps, [2] guard
// trips, [4] chains still short of n, [3] of those, chains with budget left.
struct EssTally {
    uint32_t steps = 0, guards = 0, live = 0, budget_left = 0;
};

// One wave runs chain j through FSM steps until it has used the ellipse
// window [t0, t0 + W), reached n draws, or spent its step budget.  Returns
// the number of draws it emitted; the counter contributions go to tl (the
// caller adds them to the job's counters).
// TG >= 0: the target kind fixed at compile time (the loop then holds one
// likelihood form and its registers only); TG < 0: a.target.
template <typename T, int EPL, bool FULL, int TG = -1>
__device__ __forceinline__ uint32_t ess_window_run(const EssK<T>& a, int j, int lane, EssTally& tl)
{
    const int target = TG >= 0 ? TG : a.target;
    j = uni(j);
    uint32_t t = uni(a.t[j]);
    if (t >= (uint32_t)a.n) return 0;
    const uint32_t t0 = t;
    const uint32_t wend = min(t0 + (uint32_t)a.W, (uint32_t)a.n);
    int k = uni(a.k[j]), evals = uni(a.evals[j]);
    T theta = uni(a.theta[j]), tmin = uni(a.tmin[j]), tmax = uni(a.tmax[j]), logu = uni(a.logu[j]),
      lx = uni(a.lx[j]);
    int64_t budget = uni((int64_t)a.budget[j]);

    T x[EPL], nu[EPL], xp[EPL], yv[EPL];
    const T* xj = a.x + (size_t)j * a.Dp;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        x[e] = xj[e * 64 + lane];
        yv[e] = a.y[e * 64 + lane];
    }
    unsigned long long steps = 0;
    int guards = 0;
    bool have_nu = false;
    EssLin L{0.0f, 0.0f, 0.0f, 0.0f};
    while (t < wend && budget > 0) {
        if (!have_nu) {
            const T* nj = a.nu + ((size_t)j * a.W + (t - t0)) * a.Dp;
#pragma unroll
            for (int e = 0; e < EPL; ++e) nu[e] = nj[e * 64 + lane];
            have_nu = true;
            L = ess_lin_of<T, EPL, FULL>(x, nu, yv, lane, a.D, target);
        }
        if (k == 1) {
            ess_begin<T>(a.seed, (uint32_t)j, t, logu, theta, tmin, tmax);
            evals = 0;
        } else {
            ess_shrink<T>(a.seed, (uint32_t)j, t, evals, theta, tmin, tmax);
        }
        const T lp = uni(ess_propose_eval<T, EPL, FULL>(x, nu, xp, yv, theta, lane, a.D, target, a.inv2v, L));
        ++evals;
        ++steps;
        --budget;
        const bool accept = lp - lx > logu;
        if (accept || evals >= kEssMaxEvals) {
            if (accept) {
#pragma unroll
                for (int e = 0; e < EPL; ++e) x[e] = xp[e];
                lx = lp;
            } else {
                ++guards;
            }
            ess_emit<T, EPL>(a, j, t, x, evals, lane);
            ++t;
            k = 1;
            have_nu = false;
        } else {
            k = 2;
        }
    }
    T* xo = a.x + (size_t)j * a.Dp;
#pragma unroll
    for (int e = 0; e < EPL; ++e) xo[e * 64 + lane] = x[e];
    if (lane == 0) {
        a.t[j] = t;
        a.k[j] = k;
        a.evals[j] = evals;
        a.theta[j] = theta;
        a.tmin[j] = tmin;
        a.tmax[j] = tmax;
        a.logu[j] = logu;
        a.lx[j] = lx;
        a.budget[j] = budget;
    }
    tl.steps = (uint32_t)steps;
    tl.guards = (uint32_t)guards;
    tl.live = t < (uint32_t)a.n ? 1u : 0u;
    tl.budget_left = (tl.live && budget > 0) ? 1u : 0u;
    return t - t0;
}

template <typename T, int EPL>
__device__ __forceinline__ uint32_t ess_window(const EssK<T>& a, int j, int lane, EssTally& tl)
{
    if (a.D == 64 * EPL) return ess_window_run<T, EPL, true>(a, j, lane, tl);
    return ess_window_run<T, EPL, false>(a, j, lane, tl);
}

// Add one chain's tally to the job counters (lane 0 of its wave).
template <typename T>
__device__ __forceinline__ void ess_count(const EssK<T>& a, const EssTally& tl, int lane)
{
    if (lane != 0) return;
    if (tl.steps) atomicAdd(&a.ctr[0], (unsigned long long)tl.steps);
    if (tl.guards) atomicAdd(&a.ctr[2], (unsigned long long)tl.guards);
    if (tl.live) atomicAdd(&a.ctr[4], 1ull);
    if (tl.budget_left) atomicAdd(&a.ctr[3], 1ull);
}

// ------------------------------------------------------------ host views
template <typename T>
inline EssK<T> ess_view(const JobDev& j)
{
    EssK<T> a;
    a.m = j.m;
    a.n = j.n;
    a.D = j.D;
    a.Dp = j.Dp;
    a.W = j.W;
    a.target = j.target;
    a.seed = j.seed;
    a.inv2v = (j.target == FSMMC_GP_GAUSS) ? (T)(1.0 / (2.0 * j.noise_sd * j.noise_sd)) : T(0);
    a.y = (const T*)j.y;
    a.nu = (const T*)j.nu + (size_t)j.nu_cur * j.m * j.Wcap * j.Dp;
    a.k = j.k;
    a.t = j.t;
    a.evals = j.evals;
    a.budget = j.budget;
    a.theta = (T*)j.theta;
    a.tmin = (T*)j.tmin;
    a.tmax = (T*)j.tmax;
    a.logu = (T*)j.logu;
    a.lx = (T*)j.lx;
    a.x = (T*)j.x;
    a.out = (T*)j.out;
    a.counts = j.counts;
    a.ctr = j.ctr;
    a.maxN = j.maxN;
    a.sink = (T*)j.sink;
    return a;
}

// Window product of the job's W draws per chain starting at t + tadd, into
// direction buffer `buf` (t: the chains' counters or a snapshot of them).
template <typename T>
inline NuK<T> ess_window_view(const JobDev& j, int buf = 0, const uint32_t* t = nullptr, uint32_t tadd = 0)
{
    NuK<T> a;
    a.m = j.m;
    a.n = j.n;
    a.D = j.D;
    a.Dp = j.Dp;
    a.W = j.W;
    a.seed = j.seed;
    a.role = ROLE_NU;
    a.draw_fixed = -1;
    a.tadd = tadd;
    a.t = t ? t : j.t;
    a.L = (const T*)j.L;
    a.Lp = (const uint16_t*)j.Lp;
    a.out = (T*)j.nu + (size_t)buf * j.m * j.Wcap * j.Dp;
    return a;
}


}  // namespace fsmmc
