// fsmmc_device.h -- device building blocks shared by every sampler kernel:
// counter-based random streams, wave-level reductions, target terms.
//
// Everything here is deterministic and keyed only by (seed, chain, draw,
// role, sub-step, block): nothing depends on the thread, wave, workgroup,
// launch or schedule, so a chain's draws are the same whichever kernel
// (FSM or synchronized) and whichever launch shape computes them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsmmc {

// ---------------------------------------------------------------- RNG
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): multipliers
// 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 / 0xBB67AE85.
struct Ctr4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ Ctr4 philox10(Ctr4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32 x 32 -> 64-bit product per multiplier (both halves at once)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        Ctr4 n;
        n.x = hi1 ^ c.y ^ k0;
        n.y = lo1;
        n.z = hi0 ^ c.w ^ k1;
        n.w = lo0;
        c = n;
    }
    return c;
}

enum Role : uint32_t {
    ROLE_NU = 1,
    ROLE_INIT = 2,
    ROLE_THRESH = 3,
    ROLE_ANGLE = 4,
    ROLE_MOM = 5,
    ROLE_DIR = 6,
    ROLE_LEAF = 7,
    ROLE_MERGE = 8,
    ROLE_PROP = 9,
    ROLE_ACC = 10
};

__device__ __forceinline__ Ctr4 stream_block(uint64_t seed, uint32_t chain, uint32_t draw, uint32_t role,
                                             uint32_t sub, uint32_t block)
{
    Ctr4 c{chain, draw, (role << 24) | (sub & 0xFFFFFFu), block};
    return philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// u = ((w >> 9) + 1/2) 2^-23: 24 significant bits, exact in both precisions,
// strictly inside (0, 1).
template <typename T>
__device__ __forceinline__ T u01(uint32_t w);
template <>
__device__ __forceinline__ float u01<float>(uint32_t w)
{
    return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}
template <>
__device__ __forceinline__ double u01<double>(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

template <typename T>
__device__ __forceinline__ T uniform(uint64_t seed, uint32_t chain, uint32_t draw, uint32_t role, uint32_t sub)
{
    return u01<T>(stream_block(seed, chain, draw, role, sub, 0).x);
}

// Box-Muller on one word pair: (r cos 2 pi u2, r sin 2 pi u2), r = sqrt(-2 ln u1).
__device__ __forceinline__ void box_muller(uint32_t w1, uint32_t w2, float& z0, float& z1)
{
    const float u1 = u01<float>(w1), u2 = u01<float>(w2);
    const float r = sqrtf(-2.0f * logf(u1));
    float s, c;
    sincospif(2.0f * u2, &s, &c);
    z0 = r * c;
    z1 = r * s;
}
__device__ __forceinline__ void box_muller(uint32_t w1, uint32_t w2, double& z0, double& z1)
{
    const double u1 = u01<double>(w1), u2 = u01<double>(w2);
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// The four normals d = 4b .. 4b+3 of a (role, sub) vector stream.
template <typename T>
__device__ __forceinline__ void normals4(uint64_t seed, uint32_t chain, uint32_t draw, uint32_t role,
                                         uint32_t sub, uint32_t b, T z[4])
{
    const Ctr4 w = stream_block(seed, chain, draw, role, sub, b);
    box_muller(w.x, w.y, z[0], z[1]);
    box_muller(w.z, w.w, z[2], z[3]);
}

// Normal d of a (role, sub) vector stream (computes its whole block).
template <typename T>
__device__ __forceinline__ T normal_at(uint64_t seed, uint32_t chain, uint32_t draw, uint32_t role,
                                       uint32_t sub, uint32_t d)
{
    const Ctr4 w = stream_block(seed, chain, draw, role, sub, d >> 2);
    T z0, z1;
    if ((d & 2u) == 0)
        box_muller(w.x, w.y, z0, z1);
    else
        box_muller(w.z, w.w, z0, z1);
    return (d & 1u) ? z1 : z0;
}

// ---------------------------------------------------------------- waves
// Butterfly sum over the 64 lanes of a wave: every lane ends with the same
// bits (each step adds a commutative pair), in a fixed order.
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Lane 0's copy of a value every active lane already holds (a chain's
// scalar state when one wave runs one chain).  The value is unchanged; the
// compiler may then keep it in scalar registers and run integer work on it
// (the Philox rounds of a chain's angle draws) on the scalar unit instead of
// the vector ALU.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int64_t uni(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ double uni(double v)
{
    return __longlong_as_double((long long)uni((int64_t)__double_as_longlong(v)));
}

// Wave-wide sums for counters (every lane gets the total).
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_max_i32(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide sum of per-wave counters: every thread of the block must call it
// (lane 0 of each wave contributes v); thread 0 gets the total.  Replaces one
// same-address atomic per wave by one per block.
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long* s_slot)
{
    if (threadIdx.x == 0) *s_slot = 0;
    __syncthreads();
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(s_slot, v);
    __syncthreads();
    return *s_slot;
}

__device__ __forceinline__ int block_max_i32(int v, int* s_slot)
{
    if (threadIdx.x == 0) *s_slot = 0;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) atomicMax(s_slot, v);
    __syncthreads();
    return *s_slot;
}

// A D-vector held by one wave: element d = e * 64 + lane.
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

// Dot product of two wave vectors (lane-local sum over e, then the butterfly);
// wave-uniform (called by whole waves only).
template <int EPL>
__device__ __forceinline__ float wdot(const WaveVec<EPL>& a, const WaveVec<EPL>& b)
{
    float s = 0.0f;
#pragma unroll
    for (int e = 0; e < EPL; ++e) s += a.r[e] * b.r[e];
    return uni(wave_sum(s));
}

// ---------------------------------------------------------------- math
template <typename T>
struct M;
template <>
struct M<float> {
    static __device__ __forceinline__ float exp_(float a) { return __expf(a); }
    static __device__ __forceinline__ float log_(float a) { return __logf(a); }
    static __device__ __forceinline__ float log1p_(float a) { return log1pf(a); }
    static __device__ __forceinline__ float expm1_(float a) { return expm1f(a); }
    static __device__ __forceinline__ void sincos_(float a, float* s, float* c) { sincosf(a, s, c); }
    static __device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
    // softplus(a) = max(a, 0) + log(1 + e^-|a|)
    static __device__ __forceinline__ float softplus(float a)
    {
        return fmaxf(a, 0.0f) + __logf(1.0f + __expf(-fabsf(a)));
    }
};
template <>
struct M<double> {
    static __device__ __forceinline__ double exp_(double a) { return exp(a); }
    static __device__ __forceinline__ double log_(double a) { return log(a); }
    static __device__ __forceinline__ double log1p_(double a) { return log1p(a); }
    static __device__ __forceinline__ double expm1_(double a) { return expm1(a); }
    static __device__ __forceinline__ void sincos_(double a, double* s, double* c) { sincos(a, s, c); }
    static __device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }
    static __device__ __forceinline__ double softplus(double a)
    {
        return fmax(a, 0.0) + log1p(exp(-fabs(a)));
    }
};

template <typename T>
struct Pi;
template <>
struct Pi<float> {
    static constexpr float two_pi = 6.28318530717958647692f;
};
template <>
struct Pi<double> {
    static constexpr double two_pi = 6.28318530717958647692;
};

// x = hi + mid + lo exactly, each piece a bf16 bit pattern: hi keeps the top 16
// bits of x, the remainder x - hi (at most 16 significant bits) is exact in
// FP32, mid keeps its top 16 bits and the rest (at most 8 significant bits)
// is lo.  Host-side splits follow the same rule.
__device__ __forceinline__ void split_bf16x3(float x, uint32_t& hi, uint32_t& mid, uint32_t& lo)
{
    const uint32_t uh = __float_as_uint(x) & 0xFFFF0000u;
    const float r1 = x - __uint_as_float(uh);
    const uint32_t um = __float_as_uint(r1) & 0xFFFF0000u;
    const float r2 = r1 - __uint_as_float(um);
    hi = uh >> 16;
    mid = um >> 16;
    lo = __float_as_uint(r2) >> 16;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

}  // namespace fsmmc
