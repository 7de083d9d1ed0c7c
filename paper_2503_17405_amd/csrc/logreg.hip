// logreg.hip -- the batched potential and gradient of Bayesian logistic
// regression with a N(0, I) prior, for a list of chain positions Theta:
//   eta = X Theta,  r = y - sigmoid(eta),
//   grad U = Theta - X^T r,  U = |Theta|^2 / 2 - sum_i [y_i eta_i - softplus(eta_i)].
// This is the amortized g of the NUTS FSM (one evaluation per step per chain).
//
// logreg_grad_bf16_kernel: block = 8 waves, 128 listed chains x one row slice
// of the job, on the bf16 matrix cores with FP32 results.  Every FP32 operand
// is split exactly into three bf16 pieces (hi + mid + lo, split_bf16x3) and a
// product is the sum of the six piece products that carry its first ~24 bits
// (lo*hi, mid*mid, hi*lo, mid*hi, hi*mid, hi*hi; v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation), so the arithmetic is as accurate as the FP32 path while
// the bf16 cores (16 times the FP32 rate) leave a 2.7x higher ceiling.
//   * X is split once at job setup (logreg_split_kernel) into the two
//     layouts the two contractions need, per 32-row chunk: row-major pieces
//     (eta contracts over d) and d-major pieces (X^T r contracts over rows).
//   * Waves 0-3 compute eta (Theta's pieces split in-kernel and kept in
//     registers) and r = y - sigmoid(eta) with the log-likelihood; waves 4-7
//     compute X_chunk^T r.  The two roles run one chunk apart in a software
//     pipeline with one barrier per chunk, so the residuals' vector work
//     overlaps the matrix-core work of the other waves on the same SIMD
//     (logreg_grad_tile in logreg_device.h).
// The LDS images are unpadded with XOR-permuted 16-byte units, so operand
// reads are free of bank conflicts.  Row slices are added in slice order (by
// the NUTS transition that consumes the gradient, or by logreg_reduce_kernel
// for the starting points); no float atomics, so every result is
// reproducible bit for bit.  The grouped multi-job path (batch.hip) runs the
// same device function.
#include "logreg_device.h"

namespace fsmmc {

template <int DT, int NK8>
__global__ __launch_bounds__(512) void logreg_grad_bf16_kernel(GradK a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    logreg_grad_tile<DT, NK8>(a, blockIdx.x, blockIdx.y, lds);
}

// X (Np x Dp FP32) -> three bf16 pieces in the two chunk layouts the kernel
// above loads: per 32-row chunk, [p][row][d] then [p][d][row].
template <int DP>
__global__ void logreg_split_kernel(const float* X, int Np, uint16_t* Xb)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)Np * DP) return;
    const int row = (int)(i / DP), d = (int)(i % DP);
    uint32_t pc[3];
    split_bf16x3(X[i], pc[0], pc[1], pc[2]);
    uint16_t* base = Xb + (size_t)(row / 32) * (192 * DP);
    const int r = row % 32;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        base[p * 32 * DP + r * DP + d] = (uint16_t)pc[p];
        base[96 * DP + p * DP * 32 + d * 32 + r] = (uint16_t)pc[p];
    }
}


template <int EPL>
__global__ __launch_bounds__(256) void logreg_reduce_kernel(ReduceK a)
{
    logreg_reduce_one<EPL>(a, (int)(blockIdx.x * 4 + (threadIdx.x >> 6)), threadIdx.x & 63);
}

template <int DT, int NK8>
static hipError_t grad_bf16_launch(const GradK& g, int m, int nslices, hipStream_t s, bool setup)
{
    const void* f = (const void*)logreg_grad_bf16_kernel<DT, NK8>;
    if (setup) return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, GradB<DT>::LDS);
    hipLaunchKernelGGL((logreg_grad_bf16_kernel<DT, NK8>), dim3((m + 127) / 128, nslices), dim3(512),
                       GradB<DT>::LDS, s, g);
    return hipGetLastError();
}

// setup: only raise the kernel's dynamic LDS limit (once per job).
static hipError_t grad_dispatch(const JobDev& j, const GradK& g, hipStream_t s, bool setup)
{
#define FSMMC_GRAD_CASE(K) \
    case K: return grad_bf16_launch<(K) <= 8 ? 2 : 4, K>(g, j.m, j.nslices, s, setup);
    switch ((j.D + 7) / 8) {
        FSMMC_GRAD_CASE(1) FSMMC_GRAD_CASE(2) FSMMC_GRAD_CASE(3) FSMMC_GRAD_CASE(4)
        FSMMC_GRAD_CASE(5) FSMMC_GRAD_CASE(6) FSMMC_GRAD_CASE(7) FSMMC_GRAD_CASE(8)
        FSMMC_GRAD_CASE(9) FSMMC_GRAD_CASE(10) FSMMC_GRAD_CASE(11) FSMMC_GRAD_CASE(12)
        FSMMC_GRAD_CASE(13) FSMMC_GRAD_CASE(14) FSMMC_GRAD_CASE(15) FSMMC_GRAD_CASE(16)
    default: return hipErrorInvalidValue;
    }
#undef FSMMC_GRAD_CASE
}

// Gout == nullptr: leave the row-slice partials for the consumer to add.
static hipError_t grad_launch(const JobDev& j, int dense, float* Gout, float* Uout, int gstride, hipStream_t s)
{
    const GradK g = grad_view(j, dense);
    hipError_t e = grad_dispatch(j, g, s, false);
    if (e != hipSuccess || !Gout) return e;
    const ReduceK r = reduce_view(j, dense, Gout, Uout, gstride);
    const dim3 rg((j.m + 3) / 4);
    if (j.Dp <= 64)
        hipLaunchKernelGGL(logreg_reduce_kernel<1>, rg, dim3(256), 0, s, r);
    else
        hipLaunchKernelGGL(logreg_reduce_kernel<2>, rg, dim3(256), 0, s, r);
    return hipGetLastError();
}

size_t logreg_split_bytes(const JobDev& j) { return (size_t)j.Np / 32 * 384 * j.Dp; }

// Split X into the gradient kernel's bf16 pieces (after X is in place) and
// allow the kernel its LDS.
hipError_t logreg_setup(const JobDev& j, hipStream_t s)
{
    const size_t tot = (size_t)j.Np * j.Dp;
    const dim3 grid((unsigned)((tot + 255) / 256));
    if (j.Dp == 64)
        hipLaunchKernelGGL(logreg_split_kernel<64>, grid, dim3(256), 0, s, (const float*)j.X, j.Np, (uint16_t*)j.Xb);
    else if (j.Dp == 128)
        hipLaunchKernelGGL(logreg_split_kernel<128>, grid, dim3(256), 0, s, (const float*)j.X, j.Np, (uint16_t*)j.Xb);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return grad_dispatch(j, grad_view(j, 0), s, true);
}

hipError_t nuts_gradient(const JobDev& j, hipStream_t s)
{
    return grad_launch(j, 0, nullptr, nullptr, 0, s);
}

hipError_t nuts_gradient_dense(const JobDev& j, int ncols, float* Gout, float* Uout, int gstride, hipStream_t s)
{
    return grad_launch(j, ncols, Gout, Uout, gstride, s);
}

}  // namespace fsmmc
