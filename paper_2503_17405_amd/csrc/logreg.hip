// logreg.hip -- the batched potential and gradient of Bayesian logistic
// regression with a N(0, I) prior, for a list of chain positions Theta:
//   eta = X Theta,  r = y - sigmoid(eta),
//   grad U = Theta - X^T r,  U = |Theta|^2 / 2 - sum_i [y_i eta_i - softplus(eta_i)].
// This is the amortized g of the NUTS FSM (one evaluation per step per chain).
//
// logreg_grad_kernel: block = 4 waves, 64 listed chains x one row slice of the job.
// Theta (64 x Dp) is staged in LDS once.  The slice is walked in chunks of 32
// rows; each chunk of X is loaded once (coalesced float4, double-buffered:
// the next chunk's loads are issued before this chunk's MFMAs) and shared by
// the four waves:
//   1. eta (32 rows x 64 chains) on v_mfma_f32_16x16x4_f32 with K = D rounded
//      up to 4 (not the padded Dp): wave w owns rows 16 (w & 1) .. +15 and
//      chains 32 (w >> 1) .. +31 (two 16 x 16 tiles);
//   2. r = y - sigmoid(eta) written to LDS, and the log-likelihood with one
//      log per four rows (the log of the product of the factors 1 + e^-|eta|);
//   3. X_chunk^T r on v_mfma_f32_16x16x4_f32 in 16-row tiles of d (D rounded
//      up to 16): wave w owns chains 16 w .. +15 and every d tile, so partial
//      gradients never need a cross-wave reduction.
// Row slices are added in slice order (by the NUTS transition that consumes
// the gradient, or by logreg_reduce_kernel for the starting points); no float
// atomics, so every result is reproducible bit for bit.
#include "logreg_device.h"

namespace fsmmc {

template <int DT, int NK8>
__global__ __launch_bounds__(256) void logreg_grad_kernel(GradK a)
{
    logreg_grad_tile<DT, NK8>(a, blockIdx.x, blockIdx.y);
}

template <int EPL>
__global__ __launch_bounds__(256) void logreg_reduce_kernel(ReduceK a)
{
    logreg_reduce_one<EPL>(a, (int)(blockIdx.x * 4 + (threadIdx.x >> 6)), threadIdx.x & 63);
}

// Gout == nullptr: leave the row-slice partials for the consumer to add.
static hipError_t grad_launch(const JobDev& j, int dense, float* Gout, float* Uout, int gstride, hipStream_t s)
{
    const GradK g = grad_view(j, dense);
    const dim3 grid((j.m + 63) / 64, j.nslices), block(256);
#define FSMMC_GRAD_CASE(K)                                                               \
    case K:                                                                              \
        hipLaunchKernelGGL((logreg_grad_kernel<(K) <= 8 ? 2 : 4, K>), grid, block, 0, s, g); \
        break;
    switch ((j.D + 7) / 8) {
        FSMMC_GRAD_CASE(1) FSMMC_GRAD_CASE(2) FSMMC_GRAD_CASE(3) FSMMC_GRAD_CASE(4)
        FSMMC_GRAD_CASE(5) FSMMC_GRAD_CASE(6) FSMMC_GRAD_CASE(7) FSMMC_GRAD_CASE(8)
        FSMMC_GRAD_CASE(9) FSMMC_GRAD_CASE(10) FSMMC_GRAD_CASE(11) FSMMC_GRAD_CASE(12)
        FSMMC_GRAD_CASE(13) FSMMC_GRAD_CASE(14) FSMMC_GRAD_CASE(15) FSMMC_GRAD_CASE(16)
    default: return hipErrorInvalidValue;
    }
#undef FSMMC_GRAD_CASE
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !Gout) return e;
    const ReduceK r = reduce_view(j, dense, Gout, Uout, gstride);
    const dim3 rg((j.m + 3) / 4);
    if (j.Dp <= 64)
        hipLaunchKernelGGL(logreg_reduce_kernel<1>, rg, dim3(256), 0, s, r);
    else
        hipLaunchKernelGGL(logreg_reduce_kernel<2>, rg, dim3(256), 0, s, r);
    return hipGetLastError();
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
