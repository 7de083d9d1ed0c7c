// logreg.hip -- the batched potential and gradient of Bayesian logistic
// regression with a N(0, I) prior, for a list of chain positions Theta:
//   eta = X Theta,  r = y - sigmoid(eta),
//   grad U = Theta - X^T r,  U = |Theta|^2 / 2 - sum_i [y_i eta_i - softplus(eta_i)].
// This is the amortized g of the NUTS FSM (one evaluation per step per chain).
//
// logreg_grad_kernel: block = 4 waves, 64 listed chains x one slice of 512 rows.
// The slice is walked in chunks of 32 rows; each chunk of X is staged in LDS
// once (coalesced, double-buffered) and shared by the four waves:
//   1. eta (32 rows x 64 chains) on v_mfma_f32_16x16x4_f32: wave w owns rows
//      16 (w & 1) .. +15 and chains 32 (w >> 1) .. +31 (two 16 x 16 tiles);
//   2. r = y - sigmoid(eta) and the log-likelihood terms, r written to LDS;
//   3. X_chunk^T r on v_mfma_f32_32x32x2_f32 with K = 32 rows: wave w owns
//      distinct (d, chain) output tiles, so partial gradients never need a
//      cross-wave reduction.
// Row slices are added in slice order by logreg_reduce_kernel; no float
// atomics, so every result is reproducible bit for bit.
#include "logreg_device.h"

namespace fsmmc {

template <int DT>
__global__ __launch_bounds__(256) void logreg_grad_kernel(GradK a)
{
    logreg_grad_tile<DT>(a, blockIdx.x, blockIdx.y);
}

template <int EPL>
__global__ __launch_bounds__(256) void logreg_reduce_kernel(ReduceK a)
{
    logreg_reduce_one<EPL>(a, (int)(blockIdx.x * 4 + (threadIdx.x >> 6)), threadIdx.x & 63);
}

static hipError_t grad_launch(const JobDev& j, int dense, float* Gout, float* Uout, int gstride, hipStream_t s)
{
    const GradK g = grad_view(j, dense);
    const dim3 grid((j.m + 63) / 64, j.nslices), block(256);
    switch (j.Dp / 32) {
    case 2: hipLaunchKernelGGL(logreg_grad_kernel<2>, grid, block, 0, s, g); break;
    case 4: hipLaunchKernelGGL(logreg_grad_kernel<4>, grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
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
    return grad_launch(j, 0, (float*)j.Gres, (float*)j.Ures, j.Dp, s);
}

hipError_t nuts_gradient_dense(const JobDev& j, int ncols, float* Gout, float* Uout, int gstride, hipStream_t s)
{
    return grad_launch(j, ncols, Gout, Uout, gstride, s);
}

}  // namespace fsmmc
