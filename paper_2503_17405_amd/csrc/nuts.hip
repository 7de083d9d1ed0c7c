// nuts.hip -- the no-U-turn sampler (Hoffman & Gelman 2014) as an FSM
// (Sec. 3.1, Fig. "Finite state machines ...", HMC-NUTS panel: INIT, DOUBLE,
// INTEGRATE, CHECK, DONE; Sec. 7.3: iterative form, an outer doubling loop
// and an inner integration loop), for Bayesian logistic regression.
//
// One runtime step for every chain:
//   1. nuts_step_kernel (one wavefront per chain): add up the row-slice
//      partials of the gradient that just arrived, in slice order
//      (grad U = theta - X^T r, U = |theta|^2 / 2 - loglik), finish that
//      leapfrog (second half-kick, multinomial leaf choice, U-turn
//      checkpoints), then run the cheap states back to back (CHECK, DONE,
//      INIT, DOUBLE) until the chain needs the next gradient, and issue the
//      first half of that leapfrog (Appendix, Alg. "bundled step as input to
//      amortized step").
//   2. nuts_compact_kernel: list of chains that asked for a gradient, in
//      chain order.
//   3. logreg_grad_bf16_kernel: eta = X Theta, r = y - sigmoid(eta), X^T r
//      and the log-likelihood, fused for a tile of 128 listed chains and a
//      slice of rows on the bf16 matrix cores (exact three-piece splits of
//      the FP32 operands, FP32 results); eta never leaves registers.
// The synchronized runtime uses the same kernels; a chain that finishes a
// draw waits until every chain has finished it (device-side barrier), and in
// vmap mode the gradient phase then covers every chain.
// Readings: multinomial leaf sampling inside a subtree, biased progressive
// merge of subtrees, generalized U-turn criterion on every aligned sub-span,
// divergence when H - H0 > 1000, identity mass.
#include "nuts_device.h"

namespace fsmmc {

template <int EPL>
__global__ __launch_bounds__(256) void nuts_step_kernel(NutsK a)
{
    const int lane = threadIdx.x & 63;
    const int c = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.wctr[(a.step + 1) % 3] = 0u;
        a.wctr[3 + (a.step + 1) % 3] = 0u;
    }
    int bits = 0;
    if (c < a.m) bits = nuts_chain_step<EPL>(a, c, lane);
    if (a.mode != 0) {
        // synchronized runtimes: chains alive / still inside their draw, one atomic per block
        __shared__ unsigned s_alive, s_indraw;
        if (threadIdx.x == 0) {
            s_alive = 0;
            s_indraw = 0;
        }
        __syncthreads();
        if (lane == 0 && bits) {
            atomicAdd(&s_alive, (bits & NC_ALIVE) ? 1u : 0u);
            atomicAdd(&s_indraw, (bits & NC_INDRAW) ? 1u : 0u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            if (s_alive) atomicAdd(&a.wctr[3 + a.step % 3], s_alive);
            if (s_indraw) atomicAdd(&a.wctr[a.step % 3], s_indraw);
        }
    }
}

__global__ __launch_bounds__(1024) void nuts_compact_kernel(const int32_t* req, int m, int vmap, int32_t* list,
                                                            int32_t* count, unsigned long long* ctr)
{
    nuts_compact_block<1024>(req, m, vmap, list, count, ctr);
}

// Default start: theta0 ~ N(0, I) from the INIT stream (into both buffers).
__global__ void nuts_normal_init_kernel(float* thp, int vstride, float* thq, int m, int D, int Dp, uint64_t seed)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)m * Dp) return;
    const int c = (int)(i / Dp), d = (int)(i % Dp);
    const float z = d < D ? normal_at<float>(seed, (uint32_t)c, 0, ROLE_INIT, 0, (uint32_t)d) : 0.0f;
    thp[(size_t)c * vstride + d] = z;
    thq[(size_t)c * Dp + d] = z;
}

// ------------------------------------------------------------ host side
int nuts_nvec(int max_depth) { return V_FIXED + 2 * max_depth; }

hipError_t nuts_init_state(const JobDev& j, const void* x0, hipStream_t s)
{
    float* thp = (float*)j.V + (size_t)V_THP * j.Dp;
    const int vstride = j.nvec * j.Dp;
    if (x0) {
        hipError_t e = hipMemcpy2DAsync(thp, (size_t)vstride * 4, x0, (size_t)j.D * 4, (size_t)j.D * 4, j.m,
                                        hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpy2DAsync(j.Thq, (size_t)j.Dp * 4, x0, (size_t)j.D * 4, (size_t)j.D * 4, j.m,
                             hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    } else {
        const size_t tot = (size_t)j.m * j.Dp;
        hipLaunchKernelGGL(nuts_normal_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, thp,
                           vstride, (float*)j.Thq, j.m, j.D, j.Dp, j.seed);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // grad U and U at the start, straight into the proposal slots (gP, UP)
    float* gp = (float*)j.V + (size_t)V_GP * j.Dp;
    return nuts_gradient_dense(j, j.m, gp, (float*)j.lx, vstride, s);
}

hipError_t nuts_transition(const JobDev& j, int mode, uint32_t step, hipStream_t s)
{
    NutsK a = nuts_view(j, mode, step);
    const dim3 grid((j.m + 3) / 4), block(256);
    if (j.Dp <= 64)
        hipLaunchKernelGGL(nuts_step_kernel<1>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(nuts_step_kernel<2>, grid, block, 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(nuts_compact_kernel, dim3(1), dim3(1024), 0, s, j.req, j.m, mode == 1 ? 1 : 0, j.list, j.count,
                       j.ctr);
    return hipGetLastError();
}

}  // namespace fsmmc
