// fsmmc_internal.h -- host-side declarations shared by the C ABI and the
// per-sampler launch code.  Not installed; not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fsmmc.h"

namespace fsmmc {

constexpr int kEssMaxEvals = 10000;  // evaluation guard of one ESS draw

// Device state of one job.  Chain arrays are structure-of-arrays of length m;
// vector state is m x Dp (one chain's vector contiguous, padded to Dp).
struct JobDev {
    // problem
    int kind = 0;    // sampler kind
    int target = 0;  // target kind
    int dtype = 0;
    int m = 0, n = 0, D = 0, Dp = 0, EPL = 0;
    int N = 0, Np = 0;  // LOGREG rows (padded); GP_HYPER observations
    int pdim = 0;       // GP_HYPER input dimension
    uint64_t seed = 0;
    double noise_sd = 0;
    double step_size = 0;
    int max_depth = 0, n_stages = 0;
    int fsm_states = 1;  // DRSYM: 1 condensed, 4 split loop body
    double scales[4] = {0, 0, 0, 0};

    // target data (owned copies)
    void* L = nullptr;  // Dp x Dp, zero padded (GP)
    void* Lp = nullptr; // FP32 GP with Dp > 256: L's bf16 pieces, packed (ess_lower_pieces_halfwords)
    void* y = nullptr;  // Dp (GP) or Np (LOGREG) labels / observations
    void* X = nullptr;  // LOGREG: Np x Dp, zero padded
    void* Xb = nullptr; // LOGREG: X as three bf16 pieces, row- and d-major per 32-row chunk (logreg.hip)
    void* gslot = nullptr;  // GP_HYPER with n > 128: a Cholesky work matrix per persistent block
    void* prec = nullptr;

    // common chain state
    int32_t* k = nullptr;      // FSM state label
    uint32_t* t = nullptr;     // draws done
    int32_t* evals = nullptr;  // loop count of the draw in progress
    int64_t* budget = nullptr; // steps left in the current call
    void* x = nullptr;         // m x Dp current state
    void* lx = nullptr;        // m: cached log-likelihood / log density / potential

    // ESS
    void* theta = nullptr;
    void* tmin = nullptr;
    void* tmax = nullptr;
    void* logu = nullptr;
    void* nu = nullptr;  // 2 x m x Wcap x Dp ellipse directions (double-buffered windows)
    int W = 0;           // draws per window (<= Wcap)
    int Wcap = 0;        // draws one direction buffer holds per chain
    int nu_cur = 0;      // buffer the stepping kernels read
    uint32_t* tsnap = nullptr;  // m: draw counters at the start of the running window

    // NUTS
    int32_t* jd = nullptr;     // tree depth of the subtree being built
    int32_t* vdir = nullptr;   // direction of the subtree (+1 / -1)
    int32_t* nn = nullptr;     // leaves done in the subtree
    int32_t* flags = nullptr;  // invalid / stop / diverged / turned / pending bits
    void* H0 = nullptr;        // initial Hamiltonian of the draw
    void* Wsum = nullptr;      // log-sum of leaf weights of the tree
    void* Wsub = nullptr;      // log-sum of leaf weights of the subtree
    void* US = nullptr;        // potential at the subtree proposal
    void* V = nullptr;         // m x nvec x Dp vector state
    int nvec = 0;
    void* Thq = nullptr;       // m x Dp positions whose gradient is requested
    int32_t* req = nullptr;    // m request flags
    int32_t* list = nullptr;   // m compacted requests
    int32_t* count = nullptr;  // 1
    void* Gpart = nullptr;     // nslices x m x Dp
    void* Upart = nullptr;     // nslices x m
    uint32_t* wctr = nullptr;  // [0..2] chains still in their draw, [3..5] chains alive (per step mod 3)
    int slice_rows = 0, nslices = 0;
    uint32_t tstop = 0;        // chains stop at this draw count
    void* acc = nullptr;       // m: sum over leapfrogs of min(1, e^(H0 - H)) (FP32)
    // NUTS on a Gaussian mixture (gradient computed inline by each chain's wave)
    int K = 0;                 // components
    void* mogB = nullptr;      // K x Dp: P mu_k (FP64)
    void* mogC = nullptr;      // K: log w_k - mu_k^T P mu_k / 2 (FP64)
    int32_t* queue = nullptr;  // 64 bytes: ticket counter of the persistent kernel
    int pwpb = 0, pblocks = 0; // its launch shape (waves per block, blocks)

    // outputs
    void* out = nullptr;  // m x n x D
    int32_t* counts = nullptr;  // m x n

    // counters (device): [0] steps, [1] padded steps, [2] guard trips,
    // [3] chains still short of their window / budget, [4] active chains
    unsigned long long* ctr = nullptr;
    int32_t* maxN = nullptr;  // per draw (sync)
    void* sink = nullptr;     // m, discarded results of padded bodies
};

// ESS launchers (ess.hip)
hipError_t ess_prior_draw(const JobDev& j, const void* x0, hipStream_t s);
hipError_t ess_fill_window(const JobDev& j, hipStream_t s);
// Directions of the window after the running one (draws tsnap + W ..) into buffer buf.
hipError_t ess_fill_next_window(const JobDev& j, int buf, hipStream_t s);
hipError_t copy_u32(uint32_t* dst, const uint32_t* src, int n, hipStream_t s);
hipError_t ess_fsm_round(const JobDev& j, hipStream_t s);
hipError_t ess_sync_draw(const JobDev& j, uint32_t draw, uint32_t slot, hipStream_t s);
hipError_t ess_pad_draw(const JobDev& j, uint32_t draw, uint32_t slot, hipStream_t s);
int ess_supported_epl(int D, int dtype);

// NUTS launchers (nuts.hip); mode 0 = FSM, 1 = synchronized vmap, 2 = synchronized compact
int nuts_nvec(int max_depth);
hipError_t nuts_init_state(const JobDev& j, const void* x0, hipStream_t s);
hipError_t nuts_transition(const JobDev& j, int mode, uint32_t step, hipStream_t s);
hipError_t nuts_gradient(const JobDev& j, hipStream_t s);
size_t logreg_split_bytes(const JobDev& j);
hipError_t logreg_setup(const JobDev& j, hipStream_t s);
hipError_t nuts_gradient_dense(const JobDev& j, int ncols, float* Gout, float* Uout, int gstride, hipStream_t s);

// NUTS on a Gaussian mixture (mog.hip): P (Dp x Dp) in d.prec, means in d.X
// Setup: P mu_k, the constants, and the persistent launch shape (pwpb, pblocks).
hipError_t mog_setup(JobDev& j, hipStream_t s);
hipError_t mog_init_state(const JobDev& j, const void* x0, hipStream_t s);
// sync == 0: FSM, each chain runs to tstop or through its budget; sync != 0:
// the chains' draw `draw` only (tstop = draw + 1), recording the draw's
// largest leapfrog count.  ticket: the chain queue's base, advanced here.
hipError_t mog_run(const JobDev& j, int sync, uint32_t draw, unsigned long long* ticket, hipStream_t s);
// vmap padding of draw `draw` (after mog_run of that draw).
hipError_t mog_pad(const JobDev& j, uint32_t draw, unsigned long long* ticket, hipStream_t s);
// U and grad U at n points (n x D, row-major) into G (n x D, or NULL) and U (n).
hipError_t mog_eval(const JobDev& j, int n, const float* pts, float* G, float* U, hipStream_t s);

// ESS on GP-regression hyperparameters (gph.hip); mode 0 FSM, 1 one synchronized
// draw, 2 vmap padding of that draw
int gph_max_obs();
size_t gph_slot_bytes(const JobDev& j);  // after gph_setup
int gph_max_inputs();
hipError_t gph_setup(JobDev& j);
hipError_t gph_init_state(const JobDev& j, const void* x0, hipStream_t s);
hipError_t gph_run(const JobDev& j, int mode, uint32_t draw, unsigned long long* ticket, hipStream_t s);

// Slice sampler launchers (slice.hip)
hipError_t sl_init_state(const JobDev& j, const void* x0, hipStream_t s);
hipError_t sl_dir_window(const JobDev& j, hipStream_t s);  // directions of every chain's next W draws
hipError_t sl_fsm_round(const JobDev& j, hipStream_t s);   // one window
hipError_t sl_sync_draw(const JobDev& j, uint32_t draw, hipStream_t s);
hipError_t sl_pad_draw(const JobDev& j, uint32_t draw, hipStream_t s);

// Symmetric DR launchers (drsym.hip)
hipError_t drs_init_state(const JobDev& j, const void* x0, hipStream_t s);
hipError_t drs_fsm_round(const JobDev& j, hipStream_t s);
hipError_t drs_sync_draw(const JobDev& j, uint32_t draw, hipStream_t s);
hipError_t drs_pad_draw(const JobDev& j, uint32_t draw, hipStream_t s);

// DR launchers (dr.hip)
int dr_max_dim();
hipError_t dr_init_state(const JobDev& j, const void* x0, hipStream_t s);
hipError_t dr_fsm_round(const JobDev& j, hipStream_t s);
hipError_t dr_sync_draw(const JobDev& j, uint32_t draw, hipStream_t s);
hipError_t dr_pad_draw(const JobDev& j, uint32_t draw, hipStream_t s);

// Row tiles of 32 per ellipse-GEMM wave (8 waves) for a padded dimension;
// 2 to 4 select the bf16 variant, which needs L's packed bf16 pieces.
inline int ess_gemm_rt(int Dp) { return (Dp / 32 + 7) / 8; }
// Size of L's packed bf16 pieces: per row tile ti and chunk c <= ti, two
// k-blocks of three 32 x 16 pieces.
inline size_t ess_lower_pieces_halfwords(int Dp)
{
    const size_t nt = (size_t)Dp / 32;
    return nt * (nt + 1) / 2 * 2 * 3 * 512;
}

}  // namespace fsmmc
