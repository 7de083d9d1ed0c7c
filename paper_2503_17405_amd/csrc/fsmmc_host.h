// fsmmc_host.h -- host-side internals shared by the C ABI (fsmmc_api.hip),
// the batch runtime (batch.hip) and the serving loop (serve.hip).  Not
// installed; not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <string>
#include <vector>

#include "fsmmc_internal.h"

struct fsmmc_batch;

struct fsmmc_ctx {
    int device = 0;
    size_t budget = 0;
    std::atomic<size_t> used{0};
    std::atomic<int> jobs{0};
};

namespace fsmmc {

// Record the calling thread's error message and return the status.
fsmmc_status fail(fsmmc_status s, const std::string& msg);
fsmmc_status hip_fail(hipError_t e, const char* what);

#define HIP_TRY(expr)                                                  \
    do {                                                               \
        hipError_t e__ = (expr);                                       \
        if (e__ != hipSuccess) return ::fsmmc::hip_fail(e__, #expr);   \
    } while (0)

// Argument checks of fsmmc_init_chains (sets the error message).
fsmmc_status validate_specs(const fsmmc_target_spec* t, const fsmmc_sampler_spec* s, int32_t m, int32_t n);

hipError_t fill_i64(int64_t* p, int64_t v, int n, hipStream_t s);
hipError_t fill_i32(int32_t* p, int32_t v, int n, hipStream_t s);

struct TimedLaunch {
    hipEvent_t a, b;
    int cls;
};

// Kernel classes of fsmmc_stats.kernel_ms.
enum { KC_G = 0, KC_FSM = 1, KC_SYNC = 2, KC_PAD = 3 };

}  // namespace fsmmc

struct fsmmc_job {
    fsmmc_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    fsmmc::JobDev d;
    std::vector<void*> allocs;
    size_t bytes = 0;
    unsigned long long* h_ctr = nullptr;  // pinned: [0..7] mirror of d.ctr, [8..15] scratch reads
    int launches = 0;
    uint32_t step = 0;  // NUTS runtime step counter (keys the per-step counters)
    uint32_t t_lo = 0;  // every chain holds at least t_lo draws (known without reading the device)
    unsigned long long qticket = 0;  // NUTS on a mixture: chain-queue base of the next launch
    fsmmc_batch* batch = nullptr;  // the batch or server that owns the job's stepping, if any
    // ESS: the next window's ellipse GEMM runs on a side stream while the
    // current window is stepped on `stream`
    hipStream_t side = nullptr;
    hipEvent_t ev_snap = nullptr, ev_gemm = nullptr;
    // optional per-launch device timing
    bool timing = false;
    std::vector<hipEvent_t> pool;
    std::vector<fsmmc::TimedLaunch> pending;
    double kms[4] = {0, 0, 0, 0};
    int klaunch[4] = {0, 0, 0, 0};
};

namespace fsmmc {

inline hipEvent_t ev_get(fsmmc_job* j)
{
    hipEvent_t e = nullptr;
    if (!j->pool.empty()) {
        e = j->pool.back();
        j->pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

// Queue one launcher call on stream s; with timing on, bracket it with events.
template <typename F>
inline hipError_t launch_on(fsmmc_job* j, hipStream_t s, int cls, F&& fn)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (j->timing) {
        a = ev_get(j);
        if (a) (void)hipEventRecord(a, s);
    }
    hipError_t e = fn();
    j->launches++;
    if (j->timing && a) {
        b = ev_get(j);
        if (b) {
            (void)hipEventRecord(b, s);
            j->pending.push_back({a, b, cls});
        } else {
            j->pool.push_back(a);
        }
    }
    return e;
}

template <typename F>
inline hipError_t launch(fsmmc_job* j, int cls, F&& fn)
{
    return launch_on(j, j->stream, cls, static_cast<F&&>(fn));
}

// After the stream has drained: fold the recorded intervals into the totals.
void harvest(fsmmc_job* j);

}  // namespace fsmmc
