// batch.hip -- several jobs (different targets, dimensions, chain and draw
// counts) stepped together, one captured hipGraph replay per round.
//
// A round serves every job at once:
//   1. batch_begin_kernel: reset the work queue and the per-job live counters;
//   2. batch_nu_kernel<RT, CT>: the grouped ellipse GEMM -- one launch per
//      tile shape covers the next W directions of every ESS chain of every
//      job (a table of (job, first column) tiles);
//   3. batch_fsm_kernel: persistent; each wavefront pops work items from a
//      device queue ordered longest first -- one ESS chain for W draws, or 64
//      DRMH chains (one per lane) for `chunk` draws -- and runs the chains'
//      FSM steps with the same device functions as the single-job kernels;
//   4. batch_tally_kernel: chains still short of n, per job.
// Because every random number is keyed by (seed, chain, draw, role, sub) and
// every reduction has a fixed order, a job's draws do not depend on the
// batch, the queue order or the tuning.
//
// The autotuner measures real rounds (HIP events around each replay) for a
// few values of W, the DRMH chunk and the GEMM column tile, scoring each by
// the time the same work takes when each sampler class runs alone divided by
// the measured round time, and keeps the best.
#include <algorithm>
#include <cstring>
#include <vector>

#include "dr_device.h"
#include "ess_device.h"
#include "fsmmc_host.h"

namespace fsmmc {

enum BatchCls : int32_t {
    BC_ESS1 = 0, BC_ESS2, BC_ESS4, BC_ESS6, BC_ESS8, BC_ESS12, BC_ESS16,
    BC_DR4, BC_DR8, BC_DR12, BC_DR16, BC_NONE
};

struct BJob {
    int32_t cls;
    uint32_t chunk;  // DRMH draws per chain per round
    unsigned long long* ctr;
    EssK<float> ess;
    NuK<float> nu;
    DrK dr;
};

struct BItem {
    int32_t job, first;  // ESS: chain; DRMH: first of 64 chains
};

struct BTile {
    int32_t job, col0;
};

struct BHdr {
    uint32_t next;  // work queue head
    uint32_t pad;
    unsigned long long draws_ess, draws_dr;  // draws since the last host reset
    unsigned long long live;                 // chains short of n after the round
};

__global__ void batch_begin_kernel(BHdr* h, const BJob* jobs, int njobs)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i == 0) {
        h->next = 0;
        h->live = 0;
    }
    if (i < njobs) {
        jobs[i].ctr[3] = 0;
        jobs[i].ctr[4] = 0;
    }
}

__global__ void batch_reset_kernel(BHdr* h)
{
    h->draws_ess = 0;
    h->draws_dr = 0;
}

template <int RT, int CT>
__global__ __launch_bounds__(512) void batch_nu_kernel(const BJob* jobs, const BTile* tiles)
{
    const BTile t = tiles[blockIdx.x];
    const NuK<float> a = jobs[t.job].nu;
    nu_gemm_block<RT, CT>(a, t.col0);
}

// The job table is read through the constant address space: the compiler may
// then reload a view's fields where needed instead of holding the whole view
// in registers across the chain's loop.
typedef const BJob __attribute__((address_space(4))) ConstBJob;

// WIDE: include the DRMH body for dim 13..16 (more registers per lane, one
// fewer wave per SIMD); instantiated only for batches that hold such a job.
template <bool WIDE>
__global__ __launch_bounds__(256) void batch_fsm_kernel(const BJob* jobs_in, const BItem* items, int nitems, BHdr* h)
{
    const ConstBJob* jobs = (const ConstBJob*)jobs_in;
    const int lane = threadIdx.x & 63;
    unsigned long long de = 0, dd = 0;
    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(&h->next, 1u);
        // wave-uniform from here on: the item and its job view load as scalars
        it = __builtin_amdgcn_readfirstlane(it);
        if (it >= (uint32_t)nitems) break;
        BItem item = items[it];
        item.job = __builtin_amdgcn_readfirstlane(item.job);
        item.first = __builtin_amdgcn_readfirstlane(item.first);
        const int cls = jobs[item.job].cls;
        if (cls <= BC_ESS16) {
            const EssK<float>& a = *(const EssK<float>*)&jobs[item.job].ess;
            uint32_t nd = 0;
            switch (cls) {
            case BC_ESS1: nd = ess_window<float, 1>(a, item.first, lane); break;
            case BC_ESS2: nd = ess_window<float, 2>(a, item.first, lane); break;
            case BC_ESS4: nd = ess_window<float, 4>(a, item.first, lane); break;
            case BC_ESS6: nd = ess_window<float, 6>(a, item.first, lane); break;
            case BC_ESS8: nd = ess_window<float, 8>(a, item.first, lane); break;
            case BC_ESS12: nd = ess_window<float, 12>(a, item.first, lane); break;
            default: nd = ess_window<float, 16>(a, item.first, lane); break;
            }
            if (lane == 0) de += nd;
        } else if (cls <= BC_DR16) {
            const DrK& a = *(const DrK*)&jobs[item.job].dr;
            const int c = item.first + lane;
            if (c < a.m) {
                const uint32_t stop = a.t[c] + jobs[item.job].chunk;
                if (cls == BC_DR4)
                    dd += dr_run<4>(a, c, stop);
                else if (cls == BC_DR8)
                    dd += dr_run<8>(a, c, stop);
                else if (!WIDE || cls == BC_DR12)
                    dd += dr_run<12>(a, c, stop);
                else
                    dd += dr_run<WIDE ? 16 : 12>(a, c, stop);
            }
        }
    }
    if (de) atomicAdd(&h->draws_ess, de);
    if (dd) atomicAdd(&h->draws_dr, dd);
}

__global__ void batch_tally_kernel(BHdr* h, const BJob* jobs, int njobs, unsigned long long* jlive)
{
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < njobs; i += blockDim.x) {
        const unsigned long long v = jobs[i].ctr[4];
        jlive[i] = v;
        s += v;
    }
    if (s) atomicAdd(&h->live, s);
}

// ------------------------------------------------------------ host side
namespace {

int ess_cls(int EPL)
{
    switch (EPL) {
    case 1: return BC_ESS1;
    case 2: return BC_ESS2;
    case 4: return BC_ESS4;
    case 6: return BC_ESS6;
    case 8: return BC_ESS8;
    case 12: return BC_ESS12;
    default: return BC_ESS16;
    }
}

int dr_cls(int D)
{
    switch (dr_nm(D)) {
    case 4: return BC_DR4;
    case 8: return BC_DR8;
    case 12: return BC_DR12;
    default: return BC_DR16;
    }
}

// Grouped GEMM launch shapes: (RT, CT) -> slot.
constexpr int kTileSlots = 8;
int tile_slot(int rt, int ct) { return (rt - 1) * 2 + (ct == 4 ? 1 : 0); }

hipError_t launch_tiles(int slot, int ntiles, const BJob* jobs, const BTile* tiles, hipStream_t s)
{
    const dim3 g(ntiles), b(512);
    switch (slot) {
    case 0: hipLaunchKernelGGL((batch_nu_kernel<1, 2>), g, b, 0, s, jobs, tiles); break;
    case 1: hipLaunchKernelGGL((batch_nu_kernel<1, 4>), g, b, 0, s, jobs, tiles); break;
    case 2: hipLaunchKernelGGL((batch_nu_kernel<2, 2>), g, b, 0, s, jobs, tiles); break;
    case 3: hipLaunchKernelGGL((batch_nu_kernel<2, 4>), g, b, 0, s, jobs, tiles); break;
    case 4: hipLaunchKernelGGL((batch_nu_kernel<3, 2>), g, b, 0, s, jobs, tiles); break;
    case 6: hipLaunchKernelGGL((batch_nu_kernel<4, 2>), g, b, 0, s, jobs, tiles); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

enum { MASK_ESS = 1, MASK_DR = 2 };

}  // namespace
}  // namespace fsmmc

using namespace fsmmc;

struct fsmmc_batch {
    fsmmc_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<fsmmc_job*> jobs;
    std::vector<char> live;      // job still has chains short of n
    std::vector<char> had_items; // job had work items in the current tables
    fsmmc_batch_tune tune{};
    int W = 16, chunk = 16, cols = 64, rps = 4;
    int mask = MASK_ESS | MASK_DR;  // sampler classes given work items
    bool tuned = false;
    // device tables
    BJob* d_jobs = nullptr;
    BItem* d_items = nullptr;
    size_t cap_items = 0;
    BTile* d_tiles = nullptr;
    size_t cap_tiles = 0;
    unsigned char* d_stat = nullptr;  // BHdr, then live count per job
    unsigned char* h_stat = nullptr;  // pinned mirror
    int n_items = 0, fsm_blocks = 0;
    int tile_off[kTileSlots] = {0}, tile_cnt[kTileSlots] = {0};
    hipGraphExec_t exec = nullptr;
    bool dirty = true;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int max_resident = 0;  // workgroups of the FSM kernel resident at once
    bool wide = false;     // a DRMH job has dim > 12
    // statistics
    int64_t rounds = 0, captures = 0, draws = 0;
    double gpu_ms = 0.0, tune_ms = 0.0;
    int trials = 0;
};

namespace {

size_t stat_bytes(const fsmmc_batch* b) { return sizeof(BHdr) + b->jobs.size() * sizeof(unsigned long long); }

void destroy_graph(fsmmc_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
}

template <typename T>
fsmmc_status ensure(T** p, size_t* cap, size_t n)
{
    if (n <= *cap && *p) return FSMMC_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    const size_t want = std::max<size_t>(n, 1);
    HIP_TRY(hipMalloc((void**)p, want * sizeof(T)));
    *cap = want;
    return FSMMC_OK;
}

// Rebuild the job views, the work queue and the tile tables for the live
// jobs and the current configuration, then capture the round graph.
fsmmc_status rebuild(fsmmc_batch* b)
{
    HIP_TRY(hipStreamSynchronize(b->stream));  // no replay may still read the old tables
    const int nj = (int)b->jobs.size();
    std::vector<BJob> jv(nj);
    std::vector<std::pair<double, BItem>> items;
    std::vector<BTile> tiles[kTileSlots];
    for (int i = 0; i < nj; ++i) {
        JobDev& d = b->jobs[i]->d;
        BJob& J = jv[i];
        std::memset(&J, 0, sizeof(J));
        J.ctr = d.ctr;
        J.chunk = (uint32_t)b->chunk;
        b->had_items[i] = 0;
        if (d.kind == FSMMC_ESS) {
            d.W = std::max(1, std::min(b->W, d.Wcap));
            J.cls = ess_cls(d.EPL);
            J.ess = ess_view<float>(d);
            J.nu = ess_window_view<float>(d);
            if (!b->live[i] || !(b->mask & MASK_ESS)) {
                J.cls = BC_NONE;
                continue;
            }
            b->had_items[i] = 1;
            const double cost = (double)d.W * (d.EPL + 2);
            for (int c = 0; c < d.m; ++c) items.push_back({cost, BItem{i, c}});
            const int rt = ess_gemm_rt(d.Dp);
            const int ct = (b->cols == 128 && rt <= 2) ? 4 : 2;
            const int nc = 32 * ct;
            const int ncols = d.m * d.W;
            for (int c0 = 0; c0 < ncols; c0 += nc) tiles[tile_slot(rt, ct)].push_back(BTile{i, c0});
        } else {
            J.cls = dr_cls(d.D);
            J.dr = dr_view(d);
            if (!b->live[i] || !(b->mask & MASK_DR)) {
                J.cls = BC_NONE;
                continue;
            }
            b->had_items[i] = 1;
            // 64 chains, one per lane: per draw a few stages of NM/4 Philox blocks each
            const double cost = (double)b->chunk * (dr_nm(d.D) / 4 + 1);
            for (int c = 0; c < d.m; c += 64) items.push_back({cost, BItem{i, c}});
        }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const std::pair<double, BItem>& x, const std::pair<double, BItem>& y) {
                         return x.first > y.first;
                     });
    std::vector<BItem> iv(items.size());
    for (size_t k = 0; k < items.size(); ++k) iv[k] = items[k].second;
    std::vector<BTile> tv;
    for (int s = 0; s < kTileSlots; ++s) {
        b->tile_off[s] = (int)tv.size();
        b->tile_cnt[s] = (int)tiles[s].size();
        tv.insert(tv.end(), tiles[s].begin(), tiles[s].end());
    }
    fsmmc_status st = ensure(&b->d_items, &b->cap_items, iv.size());
    if (st != FSMMC_OK) return st;
    st = ensure(&b->d_tiles, &b->cap_tiles, tv.size());
    if (st != FSMMC_OK) return st;
    HIP_TRY(hipMemcpy(b->d_jobs, jv.data(), jv.size() * sizeof(BJob), hipMemcpyHostToDevice));
    if (!iv.empty()) HIP_TRY(hipMemcpy(b->d_items, iv.data(), iv.size() * sizeof(BItem), hipMemcpyHostToDevice));
    if (!tv.empty()) HIP_TRY(hipMemcpy(b->d_tiles, tv.data(), tv.size() * sizeof(BTile), hipMemcpyHostToDevice));
    b->n_items = (int)iv.size();
    b->fsm_blocks = std::max(1, std::min(b->max_resident, (b->n_items + 3) / 4));

    destroy_graph(b);
    BHdr* h = reinterpret_cast<BHdr*>(b->d_stat);
    unsigned long long* jl = reinterpret_cast<unsigned long long*>(b->d_stat + sizeof(BHdr));
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(batch_begin_kernel, dim3((nj + 255) / 256), dim3(256), 0, b->stream, h,
                       (const BJob*)b->d_jobs, nj);
    e = hipGetLastError();
    for (int s = 0; s < kTileSlots && e == hipSuccess; ++s)
        if (b->tile_cnt[s] > 0) e = launch_tiles(s, b->tile_cnt[s], b->d_jobs, b->d_tiles + b->tile_off[s], b->stream);
    if (e == hipSuccess && b->n_items > 0) {
        if (b->wide)
            hipLaunchKernelGGL(batch_fsm_kernel<true>, dim3(b->fsm_blocks), dim3(256), 0, b->stream,
                               (const BJob*)b->d_jobs, (const BItem*)b->d_items, b->n_items, h);
        else
            hipLaunchKernelGGL(batch_fsm_kernel<false>, dim3(b->fsm_blocks), dim3(256), 0, b->stream,
                               (const BJob*)b->d_jobs, (const BItem*)b->d_items, b->n_items, h);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(batch_tally_kernel, dim3(1), dim3(256), 0, b->stream, h, (const BJob*)b->d_jobs, nj, jl);
        e = hipGetLastError();
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e, "batch round capture");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->exec = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    b->captures++;
    b->dirty = false;
    return FSMMC_OK;
}

struct RoundResult {
    double ms = 0.0;
    unsigned long long de = 0, dd = 0, live = 0;
};

// Replay the round graph k times; fold liveness into the job flags.
fsmmc_status replay(fsmmc_batch* b, int k, RoundResult* r)
{
    if (b->dirty) {
        fsmmc_status st = rebuild(b);
        if (st != FSMMC_OK) return st;
    }
    BHdr* h = reinterpret_cast<BHdr*>(b->d_stat);
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, b->stream, h);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(b->e0, b->stream));
    for (int i = 0; i < k; ++i) HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    HIP_TRY(hipEventRecord(b->e1, b->stream));
    HIP_TRY(hipMemcpyAsync(b->h_stat, b->d_stat, stat_bytes(b), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, b->e0, b->e1));
    const BHdr* hh = reinterpret_cast<const BHdr*>(b->h_stat);
    const unsigned long long* jl = reinterpret_cast<const unsigned long long*>(b->h_stat + sizeof(BHdr));
    r->ms = ms;
    r->de = hh->draws_ess;
    r->dd = hh->draws_dr;
    b->rounds += k;
    b->gpu_ms += ms;
    b->draws += (int64_t)(r->de + r->dd);
    unsigned long long live = 0;
    for (size_t i = 0; i < b->jobs.size(); ++i) {
        if (!b->had_items[i]) {
            if (b->live[i]) live += 1;  // not stepped this round: still pending
            continue;
        }
        if (b->live[i] && jl[i] == 0) {
            b->live[i] = 0;
            b->dirty = true;
        }
        live += jl[i];
    }
    r->live = live;
    return FSMMC_OK;
}

bool any_live(const fsmmc_batch* b, int kind)
{
    for (size_t i = 0; i < b->jobs.size(); ++i)
        if (b->live[i] && b->jobs[i]->d.kind == kind) return true;
    return false;
}

// Online autotuning on real rounds (see the file comment).
fsmmc_status autotune(fsmmc_batch* b)
{
    b->tuned = true;
    const bool has_ess = any_live(b, FSMMC_ESS), has_dr = any_live(b, FSMMC_DRMH);
    if (!has_ess && !has_dr) return FSMMC_OK;
    int wmax = 1;
    bool small_d = false;
    for (size_t i = 0; i < b->jobs.size(); ++i) {
        const JobDev& d = b->jobs[i]->d;
        if (d.kind == FSMMC_ESS && b->live[i]) {
            wmax = std::max(wmax, d.Wcap);
            small_d |= ess_gemm_rt(d.Dp) <= 2;
        }
    }
    RoundResult r;
    double we = 1.0, wd = 1.0;  // time per draw of each class when it runs alone
    auto run1 = [&](int W, int chunk, int cols, int mask) -> fsmmc_status {
        if (W != b->W || chunk != b->chunk || cols != b->cols || mask != b->mask) b->dirty = true;
        b->W = W;
        b->chunk = chunk;
        b->cols = cols;
        b->mask = mask;
        fsmmc_status st = replay(b, 1, &r);
        b->tune_ms += r.ms;
        b->trials++;
        return st;
    };
    fsmmc_status st;
    if (has_ess && has_dr) {
        st = run1(16, 16, 64, MASK_ESS);
        if (st != FSMMC_OK) return st;
        if (r.de) we = r.ms / (double)r.de;
        st = run1(16, 16, 64, MASK_DR);
        if (st != FSMMC_OK) return st;
        if (r.dd) wd = r.ms / (double)r.dd;
    }
    auto score = [&]() { return r.ms > 0.0 ? (we * (double)r.de + wd * (double)r.dd) / r.ms : 0.0; };
    int bestW = b->W, bestC = b->chunk, bestCols = 64;
    double best = -1.0;
    if (has_ess) {
        for (int W : {8, 16, 32, 64}) {
            if (W > std::max(8, wmax)) break;
            st = run1(W, W, 64, MASK_ESS | MASK_DR);
            if (st != FSMMC_OK) return st;
            const double sc = score();
            if (sc > best) best = sc, bestW = W, bestC = W;
        }
    }
    if (has_dr) {
        const int base = has_ess ? bestW : 16;
        for (int f : {1, 2, 4, 8}) {
            const int chunk = has_ess ? std::max(1, base * f / 2) : base * f;
            if (has_ess && chunk == bestC) continue;
            st = run1(bestW, chunk, 64, MASK_ESS | MASK_DR);
            if (st != FSMMC_OK) return st;
            const double sc = score();
            if (sc > best) best = sc, bestC = chunk;
        }
    }
    if (has_ess && small_d) {
        st = run1(bestW, bestC, 128, MASK_ESS | MASK_DR);
        if (st != FSMMC_OK) return st;
        if (score() > best) bestCols = 128;
    }
    b->W = bestW;
    b->chunk = bestC;
    b->cols = bestCols;
    b->mask = MASK_ESS | MASK_DR;
    b->dirty = true;
    return FSMMC_OK;
}

void batch_release(fsmmc_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    destroy_graph(b);
    for (fsmmc_job* j : b->jobs) {
        if (j->batch == b) {
            j->batch = nullptr;
            j->d.W = j->d.Wcap > 0 ? j->d.Wcap : j->d.W;
        }
    }
    if (b->d_jobs) (void)hipFree(b->d_jobs);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_stat) (void)hipFree(b->d_stat);
    if (b->h_stat) (void)hipHostFree(b->h_stat);
    if (b->e0) (void)hipEventDestroy(b->e0);
    if (b->e1) (void)hipEventDestroy(b->e1);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // namespace

extern "C" {

fsmmc_status fsmmc_batch_create(fsmmc_ctx* ctx, fsmmc_job* const* jobs, int32_t n_jobs, void* stream,
                                const fsmmc_batch_tune* tune, fsmmc_batch** out)
{
    if (!ctx || !jobs || !out) return fail(FSMMC_EINVAL, "ctx, jobs or out is NULL");
    *out = nullptr;
    if (n_jobs < 1) return fail(FSMMC_EINVAL, "n_jobs must be >= 1");
    for (int i = 0; i < n_jobs; ++i) {
        fsmmc_job* j = jobs[i];
        if (!j) return fail(FSMMC_EINVAL, "job is NULL");
        if (j->ctx != ctx) return fail(FSMMC_EINVAL, "job belongs to another context");
        if (j->batch) return fail(FSMMC_EBUSY, "job is already in a batch");
        for (int k = 0; k < i; ++k)
            if (jobs[k] == j) return fail(FSMMC_EINVAL, "job listed twice");
        if (j->d.kind == FSMMC_NUTS) return fail(FSMMC_ENOTSUP, "batches run ESS and DRMH jobs");
        if (j->d.dtype != FSMMC_F32) return fail(FSMMC_ENOTSUP, "batches run FP32 jobs");
    }
    if (tune && tune->gemm_cols != 0 && tune->gemm_cols != 64 && tune->gemm_cols != 128)
        return fail(FSMMC_EINVAL, "gemm_cols must be 0, 64 or 128");
    if (tune && (tune->window < 0 || tune->dr_chunk < 0 || tune->rounds_per_sync < 0))
        return fail(FSMMC_EINVAL, "tuning values must be >= 0");
    HIP_TRY(hipSetDevice(ctx->device));
    fsmmc_batch* b = new fsmmc_batch();
    b->ctx = ctx;
    if (tune) b->tune = *tune;
    b->W = b->tune.window > 0 ? b->tune.window : 16;
    b->chunk = b->tune.dr_chunk > 0 ? b->tune.dr_chunk : 16;
    b->cols = b->tune.gemm_cols > 0 ? b->tune.gemm_cols : 64;
    b->rps = b->tune.rounds_per_sync > 0 ? b->tune.rounds_per_sync : 4;
    b->jobs.assign(jobs, jobs + n_jobs);
    b->live.assign(n_jobs, 1);
    b->had_items.assign(n_jobs, 0);
    auto bail = [&](fsmmc_status s) {
        batch_release(b);
        return s;
    };
    hipError_t e = hipSuccess;
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else {
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(hip_fail(e, "hipStreamCreateWithFlags"));
        b->own_stream = true;
    }
    for (fsmmc_job* j : b->jobs) {
        e = hipStreamSynchronize(j->stream);
        if (e != hipSuccess) return bail(hip_fail(e, "hipStreamSynchronize"));
    }
    if ((e = hipMalloc((void**)&b->d_jobs, (size_t)n_jobs * sizeof(BJob))) != hipSuccess ||
        (e = hipMalloc((void**)&b->d_stat, stat_bytes(b))) != hipSuccess ||
        (e = hipHostMalloc((void**)&b->h_stat, stat_bytes(b), hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreate(&b->e0)) != hipSuccess || (e = hipEventCreate(&b->e1)) != hipSuccess)
        return bail(hip_fail(e, "batch allocation"));
    for (fsmmc_job* j : b->jobs) b->wide |= j->d.kind == FSMMC_DRMH && dr_nm(j->d.D) > 12;
    int nb = 0, cus = 0;
    if ((e = b->wide ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_fsm_kernel<true>, 256, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_fsm_kernel<false>, 256, 0)) !=
            hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device)) != hipSuccess)
        return bail(hip_fail(e, "occupancy query"));
    b->max_resident = std::max(1, nb) * std::max(1, cus);
    // every chain may run to n within a round's window: no step budget
    for (fsmmc_job* j : b->jobs) {
        e = fill_i64(j->d.budget, INT64_MAX, j->d.m, b->stream);
        if (e != hipSuccess) return bail(hip_fail(e, "budget fill"));
        j->batch = b;
    }
    *out = b;
    return FSMMC_OK;
}

fsmmc_status fsmmc_batch_run(fsmmc_batch* b, int64_t max_rounds, int32_t* all_done)
{
    if (!b) return fail(FSMMC_EINVAL, "batch is NULL");
    HIP_TRY(hipSetDevice(b->ctx->device));
    int64_t done_rounds = 0;
    if (b->tune.autotune && !b->tuned) {
        const int64_t before = b->rounds;
        fsmmc_status st = autotune(b);
        if (st != FSMMC_OK) return st;
        done_rounds += b->rounds - before;
    }
    RoundResult r;
    auto none_live = [&]() {
        for (char v : b->live)
            if (v) return false;
        return true;
    };
    bool finished = none_live();
    while (!finished && (max_rounds <= 0 || done_rounds < max_rounds)) {
        int k = b->rps;
        if (max_rounds > 0) k = (int)std::min<int64_t>(k, max_rounds - done_rounds);
        fsmmc_status st = replay(b, k, &r);
        if (st != FSMMC_OK) return st;
        done_rounds += k;
        finished = none_live();
    }
    if (all_done) *all_done = finished ? 1 : 0;
    return FSMMC_OK;
}

fsmmc_status fsmmc_batch_stats(fsmmc_batch* b, fsmmc_batch_counters* out)
{
    if (!b || !out) return fail(FSMMC_EINVAL, "batch or out is NULL");
    std::memset(out, 0, sizeof(*out));
    out->rounds = b->rounds;
    out->captures = b->captures;
    out->draws = b->draws;
    out->window = b->W;
    out->dr_chunk = b->chunk;
    out->gemm_cols = b->cols;
    int lj = 0;
    for (char v : b->live) lj += v ? 1 : 0;
    out->live_jobs = lj;
    out->gpu_ms = b->gpu_ms;
    out->tune_ms = b->tune_ms;
    out->tune_trials = b->trials;
    out->fsm_blocks = b->fsm_blocks;
    return FSMMC_OK;
}

fsmmc_status fsmmc_batch_free(fsmmc_batch* b)
{
    if (!b) return fail(FSMMC_EINVAL, "batch is NULL");
    batch_release(b);
    return FSMMC_OK;
}

}  // extern "C"
