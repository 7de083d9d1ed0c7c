// batch.hip -- several jobs (different samplers, targets, dimensions, chain
// and draw counts) stepped together, one captured hipGraph replay per round.
//
// A round serves every job at once:
//   1. batch_begin_kernel: reset the work queue;
//   2. batch_nu_kernel<RT, CT>: the grouped ellipse GEMM -- one launch per
//      tile shape covers the next W directions of every ESS chain of every
//      job (a table of (job, first column) tiles);
//   3. batch_fsm_kernel: persistent; each wavefront pops work items from a
//      device queue ordered longest first -- one ESS chain for W draws, or 64
//      DRMH chains (one per lane) for `chunk` draws -- and runs the chains'
//      FSM steps with the same device functions as the single-job kernels;
//   4. nuts_steps NUTS runtime steps for every NUTS job: grouped transition
//      (one wavefront per chain; it adds up the row-slice partials of the
//      gradient it consumes), per-job request compaction and grouped
//      logistic-regression gradient tiles;
//   5. batch_tally_kernel: per job, chains short of n and draws so far.
// Every random number is keyed by (seed, chain, draw, role, sub) and every
// reduction has a fixed order, so a job's draws do not depend on the batch,
// the queue order, the other jobs or the tuning.
//
// The autotuner measures real rounds (HIP events around each replay) for a
// few values of W, the DRMH chunk and the GEMM column tile.  It scores a
// configuration by the time the round's draws would take with each sampler
// class running alone (measured once per class) divided by the measured
// round time, and keeps the best.
#include <algorithm>
#include <cstring>
#include <vector>

#include "dr_device.h"
#include "ess_device.h"
#include "logreg_device.h"
#include "multi.h"
#include "nuts_device.h"

namespace fsmmc {

enum BatchCls : int32_t {
    BC_ESS1 = 0, BC_ESS2, BC_ESS4, BC_ESS6, BC_ESS8, BC_ESS12, BC_ESS16,
    BC_DR4, BC_DR8, BC_DR12, BC_DR16, BC_NUTS, BC_NONE
};

struct BJob {
    int32_t cls;
    uint32_t chunk;  // DRMH draws per chain per round
    int32_t m, n;
    const uint32_t* t;  // chain draw counters
    int32_t* list;      // NUTS request list and count
    int32_t* count;
    unsigned long long* ctr;
    EssK<float> ess;
    NuK<float> nu;
    DrK dr;
    NutsK nuts;
    GradK grad;
};

struct BItem {
    int32_t job, first;  // ESS: chain; DRMH: first of 64 chains; NUTS: chain / first of 4
};

struct BTile {
    int32_t job, col0;
};

struct BGrad {
    int32_t job, ct, sl, pad;
};

struct BHdr {
    uint32_t next;  // work queue head
    uint32_t pad;
    unsigned long long live;       // chains short of n after the round
    unsigned long long fsm_draws;  // draws emitted by the persistent FSM kernel
};

struct BJobStat {
    unsigned long long live, draws;
};

// The job table is read through the constant address space: the compiler may
// then reload a view's fields where needed instead of holding the whole view
// in registers across a chain's loop.
typedef const BJob __attribute__((address_space(4))) ConstBJob;

__global__ void batch_begin_kernel(BHdr* h)
{
    h->next = 0;
    h->live = 0;
    h->fsm_draws = 0;
}

template <int RT, int CT>
__global__ __launch_bounds__(512) void batch_nu_kernel(const BJob* jobs, const BTile* tiles)
{
    const BTile t = tiles[blockIdx.x];
    const NuK<float> a = jobs[t.job].nu;
    nu_gemm_block<RT, CT>(a, t.col0);
}

// WIDE: include the DRMH body for dim 13..16 (more registers per lane, one
// fewer wave per SIMD); instantiated only for batches that hold such a job.
template <bool WIDE>
__global__ __launch_bounds__(256) void batch_fsm_kernel(const BJob* jobs_in, const BItem* items, int nitems, BHdr* h)
{
    const ConstBJob* jobs = (const ConstBJob*)jobs_in;
    const int lane = threadIdx.x & 63;
    unsigned long long nd = 0;  // draws emitted by this lane's chains (ESS: lane 0 counts)
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
            uint32_t de = 0;
            EssTally tl;
            switch (cls) {
            case BC_ESS1: de = ess_window<float, 1>(a, item.first, lane, tl); break;
            case BC_ESS2: de = ess_window<float, 2>(a, item.first, lane, tl); break;
            case BC_ESS4: de = ess_window<float, 4>(a, item.first, lane, tl); break;
            case BC_ESS6: de = ess_window<float, 6>(a, item.first, lane, tl); break;
            case BC_ESS8: de = ess_window<float, 8>(a, item.first, lane, tl); break;
            case BC_ESS12: de = ess_window<float, 12>(a, item.first, lane, tl); break;
            default: de = ess_window<float, 16>(a, item.first, lane, tl); break;
            }
            ess_count(a, tl, lane);
            if (lane == 0) nd += de;
        } else if (cls <= BC_DR16) {
            const DrK& a = *(const DrK*)&jobs[item.job].dr;
            const int c = item.first + lane;
            uint32_t steps = 0, live = 0;
            if (c < a.m) {
                const uint32_t stop = a.t[c] + jobs[item.job].chunk;
                if (cls == BC_DR4)
                    nd += dr_run<4>(a, c, stop, &steps, &live);
                else if (cls == BC_DR8)
                    nd += dr_run<8>(a, c, stop, &steps, &live);
                else if (!WIDE || cls == BC_DR12)
                    nd += dr_run<12>(a, c, stop, &steps, &live);
                else
                    nd += dr_run<WIDE ? 16 : 12>(a, c, stop, &steps, &live);
            }
            // one atomic per wave and counter; lane occupancy as in dr_count_lanes
            const unsigned long long st = wave_sum_u64(steps), lv = wave_sum_u64(live);
            const unsigned long long slots = 64ull * (unsigned long long)wave_max_i32((int)steps);
            if (lane == 0) {
                if (st) atomicAdd(&a.ctr[0], st);
                if (lv) atomicAdd(&a.ctr[4], lv);
                if (st) atomicAdd(&a.ctr[5], st);
                if (slots) atomicAdd(&a.ctr[6], slots);
            }
        }
    }
    if (nd) atomicAdd(&h->fsm_draws, nd);
}

// NUTS: one wavefront per chain of the item table.
template <int EPL>
__global__ __launch_bounds__(256) void batch_nuts_step_kernel(const BJob* jobs_in, const BItem* items, int n)
{
    const ConstBJob* jobs = (const ConstBJob*)jobs_in;
    const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (w >= n) return;
    BItem it = items[w];
    it.job = __builtin_amdgcn_readfirstlane(it.job);
    it.first = __builtin_amdgcn_readfirstlane(it.first);
    const NutsK& a = *(const NutsK*)&jobs[it.job].nuts;
    nuts_chain_step<EPL>(a, it.first, threadIdx.x & 63);
}

__global__ __launch_bounds__(1024) void batch_nuts_compact_kernel(const BJob* jobs, const int32_t* njobs)
{
    const BJob& J = jobs[njobs[blockIdx.x]];
    nuts_compact_block<1024>(J.nuts.req, J.m, 0, J.list, J.count, J.ctr);
}

template <int DT>
__global__ __launch_bounds__(512) void batch_grad_kernel(const BJob* jobs_in, const BGrad* tiles)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const ConstBJob* jobs = (const ConstBJob*)jobs_in;
    const BGrad t = tiles[blockIdx.x];
    const GradK& a = *(const GradK*)&jobs[t.job].grad;
    // the job's dimension class fixed at compile time, as in the single-job
    // kernel (a runtime class leaves the tile's per-k arrays in scratch)
#define FSMMC_TILE_CASE(K) \
    case K: logreg_grad_tile<DT, (K)>(a, t.ct, t.sl, lds); break;
    if constexpr (DT == 2) {
        switch ((a.D + 7) >> 3) {
            FSMMC_TILE_CASE(1) FSMMC_TILE_CASE(2) FSMMC_TILE_CASE(3) FSMMC_TILE_CASE(4)
            FSMMC_TILE_CASE(5) FSMMC_TILE_CASE(6) FSMMC_TILE_CASE(7) default: logreg_grad_tile<DT, 8>(a, t.ct, t.sl, lds);
        }
    } else {
        switch ((a.D + 7) >> 3) {
            FSMMC_TILE_CASE(9) FSMMC_TILE_CASE(10) FSMMC_TILE_CASE(11) FSMMC_TILE_CASE(12)
            FSMMC_TILE_CASE(13) FSMMC_TILE_CASE(14) FSMMC_TILE_CASE(15) default: logreg_grad_tile<DT, 16>(a, t.ct, t.sl, lds);
        }
    }
#undef FSMMC_TILE_CASE
}

// Block i: job i's chains short of n and its draws so far.
__global__ __launch_bounds__(256) void batch_tally_kernel(BHdr* h, const BJob* jobs, BJobStat* js)
{
    __shared__ unsigned long long s_live, s_draws;
    if (threadIdx.x == 0) {
        s_live = 0;
        s_draws = 0;
    }
    __syncthreads();
    const BJob& J = jobs[blockIdx.x];
    unsigned long long live = 0, draws = 0;
    for (int c = threadIdx.x; c < J.m; c += blockDim.x) {
        const uint32_t t = J.t[c];
        draws += t;
        live += t < (uint32_t)J.n ? 1 : 0;
    }
    atomicAdd(&s_live, live);
    atomicAdd(&s_draws, draws);
    __syncthreads();
    if (threadIdx.x == 0) {
        js[blockIdx.x].live = s_live;
        js[blockIdx.x].draws = s_draws;
        if (s_live) atomicAdd(&h->live, s_live);
    }
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

int tile_slot(int rt, int ct) { return (rt - 1) * 2 + (ct == 4 ? 1 : 0); }

hipError_t launch_tiles(int slot, int ntiles, const BJob* jobs, const BTile* tiles, hipStream_t s)
{
    const dim3 g(ntiles), b(512);
    switch (slot) {
    case 0: hipLaunchKernelGGL((batch_nu_kernel<1, 2>), g, b, 0, s, jobs, tiles); break;
    case 1: hipLaunchKernelGGL((batch_nu_kernel<1, 4>), g, b, 0, s, jobs, tiles); break;
    case 2: hipLaunchKernelGGL((batch_nu_kernel<2, 2>), g, b, 0, s, jobs, tiles); break;
    case 4: hipLaunchKernelGGL((batch_nu_kernel<3, 2>), g, b, 0, s, jobs, tiles); break;
    case 6: hipLaunchKernelGGL((batch_nu_kernel<4, 2>), g, b, 0, s, jobs, tiles); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int kind_slot(int kind) { return kind == FSMMC_ESS ? 0 : (kind == FSMMC_DRMH ? 1 : 2); }
int kind_mask(int kind) { return kind == FSMMC_ESS ? MASK_ESS : (kind == FSMMC_DRMH ? MASK_DR : MASK_NUTS); }

size_t stat_bytes(size_t njobs) { return sizeof(BHdr) + njobs * sizeof(BJobStat); }

void destroy_graph(fsmmc_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
}

template <typename T>
fsmmc_status ensure(T** p, size_t* cap, size_t n)
{
    if (n <= *cap && *p) return FSMMC_OK;
    const size_t want = std::max<size_t>(std::max<size_t>(n, 2 * *cap), 1);
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    HIP_TRY(hipMalloc((void**)p, want * sizeof(T)));
    *cap = want;
    return FSMMC_OK;
}

fsmmc_status ensure_stat(fsmmc_batch* b, size_t njobs)
{
    const size_t need = stat_bytes(njobs);
    if (need <= b->cap_stat && b->d_stat) return FSMMC_OK;
    if (b->d_stat) (void)hipFree(b->d_stat);
    if (b->h_stat) (void)hipHostFree(b->h_stat);
    b->d_stat = nullptr;
    b->h_stat = nullptr;
    b->cap_stat = 0;
    const size_t want = stat_bytes(std::max<size_t>(njobs, 16) * 2);
    HIP_TRY(hipMalloc((void**)&b->d_stat, want));
    HIP_TRY(hipHostMalloc((void**)&b->h_stat, want, hipHostMallocDefault));
    b->cap_stat = want;
    return FSMMC_OK;
}

template <typename T>
fsmmc_status upload(T* dst, const std::vector<T>& v)
{
    if (!v.empty()) HIP_TRY(hipMemcpy(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return FSMMC_OK;
}

#define TRY_ST(expr)                           \
    do {                                       \
        fsmmc_status s__ = (expr);             \
        if (s__ != FSMMC_OK) return s__;       \
    } while (0)

// Rebuild the job views and work tables for the live jobs and the current
// configuration, then capture the round graph.
fsmmc_status rebuild(fsmmc_batch* b)
{
    HIP_TRY(hipStreamSynchronize(b->stream));  // no replay may still read the old tables
    const int nj = (int)b->jobs.size();
    std::vector<BJob> jv(nj);
    std::vector<std::pair<double, BItem>> items;
    std::vector<BTile> tiles[kTileSlots];
    std::vector<BItem> nsteps[2];
    std::vector<BGrad> grads[2];
    std::vector<int32_t> njobs;
    for (int i = 0; i < nj; ++i) {
        JobDev& d = b->jobs[i]->d;
        BJob& J = jv[i];
        std::memset(&J, 0, sizeof(J));
        J.ctr = d.ctr;
        J.m = d.m;
        J.n = d.n;
        J.t = d.t;
        J.chunk = (uint32_t)b->chunk;
        J.cls = BC_NONE;
        const bool on = b->live[i] && (b->mask & kind_mask(d.kind));
        b->had_items[i] = on ? 1 : 0;
        if (d.kind == FSMMC_ESS) {
            d.W = std::max(1, std::min(b->W, d.Wcap));
            d.nu_cur = 0;  // the grouped GEMM fills buffer 0
            J.ess = ess_view<float>(d);
            J.nu = ess_window_view<float>(d);
            if (!on) continue;
            J.cls = ess_cls(d.EPL);
            const double cost = (double)d.W * (d.EPL + 2);
            for (int c = 0; c < d.m; ++c) items.push_back({cost, BItem{i, c}});
            const int rt = ess_gemm_rt(d.Dp);
            const int ct = (b->cols == 128 && rt <= 1) ? 4 : 2;  // the bf16 shapes (rt >= 2) take 64
            const int ncols = d.m * d.W;
            for (int c0 = 0; c0 < ncols; c0 += 32 * ct) tiles[tile_slot(rt, ct)].push_back(BTile{i, c0});
        } else if (d.kind == FSMMC_DRMH) {
            J.dr = dr_view(d);
            if (!on) continue;
            J.cls = dr_cls(d.D);
            // 64 chains, one per lane: per draw a few stages of NM/4 Philox blocks each
            const double cost = (double)b->chunk * (dr_nm(d.D) / 4 + 1);
            for (int c = 0; c < d.m; c += 64) items.push_back({cost, BItem{i, c}});
        } else {
            J.nuts = nuts_view(d, 0, 0);
            J.grad = grad_view(d, 0);
            J.list = d.list;
            J.count = d.count;
            if (!on) continue;
            J.cls = BC_NUTS;
            const int e = d.EPL == 1 ? 0 : 1;
            for (int c = 0; c < d.m; ++c) nsteps[e].push_back(BItem{i, c});
            for (int ct = 0; ct * 128 < d.m; ++ct)
                for (int sl = 0; sl < d.nslices; ++sl) grads[e].push_back(BGrad{i, ct, sl, 0});
            njobs.push_back(i);
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
    std::vector<BItem> nv;
    for (int e = 0; e < 2; ++e) {
        b->nstep_cnt[e] = (int)nsteps[e].size();
        nv.insert(nv.end(), nsteps[e].begin(), nsteps[e].end());
    }
    std::vector<BGrad> gv;
    for (int e = 0; e < 2; ++e) {
        b->grad_cnt[e] = (int)grads[e].size();
        gv.insert(gv.end(), grads[e].begin(), grads[e].end());
    }
    b->n_nuts = (int)njobs.size();
    TRY_ST(ensure(&b->d_jobs, &b->cap_jobs, (size_t)nj));
    TRY_ST(ensure(&b->d_items, &b->cap_items, iv.size()));
    TRY_ST(ensure(&b->d_tiles, &b->cap_tiles, tv.size()));
    TRY_ST(ensure(&b->d_nitems, &b->cap_nitems, nv.size()));
    TRY_ST(ensure(&b->d_grads, &b->cap_grads, gv.size()));
    TRY_ST(ensure(&b->d_njobs, &b->cap_njobs, njobs.size()));
    TRY_ST(ensure_stat(b, (size_t)nj));
    TRY_ST(upload(b->d_jobs, jv));
    TRY_ST(upload(b->d_items, iv));
    TRY_ST(upload(b->d_tiles, tv));
    TRY_ST(upload(b->d_nitems, nv));
    TRY_ST(upload(b->d_grads, gv));
    TRY_ST(upload(b->d_njobs, njobs));
    b->n_items = (int)iv.size();
    const int resident = b->max_resident[b->wide ? 1 : 0];
    b->fsm_blocks = std::max(1, std::min(resident, (b->n_items + 3) / 4));

    destroy_graph(b);
    BHdr* h = reinterpret_cast<BHdr*>(b->d_stat);
    BJobStat* js = reinterpret_cast<BJobStat*>(b->d_stat + sizeof(BHdr));
    const BJob* jobs = b->d_jobs;
    hipStream_t s = b->stream;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    auto chk = [&]() {
        if (e == hipSuccess) e = hipGetLastError();
    };
    hipLaunchKernelGGL(batch_begin_kernel, dim3(1), dim3(1), 0, s, h);
    chk();
    for (int t = 0; t < kTileSlots && e == hipSuccess; ++t)
        if (b->tile_cnt[t] > 0) e = launch_tiles(t, b->tile_cnt[t], jobs, b->d_tiles + b->tile_off[t], s);
    if (e == hipSuccess && b->n_items > 0) {
        if (b->wide)
            hipLaunchKernelGGL(batch_fsm_kernel<true>, dim3(b->fsm_blocks), dim3(256), 0, s, jobs,
                               (const BItem*)b->d_items, b->n_items, h);
        else
            hipLaunchKernelGGL(batch_fsm_kernel<false>, dim3(b->fsm_blocks), dim3(256), 0, s, jobs,
                               (const BItem*)b->d_items, b->n_items, h);
        chk();
    }
    for (int step = 0; step < b->nuts_steps && b->n_nuts > 0 && e == hipSuccess; ++step) {
        const BItem* st1 = b->d_nitems;
        const BItem* st2 = st1 + b->nstep_cnt[0];
        if (b->nstep_cnt[0])
            hipLaunchKernelGGL(batch_nuts_step_kernel<1>, dim3((b->nstep_cnt[0] + 3) / 4), dim3(256), 0, s, jobs,
                               st1, b->nstep_cnt[0]);
        if (b->nstep_cnt[1])
            hipLaunchKernelGGL(batch_nuts_step_kernel<2>, dim3((b->nstep_cnt[1] + 3) / 4), dim3(256), 0, s, jobs,
                               st2, b->nstep_cnt[1]);
        chk();
        hipLaunchKernelGGL(batch_nuts_compact_kernel, dim3(b->n_nuts), dim3(1024), 0, s, jobs,
                           (const int32_t*)b->d_njobs);
        chk();
        if (b->grad_cnt[0])
            hipLaunchKernelGGL(batch_grad_kernel<2>, dim3(b->grad_cnt[0]), dim3(512), GradB<2>::LDS, s, jobs,
                               (const BGrad*)b->d_grads);
        if (b->grad_cnt[1])
            hipLaunchKernelGGL(batch_grad_kernel<4>, dim3(b->grad_cnt[1]), dim3(512), GradB<4>::LDS, s, jobs,
                               (const BGrad*)b->d_grads + b->grad_cnt[0]);
        chk();
    }
    if (e == hipSuccess && nj > 0) {
        hipLaunchKernelGGL(batch_tally_kernel, dim3(nj), dim3(256), 0, s, h, jobs, js);
        chk();
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &g);
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

bool any_live(const fsmmc_batch* b, int kind)
{
    for (size_t i = 0; i < b->jobs.size(); ++i)
        if (b->live[i] && b->jobs[i]->d.kind == kind) return true;
    return false;
}

uint64_t host_draws(const fsmmc_job* j)
{
    std::vector<uint32_t> t(j->d.m);
    if (hipMemcpy(t.data(), j->d.t, t.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) return 0;
    uint64_t s = 0;
    for (uint32_t v : t) s += v;
    return s;
}

}  // namespace

// ------------------------------------------------------------ internal API
fsmmc_status batch_setup(fsmmc_batch* b, fsmmc_ctx* ctx, void* stream, const fsmmc_batch_tune* tune)
{
    if (tune && tune->gemm_cols != 0 && tune->gemm_cols != 64 && tune->gemm_cols != 128)
        return fail(FSMMC_EINVAL, "gemm_cols must be 0, 64 or 128");
    if (tune && (tune->window < 0 || tune->dr_chunk < 0 || tune->rounds_per_sync < 0 || tune->nuts_steps < 0))
        return fail(FSMMC_EINVAL, "tuning values must be >= 0");
    b->ctx = ctx;
    if (tune) b->tune = *tune;
    b->W = b->tune.window > 0 ? b->tune.window : 16;
    b->chunk = b->tune.dr_chunk > 0 ? b->tune.dr_chunk : 16;
    b->cols = b->tune.gemm_cols > 0 ? b->tune.gemm_cols : 64;
    b->rps = b->tune.rounds_per_sync > 0 ? b->tune.rounds_per_sync : 4;
    b->nuts_steps = b->tune.nuts_steps > 0 ? b->tune.nuts_steps : 16;
    HIP_TRY(hipSetDevice(ctx->device));
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        b->own_stream = true;
    }
    HIP_TRY(hipEventCreate(&b->e0));
    HIP_TRY(hipEventCreate(&b->e1));
    HIP_TRY(hipFuncSetAttribute((const void*)batch_grad_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                GradB<2>::LDS));
    HIP_TRY(hipFuncSetAttribute((const void*)batch_grad_kernel<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                GradB<4>::LDS));
    int nb0 = 0, nb1 = 0, cus = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb0, batch_fsm_kernel<false>, 256, 0));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb1, batch_fsm_kernel<true>, 256, 0));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    b->max_resident[0] = std::max(1, nb0) * std::max(1, cus);
    b->max_resident[1] = std::max(1, nb1) * std::max(1, cus);
    return ensure_stat(b, 16);
}

fsmmc_status batch_admissible(const fsmmc_batch* b, const fsmmc_job* j)
{
    if (!j) return fail(FSMMC_EINVAL, "job is NULL");
    if (j->ctx != b->ctx) return fail(FSMMC_EINVAL, "job belongs to another context");
    if (j->batch) return fail(FSMMC_EBUSY, "job is already in a batch");
    if (j->d.dtype != FSMMC_F32) return fail(FSMMC_ENOTSUP, "batches run FP32 jobs");
    if (j->d.kind == FSMMC_NUTS && j->d.target != FSMMC_LOGREG)
        return fail(FSMMC_ENOTSUP, "batches run NUTS on LOGREG targets only");
    if (j->d.kind == FSMMC_ESS && j->d.target == FSMMC_GP_HYPER)
        return fail(FSMMC_ENOTSUP, "batches do not run GP_HYPER jobs");
    if (j->d.kind == FSMMC_DRSYM || j->d.kind == FSMMC_SLICE)
        return fail(FSMMC_ENOTSUP, "batches do not run DRSYM or SLICE jobs");
    return FSMMC_OK;
}

fsmmc_status batch_add(fsmmc_batch* b, fsmmc_job* j)
{
    TRY_ST(batch_admissible(b, j));
    HIP_TRY(hipStreamSynchronize(j->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    // every chain may run to n within a round: no step budget; NUTS chains run to n
    HIP_TRY(fill_i64(j->d.budget, INT64_MAX, j->d.m, b->stream));
    j->d.tstop = (uint32_t)j->d.n;
    b->jobs.push_back(j);
    b->live.push_back(1);
    b->had_items.push_back(0);
    b->tsum.push_back(host_draws(j));
    b->wide |= j->d.kind == FSMMC_DRMH && dr_nm(j->d.D) > 12;
    j->batch = b;
    b->dirty = true;
    return ensure_stat(b, b->jobs.size());
}

void batch_remove(fsmmc_batch* b, fsmmc_job* j)
{
    (void)hipStreamSynchronize(b->stream);
    for (size_t i = 0; i < b->jobs.size(); ++i) {
        if (b->jobs[i] != j) continue;
        b->jobs.erase(b->jobs.begin() + i);
        b->live.erase(b->live.begin() + i);
        b->had_items.erase(b->had_items.begin() + i);
        b->tsum.erase(b->tsum.begin() + i);
        break;
    }
    if (j->batch == b) {
        j->batch = nullptr;
        if (j->d.kind == FSMMC_ESS && j->d.Wcap > 0) j->d.W = j->d.Wcap;
    }
    b->wide = false;
    for (fsmmc_job* o : b->jobs) b->wide |= o->d.kind == FSMMC_DRMH && dr_nm(o->d.D) > 12;
    b->dirty = true;
}

bool batch_job_live(const fsmmc_batch* b, const fsmmc_job* j)
{
    for (size_t i = 0; i < b->jobs.size(); ++i)
        if (b->jobs[i] == j) return b->live[i] != 0;
    return false;
}

fsmmc_status batch_launch(fsmmc_batch* b, int k)
{
    b->pending_k = 0;
    if (b->jobs.empty()) return FSMMC_OK;
    if (b->dirty) TRY_ST(rebuild(b));
    HIP_TRY(hipEventRecord(b->e0, b->stream));
    for (int i = 0; i < k; ++i) HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    HIP_TRY(hipEventRecord(b->e1, b->stream));
    HIP_TRY(hipMemcpyAsync(b->h_stat, b->d_stat, stat_bytes(b->jobs.size()), hipMemcpyDeviceToHost, b->stream));
    b->pending_k = k;
    return FSMMC_OK;
}

fsmmc_status batch_collect(fsmmc_batch* b, RoundResult* r)
{
    *r = RoundResult();
    if (b->pending_k == 0) return FSMMC_OK;
    const int k = b->pending_k;
    b->pending_k = 0;
    HIP_TRY(hipStreamSynchronize(b->stream));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, b->e0, b->e1));
    const BJobStat* js = reinterpret_cast<const BJobStat*>(b->h_stat + sizeof(BHdr));
    r->ms = ms;
    r->fsm_draws = reinterpret_cast<const BHdr*>(b->h_stat)->fsm_draws;
    b->rounds += k;
    b->gpu_ms += ms;
    for (size_t i = 0; i < b->jobs.size(); ++i) {
        const uint64_t dd = js[i].draws - b->tsum[i];
        b->tsum[i] = js[i].draws;
        r->draws[kind_slot(b->jobs[i]->d.kind)] += dd;
        b->draws += (int64_t)dd;
        r->live += js[i].live;
        if (b->live[i] && js[i].live == 0) {
            b->live[i] = 0;
            b->dirty = true;
        }
    }
    return FSMMC_OK;
}

fsmmc_status batch_round(fsmmc_batch* b, int k, RoundResult* r)
{
    TRY_ST(batch_launch(b, k));
    return batch_collect(b, r);
}

fsmmc_status batch_autotune(fsmmc_batch* b)
{
    b->tuned = true;
    const bool has[3] = {any_live(b, FSMMC_ESS), any_live(b, FSMMC_DRMH), any_live(b, FSMMC_NUTS)};
    const int nclass = (int)has[0] + (int)has[1] + (int)has[2];
    if (!has[0] && !has[1]) return FSMMC_OK;  // nothing to tune for NUTS alone
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
    double w[3] = {1.0, 1.0, 1.0};  // device time per draw of each class running alone
    auto run1 = [&](int W, int chunk, int cols, int mask) -> fsmmc_status {
        if (W != b->W || chunk != b->chunk || cols != b->cols || mask != b->mask) b->dirty = true;
        b->W = W;
        b->chunk = chunk;
        b->cols = cols;
        b->mask = mask;
        fsmmc_status st = batch_round(b, 1, &r);
        b->tune_ms += r.ms;
        b->trials++;
        return st;
    };
    if (nclass > 1) {
        const int masks[3] = {MASK_ESS, MASK_DR, MASK_NUTS};
        for (int c = 0; c < 3; ++c) {
            if (!has[c]) continue;
            TRY_ST(run1(16, 16, 64, masks[c]));
            if (r.draws[c]) w[c] = r.ms / (double)r.draws[c];
        }
    }
    auto score = [&]() {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) s += w[c] * (double)r.draws[c];
        return r.ms > 0.0 ? s / r.ms : 0.0;
    };
    int bestW = b->W, bestC = b->chunk, bestCols = 64;
    double best = -1.0;
    if (has[0]) {
        for (int W : {8, 16, 32, 64}) {
            if (W > std::max(8, wmax)) break;
            TRY_ST(run1(W, W, 64, MASK_ALL));
            const double sc = score();
            if (sc > best) best = sc, bestW = W, bestC = W;
        }
    }
    if (has[1]) {
        const int base = has[0] ? bestW : 16;
        for (int f : {1, 2, 4, 8}) {
            const int chunk = has[0] ? std::max(1, base * f / 2) : base * f;
            if (has[0] && chunk == bestC) continue;
            TRY_ST(run1(bestW, chunk, 64, MASK_ALL));
            const double sc = score();
            if (sc > best) best = sc, bestC = chunk;
        }
    }
    if (has[0] && small_d) {
        TRY_ST(run1(bestW, bestC, 128, MASK_ALL));
        if (score() > best) bestCols = 128;
    }
    b->W = bestW;
    b->chunk = bestC;
    b->cols = bestCols;
    b->mask = MASK_ALL;
    b->dirty = true;
    return FSMMC_OK;
}

void batch_teardown(fsmmc_batch* b)
{
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    destroy_graph(b);
    while (!b->jobs.empty()) batch_remove(b, b->jobs.back());
    destroy_graph(b);
    if (b->d_jobs) (void)hipFree(b->d_jobs);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_nitems) (void)hipFree(b->d_nitems);
    if (b->d_grads) (void)hipFree(b->d_grads);
    if (b->d_njobs) (void)hipFree(b->d_njobs);
    if (b->d_stat) (void)hipFree(b->d_stat);
    if (b->h_stat) (void)hipHostFree(b->h_stat);
    if (b->e0) (void)hipEventDestroy(b->e0);
    if (b->e1) (void)hipEventDestroy(b->e1);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    b->d_jobs = nullptr;
    b->d_stat = nullptr;
    b->h_stat = nullptr;
    b->stream = nullptr;
}

}  // namespace fsmmc

using namespace fsmmc;

extern "C" {

fsmmc_status fsmmc_batch_create(fsmmc_ctx* ctx, fsmmc_job* const* jobs, int32_t n_jobs, void* stream,
                                const fsmmc_batch_tune* tune, fsmmc_batch** out)
{
    if (!ctx || !jobs || !out) return fail(FSMMC_EINVAL, "ctx, jobs or out is NULL");
    *out = nullptr;
    if (n_jobs < 1) return fail(FSMMC_EINVAL, "n_jobs must be >= 1");
    fsmmc_batch probe;
    probe.ctx = ctx;
    for (int i = 0; i < n_jobs; ++i) {
        TRY_ST(batch_admissible(&probe, jobs[i]));
        for (int k = 0; k < i; ++k)
            if (jobs[k] == jobs[i]) return fail(FSMMC_EINVAL, "job listed twice");
    }
    fsmmc_batch* b = new fsmmc_batch();
    fsmmc_status st = batch_setup(b, ctx, stream, tune);
    for (int i = 0; i < n_jobs && st == FSMMC_OK; ++i) st = batch_add(b, jobs[i]);
    if (st != FSMMC_OK) {
        batch_teardown(b);
        delete b;
        return st;
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
        TRY_ST(batch_autotune(b));
        done_rounds += b->rounds - before;
    }
    auto none_live = [&]() {
        for (char v : b->live)
            if (v) return false;
        return true;
    };
    bool finished = none_live();
    RoundResult r;
    while (!finished && (max_rounds <= 0 || done_rounds < max_rounds)) {
        int k = b->rps;
        if (max_rounds > 0) k = (int)std::min<int64_t>(k, max_rounds - done_rounds);
        TRY_ST(batch_round(b, k, &r));
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
    batch_teardown(b);
    delete b;
    return FSMMC_OK;
}

}  // extern "C"
