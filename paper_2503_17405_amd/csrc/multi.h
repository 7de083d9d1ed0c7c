// multi.h -- host-side internals of the multi-job runtime: the batch object
// stepped one graph replay per round (batch.hip) and the serving loop built
// on it (serve.hip).  Not installed; not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "fsmmc_host.h"

namespace fsmmc {

struct BJob;
struct BItem;
struct BTile;
struct BGrad;

constexpr int kTileSlots = 8;  // grouped ellipse GEMM shapes (RT, CT)

enum { MASK_ESS = 1, MASK_DR = 2, MASK_NUTS = 4, MASK_ALL = 7 };

struct RoundResult {
    double ms = 0.0;
    uint64_t draws[3] = {0, 0, 0};  // ESS, DRMH, NUTS draws produced by the replays
    uint64_t live = 0;              // chains short of n after the last replay
    uint64_t fsm_draws = 0;         // ESS + DRMH draws of the last replay (persistent kernel count)
};

}  // namespace fsmmc

struct fsmmc_batch {
    fsmmc_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<fsmmc_job*> jobs;
    std::vector<char> live;       // job still has chains short of n
    std::vector<char> had_items;  // job had work in the current tables
    std::vector<uint64_t> tsum;   // draws of the job at the last progress read
    fsmmc_batch_tune tune{};
    int W = 16, chunk = 16, cols = 64, rps = 4, nuts_steps = 16;
    int mask = fsmmc::MASK_ALL;  // sampler classes given work
    bool tuned = false;
    // device tables
    fsmmc::BJob* d_jobs = nullptr;
    size_t cap_jobs = 0;
    fsmmc::BItem* d_items = nullptr;  // persistent FSM queue (ESS chains, DRMH groups)
    size_t cap_items = 0;
    fsmmc::BTile* d_tiles = nullptr;  // ellipse GEMM tiles
    size_t cap_tiles = 0;
    fsmmc::BItem* d_nitems = nullptr;  // NUTS chains (EPL 1, then EPL 2)
    size_t cap_nitems = 0;
    fsmmc::BGrad* d_grads = nullptr;  // NUTS gradient tiles (Dp 64, then Dp 128)
    size_t cap_grads = 0;
    int32_t* d_njobs = nullptr;  // NUTS jobs (compaction blocks)
    size_t cap_njobs = 0;
    unsigned char* d_stat = nullptr;  // header, then (live, draws) per job
    unsigned char* h_stat = nullptr;  // pinned mirror
    size_t cap_stat = 0;
    int n_items = 0, fsm_blocks = 0;
    int tile_off[fsmmc::kTileSlots] = {0}, tile_cnt[fsmmc::kTileSlots] = {0};
    int nstep_cnt[2] = {0, 0}, grad_cnt[2] = {0, 0}, n_nuts = 0;
    hipGraphExec_t exec = nullptr;
    bool dirty = true;
    int pending_k = 0;  // replays launched and not yet collected
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int max_resident[2] = {0, 0};  // FSM kernel workgroups resident at once (narrow, wide)
    bool wide = false;             // a DRMH job has dim > 12
    // statistics
    int64_t rounds = 0, captures = 0, draws = 0;
    double gpu_ms = 0.0, tune_ms = 0.0;
    int trials = 0;
};

namespace fsmmc {

// Set up an empty batch on `stream` (NULL: a stream of its own).
fsmmc_status batch_setup(fsmmc_batch* b, fsmmc_ctx* ctx, void* stream, const fsmmc_batch_tune* tune);
// Check that a job may join (sampler kind, dtype, ownership).
fsmmc_status batch_admissible(const fsmmc_batch* b, const fsmmc_job* j);
// Add a job (waits for its queued initialisation); it is stepped from the next round.
fsmmc_status batch_add(fsmmc_batch* b, fsmmc_job* j);
// Remove a job between rounds; it becomes free-standing again.
void batch_remove(fsmmc_batch* b, fsmmc_job* j);
// Replay the round graph k times, then read every job's progress.
fsmmc_status batch_round(fsmmc_batch* b, int k, RoundResult* r);
// The same in two halves: queue the replays and the progress copy; then wait
// for them and fold the progress in.  Jobs may not be added or removed between.
fsmmc_status batch_launch(fsmmc_batch* b, int k);
fsmmc_status batch_collect(fsmmc_batch* b, RoundResult* r);
// Autotune window / DRMH chunk / GEMM tile on real rounds.
fsmmc_status batch_autotune(fsmmc_batch* b);
bool batch_job_live(const fsmmc_batch* b, const fsmmc_job* j);
// Free the batch's own resources (not its jobs, which are detached).
void batch_teardown(fsmmc_batch* b);

}  // namespace fsmmc
