// serve.hip -- continuous-batching server: a request loop in its own thread
// admits submitted jobs under the context's HBM budget, steps every admitted
// job in the rounds of one shared batch (batch.hip), and retires each job the
// round its last chain reaches its last draw, freeing its device memory.
//
// Loop, per iteration:
//   1. queue rounds_per_sync rounds of the batch (one graph replay each);
//   2. while the device runs them, admit pending jobs in arrival order until
//      one does not fit the budget (a job that does not fit even with nothing
//      else admitted fails with EBUDGET): admission allocates the job's state
//      and queues its initialisation on a second stream;
//   3. wait for the rounds and read every job's progress;
//   4. retire finished jobs: copy their loop counts out, detach them from the
//      batch, free them, stamp the completion time;
//   5. the jobs admitted in step 2 join the batch for the next rounds.
// Jobs never wait for each other: each chain only stops at its own n-th draw
// (Sec. 3.2), so a job's draws are the same bits alone and in any mix.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "multi.h"

using namespace fsmmc;

namespace {

struct SrvJob {
    uint64_t id = 0;
    fsmmc_target_spec target{};
    fsmmc_sampler_spec sampler{};
    int32_t m = 0, n = 0;
    uint64_t seed = 0;
    const void* x0 = nullptr;
    void* out = nullptr;
    int32_t* counts = nullptr;
    fsmmc_job* job = nullptr;
    double t_submit = 0.0, t_admit = 0.0;
};

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct fsmmc_server {
    fsmmc_ctx* ctx = nullptr;
    fsmmc_server_config cfg{};
    fsmmc_batch batch;
    hipStream_t admit_stream = nullptr;  // initialisation of admitted jobs, overlapping the rounds
    std::vector<SrvJob*> admitted_q;     // initialised, joining the batch after the current round
    std::thread thr;
    std::mutex mu;
    std::condition_variable cv_work, cv_idle;
    std::deque<SrvJob*> pending;         // guarded by mu
    std::vector<fsmmc_server_done> done; // guarded by mu
    std::vector<SrvJob*> running;        // server thread only
    bool stop = false;
    fsmmc_status fatal = FSMMC_OK;
    uint64_t next_id = 1;
    // counters, guarded by mu
    int64_t submitted = 0, admitted = 0, completed = 0, failed = 0, outstanding = 0;
    int32_t live = 0, peak_live = 0;
    uint64_t peak_bytes = 0;
    int64_t rounds = 0, draws = 0;
    double gpu_ms = 0.0;
};

namespace {

void finish(fsmmc_server* s, SrvJob* sj, fsmmc_status st)
{
    fsmmc_server_done rec{};
    rec.job_id = sj->id;
    rec.status = st;
    rec.t_submit = sj->t_submit;
    rec.t_admit = sj->t_admit;
    rec.t_done = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->done.push_back(rec);
        if (st == FSMMC_OK)
            s->completed++;
        else
            s->failed++;
        s->outstanding--;
    }
    s->cv_idle.notify_all();
    delete sj;
}

// Admit pending jobs in arrival order while the budget allows: allocate
// their state and queue their initialisation on the admission stream.
void admit(fsmmc_server* s)
{
    fsmmc_tune tune{};
    tune.window = s->cfg.ess_window > 0 ? s->cfg.ess_window : 16;
    for (;;) {
        SrvJob* sj = nullptr;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->pending.empty()) return;
            sj = s->pending.front();
        }
        fsmmc_job* job = nullptr;
        fsmmc_status st = fsmmc_init_chains(s->ctx, &sj->target, &sj->sampler, sj->m, sj->n, sj->seed, sj->x0,
                                            sj->out, s->admit_stream, &tune, &job);
        if (st == FSMMC_EBUDGET && !(s->running.empty() && s->admitted_q.empty())) return;  // wait for a retirement
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->pending.pop_front();
        }
        if (st != FSMMC_OK) {
            finish(s, sj, st);
            continue;
        }
        sj->job = job;
        sj->t_admit = now_s();
        s->admitted_q.push_back(sj);
        std::lock_guard<std::mutex> lk(s->mu);
        s->admitted++;
        s->peak_bytes = std::max<uint64_t>(s->peak_bytes, fsmmc_ctx_bytes_in_use(s->ctx));
    }
}

// Move the admitted jobs into the batch (between rounds).
void join(fsmmc_server* s)
{
    for (SrvJob* sj : s->admitted_q) {
        fsmmc_status st = batch_add(&s->batch, sj->job);  // waits for its initialisation
        if (st != FSMMC_OK) {
            fsmmc_job_free(sj->job);
            finish(s, sj, st);
            continue;
        }
        s->running.push_back(sj);
    }
    s->admitted_q.clear();
    std::lock_guard<std::mutex> lk(s->mu);
    s->live = (int32_t)s->running.size();
    s->peak_live = std::max(s->peak_live, s->live);
}

// Retire every job whose chains all have their n draws.
fsmmc_status retire(fsmmc_server* s)
{
    for (size_t i = 0; i < s->running.size();) {
        SrvJob* sj = s->running[i];
        if (batch_job_live(&s->batch, sj->job)) {
            ++i;
            continue;
        }
        fsmmc_job* job = sj->job;
        if (sj->counts)
            HIP_TRY(hipMemcpyAsync(sj->counts, job->d.counts, (size_t)job->d.m * job->d.n * 4,
                                   hipMemcpyDeviceToDevice, s->batch.stream));
        batch_remove(&s->batch, job);  // synchronises the stream
        fsmmc_job_free(job);
        s->running.erase(s->running.begin() + i);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->live = (int32_t)s->running.size();
        }
        finish(s, sj, FSMMC_OK);
    }
    return FSMMC_OK;
}

void fail_all(fsmmc_server* s, fsmmc_status st)
{
    for (SrvJob* sj : s->running) {
        batch_remove(&s->batch, sj->job);
        fsmmc_job_free(sj->job);
        finish(s, sj, st);
    }
    for (SrvJob* sj : s->admitted_q) {
        fsmmc_job_free(sj->job);
        finish(s, sj, st);
    }
    s->running.clear();
    s->admitted_q.clear();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->live = 0;
    }
    std::deque<SrvJob*> rest;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        rest.swap(s->pending);
        s->fatal = st;
    }
    for (SrvJob* sj : rest) finish(s, sj, st);
}

void serve_loop(fsmmc_server* s)
{
    if (hipSetDevice(s->ctx->device) != hipSuccess) {
        fail_all(s, FSMMC_EDEVICE);
        return;
    }
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->running.empty() && s->admitted_q.empty())
                s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty(); });
            if (s->stop && s->pending.empty() && s->running.empty() && s->admitted_q.empty()) return;
        }
        // the rounds run on the device while new arrivals are initialised
        fsmmc_status st = batch_launch(&s->batch, s->batch.rps);
        if (st == FSMMC_OK) admit(s);
        RoundResult r;
        if (st == FSMMC_OK) st = batch_collect(&s->batch, &r);
        if (st == FSMMC_OK) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->rounds = s->batch.rounds;
            s->draws = s->batch.draws;
            s->gpu_ms = s->batch.gpu_ms;
        }
        if (st == FSMMC_OK) st = retire(s);
        if (st == FSMMC_OK) join(s);
        if (st != FSMMC_OK) {
            fail_all(s, st);
            return;
        }
    }
}

}  // namespace

extern "C" {

double fsmmc_clock(void) { return now_s(); }

fsmmc_status fsmmc_server_create(fsmmc_ctx* ctx, const fsmmc_server_config* cfg, fsmmc_server** out)
{
    if (!ctx || !out) return fail(FSMMC_EINVAL, "ctx or out is NULL");
    *out = nullptr;
    if (cfg && cfg->ess_window < 0) return fail(FSMMC_EINVAL, "ess_window must be >= 0");
    fsmmc_server* s = new fsmmc_server();
    s->ctx = ctx;
    if (cfg) s->cfg = *cfg;
    fsmmc_batch_tune bt = s->cfg.batch;
    bt.autotune = 0;
    fsmmc_status st = batch_setup(&s->batch, ctx, nullptr, &bt);
    hipError_t e = hipSuccess;
    if (st == FSMMC_OK) {
        e = hipStreamCreateWithFlags(&s->admit_stream, hipStreamNonBlocking);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamCreateWithFlags");
    }
    if (st != FSMMC_OK) {
        batch_teardown(&s->batch);
        delete s;
        return st;
    }
    s->thr = std::thread(serve_loop, s);
    *out = s;
    return FSMMC_OK;
}

fsmmc_status fsmmc_server_submit(fsmmc_server* s, const fsmmc_target_spec* target, const fsmmc_sampler_spec* sampler,
                                 int32_t n_chains, int32_t n_draws, uint64_t seed, const void* x0, void* out_samples,
                                 int32_t* out_counts, uint64_t* job_id)
{
    if (!s || !job_id) return fail(FSMMC_EINVAL, "server or job_id is NULL");
    if (!out_samples) return fail(FSMMC_EINVAL, "served jobs need out_samples");
    fsmmc_status st = validate_specs(target, sampler, n_chains, n_draws);
    if (st != FSMMC_OK) return st;
    if (sampler->dtype != FSMMC_F32) return fail(FSMMC_ENOTSUP, "served jobs are FP32");
    if (sampler->kind == FSMMC_NUTS && target->kind != FSMMC_LOGREG)
        return fail(FSMMC_ENOTSUP, "served NUTS jobs are LOGREG only");
    if (target->kind == FSMMC_GP_HYPER) return fail(FSMMC_ENOTSUP, "GP_HYPER jobs are not served");
    if (sampler->kind == FSMMC_DRSYM || sampler->kind == FSMMC_SLICE)
        return fail(FSMMC_ENOTSUP, "DRSYM and SLICE jobs are not served");
    SrvJob* sj = new SrvJob();
    sj->target = *target;
    sj->sampler = *sampler;
    sj->m = n_chains;
    sj->n = n_draws;
    sj->seed = seed;
    sj->x0 = x0;
    sj->out = out_samples;
    sj->counts = out_counts;
    sj->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->fatal != FSMMC_OK) {
            delete sj;
            return fail(s->fatal, "the server stopped after a device error");
        }
        if (s->stop) {
            delete sj;
            return fail(FSMMC_EBUSY, "the server is shutting down");
        }
        sj->id = s->next_id++;
        *job_id = sj->id;
        s->pending.push_back(sj);
        s->submitted++;
        s->outstanding++;
    }
    s->cv_work.notify_one();
    return FSMMC_OK;
}

fsmmc_status fsmmc_server_poll(fsmmc_server* s, fsmmc_server_done* out, int32_t cap, int32_t* n_out)
{
    if (!s || !n_out || (cap > 0 && !out)) return fail(FSMMC_EINVAL, "server, out or n_out is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    const int32_t k = (int32_t)std::min<size_t>(s->done.size(), (size_t)std::max(cap, 0));
    for (int32_t i = 0; i < k; ++i) out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n_out = k;
    return FSMMC_OK;
}

fsmmc_status fsmmc_server_wait(fsmmc_server* s, double timeout_s, int32_t* idle)
{
    if (!s) return fail(FSMMC_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto pred = [&] { return s->outstanding == 0; };
    if (timeout_s < 0)
        s->cv_idle.wait(lk, pred);
    else
        s->cv_idle.wait_for(lk, std::chrono::duration<double>(timeout_s), pred);
    if (idle) *idle = s->outstanding == 0 ? 1 : 0;
    return FSMMC_OK;
}

fsmmc_status fsmmc_server_stats(fsmmc_server* s, fsmmc_server_counters* out)
{
    if (!s || !out) return fail(FSMMC_EINVAL, "server or out is NULL");
    std::memset(out, 0, sizeof(*out));
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->admitted = s->admitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->rounds = s->rounds;
    out->draws = s->draws;
    out->live_jobs = s->live;
    out->pending_jobs = (int32_t)s->pending.size();
    out->peak_live_jobs = s->peak_live;
    out->peak_bytes = s->peak_bytes;
    out->gpu_ms = s->gpu_ms;
    return FSMMC_OK;
}

fsmmc_status fsmmc_server_destroy(fsmmc_server* s)
{
    if (!s) return fail(FSMMC_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->thr.joinable()) s->thr.join();
    batch_teardown(&s->batch);
    if (s->admit_stream) (void)hipStreamDestroy(s->admit_stream);
    delete s;
    return FSMMC_OK;
}

}  // extern "C"
