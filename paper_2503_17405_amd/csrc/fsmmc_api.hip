// fsmmc_api.hip -- the C ABI declared in include/fsmmc.h: contexts, jobs,
// the FSM runtime loop and the synchronized runtime loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fsmmc_host.h"

using namespace fsmmc;

namespace fsmmc {
namespace {
thread_local std::string g_err;

__global__ void fill_i64_kernel(int64_t* p, int64_t v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
// *done = 1 when every chain holds n draws, else 0 (one block).
__global__ void all_done_kernel(const uint32_t* t, int m, uint32_t n, int32_t* done)
{
    int ok = 1;
    for (int i = threadIdx.x; i < m; i += blockDim.x) ok &= t[i] >= n ? 1 : 0;
    ok = __syncthreads_and(ok);
    if (threadIdx.x == 0) *done = ok;
}

}  // namespace

fsmmc_status fail(fsmmc_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

fsmmc_status hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return FSMMC_EDEVICE;
}

hipError_t fill_i64(int64_t* p, int64_t v, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t fill_i32(int32_t* p, int32_t v, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

void harvest(fsmmc_job* j)
{
    for (const TimedLaunch& t : j->pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            j->kms[t.cls] += ms;
            j->klaunch[t.cls]++;
        }
        j->pool.push_back(t.a);
        j->pool.push_back(t.b);
    }
    j->pending.clear();
}

}  // namespace fsmmc

// Workspace of fsmmc_eval_potential_noalloc: the padded gradients and
// potentials of one call before they are packed into the caller's buffers.
// One copy per device, for the life of the process; every call on a device
// shares it.  Host code never uses this name as an address: the device
// address comes from hipGetSymbolAddress, once per device (scratch_setup).
static __device__ __align__(256) unsigned char scratch[FSMMC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// theta (n x D, row-major) into the request buffer (n x Dp), zero padding.
__global__ void pack_points_kernel(const float* theta, float* thq, int n, int D, int Dp)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)n * Dp) return;
    const int r = (int)(i / Dp), d = (int)(i % Dp);
    thq[i] = d < D ? theta[(size_t)r * D + d] : 0.0f;
}

// The first D of every Dp entries of g (n rows) into out (n x D); u into U.
__global__ void unpack_potential_kernel(const float* g, const float* u, float* out, float* U, int n, int D, int Dp)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (out && i < (size_t)n * D) {
        const int r = (int)(i / D), d = (int)(i % D);
        out[i] = g[(size_t)r * Dp + d];
    }
    if (i < (size_t)n) U[i] = u[i];
}
}  // namespace

// Device address of `scratch` on `device` (the current device), looked up
// once per device.
static fsmmc_status scratch_setup(int device, void** out)
{
    if (device < 0 || device >= kMaxDevices) return fail(FSMMC_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_dev[device] = p;
    }
    if (out) *out = g_scratch_dev[device];
    return FSMMC_OK;
}

static fsmmc_status job_alloc(fsmmc_job* j, size_t bytes, void** p)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    fsmmc_ctx* c = j->ctx;
    if (c->budget) {
        size_t now = c->used.fetch_add(bytes) + bytes;
        if (now > c->budget) {
            c->used.fetch_sub(bytes);
            return fail(FSMMC_EBUDGET, "job exceeds the context's HBM budget");
        }
    } else {
        c->used.fetch_add(bytes);
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        c->used.fetch_sub(bytes);
        *p = nullptr;
        return fail(FSMMC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    j->allocs.push_back(*p);
    j->bytes += bytes;
    e = hipMemsetAsync(*p, 0, bytes, j->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    return FSMMC_OK;
}

static void job_release(fsmmc_job* j)
{
    if (!j) return;
    if (j->stream) (void)hipStreamSynchronize(j->stream);
    for (void* p : j->allocs) (void)hipFree(p);
    if (j->h_ctr) (void)hipHostFree(j->h_ctr);
    for (const TimedLaunch& t : j->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (hipEvent_t e : j->pool) (void)hipEventDestroy(e);
    if (j->side) {
        (void)hipStreamSynchronize(j->side);
        (void)hipStreamDestroy(j->side);
    }
    if (j->ev_snap) (void)hipEventDestroy(j->ev_snap);
    if (j->ev_gemm) (void)hipEventDestroy(j->ev_gemm);
    if (j->ctx) {
        j->ctx->used.fetch_sub(j->bytes);
        j->ctx->jobs.fetch_sub(1);
    }
    delete j;
}

#define ALLOC(ptr, bytes)                                               \
    do {                                                                \
        void* p__ = nullptr;                                            \
        fsmmc_status s__ = job_alloc(job, (bytes), &p__);               \
        if (s__ != FSMMC_OK) {                                          \
            job_release(job);                                           \
            return s__;                                                 \
        }                                                               \
        ptr = reinterpret_cast<decltype(ptr)>(p__);                     \
    } while (0)

#define HIP_TRY_JOB(expr)                                               \
    do {                                                                \
        hipError_t e__ = (expr);                                        \
        if (e__ != hipSuccess) {                                        \
            fsmmc_status s__ = hip_fail(e__, #expr);                    \
            job_release(job);                                           \
            return s__;                                                 \
        }                                                               \
    } while (0)

extern "C" {

const char* fsmmc_last_error(void) { return g_err.c_str(); }

const char* fsmmc_version(void) { return "fsmmc 0.1 (gfx950)"; }

fsmmc_status fsmmc_ctx_create(int device, size_t hbm_budget_bytes, fsmmc_ctx** out)
{
    if (!out) return fail(FSMMC_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(FSMMC_EINVAL, "no such device");
    HIP_TRY(hipSetDevice(device));
    fsmmc_status ss = scratch_setup(device, nullptr);
    if (ss != FSMMC_OK) return ss;
    fsmmc_ctx* c = new fsmmc_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    *out = c;
    return FSMMC_OK;
}

fsmmc_status fsmmc_ctx_destroy(fsmmc_ctx* ctx)
{
    if (!ctx) return fail(FSMMC_EINVAL, "ctx is NULL");
    if (ctx->jobs.load() != 0) return fail(FSMMC_EBUSY, "context still has jobs");
    delete ctx;
    return FSMMC_OK;
}

size_t fsmmc_ctx_bytes_in_use(const fsmmc_ctx* ctx) { return ctx ? ctx->used.load() : 0; }

}  // extern "C"

fsmmc_status fsmmc::validate_specs(const fsmmc_target_spec* t, const fsmmc_sampler_spec* s, int32_t m,
                                   int32_t n)
{
    if (!t || !s) return fail(FSMMC_EINVAL, "target or sampler spec is NULL");
    if (m < 1) return fail(FSMMC_EINVAL, "n_chains must be >= 1");
    if (n < 1) return fail(FSMMC_EINVAL, "n_draws must be >= 1");
    if (t->dim < 1) return fail(FSMMC_EINVAL, "dim must be >= 1");
    if (t->kind != FSMMC_GP_HYPER && t->aux != 0) return fail(FSMMC_EINVAL, "aux must be 0 for this target");
    if (s->dtype != FSMMC_F32 && s->dtype != FSMMC_F64) return fail(FSMMC_EINVAL, "bad dtype");
    if ((int64_t)m * (int64_t)n > (int64_t)1 << 31) return fail(FSMMC_EINVAL, "n_chains * n_draws too large");
    if (s->kind == FSMMC_ESS && t->kind == FSMMC_GP_HYPER) {
        if (s->dtype != FSMMC_F64) return fail(FSMMC_ENOTSUP, "GP_HYPER runs in FP64");
        if (t->dim != 3) return fail(FSMMC_EINVAL, "GP_HYPER has dim 3 (tau, lambda, sigma)");
        if (!t->X || !t->y) return fail(FSMMC_EINVAL, "GP_HYPER needs X and y");
        if (t->n_data < 1 || t->n_data > gph_max_obs())
            return fail(FSMMC_ENOTSUP, "GP_HYPER needs 1 to 512 observations");
        if (t->aux < 1 || t->aux > gph_max_inputs()) return fail(FSMMC_EINVAL, "GP_HYPER input dimension must be in [1, 16]");
        if (!(t->noise_sd >= 0.0) || !std::isfinite(t->noise_sd)) return fail(FSMMC_EINVAL, "jitter must be >= 0");
        return FSMMC_OK;
    }
    if (s->kind == FSMMC_ESS) {
        if (t->kind != FSMMC_GP_GAUSS && t->kind != FSMMC_GP_LOGISTIC)
            return fail(FSMMC_EINVAL, "ESS needs a GP target");
        if (!t->chol_L || !t->y) return fail(FSMMC_EINVAL, "GP target needs chol_L and y");
        if (t->kind == FSMMC_GP_GAUSS && !(t->noise_sd > 0.0))
            return fail(FSMMC_EINVAL, "GP_GAUSS needs noise_sd > 0");
        if (!ess_supported_epl(t->dim, s->dtype))
            return fail(FSMMC_ENOTSUP, "dim too large for this dtype");
        return FSMMC_OK;
    }
    if (s->kind == FSMMC_NUTS) {
        if (t->kind != FSMMC_LOGREG && t->kind != FSMMC_MOG)
            return fail(FSMMC_ENOTSUP, "NUTS is built for LOGREG and MOG targets");
        if (s->dtype != FSMMC_F32) return fail(FSMMC_ENOTSUP, "NUTS is built for FP32");
        if (t->kind == FSMMC_LOGREG) {
            if (!t->X || !t->y) return fail(FSMMC_EINVAL, "LOGREG target needs X and y");
            if (t->n_data < 1) return fail(FSMMC_EINVAL, "n_data must be >= 1");
        } else {
            if (!t->X || !t->y || !t->prec) return fail(FSMMC_EINVAL, "MOG target needs means, log weights and prec");
            if (t->n_data < 1 || t->n_data > 8) return fail(FSMMC_EINVAL, "MOG needs 1 to 8 components");
        }
        if (t->dim > 128) return fail(FSMMC_ENOTSUP, "NUTS dim must be <= 128");
        if (s->max_depth < 1 || s->max_depth > 15) return fail(FSMMC_EINVAL, "max_depth must be in [1, 15]");
        if (!(s->step_size > 0.0) || !std::isfinite(s->step_size))
            return fail(FSMMC_EINVAL, "step_size must be > 0");
        return FSMMC_OK;
    }
    if (s->kind == FSMMC_SLICE) {
        if (t->kind != FSMMC_FUNNEL && t->kind != FSMMC_GAUSS_DIAG)
            return fail(FSMMC_ENOTSUP, "SLICE is built for FUNNEL and GAUSS_DIAG targets");
        if (s->dtype != FSMMC_F32) return fail(FSMMC_ENOTSUP, "SLICE is built for FP32");
        if (t->dim > dr_max_dim()) return fail(FSMMC_ENOTSUP, "SLICE dim must be <= 16");
        if (t->kind == FSMMC_FUNNEL && t->dim < 2) return fail(FSMMC_EINVAL, "FUNNEL needs dim >= 2");
        if (t->kind == FSMMC_GAUSS_DIAG && !t->prec) return fail(FSMMC_EINVAL, "GAUSS_DIAG needs prec");
        if (!(s->scales[0] > 0.0) || !std::isfinite(s->scales[0]))
            return fail(FSMMC_EINVAL, "stepping-out width must be > 0");
        return FSMMC_OK;
    }
    if (s->kind == FSMMC_DRSYM) {
        if (t->kind != FSMMC_FUNNEL && t->kind != FSMMC_GAUSS_DIAG)
            return fail(FSMMC_ENOTSUP, "DRSYM is built for FUNNEL and GAUSS_DIAG targets");
        if (s->dtype != FSMMC_F32) return fail(FSMMC_ENOTSUP, "DRSYM is built for FP32");
        if (t->dim > dr_max_dim()) return fail(FSMMC_ENOTSUP, "DRSYM dim must be <= 16");
        if (t->kind == FSMMC_FUNNEL && t->dim < 2) return fail(FSMMC_EINVAL, "FUNNEL needs dim >= 2");
        if (t->kind == FSMMC_GAUSS_DIAG && !t->prec) return fail(FSMMC_EINVAL, "GAUSS_DIAG needs prec");
        if (s->n_stages < 1 || s->n_stages > (1 << 20)) return fail(FSMMC_EINVAL, "n_stages (tries) must be in [1, 2^20]");
        if (!(s->scales[0] > 0.0) || !std::isfinite(s->scales[0]))
            return fail(FSMMC_EINVAL, "proposal scale must be > 0");
        return FSMMC_OK;
    }
    if (s->kind == FSMMC_DRMH) {
        if (t->kind != FSMMC_FUNNEL && t->kind != FSMMC_GAUSS_DIAG)
            return fail(FSMMC_ENOTSUP, "DRMH is built for FUNNEL and GAUSS_DIAG targets");
        if (s->dtype != FSMMC_F32) return fail(FSMMC_ENOTSUP, "DRMH is built for FP32");
        if (t->dim > dr_max_dim()) return fail(FSMMC_ENOTSUP, "DRMH dim must be <= 16");
        if (t->kind == FSMMC_FUNNEL && t->dim < 2) return fail(FSMMC_EINVAL, "FUNNEL needs dim >= 2");
        if (t->kind == FSMMC_GAUSS_DIAG && !t->prec) return fail(FSMMC_EINVAL, "GAUSS_DIAG needs prec");
        if (s->n_stages < 1 || s->n_stages > 3) return fail(FSMMC_EINVAL, "n_stages must be in [1, 3]");
        for (int i = 0; i < s->n_stages; ++i)
            if (!(s->scales[i] > 0.0) || !std::isfinite(s->scales[i]))
                return fail(FSMMC_EINVAL, "proposal scales must be > 0");
        return FSMMC_OK;
    }
    return fail(FSMMC_EINVAL, "unknown sampler kind");
}

// Copy a dim x dim matrix (device, row-major) into a zero-padded Dp x Dp
// lower-triangular device buffer (entries above the diagonal dropped).
extern "C" {

// The lower triangle of L, zero padded to Dp x Dp.  With `planes`, also its
// exact three-piece bf16 split (hi, mid, lo; the same truncations as the
// device's split of z) for the bf16 ellipse GEMM, packed per (row tile ti,
// chunk c <= ti, k-block kb, piece p) as 32 x 16 blocks [row][k].
static fsmmc_status stage_lower(fsmmc_job* job, const void* src, int D, int Dp, size_t es, void* dst,
                                void* planes)
{
    std::vector<unsigned char> h((size_t)D * D * es), p((size_t)Dp * Dp * es, 0);
    HIP_TRY(hipMemcpy(h.data(), src, h.size(), hipMemcpyDeviceToHost));
    for (int r = 0; r < D; ++r) std::memcpy(&p[(size_t)r * Dp * es], &h[(size_t)r * D * es], (size_t)(r + 1) * es);
    HIP_TRY(hipMemcpyAsync(dst, p.data(), p.size(), hipMemcpyHostToDevice, job->stream));
    std::vector<uint16_t> pl;
    if (planes) {
        pl.assign(ess_lower_pieces_halfwords(Dp), 0);
        const int nt = Dp / 32;
        size_t blk = 0;  // ((ti (ti + 1) / 2 + c) 2 + kb) 3 + piece
        for (int ti = 0; ti < nt; ++ti)
            for (int c = 0; c <= ti; ++c)
                for (int kb = 0; kb < 2; ++kb, blk += 3)
                    for (int r = 0; r < 32; ++r)
                        for (int kk = 0; kk < 16; ++kk) {
                            float x;
                            std::memcpy(&x, &p[((size_t)(32 * ti + r) * Dp + 32 * c + 16 * kb + kk) * 4], 4);
                            uint32_t u, v, w;
                            std::memcpy(&u, &x, 4);
                            const uint32_t uh = u & 0xFFFF0000u;
                            float fh, fm;
                            std::memcpy(&fh, &uh, 4);
                            const float r1 = x - fh;
                            std::memcpy(&v, &r1, 4);
                            const uint32_t um = v & 0xFFFF0000u;
                            std::memcpy(&fm, &um, 4);
                            const float r2 = r1 - fm;
                            std::memcpy(&w, &r2, 4);
                            const size_t at = 16 * r + kk;
                            pl[blk * 512 + at] = (uint16_t)(uh >> 16);
                            pl[(blk + 1) * 512 + at] = (uint16_t)(um >> 16);
                            pl[(blk + 2) * 512 + at] = (uint16_t)(w >> 16);
                        }
        HIP_TRY(hipMemcpyAsync(planes, pl.data(), pl.size() * 2, hipMemcpyHostToDevice, job->stream));
    }
    HIP_TRY(hipStreamSynchronize(job->stream));
    return FSMMC_OK;
}

fsmmc_status fsmmc_init_chains(fsmmc_ctx* ctx, const fsmmc_target_spec* target,
                               const fsmmc_sampler_spec* sampler, int32_t n_chains, int32_t n_draws,
                               uint64_t seed, const void* x0, void* out_samples, void* stream,
                               const fsmmc_tune* tune, fsmmc_job** out)
{
    if (!ctx) return fail(FSMMC_EINVAL, "ctx is NULL");
    if (!out) return fail(FSMMC_EINVAL, "out is NULL");
    *out = nullptr;
    fsmmc_status st = validate_specs(target, sampler, n_chains, n_draws);
    if (st != FSMMC_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device));

    fsmmc_job* job = new fsmmc_job();
    job->ctx = ctx;
    job->timing = tune && tune->timing;
    ctx->jobs.fetch_add(1);
    job->stream = (hipStream_t)stream;
    JobDev& d = job->d;
    d.kind = sampler->kind;
    d.target = target->kind;
    d.dtype = sampler->dtype;
    d.m = n_chains;
    d.n = n_draws;
    d.D = target->dim;
    d.seed = seed;
    d.noise_sd = target->noise_sd;
    d.step_size = sampler->step_size;
    d.max_depth = sampler->max_depth;
    d.n_stages = sampler->n_stages;
    for (int i = 0; i < 4; ++i) d.scales[i] = sampler->scales[i];
    const size_t es = d.dtype == FSMMC_F32 ? 4 : 8;
    const size_t m = (size_t)d.m;

    HIP_TRY_JOB(hipHostMalloc((void**)&job->h_ctr, 16 * sizeof(unsigned long long), hipHostMallocDefault));
    ALLOC(d.ctr, 8 * sizeof(unsigned long long));
    ALLOC(d.k, m * 4);
    ALLOC(d.t, m * 4);
    ALLOC(d.evals, m * 4);
    ALLOC(d.budget, m * 8);
    ALLOC(d.lx, m * es);
    ALLOC(d.counts, m * (size_t)d.n * 4);
    if (out_samples) {
        d.out = out_samples;
    } else {
        ALLOC(d.out, m * (size_t)d.n * (size_t)d.D * es);
    }
    d.tstop = (uint32_t)d.n;

    if (d.kind == FSMMC_ESS && d.target == FSMMC_GP_HYPER) {  // FP64 Cholesky by a wave (n <= 128) or a block
        d.Dp = d.D;
        d.N = target->n_data;
        d.pdim = target->aux;
        ALLOC(d.x, m * 3 * 8);
        ALLOC(d.V, m * 3 * 8);
        ALLOC(d.theta, m * 8);
        ALLOC(d.tmin, m * 8);
        ALLOC(d.tmax, m * 8);
        ALLOC(d.logu, m * 8);
        ALLOC(d.sink, m * 8);
        ALLOC(d.maxN, (size_t)d.n * 4);
        ALLOC(d.queue, 64);
        ALLOC(d.X, (size_t)d.N * d.pdim * 8);
        ALLOC(d.y, (size_t)d.N * 8);
        HIP_TRY_JOB(hipMemcpyAsync(d.X, target->X, (size_t)d.N * d.pdim * 8, hipMemcpyDeviceToDevice, job->stream));
        HIP_TRY_JOB(hipMemcpyAsync(d.y, target->y, (size_t)d.N * 8, hipMemcpyDeviceToDevice, job->stream));
        HIP_TRY_JOB(gph_setup(d));
        if (gph_slot_bytes(d)) ALLOC(d.gslot, gph_slot_bytes(d));
        HIP_TRY_JOB(gph_init_state(d, x0, job->stream));
        job->launches += x0 ? 2 : 1;
    } else if (d.kind == FSMMC_ESS) {
        d.EPL = ess_supported_epl(d.D, d.dtype);
        d.Dp = 64 * d.EPL;
        const size_t Dp = (size_t)d.Dp;
        ALLOC(d.x, m * Dp * es);
        ALLOC(d.theta, m * es);
        ALLOC(d.tmin, m * es);
        ALLOC(d.tmax, m * es);
        ALLOC(d.logu, m * es);
        ALLOC(d.sink, m * es);
        ALLOC(d.maxN, (size_t)d.n * 4);
        ALLOC(d.L, Dp * Dp * es);
        if (d.dtype == FSMMC_F32 && ess_gemm_rt(d.Dp) >= 2) ALLOC(d.Lp, ess_lower_pieces_halfwords(d.Dp) * sizeof(uint16_t));
        ALLOC(d.y, Dp * es);
        // ellipse window: about 1 GiB of directions, 4..256 draws, at most n
        int W = tune && tune->window > 0 ? tune->window : 0;
        if (!W) {
            const double per_draw = (double)m * (double)Dp * (double)es;
            W = 4;
            while (W < 256 && 2.0 * W * per_draw <= 1073741824.0) W *= 2;
        }
        d.W = std::max(1, std::min(W, d.n));
        while ((int64_t)d.W * d.m > (int64_t)1 << 30 && d.W > 1) d.W /= 2;
        d.Wcap = d.W;
        ALLOC(d.nu, 2 * m * (size_t)d.W * Dp * es);
        ALLOC(d.tsnap, m * 4);
        HIP_TRY_JOB(hipStreamCreateWithFlags(&job->side, hipStreamNonBlocking));
        HIP_TRY_JOB(hipEventCreateWithFlags(&job->ev_snap, hipEventDisableTiming));
        HIP_TRY_JOB(hipEventCreateWithFlags(&job->ev_gemm, hipEventDisableTiming));
        fsmmc_status s2 = stage_lower(job, target->chol_L, d.D, d.Dp, es, d.L, d.Lp);
        if (s2 != FSMMC_OK) {
            job_release(job);
            return s2;
        }
        HIP_TRY_JOB(hipMemcpyAsync(d.y, target->y, (size_t)d.D * es, hipMemcpyDeviceToDevice, job->stream));
        // k = S_1 (INIT), t = 0
        hipLaunchKernelGGL(fill_i32_kernel, dim3((d.m + 255) / 256), dim3(256), 0, job->stream, d.k, 1, d.m);
        HIP_TRY_JOB(hipGetLastError());
        if (x0)
            HIP_TRY_JOB(hipMemcpy2DAsync(d.x, Dp * es, x0, (size_t)d.D * es, (size_t)d.D * es, m,
                                         hipMemcpyDeviceToDevice, job->stream));
        HIP_TRY_JOB(ess_prior_draw(d, x0, job->stream));
        job->launches += x0 ? 2 : 3;
    } else if (d.kind == FSMMC_SLICE) {  // lane per chain, [d][chain] state
        d.Dp = d.D;
        // direction window: W draws per chain, at most 32 and 256 MiB
        d.W = std::max(1, std::min(32, d.n));
        while (d.W > 1 && (double)m * d.W * d.D * 4 > 268435456.0) d.W /= 2;
        ALLOC(d.nu, m * (size_t)d.W * d.D * 4);
        ALLOC(d.tsnap, m * 4);
        ALLOC(d.x, m * (size_t)d.D * 4);
        ALLOC(d.V, 2 * m * (size_t)d.D * 4);
        ALLOC(d.logu, m * 4);
        ALLOC(d.tmin, m * 4);
        ALLOC(d.tmax, m * 4);
        ALLOC(d.theta, m * 4);
        ALLOC(d.Wsum, m * 4);
        ALLOC(d.flags, m * 4);
        ALLOC(d.nn, m * 4);
        ALLOC(d.jd, m * 4);
        ALLOC(d.vdir, m * 4);
        ALLOC(d.maxN, 2 * (size_t)d.n * 4);
        ALLOC(d.sink, m * 4);
        ALLOC(d.prec, (size_t)d.D * 4);
        if (target->kind == FSMMC_GAUSS_DIAG)
            HIP_TRY_JOB(hipMemcpyAsync(d.prec, target->prec, (size_t)d.D * 4, hipMemcpyDeviceToDevice, job->stream));
        hipLaunchKernelGGL(fill_i32_kernel, dim3((d.m + 255) / 256), dim3(256), 0, job->stream, d.k, 1, d.m);
        HIP_TRY_JOB(hipGetLastError());
        HIP_TRY_JOB(sl_init_state(d, x0, job->stream));
        job->launches += x0 ? 3 : 2;
    } else if (d.kind == FSMMC_DRSYM) {  // lane per chain, [d][chain] state
        if (tune && tune->fsm_states != 0 && tune->fsm_states != 1 && tune->fsm_states != 4) {
            job_release(job);
            return fail(FSMMC_EINVAL, "fsm_states must be 0, 1 or 4");
        }
        d.fsm_states = tune && tune->fsm_states == 4 ? 4 : 1;
        d.Dp = d.D;
        ALLOC(d.x, m * (size_t)d.D * 4);
        ALLOC(d.V, 2 * m * (size_t)d.D * 4);
        ALLOC(d.H0, m * 4);
        ALLOC(d.Wsum, m * 4);
        ALLOC(d.flags, m * 4);
        ALLOC(d.maxN, (size_t)d.n * 4);
        ALLOC(d.sink, m * 4);
        ALLOC(d.prec, (size_t)d.D * 4);
        if (target->kind == FSMMC_GAUSS_DIAG)
            HIP_TRY_JOB(hipMemcpyAsync(d.prec, target->prec, (size_t)d.D * 4, hipMemcpyDeviceToDevice, job->stream));
        HIP_TRY_JOB(drs_init_state(d, x0, job->stream));
        job->launches += x0 ? 3 : 2;
    } else if (d.kind == FSMMC_DRMH) {  // lane per chain, [d][chain] state
        d.Dp = d.D;
        ALLOC(d.x, m * (size_t)d.D * 4);
        ALLOC(d.V, 2 * m * (size_t)d.D * 4);
        ALLOC(d.H0, m * 4);
        ALLOC(d.Wsum, m * 4);
        ALLOC(d.maxN, (size_t)d.n * 4);
        ALLOC(d.sink, m * 4);
        ALLOC(d.prec, (size_t)d.D * 4);
        if (target->kind == FSMMC_GAUSS_DIAG)
            HIP_TRY_JOB(hipMemcpyAsync(d.prec, target->prec, (size_t)d.D * 4, hipMemcpyDeviceToDevice, job->stream));
        hipLaunchKernelGGL(fill_i32_kernel, dim3((d.m + 255) / 256), dim3(256), 0, job->stream, d.k, 1, d.m);
        HIP_TRY_JOB(hipGetLastError());
        HIP_TRY_JOB(dr_init_state(d, x0, job->stream));
        job->launches += x0 ? 3 : 2;
    } else if (target->kind == FSMMC_MOG) {  // NUTS on a mixture: persistent kernel, inline gradient
        d.EPL = d.D <= 64 ? 1 : 2;
        d.Dp = 64 * d.EPL;
        const size_t Dp = (size_t)d.Dp;
        d.K = target->n_data;
        d.nvec = nuts_nvec(d.max_depth);
        ALLOC(d.jd, m * 4);
        ALLOC(d.vdir, m * 4);
        ALLOC(d.nn, m * 4);
        ALLOC(d.flags, m * 4);
        ALLOC(d.H0, m * 4);
        ALLOC(d.Wsum, m * 4);
        ALLOC(d.Wsub, m * 4);
        ALLOC(d.US, m * 4);
        ALLOC(d.acc, m * 4);
        ALLOC(d.V, m * (size_t)d.nvec * Dp * 4);
        ALLOC(d.Thq, m * Dp * 4);
        ALLOC(d.req, m * 4);
        ALLOC(d.wctr, 64);
        ALLOC(d.queue, 64);
        ALLOC(d.maxN, (size_t)d.n * 4);
        ALLOC(d.sink, m * 4);
        ALLOC(d.prec, Dp * Dp * 4);
        ALLOC(d.X, (size_t)d.K * d.D * 4);
        ALLOC(d.y, (size_t)d.K * 4);
        ALLOC(d.mogB, (size_t)d.K * Dp * 8);
        ALLOC(d.mogC, (size_t)d.K * 8);
        HIP_TRY_JOB(hipMemcpy2DAsync(d.prec, Dp * 4, target->prec, (size_t)d.D * 4, (size_t)d.D * 4, (size_t)d.D,
                                     hipMemcpyDeviceToDevice, job->stream));
        HIP_TRY_JOB(hipMemcpyAsync(d.X, target->X, (size_t)d.K * d.D * 4, hipMemcpyDeviceToDevice, job->stream));
        HIP_TRY_JOB(hipMemcpyAsync(d.y, target->y, (size_t)d.K * 4, hipMemcpyDeviceToDevice, job->stream));
        HIP_TRY_JOB(mog_setup(d, job->stream));
        hipLaunchKernelGGL(fill_i32_kernel, dim3((d.m + 255) / 256), dim3(256), 0, job->stream, d.k, 1, d.m);
        HIP_TRY_JOB(hipGetLastError());
        HIP_TRY_JOB(mog_init_state(d, x0, job->stream));
        job->launches += x0 ? 3 : 4;
    } else {  // NUTS on logistic regression
        d.EPL = d.D <= 64 ? 1 : 2;
        d.Dp = 64 * d.EPL;
        const size_t Dp = (size_t)d.Dp;
        d.N = target->n_data;
        // Row slices of the gradient: about 256 (128-chain tile, slice) blocks at
        // full load -- one round of the blocks the chip holds at once (one per
        // CU) -- with slices of up to 1280 rows, a multiple of the 32-row chunk
        // (N = 10^4: at 4096 chains 8 slices of 1280 rows run the NUTS job 7%
        // faster than 16 of 640; at 8192 chains 4 slices of 2528 rows match 8
        // of 1280 in the FSM runtime but slow the compacted baseline's partial
        // steps by 40%, so the cap stays at 1280).  Slices go below 256 rows only while
        // the partial sums the transition adds stay within 2^20 floats per step:
        // a job of few chains then spreads its rows over many blocks instead of
        // walking them chunk after chunk in a handful (16 chains, N = 1000: 32
        // blocks of one chunk instead of 4 of eight).
        {
            const int tiles = (m + 127) / 128;
            const int want = std::max(1, (256 + tiles - 1) / tiles);
            const int rows = ((d.N + want - 1) / want + 31) / 32 * 32;
            const int cap = std::max(1, (1 << 20) / ((int)m * (int)Dp));
            const int rows_min = std::min(256, std::max(32, ((d.N + cap - 1) / cap + 31) / 32 * 32));
            d.slice_rows = std::min(1280, std::max(rows_min, rows));
        }
        d.nslices = (d.N + d.slice_rows - 1) / d.slice_rows;
        d.Np = d.nslices * d.slice_rows;
        d.nvec = nuts_nvec(d.max_depth);
        ALLOC(d.jd, m * 4);
        ALLOC(d.vdir, m * 4);
        ALLOC(d.nn, m * 4);
        ALLOC(d.flags, m * 4);
        ALLOC(d.H0, m * 4);
        ALLOC(d.Wsum, m * 4);
        ALLOC(d.Wsub, m * 4);
        ALLOC(d.US, m * 4);
        ALLOC(d.acc, m * 4);
        ALLOC(d.V, m * (size_t)d.nvec * Dp * 4);
        ALLOC(d.Thq, m * Dp * 4);
        ALLOC(d.req, m * 4);
        ALLOC(d.list, m * 4);
        ALLOC(d.count, 64);
        ALLOC(d.Gpart, (size_t)d.nslices * m * Dp * 4);
        ALLOC(d.Upart, (size_t)d.nslices * m * 4);
        ALLOC(d.wctr, 64);
        ALLOC(d.X, (size_t)d.Np * Dp * 4);
        ALLOC(d.Xb, logreg_split_bytes(d));
        ALLOC(d.y, (size_t)d.Np * 4);
        HIP_TRY_JOB(hipMemcpy2DAsync(d.X, Dp * 4, target->X, (size_t)d.D * 4, (size_t)d.D * 4, (size_t)d.N,
                                     hipMemcpyDeviceToDevice, job->stream));
        HIP_TRY_JOB(hipMemcpyAsync(d.y, target->y, (size_t)d.N * 4, hipMemcpyDeviceToDevice, job->stream));
        HIP_TRY_JOB(logreg_setup(d, job->stream));
        hipLaunchKernelGGL(fill_i32_kernel, dim3((d.m + 255) / 256), dim3(256), 0, job->stream, d.k, 1, d.m);
        HIP_TRY_JOB(hipGetLastError());
        HIP_TRY_JOB(nuts_init_state(d, x0, job->stream));
        job->launches += 3;
    }
    *out = job;
    return FSMMC_OK;
}

static fsmmc_status read_ctr(fsmmc_job* job)
{
    HIP_TRY(hipMemcpyAsync(job->h_ctr, job->d.ctr, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           job->stream));
    HIP_TRY(hipStreamSynchronize(job->stream));
    harvest(job);
    return FSMMC_OK;
}

static fsmmc_status progress(fsmmc_job* job, std::vector<uint32_t>& t, std::vector<int32_t>* k)
{
    t.resize(job->d.m);
    HIP_TRY(hipMemcpyAsync(t.data(), job->d.t, t.size() * 4, hipMemcpyDeviceToHost, job->stream));
    if (k) {
        k->resize(job->d.m);
        HIP_TRY(hipMemcpyAsync(k->data(), job->d.k, k->size() * 4, hipMemcpyDeviceToHost, job->stream));
    }
    HIP_TRY(hipStreamSynchronize(job->stream));
    return FSMMC_OK;
}

// NUTS runtime: steps of {transition, compaction, gradient, reduce}, issued in
// batches; after each batch the host reads how many chains are still alive
// and how many asked for a gradient in the last step.
static fsmmc_status nuts_run(fsmmc_job* job, int mode, int64_t max_steps, uint32_t tstop, int32_t* all_done)
{
    JobDev& d = job->d;
    d.tstop = tstop;
    const int64_t b = max_steps > 0 ? max_steps : INT64_MAX;
    hipLaunchKernelGGL(fill_i64_kernel, dim3((d.m + 255) / 256), dim3(256), 0, job->stream, d.budget, b, d.m);
    HIP_TRY(hipGetLastError());
    job->launches++;
    const int batch = 16;
    uint32_t* h = reinterpret_cast<uint32_t*>(job->h_ctr + 8);
    uint32_t alive = 1;
    for (;;) {
        for (int i = 0; i < batch; ++i) {
            const uint32_t s = job->step;
            HIP_TRY(launch(job, mode == 0 ? KC_FSM : KC_SYNC, [&] { return nuts_transition(d, mode, s, job->stream); }));
            HIP_TRY(launch(job, KC_G, [&] { return nuts_gradient(d, job->stream); }));
            job->step++;
        }
        HIP_TRY(hipMemcpyAsync(h, d.wctr, 6 * 4, hipMemcpyDeviceToHost, job->stream));
        HIP_TRY(hipMemcpyAsync(h + 6, d.count, 4, hipMemcpyDeviceToHost, job->stream));
        HIP_TRY(hipStreamSynchronize(job->stream));
        harvest(job);
        const uint32_t reqs = h[6];
        if (mode == 0) {
            // FSM: a chain short of tstop requests a gradient every step unless its
            // budget is spent, so no request means every chain is done or out of budget
            if (reqs == 0) break;
            continue;
        }
        alive = h[3 + (job->step - 1) % 3];
        if (alive == 0) break;
    }
    if (all_done) {
        std::vector<uint32_t> t(d.m);
        HIP_TRY(hipMemcpy(t.data(), d.t, t.size() * 4, hipMemcpyDeviceToHost));
        int done = 1;
        for (uint32_t v : t) done &= v >= (uint32_t)d.n;
        *all_done = done;
    }
    return FSMMC_OK;
}

// NUTS on a mixture.  FSM: one launch of the persistent kernel; every chain
// runs to tstop or through max_steps gradient evaluations.  Synchronized:
// one launch per draw (and in vmap mode one padding launch per draw).
static fsmmc_status mog_fsm(fsmmc_job* job, int64_t max_steps, int32_t* all_done)
{
    JobDev& d = job->d;
    d.tstop = (uint32_t)d.n;
    const int64_t b = max_steps > 0 ? max_steps : INT64_MAX;
    HIP_TRY(fill_i64(d.budget, b, d.m, job->stream));
    job->launches++;
    HIP_TRY(launch(job, KC_FSM, [&] { return mog_run(d, 0, 0, &job->qticket, job->stream); }));
    std::vector<uint32_t> t;
    fsmmc_status s = progress(job, t, nullptr);
    if (s != FSMMC_OK) return s;
    harvest(job);
    if (all_done) {
        int done = 1;
        for (uint32_t v : t) done &= v >= (uint32_t)d.n;
        *all_done = done;
    }
    return FSMMC_OK;
}

static fsmmc_status mog_sync(fsmmc_job* job, int mode, uint32_t t0, uint32_t t1, int32_t* all_done)
{
    JobDev& d = job->d;
    HIP_TRY(fill_i64(d.budget, INT64_MAX, d.m, job->stream));
    job->launches++;
    for (uint32_t dr = t0; dr < t1; ++dr) {
        HIP_TRY(launch(job, KC_SYNC, [&] { return mog_run(d, 1, dr, &job->qticket, job->stream); }));
        if (mode == FSMMC_SYNC_VMAP)
            HIP_TRY(launch(job, KC_PAD, [&] { return mog_pad(d, dr, &job->qticket, job->stream); }));
    }
    std::vector<uint32_t> t;
    fsmmc_status s = progress(job, t, nullptr);
    if (s != FSMMC_OK) return s;
    harvest(job);
    for (uint32_t v : t)
        if (v != t1) return fail(FSMMC_EDEVICE, "synchronized NUTS: a chain did not complete its draw");
    if (all_done) *all_done = t1 >= (uint32_t)d.n ? 1 : 0;
    return FSMMC_OK;
}

// ESS on GP hyperparameters: FSM = one persistent launch; synchronized = one
// launch per draw (plus the vmap padding launch).
static fsmmc_status gph_fsm(fsmmc_job* job, int64_t max_steps, int32_t* all_done)
{
    JobDev& d = job->d;
    d.tstop = (uint32_t)d.n;
    HIP_TRY(fill_i64(d.budget, max_steps > 0 ? max_steps : INT64_MAX, d.m, job->stream));
    job->launches++;
    HIP_TRY(launch(job, KC_FSM, [&] { return gph_run(d, 0, 0, &job->qticket, job->stream); }));
    std::vector<uint32_t> t;
    fsmmc_status s = progress(job, t, nullptr);
    if (s != FSMMC_OK) return s;
    harvest(job);
    if (all_done) {
        int done = 1;
        for (uint32_t v : t) done &= v >= (uint32_t)d.n;
        *all_done = done;
    }
    return FSMMC_OK;
}

static fsmmc_status gph_sync(fsmmc_job* job, int mode, uint32_t t0, uint32_t t1, int32_t* all_done)
{
    JobDev& d = job->d;
    HIP_TRY(fill_i64(d.budget, INT64_MAX, d.m, job->stream));
    job->launches++;
    for (uint32_t dr = t0; dr < t1; ++dr) {
        HIP_TRY(launch(job, KC_SYNC, [&] { return gph_run(d, 1, dr, &job->qticket, job->stream); }));
        if (mode == FSMMC_SYNC_VMAP)
            HIP_TRY(launch(job, KC_PAD, [&] { return gph_run(d, 2, dr, &job->qticket, job->stream); }));
    }
    std::vector<uint32_t> t;
    fsmmc_status s = progress(job, t, nullptr);
    if (s != FSMMC_OK) return s;
    harvest(job);
    for (uint32_t v : t)
        if (v != t1) return fail(FSMMC_EDEVICE, "synchronized ESS: a chain did not complete its draw");
    if (all_done) *all_done = t1 >= (uint32_t)d.n ? 1 : 0;
    return FSMMC_OK;
}

// ESS windows [t0 + kW, t0 + (k+1)W): while window k is stepped on the job's
// stream, the ellipse GEMM of window k+1 runs on the side stream from a
// snapshot of the draw counters taken at the start of window k (every chain
// either completes window k or reaches n, so window k+1 starts at the
// snapshot + W).  Directions are double-buffered.  mode < 0: FSM runtime;
// otherwise synchronized (FSMMC_SYNC_VMAP / COMPACT) from draw t0 to t1.
static fsmmc_status ess_windows(fsmmc_job* job, int mode, uint32_t t0, uint32_t t1, int K)
{
    JobDev& d = job->d;
    hipStream_t s = job->stream;
    d.nu_cur = 0;
    HIP_TRY(launch(job, KC_G, [&] { return ess_fill_window(d, s); }));
    for (int k = 0; k < K; ++k) {
        const bool next = k + 1 < K;
        if (next) {
            HIP_TRY(copy_u32(d.tsnap, d.t, d.m, s));
            HIP_TRY(hipEventRecord(job->ev_snap, s));
            HIP_TRY(hipStreamWaitEvent(job->side, job->ev_snap, 0));
            const int nb = (k + 1) & 1;
            HIP_TRY(launch_on(job, job->side, KC_G, [&] { return ess_fill_next_window(d, nb, job->side); }));
            HIP_TRY(hipEventRecord(job->ev_gemm, job->side));
        }
        d.nu_cur = k & 1;
        if (mode < 0) {
            HIP_TRY(hipMemsetAsync(d.ctr + 3, 0, 2 * sizeof(unsigned long long), s));
            HIP_TRY(launch(job, KC_FSM, [&] { return ess_fsm_round(d, s); }));
        } else {
            const uint32_t w0 = t0 + (uint32_t)k * (uint32_t)d.W;
            const uint32_t w1 = std::min(t1, w0 + (uint32_t)d.W);
            for (uint32_t dr = w0; dr < w1; ++dr) {
                HIP_TRY(launch(job, KC_SYNC, [&] { return ess_sync_draw(d, dr, dr - w0, s); }));
                if (mode == FSMMC_SYNC_VMAP)
                    HIP_TRY(launch(job, KC_PAD, [&] { return ess_pad_draw(d, dr, dr - w0, s); }));
            }
        }
        if (next) HIP_TRY(hipStreamWaitEvent(s, job->ev_gemm, 0));
    }
    d.nu_cur = 0;
    return FSMMC_OK;
}

fsmmc_status fsmmc_step_fsm(fsmmc_job* job, int64_t max_steps, int32_t* all_done)
{
    if (!job) return fail(FSMMC_EINVAL, "job is NULL");
    if (job->batch) return fail(FSMMC_EBUSY, "job is stepped by a batch or server");
    JobDev& d = job->d;
    HIP_TRY(hipSetDevice(job->ctx->device));
    if (d.kind == FSMMC_NUTS && d.target == FSMMC_MOG) return mog_fsm(job, max_steps, all_done);
    if (d.kind == FSMMC_ESS && d.target == FSMMC_GP_HYPER) return gph_fsm(job, max_steps, all_done);
    if (d.kind == FSMMC_NUTS) return nuts_run(job, 0, max_steps, (uint32_t)d.n, all_done);
    if (d.kind == FSMMC_SLICE) {  // window by window: directions, then the FSM kernel
        d.tstop = (uint32_t)d.n;
        HIP_TRY(fill_i64(d.budget, max_steps > 0 ? max_steps : INT64_MAX, d.m, job->stream));
        job->launches++;
        for (;;) {
            HIP_TRY(hipMemsetAsync(d.ctr + 3, 0, 2 * sizeof(unsigned long long), job->stream));
            HIP_TRY(launch(job, KC_G, [&] { return sl_dir_window(d, job->stream); }));
            HIP_TRY(launch(job, KC_FSM, [&] { return sl_fsm_round(d, job->stream); }));
            fsmmc_status s = read_ctr(job);
            if (s != FSMMC_OK) return s;
            if (job->h_ctr[3] == 0) break;  // no chain short of n with budget left
        }
        if (all_done) *all_done = job->h_ctr[4] == 0 ? 1 : 0;
        return FSMMC_OK;
    }
    if (d.kind == FSMMC_DRSYM) {
        d.tstop = (uint32_t)d.n;
        const int64_t b = max_steps > 0 ? max_steps : INT64_MAX;
        HIP_TRY(fill_i64(d.budget, b, d.m, job->stream));
        job->launches++;
        HIP_TRY(hipMemsetAsync(d.ctr + 3, 0, 2 * sizeof(unsigned long long), job->stream));
        HIP_TRY(launch(job, KC_FSM, [&] { return drs_fsm_round(d, job->stream); }));
        fsmmc_status s = read_ctr(job);
        if (s != FSMMC_OK) return s;
        if (all_done) *all_done = job->h_ctr[4] == 0 ? 1 : 0;
        return FSMMC_OK;
    }
    if (d.kind == FSMMC_DRMH) {
        // one persistent launch: every lane runs its chain to n draws or to its budget
        d.tstop = (uint32_t)d.n;
        const int64_t b = max_steps > 0 ? max_steps : INT64_MAX;
        hipLaunchKernelGGL(fill_i64_kernel, dim3((d.m + 255) / 256), dim3(256), 0, job->stream, d.budget, b, d.m);
        HIP_TRY(hipGetLastError());
        job->launches++;
        HIP_TRY(hipMemsetAsync(d.ctr + 3, 0, 2 * sizeof(unsigned long long), job->stream));
        HIP_TRY(launch(job, KC_FSM, [&] { return dr_fsm_round(d, job->stream); }));
        fsmmc_status s = read_ctr(job);
        if (s != FSMMC_OK) return s;
        if (all_done) *all_done = job->h_ctr[4] == 0 ? 1 : 0;
        return FSMMC_OK;
    }
    const int64_t b = max_steps > 0 ? max_steps : INT64_MAX;
    HIP_TRY(fill_i64(d.budget, b, d.m, job->stream));
    job->launches++;
    if (max_steps <= 0) {
        // every chain runs to n: the number of windows is known up front
        std::vector<uint32_t> t;
        fsmmc_status s = progress(job, t, nullptr);
        if (s != FSMMC_OK) return s;
        uint32_t rem = 0;
        for (uint32_t v : t) rem = std::max(rem, (uint32_t)d.n - std::min(v, (uint32_t)d.n));
        const int K = (int)((rem + (uint32_t)d.W - 1) / (uint32_t)d.W);
        if (K > 0) {
            s = ess_windows(job, -1, 0, 0, K);
            if (s != FSMMC_OK) return s;
        }
        s = read_ctr(job);
        if (s != FSMMC_OK) return s;
        if (all_done) *all_done = (K == 0 || job->h_ctr[4] == 0) ? 1 : 0;
        return FSMMC_OK;
    }
    unsigned long long active = 1;
    for (;;) {
        HIP_TRY(hipMemsetAsync(d.ctr + 3, 0, 2 * sizeof(unsigned long long), job->stream));
        HIP_TRY(launch(job, KC_G, [&] { return ess_fill_window(d, job->stream); }));
        HIP_TRY(launch(job, KC_FSM, [&] { return ess_fsm_round(d, job->stream); }));
        fsmmc_status s = read_ctr(job);
        if (s != FSMMC_OK) return s;
        active = job->h_ctr[4];
        if (active == 0 || job->h_ctr[3] == 0) break;
    }
    if (all_done) *all_done = active == 0 ? 1 : 0;
    return FSMMC_OK;
}

// The FSM runtime without host reads: every round a chain runs to the end of
// its window (W draws) or of its budget, so ceil((n - t_lo) / W) rounds take
// every chain to n or to the end of its budget; rounds past that find no
// chain to step (their kernels return at once).  NUTS: a live chain with
// budget asks for one gradient per runtime step, so max_steps + 1 steps (the
// last one consumes the last gradient) leave it where fsmmc_step_fsm would.
fsmmc_status fsmmc_step_fsm_async(fsmmc_job* job, int64_t max_steps, int32_t* done)
{
    if (!job) return fail(FSMMC_EINVAL, "job is NULL");
    if (job->batch) return fail(FSMMC_EBUSY, "job is stepped by a batch or server");
    if (!done) return fail(FSMMC_EINVAL, "done is NULL");
    JobDev& d = job->d;
    HIP_TRY(hipSetDevice(job->ctx->device));
    hipPointerAttribute_t pa{};
    if (hipPointerGetAttributes(&pa, done) != hipSuccess ||
        (pa.type != hipMemoryTypeDevice && pa.type != hipMemoryTypeHost && pa.type != hipMemoryTypeManaged) ||
        !pa.devicePointer) {
        (void)hipGetLastError();
        return fail(FSMMC_EINVAL, "done must be device memory or pinned (hipHostMalloc) host memory");
    }
    const bool nuts_lr = d.kind == FSMMC_NUTS && d.target == FSMMC_LOGREG;
    if (nuts_lr && max_steps <= 0)
        return fail(FSMMC_EINVAL, "asynchronous NUTS on logistic regression needs max_steps > 0 (its length is "
                                  "not known ahead)");
    hipStream_t s = job->stream;
    const uint32_t n = (uint32_t)d.n;
    const int64_t b = max_steps > 0 ? max_steps : INT64_MAX;
    const int K = (int)((n - std::min(job->t_lo, n) + (uint32_t)d.W - 1) / (uint32_t)std::max(1, d.W));
    d.tstop = n;
    HIP_TRY(fill_i64(d.budget, b, d.m, s));
    job->launches++;
    if (nuts_lr) {
        for (int64_t i = 0; i <= max_steps; ++i) {
            const uint32_t st = job->step;
            HIP_TRY(launch(job, KC_FSM, [&] { return nuts_transition(d, 0, st, s); }));
            HIP_TRY(launch(job, KC_G, [&] { return nuts_gradient(d, s); }));
            job->step++;
        }
    } else if (d.kind == FSMMC_NUTS) {  // mixture: one persistent launch
        HIP_TRY(launch(job, KC_FSM, [&] { return mog_run(d, 0, 0, &job->qticket, s); }));
    } else if (d.kind == FSMMC_ESS && d.target == FSMMC_GP_HYPER) {
        HIP_TRY(launch(job, KC_FSM, [&] { return gph_run(d, 0, 0, &job->qticket, s); }));
    } else if (d.kind == FSMMC_DRSYM) {
        HIP_TRY(hipMemsetAsync(d.ctr + 3, 0, 2 * sizeof(unsigned long long), s));
        HIP_TRY(launch(job, KC_FSM, [&] { return drs_fsm_round(d, s); }));
    } else if (d.kind == FSMMC_DRMH) {
        HIP_TRY(hipMemsetAsync(d.ctr + 3, 0, 2 * sizeof(unsigned long long), s));
        HIP_TRY(launch(job, KC_FSM, [&] { return dr_fsm_round(d, s); }));
    } else if (d.kind == FSMMC_SLICE) {
        for (int k = 0; k < K; ++k) {
            HIP_TRY(hipMemsetAsync(d.ctr + 3, 0, 2 * sizeof(unsigned long long), s));
            HIP_TRY(launch(job, KC_G, [&] { return sl_dir_window(d, s); }));
            HIP_TRY(launch(job, KC_FSM, [&] { return sl_fsm_round(d, s); }));
        }
    } else if (max_steps <= 0) {  // ESS, every chain to n: pipelined windows
        if (K > 0) {
            fsmmc_status st = ess_windows(job, -1, 0, 0, K);
            if (st != FSMMC_OK) return st;
        }
    } else {  // ESS with a budget: windows one after another
        for (int k = 0; k < K; ++k) {
            HIP_TRY(hipMemsetAsync(d.ctr + 3, 0, 2 * sizeof(unsigned long long), s));
            HIP_TRY(launch(job, KC_G, [&] { return ess_fill_window(d, s); }));
            HIP_TRY(launch(job, KC_FSM, [&] { return ess_fsm_round(d, s); }));
        }
    }
    hipLaunchKernelGGL(all_done_kernel, dim3(1), dim3(256), 0, s, (const uint32_t*)d.t, d.m, n,
                       (int32_t*)pa.devicePointer);
    HIP_TRY(hipGetLastError());
    if (max_steps <= 0) job->t_lo = n;
    return FSMMC_OK;
}

fsmmc_status fsmmc_step_synchronized(fsmmc_job* job, int32_t n_draws, int32_t mode, int32_t* all_done)
{
    if (!job) return fail(FSMMC_EINVAL, "job is NULL");
    if (job->batch) return fail(FSMMC_EBUSY, "job is stepped by a batch or server");
    if (mode != FSMMC_SYNC_VMAP && mode != FSMMC_SYNC_COMPACT) return fail(FSMMC_EINVAL, "bad mode");
    JobDev& d = job->d;
    HIP_TRY(hipSetDevice(job->ctx->device));
    std::vector<uint32_t> t;
    std::vector<int32_t> k;
    fsmmc_status s = progress(job, t, &k);
    if (s != FSMMC_OK) return s;
    if (d.kind == FSMMC_DRMH) {  // the stage counter marks a draw in progress
        HIP_TRY(hipMemcpy(k.data(), d.evals, k.size() * 4, hipMemcpyDeviceToHost));
        for (int32_t& v : k) v = v == 0 ? 1 : 0;
    }
    if (d.kind == FSMMC_DRSYM) {  // no try made and no split sub-state pending
        std::vector<int32_t> e(k.size());
        HIP_TRY(hipMemcpy(e.data(), d.evals, e.size() * 4, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < k.size(); ++i) k[i] = (e[i] == 0 && k[i] == 0) ? 1 : 0;
    }
    const uint32_t t0 = t[0];
    for (int i = 0; i < d.m; ++i)
        if (t[i] != t0 || k[i] != 1)
            return fail(FSMMC_EINVAL, "chains are not synchronized at a draw boundary");
    const uint32_t t1 = std::min<uint32_t>((uint32_t)d.n, t0 + (uint32_t)std::max(n_draws, 0));
    if (d.kind == FSMMC_NUTS) {
        if (t1 == t0) {
            if (all_done) *all_done = t1 >= (uint32_t)d.n ? 1 : 0;
            return FSMMC_OK;
        }
        if (d.target == FSMMC_MOG) return mog_sync(job, mode, t0, t1, all_done);
        return nuts_run(job, mode == FSMMC_SYNC_VMAP ? 1 : 2, 0, t1, all_done);
    }
    if (d.kind == FSMMC_ESS && d.target == FSMMC_GP_HYPER) {
        if (t1 == t0) {
            if (all_done) *all_done = t1 >= (uint32_t)d.n ? 1 : 0;
            return FSMMC_OK;
        }
        return gph_sync(job, mode, t0, t1, all_done);
    }
    if (d.kind == FSMMC_DRSYM || d.kind == FSMMC_SLICE) {
        const bool sl = d.kind == FSMMC_SLICE;
        for (uint32_t dr = t0; dr < t1; ++dr) {
            if (sl && (dr - t0) % (uint32_t)d.W == 0)
                HIP_TRY(launch(job, KC_G, [&] { return sl_dir_window(d, job->stream); }));
            HIP_TRY(launch(job, KC_SYNC, [&] {
                return sl ? sl_sync_draw(d, dr, job->stream) : drs_sync_draw(d, dr, job->stream);
            }));
            if (mode == FSMMC_SYNC_VMAP)
                HIP_TRY(launch(job, KC_PAD, [&] {
                    return sl ? sl_pad_draw(d, dr, job->stream) : drs_pad_draw(d, dr, job->stream);
                }));
        }
        HIP_TRY(hipStreamSynchronize(job->stream));
        harvest(job);
        if (all_done) *all_done = t1 >= (uint32_t)d.n ? 1 : 0;
        return FSMMC_OK;
    }
    if (d.kind == FSMMC_DRMH) {
        for (uint32_t dr = t0; dr < t1; ++dr) {
            HIP_TRY(launch(job, KC_SYNC, [&] { return dr_sync_draw(d, dr, job->stream); }));
            if (mode == FSMMC_SYNC_VMAP)
                HIP_TRY(launch(job, KC_PAD, [&] { return dr_pad_draw(d, dr, job->stream); }));
        }
        HIP_TRY(hipStreamSynchronize(job->stream));
        harvest(job);
        if (all_done) *all_done = t1 >= (uint32_t)d.n ? 1 : 0;
        return FSMMC_OK;
    }
    if (t1 > t0) {
        const int K = (int)((t1 - t0 + (uint32_t)d.W - 1) / (uint32_t)d.W);
        fsmmc_status s2 = ess_windows(job, mode, t0, t1, K);
        if (s2 != FSMMC_OK) return s2;
    }
    HIP_TRY(hipStreamSynchronize(job->stream));
    harvest(job);
    if (all_done) *all_done = t1 >= (uint32_t)d.n ? 1 : 0;
    return FSMMC_OK;
}

fsmmc_status fsmmc_collect_samples(fsmmc_job* job, int32_t b, int32_t e, void* dst, int32_t dst_is_host)
{
    if (!job || !dst) return fail(FSMMC_EINVAL, "job or dst is NULL");
    JobDev& d = job->d;
    if (b < 0 || e > d.n || b >= e) return fail(FSMMC_EINVAL, "bad draw range");
    std::vector<uint32_t> t;
    fsmmc_status s = progress(job, t, nullptr);
    if (s != FSMMC_OK) return s;
    for (uint32_t v : t)
        if (v < (uint32_t)e) return fail(FSMMC_ENOTDONE, "draws not produced yet");
    const size_t es = d.dtype == FSMMC_F32 ? 4 : 8;
    const size_t row = (size_t)d.D * es;
    HIP_TRY(hipMemcpy2DAsync(dst, (size_t)(e - b) * row, (const char*)d.out + (size_t)b * row, (size_t)d.n * row,
                             (size_t)(e - b) * row, (size_t)d.m,
                             dst_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, job->stream));
    HIP_TRY(hipStreamSynchronize(job->stream));
    return FSMMC_OK;
}

fsmmc_status fsmmc_collect_counts(fsmmc_job* job, int32_t* dst)
{
    if (!job || !dst) return fail(FSMMC_EINVAL, "job or dst is NULL");
    HIP_TRY(hipMemcpyAsync(dst, job->d.counts, (size_t)job->d.m * job->d.n * 4, hipMemcpyDeviceToHost,
                           job->stream));
    HIP_TRY(hipStreamSynchronize(job->stream));
    return FSMMC_OK;
}

fsmmc_status fsmmc_eval_potential(fsmmc_job* job, int32_t n_points, const void* theta, void* grad, void* U)
{
    if (!job || !theta || !U) return fail(FSMMC_EINVAL, "job, theta or U is NULL");
    if (job->batch) return fail(FSMMC_EBUSY, "job is stepped by a batch or server");
    JobDev& d = job->d;
    if (d.kind != FSMMC_NUTS) return fail(FSMMC_ENOTSUP, "only NUTS jobs evaluate a potential");
    if (n_points < 1 || n_points > d.m) return fail(FSMMC_EINVAL, "n_points must be in [1, n_chains]");
    HIP_TRY(hipSetDevice(job->ctx->device));
    if (d.target == FSMMC_MOG) {
        HIP_TRY(mog_eval(d, n_points, (const float*)theta, (float*)grad, (float*)U, job->stream));
        HIP_TRY(hipStreamSynchronize(job->stream));
        return FSMMC_OK;
    }
    // The positions go through the request buffer, which only the gradient
    // kernels read; results land in temporary buffers so the gradients of
    // chains with a leapfrog in flight are kept.
    void *tg = nullptr, *tu = nullptr;
    HIP_TRY(hipMalloc(&tg, (size_t)n_points * d.Dp * 4));
    hipError_t e = hipMalloc(&tu, (size_t)n_points * 4);
    if (e == hipSuccess) e = hipMemsetAsync(d.Thq, 0, (size_t)d.m * d.Dp * 4, job->stream);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(d.Thq, (size_t)d.Dp * 4, theta, (size_t)d.D * 4, (size_t)d.D * 4, (size_t)n_points,
                             hipMemcpyDeviceToDevice, job->stream);
    if (e == hipSuccess) e = nuts_gradient_dense(d, n_points, (float*)tg, (float*)tu, d.Dp, job->stream);
    if (e == hipSuccess && grad)
        e = hipMemcpy2DAsync(grad, (size_t)d.D * 4, tg, (size_t)d.Dp * 4, (size_t)d.D * 4, (size_t)n_points,
                             hipMemcpyDeviceToDevice, job->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(U, tu, (size_t)n_points * 4, hipMemcpyDeviceToDevice, job->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(job->stream);
    (void)hipFree(tg);
    if (tu) (void)hipFree(tu);
    if (e != hipSuccess) return hip_fail(e, "fsmmc_eval_potential");
    return FSMMC_OK;
}

fsmmc_status fsmmc_eval_potential_noalloc(fsmmc_job* job, int32_t n_points, const void* theta, void* grad, void* U)
{
    if (!job || !theta || !U) return fail(FSMMC_EINVAL, "job, theta or U is NULL");
    if (job->batch) return fail(FSMMC_EBUSY, "job is stepped by a batch or server");
    JobDev& d = job->d;
    if (d.kind != FSMMC_NUTS) return fail(FSMMC_ENOTSUP, "only NUTS jobs evaluate a potential");
    if (n_points < 1 || n_points > d.m) return fail(FSMMC_EINVAL, "n_points must be in [1, n_chains]");
    if (d.target == FSMMC_MOG) {  // no workspace: the evaluation kernel writes the outputs directly
        HIP_TRY(hipSetDevice(job->ctx->device));
        HIP_TRY(mog_eval(d, n_points, (const float*)theta, (float*)grad, (float*)U, job->stream));
        return FSMMC_OK;
    }
    // padded gradients, then the potentials at the next 256-byte boundary
    const size_t gbytes = ((size_t)n_points * d.Dp * 4 + 255) & ~(size_t)255;
    if (gbytes + (size_t)n_points * 4 > (size_t)FSMMC_NOALLOC_SCRATCH_BYTES)
        return fail(FSMMC_EINVAL, "n_points x (padded dim + 1) x 4 bytes exceeds the allocation-free workspace "
                                  "(FSMMC_NOALLOC_SCRATCH_BYTES)");
    HIP_TRY(hipSetDevice(job->ctx->device));
    void* base = nullptr;
    fsmmc_status st = scratch_setup(job->ctx->device, &base);
    if (st != FSMMC_OK) return st;
    float* tg = static_cast<float*>(base);
    float* tu = reinterpret_cast<float*>(static_cast<unsigned char*>(base) + gbytes);
    const size_t np = (size_t)n_points * d.Dp;
    hipLaunchKernelGGL(pack_points_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, job->stream,
                       (const float*)theta, (float*)d.Thq, n_points, d.D, d.Dp);
    HIP_TRY(hipGetLastError());
    HIP_TRY(nuts_gradient_dense(d, n_points, tg, tu, d.Dp, job->stream));
    const size_t nu = std::max((size_t)n_points * d.D, (size_t)n_points);
    hipLaunchKernelGGL(unpack_potential_kernel, dim3((unsigned)((nu + 255) / 256)), dim3(256), 0, job->stream,
                       (const float*)tg, (const float*)tu, (float*)grad, (float*)U, n_points, d.D, d.Dp);
    HIP_TRY(hipGetLastError());
    return FSMMC_OK;
}

fsmmc_status fsmmc_chain_progress(fsmmc_job* job, uint32_t* dst)
{
    if (!job || !dst) return fail(FSMMC_EINVAL, "job or dst is NULL");
    std::vector<uint32_t> t;
    fsmmc_status s = progress(job, t, nullptr);
    if (s != FSMMC_OK) return s;
    std::memcpy(dst, t.data(), t.size() * 4);
    return FSMMC_OK;
}

fsmmc_status fsmmc_job_stats(fsmmc_job* job, fsmmc_stats* out)
{
    if (!job || !out) return fail(FSMMC_EINVAL, "job or out is NULL");
    std::vector<uint32_t> t;
    fsmmc_status s = progress(job, t, nullptr);
    if (s != FSMMC_OK) return s;
    s = read_ctr(job);
    if (s != FSMMC_OK) return s;
    std::memset(out, 0, sizeof(*out));
    out->steps = (int64_t)job->h_ctr[0];
    out->padded_steps = (int64_t)job->h_ctr[1];
    out->guard_trips = (int32_t)job->h_ctr[2];
    for (uint32_t v : t) {
        out->draws += v;
        out->chains_done += v >= (uint32_t)job->d.n;
    }
    out->launches = job->launches;
    for (int c = 0; c < 4; ++c) {
        out->kernel_ms[c] = job->kms[c];
        out->kernel_launches[c] = job->klaunch[c];
    }
    const JobDev& d = job->d;
    // loop counts of the produced draws: histogram, mean, per-draw max over chains
    std::vector<int32_t> cnt((size_t)d.m * d.n);
    HIP_TRY(hipMemcpy(cnt.data(), d.counts, cnt.size() * 4, hipMemcpyDeviceToHost));
    uint32_t tmin = UINT32_MAX;
    double sum = 0.0;
    int64_t nd = 0;
    for (int c = 0; c < d.m; ++c) {
        tmin = std::min(tmin, t[c]);
        const int32_t* row = &cnt[(size_t)c * d.n];
        for (uint32_t i = 0; i < t[c] && i < (uint32_t)d.n; ++i) {
            const int32_t v = std::max(row[i], 0);
            out->hist[std::min(v, FSMMC_HIST_BINS - 1)]++;
            sum += v;
            ++nd;
        }
    }
    out->mean_loops = nd ? sum / (double)nd : 0.0;
    if (tmin != UINT32_MAX && tmin > 0) {
        double smax = 0.0, sall = 0.0;
        for (uint32_t i = 0; i < tmin; ++i) {
            int32_t mx = 0;
            for (int c = 0; c < d.m; ++c) {
                const int32_t v = std::max(cnt[(size_t)c * d.n + i], 0);
                mx = std::max(mx, v);
                sall += v;
            }
            smax += mx;
        }
        out->mean_max_loops = smax / (double)tmin;
        const double mean_common = sall / ((double)tmin * (double)d.m);
        out->r_hat = mean_common > 0.0 ? out->mean_max_loops / mean_common : 0.0;
    }
    if (d.kind == FSMMC_DRMH || d.kind == FSMMC_DRSYM || d.kind == FSMMC_SLICE) {
        out->active_lanes = (int64_t)job->h_ctr[5];
        out->lane_slots = (int64_t)job->h_ctr[6];
    } else {
        out->active_lanes = out->steps * (int64_t)d.D;
        out->lane_slots = (out->steps + out->padded_steps) * (int64_t)d.Dp;
    }
    if (d.kind == FSMMC_NUTS && d.acc) {
        std::vector<float> acc((size_t)d.m);
        HIP_TRY(hipMemcpy(acc.data(), d.acc, acc.size() * 4, hipMemcpyDeviceToHost));
        double a = 0.0;
        for (float v : acc) a += (double)v;
        out->accept_sum = a;
    }
    return FSMMC_OK;
}

fsmmc_status fsmmc_job_sync(fsmmc_job* job)
{
    if (!job) return fail(FSMMC_EINVAL, "job is NULL");
    HIP_TRY(hipStreamSynchronize(job->stream));
    return FSMMC_OK;
}

fsmmc_status fsmmc_job_free(fsmmc_job* job)
{
    if (!job) return fail(FSMMC_EINVAL, "job is NULL");
    if (job->batch) return fail(FSMMC_EBUSY, "job is stepped by a batch or server");
    job_release(job);
    return FSMMC_OK;
}

}  // extern "C"
