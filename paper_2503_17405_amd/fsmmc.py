"""Thin ctypes binding of libfsmmc (include/fsmmc.h).

Argument marshalling only: every step of the sampling path runs in the HIP
library.  PyTorch supplies device memory (tensors' data pointers) and the
stream.  Importing this module loads ``libfsmmc.so``; if it is missing the
import raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfsmmc.so")

OK, EINVAL, ENOMEM, EBUDGET, EDEVICE, EBUSY, ENOTDONE, ENOTSUP = range(8)
GP_GAUSS, GP_LOGISTIC, LOGREG, FUNNEL, GAUSS_DIAG, MOG, GP_HYPER = range(7)
HIST_BINS = 1025
ESS, NUTS, DRMH, DRSYM, SLICE = range(5)
F32, F64 = 0, 1
SYNC_VMAP, SYNC_COMPACT = 0, 1

# every symbol the header declares
EXPORTS = [
    "fsmmc_ctx_create", "fsmmc_ctx_destroy", "fsmmc_ctx_bytes_in_use", "fsmmc_init_chains",
    "fsmmc_step_fsm", "fsmmc_step_fsm_async", "fsmmc_step_synchronized", "fsmmc_collect_samples",
    "fsmmc_collect_counts",
    "fsmmc_chain_progress", "fsmmc_job_stats", "fsmmc_job_sync", "fsmmc_job_free",
    "fsmmc_last_error", "fsmmc_version", "fsmmc_eval_potential", "fsmmc_eval_potential_noalloc",
    "fsmmc_batch_create", "fsmmc_batch_run", "fsmmc_batch_stats", "fsmmc_batch_free",
    "fsmmc_clock", "fsmmc_server_create", "fsmmc_server_submit", "fsmmc_server_poll",
    "fsmmc_server_wait", "fsmmc_server_stats", "fsmmc_server_destroy", "fsmmc_measure_ceilings",
]


class TargetSpec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("n_data", C.c_int32),
                ("aux", C.c_int32), ("X", C.c_void_p), ("y", C.c_void_p),
                ("chol_L", C.c_void_p), ("prec", C.c_void_p), ("noise_sd", C.c_double)]


class SamplerSpec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32), ("max_depth", C.c_int32),
                ("n_stages", C.c_int32), ("step_size", C.c_double), ("scales", C.c_double * 4)]


class Tune(C.Structure):
    _fields_ = [("window", C.c_int32), ("timing", C.c_int32), ("fsm_states", C.c_int32),
                ("reserved", C.c_int32 * 5)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("padded_steps", C.c_int64), ("draws", C.c_int64),
                ("chains_done", C.c_int32), ("guard_trips", C.c_int32), ("launches", C.c_int32),
                ("reserved", C.c_int32), ("kernel_ms", C.c_double * 4),
                ("kernel_launches", C.c_int32 * 4), ("mean_loops", C.c_double),
                ("mean_max_loops", C.c_double), ("r_hat", C.c_double), ("active_lanes", C.c_int64),
                ("lane_slots", C.c_int64), ("accept_sum", C.c_double), ("hist", C.c_int64 * HIST_BINS)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        d["kernel_ms"] = list(self.kernel_ms)
        d["kernel_launches"] = list(self.kernel_launches)
        d["hist"] = np.frombuffer(self.hist, dtype=np.int64).copy()
        return d


class BatchTune(C.Structure):
    _fields_ = [("autotune", C.c_int32), ("window", C.c_int32), ("dr_chunk", C.c_int32),
                ("gemm_cols", C.c_int32), ("rounds_per_sync", C.c_int32), ("nuts_steps", C.c_int32),
                ("reserved", C.c_int32 * 2)]


class BatchCounters(C.Structure):
    _fields_ = [("rounds", C.c_int64), ("captures", C.c_int64), ("draws", C.c_int64),
                ("window", C.c_int32), ("dr_chunk", C.c_int32), ("gemm_cols", C.c_int32),
                ("live_jobs", C.c_int32), ("gpu_ms", C.c_double), ("tune_ms", C.c_double),
                ("tune_trials", C.c_int32), ("fsm_blocks", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(C.Structure):
    _fields_ = [("batch", BatchTune), ("ess_window", C.c_int32), ("reserved", C.c_int32 * 7)]


class ServerDone(C.Structure):
    _fields_ = [("job_id", C.c_uint64), ("status", C.c_int32), ("reserved", C.c_int32),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


class ServerCounters(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("failed", C.c_int64), ("rounds", C.c_int64), ("draws", C.c_int64),
                ("live_jobs", C.c_int32), ("pending_jobs", C.c_int32), ("peak_live_jobs", C.c_int32),
                ("reserved", C.c_int32), ("peak_bytes", C.c_uint64), ("gpu_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Ceilings(C.Structure):
    _fields_ = [("hbm_copy_gbps", C.c_double), ("mfma_bf16_tflops", C.c_double), ("mfma_f32_tflops", C.c_double),
                ("valu_f32_tflops", C.c_double), ("valu_f64_tflops", C.c_double), ("exp_f32_gops", C.c_double),
                ("cus", C.c_int32), ("clock_mhz", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FsmmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("fsmmc error %d: %s" % (status, msg))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfsmmc.so is not built (run __graft_entry__.build() or "
                          "python paper_2503_17405_amd/build.py)")
    L = C.CDLL(LIB_PATH)
    p, i32, i64, u64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_size_t
    pp = C.POINTER(C.c_void_p)
    sigs = {
        "fsmmc_ctx_create": ([C.c_int, sz, pp], C.c_int),
        "fsmmc_ctx_destroy": ([p], C.c_int),
        "fsmmc_ctx_bytes_in_use": ([p], sz),
        "fsmmc_init_chains": ([p, p, p, i32, i32, u64, p, p, p, p, pp], C.c_int),
        "fsmmc_step_fsm": ([p, i64, p], C.c_int),
        "fsmmc_step_fsm_async": ([p, i64, p], C.c_int),
        "fsmmc_step_synchronized": ([p, i32, i32, p], C.c_int),
        "fsmmc_collect_samples": ([p, i32, i32, p, i32], C.c_int),
        "fsmmc_collect_counts": ([p, p], C.c_int),
        "fsmmc_chain_progress": ([p, p], C.c_int),
        "fsmmc_eval_potential": ([p, i32, p, p, p], C.c_int),
        "fsmmc_eval_potential_noalloc": ([p, i32, p, p, p], C.c_int),
        "fsmmc_job_stats": ([p, p], C.c_int),
        "fsmmc_job_sync": ([p], C.c_int),
        "fsmmc_job_free": ([p], C.c_int),
        "fsmmc_batch_create": ([p, pp, i32, p, p, pp], C.c_int),
        "fsmmc_batch_run": ([p, i64, p], C.c_int),
        "fsmmc_batch_stats": ([p, p], C.c_int),
        "fsmmc_batch_free": ([p], C.c_int),
        "fsmmc_clock": ([], C.c_double),
        "fsmmc_server_create": ([p, p, pp], C.c_int),
        "fsmmc_server_submit": ([p, p, p, i32, i32, u64, p, p, p, C.POINTER(C.c_uint64)], C.c_int),
        "fsmmc_server_poll": ([p, p, i32, C.POINTER(C.c_int32)], C.c_int),
        "fsmmc_server_wait": ([p, C.c_double, p], C.c_int),
        "fsmmc_server_stats": ([p, p], C.c_int),
        "fsmmc_server_destroy": ([p], C.c_int),
        "fsmmc_last_error": ([], C.c_char_p),
        "fsmmc_version": ([], C.c_char_p),
        "fsmmc_measure_ceilings": ([C.c_int, sz, p], C.c_int),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes, f.restype = args, res
    return L


lib = _load()


def _check(status):
    if status != OK:
        raise FsmmcError(status, lib.fsmmc_last_error().decode())


def measure_ceilings(device=0, copy_bytes=2 << 30):
    out = Ceilings()
    _check(lib.fsmmc_measure_ceilings(device, copy_bytes, C.byref(out)))
    return out.as_dict()


def version():
    return lib.fsmmc_version().decode()


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("fsmmc needs contiguous row-major tensors (call .contiguous())")
    return C.c_void_p(t.data_ptr())


def _dense(t):
    return None if t is None else t.contiguous()


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------- C names
def fsmmc_ctx_create(device=0, hbm_budget_bytes=0):
    out = C.c_void_p()
    _check(lib.fsmmc_ctx_create(device, hbm_budget_bytes, C.byref(out)))
    return out


def fsmmc_ctx_destroy(ctx):
    _check(lib.fsmmc_ctx_destroy(ctx))


def fsmmc_init_chains(ctx, target, sampler, n_chains, n_draws, seed, x0=None, out_samples=None,
                      stream=None, tune=None):
    out = C.c_void_p()
    _check(lib.fsmmc_init_chains(ctx, C.byref(target), C.byref(sampler), n_chains, n_draws,
                                 seed, _ptr(x0), _ptr(out_samples), _stream_ptr(stream),
                                 None if tune is None else C.byref(tune), C.byref(out)))
    return out


def fsmmc_step_fsm(job, max_steps=0):
    done = C.c_int32()
    _check(lib.fsmmc_step_fsm(job, max_steps, C.byref(done)))
    return bool(done.value)


def fsmmc_step_fsm_async(job, max_steps, done):
    """done: an int32 tensor on the device or in pinned host memory (the
    library rejects pageable memory); its first element is written when the
    queued steps have run."""
    import torch
    if done.dtype != torch.int32 or done.numel() < 1:
        raise ValueError("done must be an int32 tensor with at least one element")
    _check(lib.fsmmc_step_fsm_async(job, max_steps, C.c_void_p(done.data_ptr())))


def fsmmc_step_synchronized(job, n_draws, mode=SYNC_VMAP):
    done = C.c_int32()
    _check(lib.fsmmc_step_synchronized(job, n_draws, mode, C.byref(done)))
    return bool(done.value)


def fsmmc_collect_samples(job, draw_begin, draw_end, dst, dst_is_host):
    ptr = C.c_void_p(dst.ctypes.data) if dst_is_host else _ptr(dst)
    _check(lib.fsmmc_collect_samples(job, draw_begin, draw_end, ptr, 1 if dst_is_host else 0))


def fsmmc_collect_counts(job, dst):
    _check(lib.fsmmc_collect_counts(job, C.c_void_p(dst.ctypes.data)))


def fsmmc_chain_progress(job, dst):
    _check(lib.fsmmc_chain_progress(job, C.c_void_p(dst.ctypes.data)))


def fsmmc_eval_potential(job, theta, grad, U):
    _check(lib.fsmmc_eval_potential(job, int(theta.shape[0]), _ptr(theta), _ptr(grad), _ptr(U)))


def fsmmc_eval_potential_noalloc(job, theta, grad, U):
    _check(lib.fsmmc_eval_potential_noalloc(job, int(theta.shape[0]), _ptr(theta), _ptr(grad), _ptr(U)))


def fsmmc_job_stats(job):
    s = Stats()
    _check(lib.fsmmc_job_stats(job, C.byref(s)))
    return s.as_dict()


def fsmmc_job_sync(job):
    _check(lib.fsmmc_job_sync(job))


def fsmmc_job_free(job):
    _check(lib.fsmmc_job_free(job))


def fsmmc_batch_create(ctx, jobs, stream=None, tune=None):
    arr = (C.c_void_p * len(jobs))(*[j.value for j in jobs])
    out = C.c_void_p()
    st = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(lib.fsmmc_batch_create(ctx, C.cast(arr, C.POINTER(C.c_void_p)), len(jobs), st,
                                  None if tune is None else C.byref(tune), C.byref(out)))
    return out


def fsmmc_batch_run(batch, max_rounds=0):
    done = C.c_int32()
    _check(lib.fsmmc_batch_run(batch, max_rounds, C.byref(done)))
    return bool(done.value)


def fsmmc_batch_stats(batch):
    s = BatchCounters()
    _check(lib.fsmmc_batch_stats(batch, C.byref(s)))
    return s.as_dict()


def fsmmc_batch_free(batch):
    _check(lib.fsmmc_batch_free(batch))


# ------------------------------------------------------------- convenience
class Context:
    def __init__(self, device=0, hbm_budget_bytes=0):
        self.handle = fsmmc_ctx_create(device, hbm_budget_bytes)
        self.device = device

    def bytes_in_use(self):
        return lib.fsmmc_ctx_bytes_in_use(self.handle)

    def close(self):
        if self.handle is not None:
            fsmmc_ctx_destroy(self.handle)
            self.handle = None


def gp_target(chol_L, y, noise_sd=None):
    """Target spec of a latent GP (tensors on the device, in the job dtype)."""
    kind = GP_LOGISTIC if noise_sd is None else GP_GAUSS
    chol_L, y = _dense(chol_L), _dense(y)
    spec = TargetSpec(kind, int(y.numel()), 0, 0, None, _ptr(y), _ptr(chol_L), None,
                      float(noise_sd or 0.0))
    return spec, (chol_L, y)


def ess_sampler(dtype=F32):
    return SamplerSpec(ESS, dtype, 0, 0, 0.0, (C.c_double * 4)())


def logreg_target(X, y):
    """Bayesian logistic regression with a N(0, I) prior: X (N x D), labels y (N,)."""
    X, y = _dense(X), _dense(y)
    spec = TargetSpec(LOGREG, int(X.shape[1]), int(X.shape[0]), 0, _ptr(X), _ptr(y), None, None, 0.0)
    return spec, (X, y)


def mog_target(means, log_weights, prec):
    """Mixture of K Gaussians sharing the precision matrix prec (D x D):
    means (K x D), log_weights (K,)."""
    means, log_weights, prec = _dense(means), _dense(log_weights), _dense(prec)
    spec = TargetSpec(MOG, int(means.shape[1]), int(means.shape[0]), 0, _ptr(means), _ptr(log_weights), None,
                      _ptr(prec), 0.0)
    return spec, (means, log_weights, prec)


def gp_hyper_target(X, y, jitter=1e-6):
    """GP-regression hyperparameters (tau, lambda, sigma) with the N(0, I)
    prior: X (n x p) inputs and y (n,) outputs, FP64 device tensors."""
    X, y = _dense(X), _dense(y)
    spec = TargetSpec(GP_HYPER, 3, int(X.shape[0]), int(X.shape[1]), _ptr(X), _ptr(y), None, None,
                      float(jitter))
    return spec, (X, y)


def nuts_sampler(step_size, max_depth=10, dtype=F32):
    return SamplerSpec(NUTS, dtype, int(max_depth), 0, float(step_size), (C.c_double * 4)())


def funnel_target(dim=10):
    """Neal's funnel: v ~ N(0, 9), x_i | v ~ N(0, e^v), i = 1 .. dim-1."""
    return TargetSpec(FUNNEL, int(dim), 0, 0, None, None, None, None, 0.0), ()


def gauss_target(prec):
    """N(0, diag(prec)^-1); prec is a device tensor of precisions."""
    prec = _dense(prec)
    return TargetSpec(GAUSS_DIAG, int(prec.numel()), 0, 0, None, None, None, _ptr(prec), 0.0), (prec,)


def drsym_sampler(n_tries=100, sigma=0.1, dtype=F32):
    """Symmetric delayed rejection: up to n_tries proposals per draw, each
    re-centred on the last rejected one, standard deviation sigma."""
    return SamplerSpec(DRSYM, dtype, 0, int(n_tries), 0.0, (C.c_double * 4)(float(sigma), 0.0, 0.0, 0.0))


def slice_sampler(width=1.0, dtype=F32):
    """Slice sampling along a random direction, stepping-out width `width`."""
    return SamplerSpec(SLICE, dtype, 0, 0, 0.0, (C.c_double * 4)(float(width), 0.0, 0.0, 0.0))


def dr_sampler(scales=(1.0, 0.3, 0.1), dtype=F32):
    sc = list(scales) + [0.0] * (4 - len(scales))
    return SamplerSpec(DRMH, dtype, 0, len(scales), 0.0, (C.c_double * 4)(*sc))


class Job:
    """One sampling job: n_chains chains x n_draws draws of one target."""

    def __init__(self, ctx, target, sampler, n_chains, n_draws, seed, x0=None, out=None,
                 stream=None, window=0, timing=False, fsm_states=0):
        import torch
        spec, self._keep = target
        self.sampler = sampler
        self.m, self.n, self.dim = n_chains, n_draws, spec.dim
        self.dtype = torch.float32 if sampler.dtype == F32 else torch.float64
        tune = Tune(window, 1 if timing else 0, fsm_states) if (window or timing or fsm_states) else None
        torch.cuda.synchronize()
        # x0 is read asynchronously on the job's stream: keep a dense copy alive with the job
        self._x0 = _dense(x0)
        if out is not None and not out.is_contiguous():
            raise ValueError("out must be a contiguous (n_chains, n_draws, dim) tensor")
        self.handle = fsmmc_init_chains(ctx.handle, spec, sampler, n_chains, n_draws, seed, self._x0,
                                        out, stream, tune)
        self.out = out

    def step_fsm(self, max_steps=0):
        return fsmmc_step_fsm(self.handle, max_steps)

    def step_fsm_async(self, max_steps, done):
        fsmmc_step_fsm_async(self.handle, max_steps, done)

    def step_synchronized(self, n_draws, mode=SYNC_VMAP):
        return fsmmc_step_synchronized(self.handle, n_draws, mode)

    def samples(self, b=0, e=None):
        e = self.n if e is None else e
        dst = np.zeros((self.m, e - b, self.dim),
                       dtype=np.float32 if self.sampler.dtype == F32 else np.float64)
        fsmmc_collect_samples(self.handle, b, e, dst, True)
        return dst

    def counts(self):
        dst = np.zeros((self.m, self.n), dtype=np.int32)
        fsmmc_collect_counts(self.handle, dst)
        return dst

    def progress(self):
        dst = np.zeros(self.m, dtype=np.uint32)
        fsmmc_chain_progress(self.handle, dst)
        return dst

    def stats(self):
        return fsmmc_job_stats(self.handle)

    def potential(self, theta):
        """U and grad U of the job's target at theta (device tensor, points x dim)."""
        import torch
        theta = theta.contiguous()
        g = torch.empty_like(theta)
        U = torch.empty(theta.shape[0], dtype=theta.dtype, device=theta.device)
        fsmmc_eval_potential(self.handle, theta, g, U)
        return U, g

    def potential_noalloc(self, theta, g, U):
        """fsmmc_eval_potential_noalloc into caller-provided g and U (queued on
        the job's stream; call sync() before reading them)."""
        fsmmc_eval_potential_noalloc(self.handle, theta.contiguous(), g, U)

    def sync(self):
        fsmmc_job_sync(self.handle)

    def free(self):
        if self.handle is not None:
            fsmmc_job_free(self.handle)
            self.handle = None


class Batch:
    """Several jobs stepped together (one graph replay per round)."""

    def __init__(self, ctx, jobs, stream=None, autotune=False, window=0, dr_chunk=0, gemm_cols=0,
                 rounds_per_sync=0, nuts_steps=0):
        self.jobs = list(jobs)
        tune = BatchTune(1 if autotune else 0, window, dr_chunk, gemm_cols, rounds_per_sync, nuts_steps)
        self.handle = fsmmc_batch_create(ctx.handle, [j.handle for j in self.jobs], stream, tune)

    def run(self, max_rounds=0):
        return fsmmc_batch_run(self.handle, max_rounds)

    def stats(self):
        return fsmmc_batch_stats(self.handle)

    def free(self):
        if self.handle is not None:
            fsmmc_batch_free(self.handle)
            self.handle = None


def clock():
    """The monotonic host clock (seconds) the server stamps its records with."""
    return lib.fsmmc_clock()


class Server:
    """Continuous-batching server: jobs submitted at any time are admitted
    under the context's HBM budget, stepped together and retired as they
    finish.  Device buffers handed to submit() are kept alive here until the
    job is reported by poll()."""

    def __init__(self, ctx, ess_window=0, nuts_steps=0, rounds_per_sync=0, window=0, dr_chunk=0,
                 gemm_cols=0):
        cfg = ServerConfig(BatchTune(0, window, dr_chunk, gemm_cols, rounds_per_sync, nuts_steps), ess_window)
        out = C.c_void_p()
        _check(lib.fsmmc_server_create(ctx.handle, C.byref(cfg), C.byref(out)))
        self.handle = out
        self._keep = {}

    def submit(self, target, sampler, n_chains, n_draws, seed, out, x0=None, counts=None):
        spec, keep = target
        x0 = _dense(x0)
        if not out.is_contiguous() or (counts is not None and not counts.is_contiguous()):
            raise ValueError("out and counts must be contiguous device tensors")
        jid = C.c_uint64()
        _check(lib.fsmmc_server_submit(self.handle, C.byref(spec), C.byref(sampler), n_chains, n_draws, seed,
                                       _ptr(x0), _ptr(out), _ptr(counts), C.byref(jid)))
        self._keep[jid.value] = (keep, x0, out, counts)
        return jid.value

    def poll(self, cap=1024):
        buf = (ServerDone * cap)()
        n = C.c_int32()
        _check(lib.fsmmc_server_poll(self.handle, buf, cap, C.byref(n)))
        recs = []
        for i in range(n.value):
            r = buf[i]
            self._keep.pop(r.job_id, None)
            recs.append(dict(job_id=r.job_id, status=r.status, t_submit=r.t_submit, t_admit=r.t_admit,
                             t_done=r.t_done))
        return recs

    def wait(self, timeout=-1.0):
        idle = C.c_int32()
        _check(lib.fsmmc_server_wait(self.handle, float(timeout), C.byref(idle)))
        return bool(idle.value)

    def stats(self):
        s = ServerCounters()
        _check(lib.fsmmc_server_stats(self.handle, C.byref(s)))
        return s.as_dict()

    def close(self):
        if self.handle is not None:
            _check(lib.fsmmc_server_destroy(self.handle))
            self.handle = None
            self._keep.clear()
