"""FP64 CPU oracle: build and ctypes wrapper.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the HIP path and imports nothing from it.

The arithmetic lives in ``fsmmc_oracle.c`` (plain C, FP64, one chain at a
time); this file only compiles it and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fsmmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# target kinds
GP_GAUSS, GP_LOGISTIC, LOGREG, FUNNEL, GAUSS_DIAG, MOG, GP_HYPER = 0, 1, 2, 3, 4, 5, 6
# sampler kinds
ESS, NUTS, DRMH, DRSYM, SLICE = 0, 1, 2, 3, 4
# stream roles
ROLE_NU, ROLE_INIT, ROLE_THRESH, ROLE_ANGLE = 1, 2, 3, 4
ROLE_MOM, ROLE_DIR, ROLE_LEAF, ROLE_MERGE, ROLE_PROP, ROLE_ACC = 5, 6, 7, 8, 9, 10


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Target(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("n_data", C.c_int32),
                ("aux", C.c_int32), ("X", C.c_void_p), ("y", C.c_void_p),
                ("prec", C.c_void_p), ("noise_sd", C.c_double)]


class _Sampler(C.Structure):
    _fields_ = [("kind", C.c_int32), ("max_depth", C.c_int32), ("n_stages", C.c_int32),
                ("pad_", C.c_int32), ("step_size", C.c_double), ("scales", C.c_double * 4),
                ("chol_L", C.c_void_p)]


class _NutsInfo(C.Structure):
    _fields_ = [("n_leapfrog", C.c_int32), ("depth", C.c_int32), ("diverged", C.c_int32),
                ("turned", C.c_int32), ("accept", C.c_double)]


_lib = None
_lock = threading.Lock()


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB)
            d, p, u32, u64, i32 = C.c_double, C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
            L.orc_philox4x32_10.argtypes = [p, p, p]
            L.orc_u01.restype = d
            L.orc_u01.argtypes = [u32]
            L.orc_uniform.restype = d
            L.orc_uniform.argtypes = [u64, u32, u32, u32, u32]
            L.orc_normals.argtypes = [u64, u32, u32, u32, u32, i32, p]
            L.orc_gp_hyper_loglik.restype = d
            L.orc_gp_hyper_loglik.argtypes = [p, p, p, p]
            L.orc_gp_loglik.restype = d
            L.orc_gp_loglik.argtypes = [p, p]
            L.orc_potential.restype = d
            L.orc_potential.argtypes = [p, p, p]
            L.orc_logpdf.restype = d
            L.orc_logpdf.argtypes = [p, p]
            L.orc_log1mexp.restype = d
            L.orc_log1mexp.argtypes = [d]
            L.orc_dr_log_alpha1.restype = d
            L.orc_dr_log_alpha1.argtypes = [d, d]
            L.orc_drsym_alpha.restype = d
            L.orc_drsym_alpha.argtypes = [d, d, d]
            L.orc_drsym_sample.restype = i32
            L.orc_drsym_sample.argtypes = [p, i32, d, u64, u32, u32, p, p, p]
            L.orc_dr_log_alpha2.restype = d
            L.orc_dr_log_alpha2.argtypes = [d, d, d, d, d]
            L.orc_dr_log_alpha3.restype = d
            L.orc_dr_log_alpha3.argtypes = [d, d, d, d, p]
            L.orc_leapfrog.restype = d
            L.orc_leapfrog.argtypes = [p, d, p, p, p, p]
            L.orc_nuts_subtree_first_turn.restype = i32
            L.orc_nuts_subtree_first_turn.argtypes = [i32, i32, p]
            L.orc_nuts_sample.restype = i32
            L.orc_nuts_sample.argtypes = [p, d, i32, u64, u32, u32, p, p, p, p, p]
            L.orc_draw_traced.restype = i32
            L.orc_draw_traced.argtypes = [p, p, u64, u32, u32, p, p, p, i32, p, i32]
            L.orc_ess_sample.restype = i32
            L.orc_ess_sample.argtypes = [p, p, u64, u32, u32, p, p, p]
            L.orc_dr_sample.restype = i32
            L.orc_dr_sample.argtypes = [p, i32, p, u64, u32, u32, p, p, p]
            L.orc_run_chain.restype = i32
            L.orc_run_chain.argtypes = [p, p, u64, u32, i32, p, p, p, i32, p, p]
            L.orc_ess_init.argtypes = [p, i32, u64, u32, p, p]
            L.orc_funnel_init.argtypes = [i32, u64, u32, p]
            L.orc_normal_init.argtypes = [i32, u64, u32, p]
            _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class Target:
    """A target density (kept alive together with its arrays)."""

    def __init__(self, kind, dim, X=None, y=None, prec=None, noise_sd=0.0):
        self.kind, self.dim = kind, int(dim)
        self.X, self.y, self.prec = _f64(X), _f64(y), _f64(prec)
        n_data = 0 if self.X is None else self.X.shape[0]
        aux = self.X.shape[1] if (self.X is not None and self.X.ndim == 2) else 0
        self.s = _Target(kind, self.dim, n_data, aux, _ptr(self.X), _ptr(self.y), _ptr(self.prec),
                         float(noise_sd))

    @property
    def ref(self):
        return C.byref(self.s)


def gp_target(y, noise_sd=None):
    """GP latent target: Gaussian likelihood if noise_sd is given, else Bernoulli-logistic."""
    y = np.asarray(y, dtype=np.float64)
    if noise_sd is None:
        return Target(GP_LOGISTIC, y.size, y=y)
    return Target(GP_GAUSS, y.size, y=y, noise_sd=noise_sd)


def logreg_target(X, y):
    X = np.asarray(X, dtype=np.float64)
    return Target(LOGREG, X.shape[1], X=X, y=y)


def funnel_target(dim=10):
    return Target(FUNNEL, dim)


def mog_target(means, log_weights, prec):
    """Mixture of K Gaussians sharing one precision matrix P (Sec. 7.3):
    pi(x) ∝ sum_k w_k exp(-(x - mu_k)^T P (x - mu_k) / 2).  means (K, D)."""
    means = np.atleast_2d(np.asarray(means, dtype=np.float64))
    return Target(MOG, means.shape[1], X=means, y=np.asarray(log_weights, dtype=np.float64),
                  prec=np.asarray(prec, dtype=np.float64))


def gp_hyper_target(X, y, jitter=1e-6):
    """GP regression hyperparameters theta = (tau, lambda, sigma): the marginal
    likelihood N(y; 0, tau^2 exp(-lambda^2 |a - b|^2) + (sigma^2 + jitter) I)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    return Target(GP_HYPER, 3, X=X, y=np.asarray(y, dtype=np.float64), noise_sd=jitter)


def gp_hyper_loglik(target, th):
    return lib().orc_gp_hyper_loglik(target.ref, _ptr(_f64(th)), None, None)


def gauss_target(prec):
    prec = np.asarray(prec, dtype=np.float64)
    return Target(GAUSS_DIAG, prec.size, prec=prec)


class Sampler:
    def __init__(self, kind, chol_L=None, step_size=0.0, max_depth=10, n_stages=3,
                 scales=(1.0, 0.3, 0.1)):
        self.kind = kind
        self.L = _f64(chol_L)
        sc = (C.c_double * 4)(*(list(scales) + [0.0] * (4 - len(scales))))
        self.s = _Sampler(kind, int(max_depth), int(n_stages), 0, float(step_size), sc, _ptr(self.L))

    @property
    def ref(self):
        return C.byref(self.s)


def ess_sampler(chol_L):
    return Sampler(ESS, chol_L=chol_L)


def nuts_sampler(step_size, max_depth=10):
    return Sampler(NUTS, step_size=step_size, max_depth=max_depth)


def dr_sampler(scales=(1.0, 0.3, 0.1), n_stages=None):
    n = len(scales) if n_stages is None else n_stages
    return Sampler(DRMH, n_stages=n, scales=scales)


def slice_sampler(width=1.0):
    """Slice sampling along a random direction, stepping-out width `width`."""
    return Sampler(SLICE, scales=(float(width),))


def drsym_sampler(n_tries=100, sigma=0.1):
    """Symmetric delayed rejection: up to n_tries re-centred proposals of
    standard deviation sigma per draw."""
    return Sampler(DRSYM, n_stages=int(n_tries), scales=(float(sigma),))


# ---------------------------------------------------------------- RNG
def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed, chain, draw, role, sub=0):
    return lib().orc_uniform(seed, chain, draw, role, sub)


def normals(seed, chain, draw, role, sub, n):
    z = np.zeros(n)
    lib().orc_normals(seed, chain, draw, role, sub, n, _ptr(z))
    return z


# ---------------------------------------------------------------- targets
def gp_loglik(target, f):
    f = _f64(f)
    return lib().orc_gp_loglik(target.ref, _ptr(f))


def potential(target, th, grad=False):
    th = _f64(th)
    g = np.zeros_like(th) if grad else None
    U = lib().orc_potential(target.ref, _ptr(th), _ptr(g))
    return (U, g) if grad else U


def logpdf(target, x):
    x = _f64(x)
    return lib().orc_logpdf(target.ref, _ptr(x))


# ---------------------------------------------------------------- pieces
def log1mexp(a):
    return lib().orc_log1mexp(float(a))


def drsym_alpha(lx, ly, lstar):
    return lib().orc_drsym_alpha(float(lx), float(ly), float(lstar))


def drsym_sample(target, n_tries, sigma, seed, chain, draw, x):
    x = _f64(x).copy()
    lx = C.c_double(logpdf(target, x))
    work = np.zeros(2 * target.dim)
    s = lib().orc_drsym_sample(target.ref, int(n_tries), float(sigma), seed, chain, draw, _ptr(x),
                               C.byref(lx), _ptr(work))
    return x, s


def dr_log_alpha1(la, lb):
    return lib().orc_dr_log_alpha1(la, lb)


def dr_log_alpha2(la, lb, lc, lq1_ab, lq1_cb):
    return lib().orc_dr_log_alpha2(la, lb, lc, lq1_ab, lq1_cb)


def dr_log_alpha3(lx, l1, l2, l3, q):
    q = _f64(q)
    return lib().orc_dr_log_alpha3(lx, l1, l2, l3, _ptr(q))


def leapfrog(target, veps, th, p, g):
    th, p, g = _f64(th).copy(), _f64(p).copy(), _f64(g).copy()
    ph = np.zeros_like(th)
    U = lib().orc_leapfrog(target.ref, float(veps), _ptr(th), _ptr(p), _ptr(g), _ptr(ph))
    return th, p, g, U


def nuts_subtree_first_turn(moms):
    moms = _f64(moms)
    n, D = moms.shape
    j = int(np.log2(n))
    assert 1 << j == n
    return lib().orc_nuts_subtree_first_turn(D, j, _ptr(moms))


def nuts_sample(target, eps, max_depth, seed, chain, draw, th, U, g):
    D = target.dim
    th, g = _f64(th).copy(), _f64(g).copy()
    Uc = C.c_double(U)
    ws = np.zeros(D * (13 + 2 * 16))
    info = _NutsInfo()
    lib().orc_nuts_sample(target.ref, float(eps), int(max_depth), seed, chain, draw, _ptr(th),
                          C.byref(Uc), _ptr(g), _ptr(ws), C.byref(info))
    return th, Uc.value, g, dict(n_leapfrog=info.n_leapfrog, depth=info.depth,
                                  diverged=info.diverged, turned=info.turned, accept=info.accept)


def draw_traced(target, sampler, seed, chain, draw, x_prev, flip_at=-1, cap=1 << 16):
    """One draw from x_prev with its branch decisions recorded; with
    flip_at >= 0 the outcome of decision number flip_at is inverted.
    Returns (x, loop count, margins, scales): margin k is the distance of
    decision k's compared quantity from its threshold, scale k the magnitude
    of the terms it was formed from."""
    x = _f64(x_prev).copy()
    mar, sca = np.zeros(cap), np.zeros(cap)
    nd = C.c_int32()
    cnt = lib().orc_draw_traced(target.ref, sampler.ref, seed, chain, draw, _ptr(x), _ptr(mar),
                                _ptr(sca), cap, C.byref(nd), int(flip_at))
    if cnt == 0:
        raise ValueError("oracle rejected the arguments")
    k = min(nd.value, cap)
    return x, abs(int(cnt)), mar[:k], sca[:k]


def ess_init(chol_L, seed, chain):
    L = _f64(chol_L)
    D = L.shape[0]
    x, z = np.zeros(D), np.zeros(D)
    lib().orc_ess_init(_ptr(L), D, seed, chain, _ptr(x), _ptr(z))
    return x


def funnel_init(dim, seed, chain):
    x = np.zeros(dim)
    lib().orc_funnel_init(dim, seed, chain, _ptr(x))
    return x


def normal_init(dim, seed, chain):
    x = np.zeros(dim)
    lib().orc_normal_init(dim, seed, chain, _ptr(x))
    return x


# ---------------------------------------------------------------- chains
def run_chain(target, sampler, seed, chain, n, x0=None, use_fsm=False, want_edges=False):
    """One chain of n draws.  Returns dict(draws (n, D), counts (n,), guards,
    edges, steps)."""
    D = target.dim
    out = np.zeros((n, D))
    counts = np.zeros(n, dtype=np.int32)
    edges = np.zeros(36, dtype=np.int64)
    steps = np.zeros(1, dtype=np.int64)
    x0 = _f64(x0)
    g = lib().orc_run_chain(target.ref, sampler.ref, seed, chain, n, _ptr(x0), _ptr(out),
                            _ptr(counts), int(use_fsm), _ptr(edges), _ptr(steps))
    if g < 0:
        raise ValueError("oracle rejected the arguments")
    res = dict(draws=out, counts=counts, guards=g, steps=int(steps[0]))
    if want_edges:
        K = 6 if sampler.kind in (NUTS, SLICE) else 4
        res["edges"] = edges[:K * K].reshape(K, K)
    return res


def run_chains(target, sampler, seed, chains, n, x0=None, use_fsm=False, threads=None):
    """Many independent chains, one per worker thread (ctypes drops the GIL).
    x0: (len(chains), D) or None.  Returns (draws (m, n, D), counts (m, n), guards)."""
    chains = list(chains)
    m, D = len(chains), target.dim
    draws = np.zeros((m, n, D))
    counts = np.zeros((m, n), dtype=np.int32)
    guards = np.zeros(m, dtype=np.int64)
    lib()

    def one(i):
        r = run_chain(target, sampler, seed, chains[i], n,
                      None if x0 is None else x0[i], use_fsm)
        draws[i], counts[i], guards[i] = r["draws"], r["counts"], r["guards"]

    nt = threads or min(m, os.cpu_count() or 1)
    if nt <= 1:
        for i in range(m):
            one(i)
    else:
        with ThreadPoolExecutor(nt) as ex:
            list(ex.map(one, range(m)))
    return draws, counts, int(guards.sum())
