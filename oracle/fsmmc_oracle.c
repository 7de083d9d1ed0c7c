/*
 * fsmmc_oracle.c -- plain FP64 CPU oracle for FSM-scheduled multi-chain MCMC
 * (Dance, Glaser, Orbanz, Adams, "Efficiently Vectorized MCMC on Modern
 * Accelerators", ICML 2025).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The product (HIP) path
 * never links, loads or calls it, and the two share no code: this file has
 * its own Philox, its own targets and its own samplers, written from the
 * paper and from the published definitions named below.
 *
 * Everything is one chain at a time, FP64, no blocking, no fusion.  Each
 * sampler exists twice:
 *   - `*_sample`: the single-chain transition kernel `sample` (Sec. 2.1,
 *     Alg. "MCMC algorithm with sample function"), loops written as loops;
 *   - `*_fsm_step`: the same kernel cut into while-loop-free blocks S_1..S_K
 *     with a transition function delta (Sec. 3.1, Fig. "FSM of an MCMC
 *     algorithm with a single while loop"; Sec. 3.2, Alg. "step function
 *     for FSM"), driven by the FSM runtime of Alg. "FSM MCMC algorithm".
 * The two must agree bit for bit: the FSM changes the schedule, not the
 * draws (Sec. 1, "equivalent samplers"; Sec. 3.2 final paragraph).
 *
 * Randomness contract (shared specification, separate implementation):
 *   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  key = (seed lo32,
 *   seed hi32); counter = (chain, draw, role<<24 | sub, block).  A uniform
 *   is ((w >> 9) + 0.5) * 2^-23 (24 significant bits, exact in FP32).
 *   Normal d of a vector uses block d/4, words 2q and 2q+1 with
 *   q = (d mod 4) div 2, Box-Muller: even d -> r cos(2 pi u2),
 *   odd d -> r sin(2 pi u2), r = sqrt(-2 ln u1).
 *
 * Compile: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011): 10 rounds of the 4x32 Philox S-box;
 * multipliers 0xD2511F53, 0xCD9E8D57; Weyl key increments 0x9E3779B9,
 * 0xBB67AE85 applied between rounds.                                   */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Roles of the random streams. */
enum {
    ORC_ROLE_NU = 1,     /* ESS ellipse normals               */
    ORC_ROLE_INIT = 2,   /* default initial state normals      */
    ORC_ROLE_THRESH = 3, /* ESS slice threshold u              */
    ORC_ROLE_ANGLE = 4,  /* ESS angle at shrink s              */
    ORC_ROLE_MOM = 5,    /* NUTS momentum                      */
    ORC_ROLE_DIR = 6,    /* NUTS direction at depth j          */
    ORC_ROLE_LEAF = 7,   /* NUTS leaf pick at (j, n)           */
    ORC_ROLE_MERGE = 8,  /* NUTS subtree merge at depth j      */
    ORC_ROLE_PROP = 9,   /* DR proposal normals at stage s     */
    ORC_ROLE_ACC = 10    /* DR acceptance uniform at stage s   */
};

static void stream_block(uint64_t seed, uint32_t chain, uint32_t draw, uint32_t role,
                         uint32_t sub, uint32_t block, uint32_t w[4])
{
    uint32_t ctr[4] = {chain, draw, (role << 24) | (sub & 0xFFFFFFu), block};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, w);
}

double orc_u01(uint32_t w) { return ((double)(w >> 9) + 0.5) * 0x1p-23; }

/* One uniform: word 0 of block 0. */
double orc_uniform(uint64_t seed, uint32_t chain, uint32_t draw, uint32_t role, uint32_t sub)
{
    uint32_t w[4];
    stream_block(seed, chain, draw, role, sub, 0, w);
    return orc_u01(w[0]);
}

/* n standard normals of one (role, sub) stream, Box-Muller per word pair. */
void orc_normals(uint64_t seed, uint32_t chain, uint32_t draw, uint32_t role, uint32_t sub,
                 int n, double* z)
{
    uint32_t w[4];
    for (int d = 0; d < n; ++d) {
        if ((d & 3) == 0) stream_block(seed, chain, draw, role, sub, (uint32_t)(d >> 2), w);
        int q = (d & 3) >> 1;
        double u1 = orc_u01(w[2 * q]);
        double u2 = orc_u01(w[2 * q + 1]);
        double r = sqrt(-2.0 * log(u1));
        double a = 2.0 * ORC_PI * u2;
        z[d] = (d & 1) ? r * sin(a) : r * cos(a);
    }
}

/* ------------------------------------------------------------------ */
/* Optional record of the branch decisions of one draw (test support; the
 * arithmetic is the same with or without it).  Every floating-point
 * comparison that picks a branch goes through decide(): with a record
 * attached it stores the distance of the compared quantity from its
 * threshold and the magnitude of the terms that quantity was formed from,
 * and it can invert the outcome of decision number flip_at, so the tests can
 * replay a draw as if one comparison had gone the other way.             */
typedef struct {
    double* margin;
    double* scale;
    int32_t cap, n;
    int32_t flip_at; /* index of the decision to invert, -1 for none */
} orc_trace;

static __thread orc_trace* g_trace = NULL;

static int decide(int outcome, double margin, double scale)
{
    if (!g_trace) return outcome;
    int32_t i = g_trace->n++;
    if (i < g_trace->cap) {
        g_trace->margin[i] = fabs(margin);
        g_trace->scale[i] = fabs(scale);
    }
    return (i == g_trace->flip_at) ? !outcome : outcome;
}

/* ------------------------------------------------------------------ */
/* Targets.                                                            */
enum { ORC_GP_GAUSS = 0, ORC_GP_LOGISTIC = 1, ORC_LOGREG = 2, ORC_FUNNEL = 3, ORC_GAUSS_DIAG = 4,
       ORC_MOG = 5, ORC_GP_HYPER = 6 };

typedef struct {
    int32_t kind;
    int32_t dim;
    int32_t n_data;     /* LOGREG: rows of X; MOG: number of components K;
                           GP_HYPER: number of observations n                  */
    int32_t aux;        /* GP_HYPER: input dimension p of the rows of X        */
    const double* X;    /* LOGREG: n_data x dim, row-major; MOG: K x dim means */
    const double* y;    /* GP: dim observations/labels; LOGREG: n_data labels;
                           MOG: K log mixture weights                          */
    const double* prec; /* GAUSS_DIAG: dim precisions; MOG: dim x dim shared
                           precision matrix (inverse covariance), row-major    */
    double noise_sd;    /* GP_GAUSS observation noise standard deviation;
                           GP_HYPER: jitter added to the diagonal              */
} orc_target;

/* GP regression marginal likelihood of the hyperparameters (Sec. 7.2):
 * theta = (tau, lambda, sigma), k(a, b) = tau^2 exp(-lambda^2 |a - b|^2),
 * y ~ N(0, C), C = tau^2 K + (sigma^2 + jitter) I.  Returns
 * -y^T C^-1 y / 2 - log det C / 2 (no 2 pi term), -inf if C is not positive
 * definite in floating point; *quad and *logdet receive the two terms.
 * Cholesky C = L L^T row by row (Cholesky-Banachiewicz), forward solve
 * L z = y, quad = |z|^2, log det = 2 sum log L_ii.                      */
double orc_gp_hyper_loglik(const orc_target* t, const double* th, double* quad, double* logdet)
{
    int n = t->n_data, p = t->aux;
    double tau2 = th[0] * th[0], lam2 = th[1] * th[1], s2 = th[2] * th[2] + t->noise_sd;
    double* L = (double*)calloc((size_t)n * n, sizeof(double));
    double* z = (double*)calloc((size_t)n, sizeof(double));
    double ld = 0.0, q = 0.0;
    int ok = 1;
    for (int i = 0; i < n && ok; ++i) {
        for (int k = 0; k <= i; ++k) {
            double r2 = 0.0;
            for (int d = 0; d < p; ++d) {
                double e = t->X[(size_t)i * p + d] - t->X[(size_t)k * p + d];
                r2 += e * e;
            }
            double c = tau2 * exp(-lam2 * r2) + (i == k ? s2 : 0.0);
            for (int j = 0; j < k; ++j) c -= L[(size_t)i * n + j] * L[(size_t)k * n + j];
            if (i == k) {
                if (!(c > 0.0)) {
                    ok = 0;
                    break;
                }
                L[(size_t)i * n + i] = sqrt(c);
            } else {
                L[(size_t)i * n + k] = c / L[(size_t)k * n + k];
            }
        }
    }
    if (ok) {
        for (int i = 0; i < n; ++i) {
            double r = t->y[i];
            for (int j = 0; j < i; ++j) r -= L[(size_t)i * n + j] * z[j];
            z[i] = r / L[(size_t)i * n + i];
            q += z[i] * z[i];
            ld += 2.0 * log(L[(size_t)i * n + i]);
        }
    }
    free(L);
    free(z);
    if (quad) *quad = ok ? q : INFINITY;
    if (logdet) *logdet = ok ? ld : INFINITY;
    return ok ? -0.5 * q - 0.5 * ld : -INFINITY;
}

static double softplus(double a) { return (a > 0.0 ? a : 0.0) + log1p(exp(-fabs(a))); }

static double sigmoid(double a)
{
    if (a >= 0.0) return 1.0 / (1.0 + exp(-a));
    double e = exp(a);
    return e / (1.0 + e);
}

/* Log-likelihood factor f of p(x) ∝ f(x) N(x | 0, Sigma) (Sec. 2.2, Example). */
double orc_gp_loglik(const orc_target* t, const double* f)
{
    double s = 0.0;
    if (t->kind == ORC_GP_HYPER) return orc_gp_hyper_loglik(t, f, NULL, NULL);
    if (t->kind == ORC_GP_GAUSS) {
        double inv2v = 1.0 / (2.0 * t->noise_sd * t->noise_sd);
        for (int i = 0; i < t->dim; ++i) {
            double r = t->y[i] - f[i];
            s -= r * r * inv2v;
        }
    } else {
        for (int i = 0; i < t->dim; ++i) s += t->y[i] * f[i] - softplus(f[i]);
    }
    return s;
}

/* Sum of the absolute values of the summands of orc_gp_loglik at f. */
static double gp_loglik_absterms(const orc_target* t, const double* f)
{
    double s = 0.0;
    if (t->kind == ORC_GP_HYPER) {
        double q = 0.0, ld = 0.0;
        orc_gp_hyper_loglik(t, f, &q, &ld);
        return 0.5 * fabs(q) + 0.5 * fabs(ld);
    }
    if (t->kind == ORC_GP_GAUSS) {
        double inv2v = 1.0 / (2.0 * t->noise_sd * t->noise_sd);
        for (int i = 0; i < t->dim; ++i) {
            double r = t->y[i] - f[i];
            s += r * r * inv2v;
        }
    } else {
        for (int i = 0; i < t->dim; ++i) s += fabs(t->y[i] * f[i]) + softplus(f[i]);
    }
    return s;
}

/* Potential U = -log pi (up to a constant) and, if g != NULL, its gradient. */
double orc_potential(const orc_target* t, const double* th, double* g)
{
    int D = t->dim;
    double U = 0.0;
    if (t->kind == ORC_LOGREG) {
        if (g)
            for (int d = 0; d < D; ++d) g[d] = th[d];
        for (int d = 0; d < D; ++d) U += 0.5 * th[d] * th[d];
        for (int i = 0; i < t->n_data; ++i) {
            const double* xi = t->X + (size_t)i * D;
            double eta = 0.0;
            for (int d = 0; d < D; ++d) eta += xi[d] * th[d];
            U -= t->y[i] * eta - softplus(eta);
            if (g) {
                double r = t->y[i] - sigmoid(eta);
                for (int d = 0; d < D; ++d) g[d] -= xi[d] * r;
            }
        }
    } else if (t->kind == ORC_GAUSS_DIAG) {
        for (int d = 0; d < D; ++d) {
            U += 0.5 * t->prec[d] * th[d] * th[d];
            if (g) g[d] = t->prec[d] * th[d];
        }
    } else if (t->kind == ORC_MOG) {
        /* Mixture of K Gaussians with one shared covariance (Sec. 7.3):
         * pi(x) ∝ sum_k w_k exp(-q_k / 2), q_k = (x - mu_k)^T P (x - mu_k).
         * U = -log sum_k exp(log w_k - q_k / 2), taken relative to the largest
         * term; grad U = sum_k r_k P (x - mu_k), r_k the component weights. */
        int K = t->n_data;
        double* a = (double*)malloc(sizeof(double) * (size_t)K);
        double* dx = (double*)malloc(sizeof(double) * (size_t)D);
        double* Pd = (double*)malloc(sizeof(double) * (size_t)D * (size_t)K);
        double amax = -INFINITY;
        for (int k = 0; k < K; ++k) {
            const double* mu = t->X + (size_t)k * D;
            for (int d = 0; d < D; ++d) dx[d] = th[d] - mu[d];
            double q = 0.0;
            for (int i = 0; i < D; ++i) {
                double s = 0.0;
                for (int j = 0; j < D; ++j) s += t->prec[(size_t)i * D + j] * dx[j];
                Pd[(size_t)k * D + i] = s;
                q += dx[i] * s;
            }
            a[k] = t->y[k] - 0.5 * q;
            if (a[k] > amax) amax = a[k];
        }
        double z = 0.0;
        for (int k = 0; k < K; ++k) z += exp(a[k] - amax);
        double lse = amax + log(z);
        U = -lse;
        if (g) {
            for (int d = 0; d < D; ++d) g[d] = 0.0;
            for (int k = 0; k < K; ++k) {
                double r = exp(a[k] - lse);
                for (int d = 0; d < D; ++d) g[d] += r * Pd[(size_t)k * D + d];
            }
        }
        free(a);
        free(dx);
        free(Pd);
    } else if (t->kind == ORC_FUNNEL) {
        /* Neal's funnel: v ~ N(0, 9), x_i | v ~ N(0, e^v), i = 1..D-1. */
        double v = th[0], ss = 0.0;
        for (int d = 1; d < D; ++d) ss += th[d] * th[d];
        double ev = exp(-v);
        U = v * v / 18.0 + 0.5 * (double)(D - 1) * v + 0.5 * ev * ss;
        if (g) {
            g[0] = v / 9.0 + 0.5 * (double)(D - 1) - 0.5 * ev * ss;
            for (int d = 1; d < D; ++d) g[d] = ev * th[d];
        }
    } else {
        U = -orc_gp_loglik(t, th);
    }
    return U;
}

double orc_logpdf(const orc_target* t, const double* x) { return -orc_potential(t, x, NULL); }

/* ------------------------------------------------------------------ */
/* Default initial states (role INIT, draw 0).                          */

/* ESS: a draw from the Gaussian prior, x0 = L z. */
void orc_ess_init(const double* L, int D, uint64_t seed, uint32_t chain, double* x0, double* z)
{
    orc_normals(seed, chain, 0, ORC_ROLE_INIT, 0, D, z);
    for (int i = 0; i < D; ++i) {
        double s = 0.0;
        for (int k = 0; k <= i; ++k) s += L[(size_t)i * D + k] * z[k];
        x0[i] = s;
    }
}

/* Funnel: an exact draw, v = 3 z_0, x_i = e^{v/2} z_i. */
void orc_funnel_init(int D, uint64_t seed, uint32_t chain, double* x0)
{
    orc_normals(seed, chain, 0, ORC_ROLE_INIT, 0, D, x0);
    double v = 3.0 * x0[0];
    x0[0] = v;
    double s = exp(0.5 * v);
    for (int d = 1; d < D; ++d) x0[d] *= s;
}

/* Standard normal start (NUTS default when no x0 is given). */
void orc_normal_init(int D, uint64_t seed, uint32_t chain, double* x0)
{
    orc_normals(seed, chain, 0, ORC_ROLE_INIT, 0, D, x0);
}

/* ------------------------------------------------------------------ */
/* Elliptical slice sampling (Murray, Adams, MacKay 2010; Appendix,
 * Alg. "Transition kernel for elliptical slice sampler").
 * Readings: the loop continues while log L(x') <= log y (the printed
 * condition is inverted); the threshold uses the log-likelihood factor,
 * not the full density; ties reject.                                   */

#define ORC_ESS_MAX_EVALS 10000

/* Returns the number of log-likelihood evaluations N (>= 1) of this draw;
 * -N if the evaluation guard tripped (x left unchanged).  work: 3*D.   */
int orc_ess_sample(const orc_target* t, const double* L, uint64_t seed, uint32_t chain,
                   uint32_t draw, double* x, double* lx, double* work)
{
    int D = t->dim;
    double *nu = work, *xp = work + D, *z = work + 2 * D;
    orc_normals(seed, chain, draw, ORC_ROLE_NU, 0, D, z);
    for (int i = 0; i < D; ++i) {
        double s = 0.0;
        for (int k = 0; k <= i; ++k) s += L[(size_t)i * D + k] * z[k];
        nu[i] = s;
    }
    double logy = *lx + log(orc_uniform(seed, chain, draw, ORC_ROLE_THRESH, 0));
    double theta = 2.0 * ORC_PI * orc_uniform(seed, chain, draw, ORC_ROLE_ANGLE, 0);
    double tmin = theta - 2.0 * ORC_PI, tmax = theta;
    int evals = 0;
    for (;;) {
        double c = cos(theta), s = sin(theta);
        for (int i = 0; i < D; ++i) xp[i] = x[i] * c + nu[i] * s;
        double lp = orc_gp_loglik(t, xp);
        ++evals;
        if (decide(lp > logy, lp - logy, g_trace ? gp_loglik_absterms(t, xp) + fabs(logy) : 0.0)) {
            memcpy(x, xp, sizeof(double) * (size_t)D);
            *lx = lp;
            return evals;
        }
        if (evals >= ORC_ESS_MAX_EVALS) return -evals;
        if (decide(theta < 0.0, theta, fabs(tmin) + fabs(tmax)))
            tmin = theta;
        else
            tmax = theta;
        theta = tmin + (tmax - tmin) * orc_uniform(seed, chain, draw, ORC_ROLE_ANGLE, (uint32_t)evals);
    }
}

/* ESS as an FSM: S1 INIT, S2 SHRINK, S3 DONE (Fig. "Finite state machines
 * for the sample function ...", elliptical slice sampling panel).        */
enum { ESS_INIT = 1, ESS_SHRINK = 2, ESS_DONE = 3 };

typedef struct {
    int k;
    uint32_t t; /* draw index the chain is working on */
    int evals;
    double theta, tmin, tmax, logy, lp, lx;
    double *x, *nu, *xp, *z;
} ess_fsm;

static void ess_propose(const orc_target* t, ess_fsm* f)
{
    int D = t->dim;
    double c = cos(f->theta), s = sin(f->theta);
    for (int i = 0; i < D; ++i) f->xp[i] = f->x[i] * c + f->nu[i] * s;
    f->lp = orc_gp_loglik(t, f->xp);
    f->evals++;
}

/* One FSM step (Alg. "step function for FSM"): run S_k, then k <- delta(k, z).
 * Returns isSample = [k == K] evaluated before the block runs.           */
static int ess_fsm_step(const orc_target* t, const double* L, uint64_t seed, uint32_t chain,
                        ess_fsm* f, int* guard)
{
    int D = t->dim;
    int is_sample = (f->k == ESS_DONE);
    switch (f->k) {
    case ESS_INIT: {
        orc_normals(seed, chain, f->t, ORC_ROLE_NU, 0, D, f->z);
        for (int i = 0; i < D; ++i) {
            double s = 0.0;
            for (int k = 0; k <= i; ++k) s += L[(size_t)i * D + k] * f->z[k];
            f->nu[i] = s;
        }
        f->logy = f->lx + log(orc_uniform(seed, chain, f->t, ORC_ROLE_THRESH, 0));
        f->theta = 2.0 * ORC_PI * orc_uniform(seed, chain, f->t, ORC_ROLE_ANGLE, 0);
        f->tmin = f->theta - 2.0 * ORC_PI;
        f->tmax = f->theta;
        f->evals = 0;
        ess_propose(t, f);
        break;
    }
    case ESS_SHRINK:
        if (f->theta < 0.0)
            f->tmin = f->theta;
        else
            f->tmax = f->theta;
        f->theta = f->tmin + (f->tmax - f->tmin) *
                                 orc_uniform(seed, chain, f->t, ORC_ROLE_ANGLE, (uint32_t)f->evals);
        ess_propose(t, f);
        break;
    case ESS_DONE:
        if (!*guard) {
            memcpy(f->x, f->xp, sizeof(double) * (size_t)D);
            f->lx = f->lp;
        }
        break;
    }
    /* delta */
    switch (f->k) {
    case ESS_INIT:
    case ESS_SHRINK:
        if (f->lp > f->logy)
            f->k = ESS_DONE;
        else if (f->evals >= ORC_ESS_MAX_EVALS) {
            *guard = 1;
            f->k = ESS_DONE;
        } else
            f->k = ESS_SHRINK;
        break;
    case ESS_DONE:
        f->k = ESS_INIT;
        break;
    }
    return is_sample;
}

/* ------------------------------------------------------------------ */
/* Delayed-rejection Metropolis-Hastings, n_stages <= 3 (Tierney & Mira
 * 1999; Mira 2001), every stage's Gaussian proposal centred at the current
 * state x: y_s = x + scale_s z_s.  Acceptance in log space; with symmetric
 * centred proposals the last-stage kernel cancels.                        */

/* log(1 - e^a) for a <= 0 (Maechler 2012): -inf at a = 0. */
double orc_log1mexp(double a)
{
    if (a > -0.6931471805599453) return log(-expm1(a));
    return log1p(-exp(a));
}

/* log min(1, e^d) with NaN mapped to NaN (a NaN never accepts). */
static double log_min1(double d) { return (d >= 0.0) ? 0.0 : d; }

/* log alpha_1(a -> b) = min(0, l_b - l_a). */
double orc_dr_log_alpha1(double la, double lb) { return log_min1(lb - la); }

/* log alpha_2(a, b, c): from a, b rejected at stage 1, c proposed at stage 2.
 * lq1_ab = log q1(a -> b), lq1_cb = log q1(c -> b).                       */
double orc_dr_log_alpha2(double la, double lb, double lc, double lq1_ab, double lq1_cb)
{
    double num = lc + lq1_cb + orc_log1mexp(orc_dr_log_alpha1(lc, lb));
    double den = la + lq1_ab + orc_log1mexp(orc_dr_log_alpha1(la, lb));
    return log_min1(num - den);
}

/* log alpha_3(x, y1, y2, y3).  q holds the proposal log-densities:
 *  q[0] = log q1(x -> y1), q[1] = log q1(y2 -> y1), q[2] = log q2(x -> y2),
 *  q[3] = log q1(y3 -> y2), q[4] = log q2(y3 -> y1), q[5] = log q1(y1 -> y2). */
double orc_dr_log_alpha3(double lx, double l1, double l2, double l3, const double* q)
{
    double la1_x1 = orc_dr_log_alpha1(lx, l1);
    double la2_x12 = orc_dr_log_alpha2(lx, l1, l2, q[0], q[1]);
    double la1_32 = orc_dr_log_alpha1(l3, l2);
    /* A zero factor of the reverse path (an impossible reverse proposal, or
     * alpha_1(y3, y2) = 1) makes alpha_3 = 0 whatever the bounded factor
     * 1 - alpha_2(y3, y2, y1) is; decide it before that factor is formed. */
    double part = q[3] + q[4] + orc_log1mexp(la1_32);
    if (part == -INFINITY) return -INFINITY;
    double la2_321 = orc_dr_log_alpha2(l3, l2, l1, q[3], q[5]);
    double num = l3 + part + orc_log1mexp(la2_321);
    double den = lx + q[0] + q[2] + orc_log1mexp(la1_x1) + orc_log1mexp(la2_x12);
    return log_min1(num - den);
}

static double lq_gauss(const double* a, const double* b, int D, double sc)
{
    double s = 0.0;
    for (int i = 0; i < D; ++i) {
        double r = b[i] - a[i];
        s += r * r;
    }
    return -s / (2.0 * sc * sc);
}

static void dr_propose(const orc_target* t, const double* scales, uint64_t seed, uint32_t chain,
                       uint32_t draw, int s, const double* x, double* y)
{
    int D = t->dim;
    orc_normals(seed, chain, draw, ORC_ROLE_PROP, (uint32_t)s, D, y);
    for (int i = 0; i < D; ++i) y[i] = x[i] + scales[s] * y[i];
}

static double dr_log_alpha_stage(int s, int D, const double* scales, const double* x,
                                 const double* y1, const double* y2, const double* y3,
                                 double lx, double l1, double l2, double l3)
{
    if (s == 0) return orc_dr_log_alpha1(lx, l1);
    if (s == 1)
        return orc_dr_log_alpha2(lx, l1, l2, lq_gauss(x, y1, D, scales[0]),
                                 lq_gauss(y2, y1, D, scales[0]));
    double q[6];
    q[0] = lq_gauss(x, y1, D, scales[0]);
    q[1] = lq_gauss(y2, y1, D, scales[0]);
    q[2] = lq_gauss(x, y2, D, scales[1]);
    q[3] = lq_gauss(y3, y2, D, scales[0]);
    q[4] = lq_gauss(y3, y1, D, scales[1]);
    q[5] = lq_gauss(y1, y2, D, scales[0]);
    return orc_dr_log_alpha3(lx, l1, l2, l3, q);
}

/* Magnitude of the log terms that the stage-s acceptance is formed from:
 * |log pi| of x and of the proposals so far, and |log q| of every proposal
 * density that alpha_s uses.  Used only for a decision record.          */
static double dr_stage_absterms(int s, int D, const double* scales, const double* x,
                                const double* y1, const double* y2, const double* y3, double lx,
                                const double* l)
{
    double a = fabs(lx);
    for (int i = 0; i <= s; ++i) a += fabs(l[i]);
    if (s >= 1) a += fabs(lq_gauss(x, y1, D, scales[0])) + fabs(lq_gauss(y2, y1, D, scales[0]));
    if (s >= 2)
        a += fabs(lq_gauss(x, y2, D, scales[1])) + fabs(lq_gauss(y3, y2, D, scales[0])) +
             fabs(lq_gauss(y3, y1, D, scales[1])) + fabs(lq_gauss(y1, y2, D, scales[0]));
    return a;
}

/* One DR draw.  Returns the number of stages evaluated (1..n_stages);
 * x, lx updated on acceptance.  work: 3*D.                               */
int orc_dr_sample(const orc_target* t, int n_stages, const double* scales, uint64_t seed,
                  uint32_t chain, uint32_t draw, double* x, double* lx, double* work)
{
    int D = t->dim;
    double* y[3] = {work, work + D, work + 2 * D};
    double l[3] = {0.0, 0.0, 0.0};
    int s = 0;
    while (s < n_stages) {
        dr_propose(t, scales, seed, chain, draw, s, x, y[s]);
        l[s] = orc_logpdf(t, y[s]);
        double la = dr_log_alpha_stage(s, D, scales, x, y[0], y[1], y[2], *lx, l[0], l[1], l[2]);
        double u = orc_uniform(seed, chain, draw, ORC_ROLE_ACC, (uint32_t)s);
        double sc = g_trace ? dr_stage_absterms(s, D, scales, x, y[0], y[1], y[2], *lx, l) : 0.0;
        ++s;
        if (decide(log(u) < la, log(u) - la, sc)) {
            memcpy(x, y[s - 1], sizeof(double) * (size_t)D);
            *lx = l[s - 1];
            break;
        }
    }
    return s;
}

/* DR as an FSM: S1 INIT, S2 PROPOSE (one stage per visit), S3 DONE
 * (Fig. "Finite state machines ...", delayed rejection panel).          */
enum { DR_INIT = 1, DR_PROPOSE = 2, DR_DONE = 3 };

typedef struct {
    int k, s, accepted;
    uint32_t t;
    double lx, l[3];
    double *x, *y[3];
} dr_fsm;

static int dr_fsm_step(const orc_target* t, int n_stages, const double* scales, uint64_t seed,
                       uint32_t chain, dr_fsm* f)
{
    int D = t->dim;
    int is_sample = (f->k == DR_DONE);
    switch (f->k) {
    case DR_INIT:
        f->s = 0;
        f->accepted = 0;
        break;
    case DR_PROPOSE: {
        int s = f->s;
        dr_propose(t, scales, seed, chain, f->t, s, f->x, f->y[s]);
        f->l[s] = orc_logpdf(t, f->y[s]);
        double la = dr_log_alpha_stage(s, D, scales, f->x, f->y[0], f->y[1], f->y[2], f->lx,
                                       f->l[0], f->l[1], f->l[2]);
        double u = orc_uniform(seed, chain, f->t, ORC_ROLE_ACC, (uint32_t)s);
        f->accepted = (log(u) < la);
        f->s = s + 1;
        break;
    }
    case DR_DONE:
        if (f->accepted) {
            memcpy(f->x, f->y[f->s - 1], sizeof(double) * (size_t)D);
            f->lx = f->l[f->s - 1];
        }
        break;
    }
    switch (f->k) {
    case DR_INIT:
        f->k = (n_stages > 0) ? DR_PROPOSE : DR_DONE;
        break;
    case DR_PROPOSE:
        f->k = (f->accepted || f->s >= n_stages) ? DR_DONE : DR_PROPOSE;
        break;
    case DR_DONE:
        f->k = DR_INIT;
        break;
    }
    return is_sample;
}

/* ------------------------------------------------------------------ */
/* Symmetric delayed rejection (Mira 2001; Sec. 7.1): up to M tries per
 * draw, each proposal re-centred on the previous (rejected) one,
 *   y_0 = x + sigma z_0,  y_s = y_{s-1} + sigma z_s,
 * accepted with probability
 *   alpha_s = min(1, max(0, pi(y_s) - pi*_s) / (pi(x) - pi*_s)),
 *   pi*_s = max_{j<s} pi(y_j)  (pi*_0 = 0: alpha_0 is the Metropolis ratio).
 * After M rejections x is kept.  Both densities are taken relative to pi(x)
 * (the ratio is unchanged), so only differences of log densities are
 * exponentiated.  Reading: sigma is a standard deviation.               */

/* alpha_s from log pi(x), log pi(y_s) and log pi*_s (-inf for s = 0). */
double orc_drsym_alpha(double lx, double ly, double lstar)
{
    double r = exp(ly - lx), rs = exp(lstar - lx);
    double a = (r - rs) / (1.0 - rs);
    if (!(a > 0.0)) a = 0.0;
    if (a > 1.0) a = 1.0;
    return a;
}

static void drsym_propose(const orc_target* t, double sigma, uint64_t seed, uint32_t chain,
                          uint32_t draw, int s, const double* c, double* y)
{
    int D = t->dim;
    orc_normals(seed, chain, draw, ORC_ROLE_PROP, (uint32_t)s, D, y);
    for (int i = 0; i < D; ++i) y[i] = c[i] + sigma * y[i];
}

/* One draw.  Returns the number of tries (1..M); x, lx updated on
 * acceptance.  work: 2*D.                                               */
int orc_drsym_sample(const orc_target* t, int M, double sigma, uint64_t seed, uint32_t chain,
                     uint32_t draw, double* x, double* lx, double* work)
{
    int D = t->dim;
    double *c = work, *y = work + D;
    memcpy(c, x, sizeof(double) * (size_t)D);
    double lstar = -INFINITY;
    int s = 0;
    while (s < M) {
        drsym_propose(t, sigma, seed, chain, draw, s, c, y);
        double ly = orc_logpdf(t, y);
        double a = orc_drsym_alpha(*lx, ly, lstar);
        double u = orc_uniform(seed, chain, draw, ORC_ROLE_ACC, (uint32_t)s);
        ++s;
        if (decide(u < a, u - a, 1.0)) {
            memcpy(x, y, sizeof(double) * (size_t)D);
            *lx = ly;
            break;
        }
        if (ly > lstar) lstar = ly;
        memcpy(c, y, sizeof(double) * (size_t)D);
    }
    return s;
}

/* As an FSM: the loop body (one try) is the single PROPOSE state with INIT
 * and DONE bundled into it (Sec. 7.1: they are essentially empty).  One
 * step = one try; returns 1 when the step ends a draw.                    */
typedef struct {
    int s;
    uint32_t t;
    double lx, lstar;
    double *x, *c, *y;
} drsym_fsm;

static int drsym_fsm_step(const orc_target* t, int M, double sigma, uint64_t seed, uint32_t chain,
                          drsym_fsm* f)
{
    int D = t->dim;
    drsym_propose(t, sigma, seed, chain, f->t, f->s, f->c, f->y);
    double ly = orc_logpdf(t, f->y);
    double a = orc_drsym_alpha(f->lx, ly, f->lstar);
    double u = orc_uniform(seed, chain, f->t, ORC_ROLE_ACC, (uint32_t)f->s);
    f->s++;
    int end = 0;
    if (u < a) {
        memcpy(f->x, f->y, sizeof(double) * (size_t)D);
        f->lx = ly;
        end = 1;
    } else if (f->s >= M) {
        end = 1;
    } else {
        if (ly > f->lstar) f->lstar = ly;
        memcpy(f->c, f->y, sizeof(double) * (size_t)D);
    }
    if (end) { /* DONE, then INIT of the next draw */
        memcpy(f->c, f->x, sizeof(double) * (size_t)D);
        f->lstar = -INFINITY;
    }
    return end;
}

/* ------------------------------------------------------------------ */
/* Slice sampling along a random direction (Neal 2003: stepping out and
 * shrinkage, Sec. 4; a random line through x for a multivariate target,
 * Sec. 5.1).  Sec. 3.1's slice panel: S1 INIT E, S2 EXPAND, S3 INIT S,
 * S4 SHRINK, S5 DONE.  Draw t from x:
 *   log y = log pi(x) + ln u;  d = z / |z|;  L = -w u', R = L + w;
 *   while an end is inside the slice (log pi > log y): step out the left end
 *   if it is inside, else the right one, by w;
 *   point x' = x + t d, t uniform on [L, R]; while log pi(x') <= log y:
 *   shrink the side of t (t < 0: L = t, else R = t) and draw again.
 * Loop count N = log-density evaluations (2 + steps out + 1 + shrinks).
 * Guard: a draw stops (x kept) after ORC_ESS_MAX_EVALS evaluations.      */

static double slice_eval(const orc_target* t, const double* x, const double* d, double s, double* xp)
{
    for (int i = 0; i < t->dim; ++i) xp[i] = x[i] + s * d[i];
    return orc_logpdf(t, xp);
}

static void slice_direction(int D, uint64_t seed, uint32_t chain, uint32_t draw, double* d)
{
    orc_normals(seed, chain, draw, ORC_ROLE_NU, 0, D, d);
    double n = 0.0;
    for (int i = 0; i < D; ++i) n += d[i] * d[i];
    n = sqrt(n);
    for (int i = 0; i < D; ++i) d[i] /= n;
}

/* Returns N (> 0), or -N when the guard stopped the draw.  work: 3*D.   */
int orc_slice_sample(const orc_target* t, double w, uint64_t seed, uint32_t chain, uint32_t draw,
                     double* x, double* lx, double* work)
{
    int D = t->dim;
    double *d = work, *xp = work + D, *xb = work + 2 * D;
    double logy = *lx + log(orc_uniform(seed, chain, draw, ORC_ROLE_THRESH, 0));
    slice_direction(D, seed, chain, draw, d);
    double L = -w * orc_uniform(seed, chain, draw, ORC_ROLE_ANGLE, 0), R = L + w;
    double lL = slice_eval(t, x, d, L, xp), lR = slice_eval(t, x, d, R, xp);
    int evals = 2;
    int inL = decide(lL > logy, lL - logy, 1.0 + fabs(lL) + fabs(logy));
    int inR = decide(lR > logy, lR - logy, 1.0 + fabs(lR) + fabs(logy));
    while (inL || inR) {
        if (evals >= ORC_ESS_MAX_EVALS) return -evals;
        if (inL) {
            L -= w;
            lL = slice_eval(t, x, d, L, xp);
            inL = decide(lL > logy, lL - logy, 1.0 + fabs(lL) + fabs(logy));
        } else {
            R += w;
            lR = slice_eval(t, x, d, R, xp);
            inR = decide(lR > logy, lR - logy, 1.0 + fabs(lR) + fabs(logy));
        }
        ++evals;
    }
    for (int s = 0;; ++s) {
        if (evals >= ORC_ESS_MAX_EVALS) return -evals;
        double tt = L + (R - L) * orc_uniform(seed, chain, draw, ORC_ROLE_ANGLE, (uint32_t)(1 + s));
        double lp = slice_eval(t, x, d, tt, xb);
        ++evals;
        if (decide(lp > logy, lp - logy, 1.0 + fabs(lp) + fabs(logy))) {
            memcpy(x, xb, sizeof(double) * (size_t)D);
            *lx = lp;
            return evals;
        }
        if (decide(tt < 0.0, tt, fabs(L) + fabs(R)))
            L = tt;
        else
            R = tt;
    }
}

/* The same draw as an FSM, one block per step (INIT E, EXPAND, INIT S,
 * SHRINK, DONE).                                                          */
enum { SL_INITE = 1, SL_EXPAND = 2, SL_INITS = 3, SL_SHRINK = 4, SL_DONE = 5 };

typedef struct {
    int k, evals, inL, inR, acc, s, guard;
    uint32_t t;
    double lx, logy, L, R, tt, lp;
    double *x, *d, *xp, *xb;
} slice_fsm;

static int slice_fsm_step(const orc_target* t, double w, uint64_t seed, uint32_t chain, slice_fsm* f)
{
    int D = t->dim;
    int is_sample = 0;
    switch (f->k) {
    case SL_INITE: {
        f->logy = f->lx + log(orc_uniform(seed, chain, f->t, ORC_ROLE_THRESH, 0));
        slice_direction(D, seed, chain, f->t, f->d);
        f->L = -w * orc_uniform(seed, chain, f->t, ORC_ROLE_ANGLE, 0);
        f->R = f->L + w;
        f->inL = slice_eval(t, f->x, f->d, f->L, f->xp) > f->logy;
        f->inR = slice_eval(t, f->x, f->d, f->R, f->xp) > f->logy;
        f->evals = 2;
        f->guard = 0;
        f->k = (f->inL || f->inR) ? SL_EXPAND : SL_INITS;
        break;
    }
    case SL_EXPAND:
        if (f->evals >= ORC_ESS_MAX_EVALS) {
            f->guard = 1;
            f->k = SL_DONE;
            break;
        }
        if (f->inL) {
            f->L -= w;
            f->inL = slice_eval(t, f->x, f->d, f->L, f->xp) > f->logy;
        } else {
            f->R += w;
            f->inR = slice_eval(t, f->x, f->d, f->R, f->xp) > f->logy;
        }
        f->evals++;
        f->k = (f->inL || f->inR) ? SL_EXPAND : SL_INITS;
        break;
    case SL_INITS:
    case SL_SHRINK:
        if (f->k == SL_SHRINK) {
            if (f->tt < 0.0)
                f->L = f->tt;
            else
                f->R = f->tt;
            f->s++;
        } else {
            f->s = 0;
        }
        if (f->evals >= ORC_ESS_MAX_EVALS) {
            f->guard = 1;
            f->k = SL_DONE;
            break;
        }
        f->tt = f->L + (f->R - f->L) * orc_uniform(seed, chain, f->t, ORC_ROLE_ANGLE, (uint32_t)(1 + f->s));
        f->lp = slice_eval(t, f->x, f->d, f->tt, f->xb);
        f->evals++;
        f->acc = f->lp > f->logy;
        f->k = f->acc ? SL_DONE : SL_SHRINK;
        break;
    case SL_DONE:
        if (!f->guard) {
            memcpy(f->x, f->xb, sizeof(double) * (size_t)D);
            f->lx = f->lp;
        }
        is_sample = 1;
        f->k = SL_INITE;
        break;
    }
    return is_sample;
}

/* ------------------------------------------------------------------ */
/* No-U-Turn sampler (Hoffman & Gelman 2014) in the iterative two-nested-
 * loop form the paper converts (Sec. 7.3: an outer loop that doubles the
 * trajectory, an inner loop that integrates it while watching for U-turns
 * and divergence).  Reading: multinomial leaf sampling inside a subtree,
 * biased progressive merge of subtrees, generalized U-turn criterion on
 * every aligned sub-span, divergence when H - H0 > 1000; identity mass. */

#define ORC_NUTS_DMAX 1000.0
#define ORC_NUTS_MAXJ 15

static double logaddexp(double a, double b)
{
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    double m = a > b ? a : b;
    return m + log1p(exp(-fabs(a - b)));
}

static double dot(const double* a, const double* b, int D)
{
    double s = 0.0;
    for (int i = 0; i < D; ++i) s += a[i] * b[i];
    return s;
}

/* Workspace of one NUTS chain. */
typedef struct {
    double *thL, *pL, *gL, *thR, *pR, *gR; /* trajectory edges          */
    double *thP, *gP;                      /* tree proposal             */
    double *thS, *gS;                      /* subtree proposal          */
    double *rho, *rhoS;                    /* momentum sums             */
    double *ckp, *ckr;                     /* per-level checkpoints      */
    double *ph;                            /* half-step momentum         */
    double UP, US;
} nuts_ws;

static size_t nuts_ws_len(int D) { return (size_t)D * (13 + 2 * (ORC_NUTS_MAXJ + 1)); }

static void nuts_ws_bind(nuts_ws* w, double* buf, int D)
{
    double* p = buf;
    w->thL = p; p += D; w->pL = p; p += D; w->gL = p; p += D;
    w->thR = p; p += D; w->pR = p; p += D; w->gR = p; p += D;
    w->thP = p; p += D; w->gP = p; p += D;
    w->thS = p; p += D; w->gS = p; p += D;
    w->rho = p; p += D; w->rhoS = p; p += D;
    w->ph = p; p += D;
    w->ckp = p; p += (size_t)D * (ORC_NUTS_MAXJ + 1);
    w->ckr = p;
}

/* One leapfrog step of size v*eps from (th, p, g); th, p, g updated in place.
 * Returns U at the new position.                                          */
double orc_leapfrog(const orc_target* t, double veps, double* th, double* p, double* g,
                    double* ph)
{
    int D = t->dim;
    for (int i = 0; i < D; ++i) ph[i] = p[i] - 0.5 * veps * g[i];
    for (int i = 0; i < D; ++i) th[i] = th[i] + veps * ph[i];
    double U = orc_potential(t, th, g);
    for (int i = 0; i < D; ++i) p[i] = ph[i] - 0.5 * veps * g[i];
    return U;
}

static double abs_dot(const double* a, const double* b, int D)
{
    double s = 0.0;
    for (int i = 0; i < D; ++i) s += fabs(a[i] * b[i]);
    return s;
}

/* Store checkpoints for spans starting at leaf n, then test every aligned
 * span of size 2^k (k >= 1) ending at leaf n.  rhoS already includes p_n.
 * Returns 1 when some span is turning.                                   */
static int nuts_leaf_uturn(int D, int j, uint32_t n, const double* p, const double* rhoS,
                           double* ckp, double* ckr, double* tmp)
{
    for (int k = 1; k <= j; ++k) {
        if ((n & ((1u << k) - 1u)) == 0u) {
            memcpy(ckp + (size_t)k * D, p, sizeof(double) * (size_t)D);
            for (int i = 0; i < D; ++i) ckr[(size_t)k * D + i] = rhoS[i] - p[i];
        }
    }
    int turn = 0;
    for (int k = 1; k <= j; ++k) {
        if (((n + 1u) & ((1u << k) - 1u)) == 0u) {
            for (int i = 0; i < D; ++i) tmp[i] = rhoS[i] - ckr[(size_t)k * D + i];
            double d0 = dot(ckp + (size_t)k * D, tmp, D), d1 = dot(p, tmp, D);
            int t0 = decide(d0 <= 0.0, d0, g_trace ? abs_dot(ckp + (size_t)k * D, tmp, D) : 0.0);
            int t1 = decide(d1 <= 0.0, d1, g_trace ? abs_dot(p, tmp, D) : 0.0);
            if (t0 || t1) turn = 1;
        }
    }
    return turn;
}

/* Exposed for the test of the checkpoint bookkeeping: given the momenta of
 * the 2^j leaves of one subtree (in integration order, row-major), return
 * the first leaf index at which a span turns, or 2^j if none does.      */
int orc_nuts_subtree_first_turn(int D, int j, const double* moms)
{
    double* buf = (double*)calloc((size_t)D * (3 + 2 * (ORC_NUTS_MAXJ + 1)), sizeof(double));
    double *rho = buf, *tmp = buf + D, *ckp = buf + 2 * D, *ckr = ckp + (size_t)D * (ORC_NUTS_MAXJ + 1);
    uint32_t leaves = 1u << j;
    uint32_t n;
    for (n = 0; n < leaves; ++n) {
        const double* p = moms + (size_t)n * D;
        for (int i = 0; i < D; ++i) rho[i] += p[i];
        if (nuts_leaf_uturn(D, j, n, p, rho, ckp, ckr, tmp)) break;
    }
    free(buf);
    return (int)n;
}

/* Per-draw diagnostics of NUTS. */
typedef struct {
    int32_t n_leapfrog;
    int32_t depth;     /* number of subtrees built */
    int32_t diverged;
    int32_t turned;
    double accept;     /* sum over the draw's leapfrogs of min(1, exp(H0 - H)),
                          a divergent or undefined energy counting 0: the
                          acceptance statistic that step-size adaptation
                          targets (Hoffman & Gelman 2014, Sec. 3.2)       */
} orc_nuts_info;

/* One NUTS draw as nested while loops.  th, U, g: current state (g = grad U
 * at th), updated in place.  ws: nuts_ws_len(D) doubles.                */
int orc_nuts_sample(const orc_target* t, double eps, int max_depth, uint64_t seed,
                    uint32_t chain, uint32_t draw, double* th, double* U, double* g, double* wsbuf,
                    orc_nuts_info* info)
{
    int D = t->dim;
    nuts_ws w;
    nuts_ws_bind(&w, wsbuf, D);
    double* tmp = w.ph; /* ph is dead between leapfrogs */

    /* INIT */
    orc_normals(seed, chain, draw, ORC_ROLE_MOM, 0, D, w.pL);
    double H0 = *U + 0.5 * dot(w.pL, w.pL, D);
    memcpy(w.pR, w.pL, sizeof(double) * D);
    memcpy(w.rho, w.pL, sizeof(double) * D);
    memcpy(w.thL, th, sizeof(double) * D);
    memcpy(w.thR, th, sizeof(double) * D);
    memcpy(w.gL, g, sizeof(double) * D);
    memcpy(w.gR, g, sizeof(double) * D);
    memcpy(w.thP, th, sizeof(double) * D);
    memcpy(w.gP, g, sizeof(double) * D);
    w.UP = *U;
    double W = 0.0, acc = 0.0;
    int j = 0, stop = 0, nleap = 0, diverged = 0, turned = 0;

    while (!stop && j < max_depth) {
        /* DOUBLE */
        int v = (orc_uniform(seed, chain, draw, ORC_ROLE_DIR, (uint32_t)j) < 0.5) ? 1 : -1;
        double *the = v > 0 ? w.thR : w.thL, *pe = v > 0 ? w.pR : w.pL, *ge = v > 0 ? w.gR : w.gL;
        double Ws = -INFINITY;
        memset(w.rhoS, 0, sizeof(double) * D);
        uint32_t n = 0, leaves = 1u << j;
        int invalid = 0;
        while (!invalid && n < leaves) {
            /* INTEGRATE: one leapfrog, leaf bookkeeping, U-turn checks */
            double Un = orc_leapfrog(t, v * eps, the, pe, ge, w.ph);
            ++nleap;
            double wn = H0 - (Un + 0.5 * dot(pe, pe, D));
            if (wn >= 0.0)
                acc += 1.0;
            else if (wn > -INFINITY)
                acc += exp(wn);
            const double escale = fabs(H0) + fabs(Un) + 0.5 * dot(pe, pe, D);
            if (decide(!(-wn <= ORC_NUTS_DMAX), -wn - ORC_NUTS_DMAX, escale)) {
                invalid = 1;
                diverged = 1;
                break;
            }
            double Wn = logaddexp(Ws, wn);
            double lu = log(orc_uniform(seed, chain, draw, ORC_ROLE_LEAF, ((uint32_t)j << 16) | n));
            /* the first leaf of a subtree is always taken (wn - Wn = 0 > lu):
             * not a decision that rounding can invert, so it is not recorded */
            if (n == 0 ? (lu < wn - Wn) : decide(lu < wn - Wn, lu - (wn - Wn), escale)) {
                memcpy(w.thS, the, sizeof(double) * D);
                memcpy(w.gS, ge, sizeof(double) * D);
                w.US = Un;
            }
            Ws = Wn;
            for (int i = 0; i < D; ++i) w.rhoS[i] += pe[i];
            if (nuts_leaf_uturn(D, j, n, pe, w.rhoS, w.ckp, w.ckr, tmp)) {
                invalid = 1;
                turned = 1;
                break;
            }
            ++n;
        }
        /* CHECK */
        if (invalid) {
            stop = 1;
        } else {
            double lu = log(orc_uniform(seed, chain, draw, ORC_ROLE_MERGE, (uint32_t)j));
            if (decide(lu < Ws - W, lu - (Ws - W), fabs(H0) + 1.0)) {
                memcpy(w.thP, w.thS, sizeof(double) * D);
                memcpy(w.gP, w.gS, sizeof(double) * D);
                w.UP = w.US;
            }
            W = logaddexp(W, Ws);
            for (int i = 0; i < D; ++i) w.rho[i] += w.rhoS[i];
            double dl = dot(w.pL, w.rho, D), dr = dot(w.pR, w.rho, D);
            int tl = decide(dl <= 0.0, dl, g_trace ? abs_dot(w.pL, w.rho, D) : 0.0);
            int tr = decide(dr <= 0.0, dr, g_trace ? abs_dot(w.pR, w.rho, D) : 0.0);
            if (tl || tr) {
                stop = 1;
                turned = 1;
            }
        }
        ++j;
    }
    /* DONE */
    memcpy(th, w.thP, sizeof(double) * D);
    memcpy(g, w.gP, sizeof(double) * D);
    *U = w.UP;
    if (info) {
        info->n_leapfrog = nleap;
        info->depth = j;
        info->diverged = diverged;
        info->turned = turned;
        info->accept = acc;
    }
    return nleap;
}

/* NUTS as an FSM: S1 INIT, S2 DOUBLE, S3 INTEGRATE, S4 CHECK, S5 DONE
 * (Fig. "Finite state machines ...", HMC-NUTS panel; Appendix, nested
 * while-loop construction).                                              */
enum { NUTS_INIT = 1, NUTS_DOUBLE = 2, NUTS_INTEGRATE = 3, NUTS_CHECK = 4, NUTS_DONE = 5 };

typedef struct {
    int k;
    uint32_t t;
    int j, v, stop, invalid, nleap, diverged, turned;
    uint32_t n;
    double H0, W, Ws, U;
    double *th, *g;
    nuts_ws w;
} nuts_fsm;

static int nuts_fsm_step(const orc_target* t, double eps, int max_depth, uint64_t seed,
                         uint32_t chain, nuts_fsm* f)
{
    int D = t->dim;
    nuts_ws* w = &f->w;
    int is_sample = (f->k == NUTS_DONE);
    switch (f->k) {
    case NUTS_INIT:
        orc_normals(seed, chain, f->t, ORC_ROLE_MOM, 0, D, w->pL);
        f->H0 = f->U + 0.5 * dot(w->pL, w->pL, D);
        memcpy(w->pR, w->pL, sizeof(double) * D);
        memcpy(w->rho, w->pL, sizeof(double) * D);
        memcpy(w->thL, f->th, sizeof(double) * D);
        memcpy(w->thR, f->th, sizeof(double) * D);
        memcpy(w->gL, f->g, sizeof(double) * D);
        memcpy(w->gR, f->g, sizeof(double) * D);
        memcpy(w->thP, f->th, sizeof(double) * D);
        memcpy(w->gP, f->g, sizeof(double) * D);
        w->UP = f->U;
        f->W = 0.0;
        f->j = 0;
        f->stop = 0;
        f->nleap = 0;
        f->diverged = 0;
        f->turned = 0;
        break;
    case NUTS_DOUBLE:
        f->v = (orc_uniform(seed, chain, f->t, ORC_ROLE_DIR, (uint32_t)f->j) < 0.5) ? 1 : -1;
        f->Ws = -INFINITY;
        memset(w->rhoS, 0, sizeof(double) * D);
        f->n = 0;
        f->invalid = 0;
        break;
    case NUTS_INTEGRATE: {
        double *the = f->v > 0 ? w->thR : w->thL, *pe = f->v > 0 ? w->pR : w->pL;
        double* ge = f->v > 0 ? w->gR : w->gL;
        double Un = orc_leapfrog(t, f->v * eps, the, pe, ge, w->ph);
        f->nleap++;
        double wn = f->H0 - (Un + 0.5 * dot(pe, pe, D));
        if (!(-wn <= ORC_NUTS_DMAX)) {
            f->invalid = 1;
            f->diverged = 1;
            break;
        }
        double Wn = logaddexp(f->Ws, wn);
        if (log(orc_uniform(seed, chain, f->t, ORC_ROLE_LEAF, ((uint32_t)f->j << 16) | f->n)) <
            wn - Wn) {
            memcpy(w->thS, the, sizeof(double) * D);
            memcpy(w->gS, ge, sizeof(double) * D);
            w->US = Un;
        }
        f->Ws = Wn;
        for (int i = 0; i < D; ++i) w->rhoS[i] += pe[i];
        if (nuts_leaf_uturn(D, f->j, f->n, pe, w->rhoS, w->ckp, w->ckr, w->ph)) {
            f->invalid = 1;
            f->turned = 1;
            break;
        }
        f->n++;
        break;
    }
    case NUTS_CHECK:
        if (f->invalid) {
            f->stop = 1;
        } else {
            if (log(orc_uniform(seed, chain, f->t, ORC_ROLE_MERGE, (uint32_t)f->j)) < f->Ws - f->W) {
                memcpy(w->thP, w->thS, sizeof(double) * D);
                memcpy(w->gP, w->gS, sizeof(double) * D);
                w->UP = w->US;
            }
            f->W = logaddexp(f->W, f->Ws);
            for (int i = 0; i < D; ++i) w->rho[i] += w->rhoS[i];
            if (dot(w->pL, w->rho, D) <= 0.0 || dot(w->pR, w->rho, D) <= 0.0) {
                f->stop = 1;
                f->turned = 1;
            }
        }
        f->j++;
        break;
    case NUTS_DONE:
        memcpy(f->th, w->thP, sizeof(double) * D);
        memcpy(f->g, w->gP, sizeof(double) * D);
        f->U = w->UP;
        break;
    }
    /* delta: the outer loop condition after INIT and CHECK, the inner loop
     * condition after DOUBLE and INTEGRATE.                              */
    switch (f->k) {
    case NUTS_INIT:
    case NUTS_CHECK:
        f->k = (!f->stop && f->j < max_depth) ? NUTS_DOUBLE : NUTS_DONE;
        break;
    case NUTS_DOUBLE:
    case NUTS_INTEGRATE:
        f->k = (!f->invalid && f->n < (1u << f->j)) ? NUTS_INTEGRATE : NUTS_CHECK;
        break;
    case NUTS_DONE:
        f->k = NUTS_INIT;
        break;
    }
    return is_sample;
}

/* ------------------------------------------------------------------ */
/* Chain runners: Alg. "MCMC algorithm with sample function" (use_fsm = 0)
 * or Alg. "FSM MCMC algorithm" (use_fsm = 1).                          */
enum { ORC_ESS = 0, ORC_NUTS = 1, ORC_DRMH = 2, ORC_DRSYM = 3, ORC_SLICE = 4 };

typedef struct {
    int32_t kind;
    int32_t max_depth;
    int32_t n_stages;
    int32_t pad_;
    double step_size;
    double scales[4];
    const double* chol_L; /* ESS: D x D lower Cholesky factor of the prior covariance */
} orc_sampler;

/*
 * Run one chain for n draws.
 *   x0:     initial state (dim) or NULL for the default initialisation.
 *   out:    n x dim draws (row-major).
 *   counts: n loop counts N_t (ESS: log-likelihood evaluations; NUTS:
 *           leapfrog steps; DR: stages evaluated), may be NULL.
 *   edges:  (K+1) x (K+1) counts of observed FSM transitions k -> k'
 *           (FSM mode only), may be NULL.
 *   steps:  total FSM steps taken (FSM mode only), may be NULL.
 * Returns 0, or -1 on a bad argument, or the number of guard trips (> 0).
 */
int orc_run_chain(const orc_target* t, const orc_sampler* sp, uint64_t seed, uint32_t chain,
                  int n, const double* x0, double* out, int32_t* counts, int use_fsm,
                  int64_t* edges, int64_t* steps)
{
    int D = t->dim;
    if (D <= 0 || n < 0 || !out) return -1;
    int guards = 0;
    int64_t nsteps = 0;
    if (sp->kind == ORC_ESS) {
        double* buf = (double*)malloc(sizeof(double) * (size_t)D * 5);
        double *x = buf, *work = buf + D, *z = buf + 4 * D;
        if (x0)
            memcpy(x, x0, sizeof(double) * D);
        else
            orc_ess_init(sp->chol_L, D, seed, chain, x, z);
        double lx = orc_gp_loglik(t, x);
        if (!use_fsm) {
            for (int i = 0; i < n; ++i) {
                int e = orc_ess_sample(t, sp->chol_L, seed, chain, (uint32_t)i, x, &lx, work);
                if (e < 0) {
                    ++guards;
                    e = -e;
                }
                if (counts) counts[i] = e;
                memcpy(out + (size_t)i * D, x, sizeof(double) * D);
            }
        } else {
            ess_fsm f;
            memset(&f, 0, sizeof(f));
            f.k = ESS_INIT;
            f.t = 0;
            f.x = x;
            f.nu = work;
            f.xp = work + D;
            f.z = work + 2 * D;
            f.lx = lx;
            int guard = 0;
            while ((int)f.t < n) {
                int k0 = f.k;
                int is_sample = ess_fsm_step(t, sp->chol_L, seed, chain, &f, &guard);
                ++nsteps;
                if (edges) edges[k0 * 4 + f.k]++;
                if (is_sample) {
                    if (counts) counts[f.t] = f.evals;
                    if (guard) ++guards;
                    guard = 0;
                    memcpy(out + (size_t)f.t * D, f.x, sizeof(double) * D);
                    f.t++;
                }
            }
        }
        free(buf);
    } else if (sp->kind == ORC_DRMH) {
        double* buf = (double*)malloc(sizeof(double) * (size_t)D * 4);
        double *x = buf, *work = buf + D;
        if (x0)
            memcpy(x, x0, sizeof(double) * D);
        else if (t->kind == ORC_FUNNEL)
            orc_funnel_init(D, seed, chain, x);
        else
            orc_normal_init(D, seed, chain, x);
        double lx = orc_logpdf(t, x);
        if (!use_fsm) {
            for (int i = 0; i < n; ++i) {
                int s = orc_dr_sample(t, sp->n_stages, sp->scales, seed, chain, (uint32_t)i, x, &lx, work);
                if (counts) counts[i] = s;
                memcpy(out + (size_t)i * D, x, sizeof(double) * D);
            }
        } else {
            dr_fsm f;
            memset(&f, 0, sizeof(f));
            f.k = DR_INIT;
            f.t = 0;
            f.x = x;
            f.lx = lx;
            f.y[0] = work;
            f.y[1] = work + D;
            f.y[2] = work + 2 * D;
            while ((int)f.t < n) {
                int k0 = f.k;
                int is_sample = dr_fsm_step(t, sp->n_stages, sp->scales, seed, chain, &f);
                ++nsteps;
                if (edges) edges[k0 * 4 + f.k]++;
                if (is_sample) {
                    if (counts) counts[f.t] = f.s;
                    memcpy(out + (size_t)f.t * D, f.x, sizeof(double) * D);
                    f.t++;
                }
            }
        }
        free(buf);
    } else if (sp->kind == ORC_SLICE) {
        /* scales[0] = w, the stepping-out width */
        if (!(sp->scales[0] > 0.0)) return -1;
        double* buf = (double*)malloc(sizeof(double) * (size_t)D * 4);
        double *x = buf, *work = buf + D;
        if (x0)
            memcpy(x, x0, sizeof(double) * D);
        else if (t->kind == ORC_FUNNEL)
            orc_funnel_init(D, seed, chain, x);
        else
            orc_normal_init(D, seed, chain, x);
        double lx = orc_logpdf(t, x);
        if (!use_fsm) {
            for (int i = 0; i < n; ++i) {
                int s = orc_slice_sample(t, sp->scales[0], seed, chain, (uint32_t)i, x, &lx, work);
                if (s < 0) {
                    ++guards;
                    s = -s;
                }
                if (counts) counts[i] = s;
                memcpy(out + (size_t)i * D, x, sizeof(double) * D);
            }
        } else {
            slice_fsm f;
            memset(&f, 0, sizeof(f));
            f.k = SL_INITE;
            f.lx = lx;
            f.x = x;
            f.d = work;
            f.xp = work + D;
            f.xb = work + 2 * D;
            while ((int)f.t < n) {
                int k0 = f.k;
                int is_sample = slice_fsm_step(t, sp->scales[0], seed, chain, &f);
                ++nsteps;
                if (edges) edges[k0 * 6 + f.k]++;
                if (is_sample) {
                    if (f.guard) ++guards;
                    if (counts) counts[f.t] = f.evals;
                    memcpy(out + (size_t)f.t * D, f.x, sizeof(double) * D);
                    f.t++;
                }
            }
        }
        free(buf);
    } else if (sp->kind == ORC_DRSYM) {
        /* n_stages = M tries, scales[0] = sigma */
        if (sp->n_stages < 1) return -1;
        double* buf = (double*)malloc(sizeof(double) * (size_t)D * 3);
        double *x = buf, *work = buf + D;
        if (x0)
            memcpy(x, x0, sizeof(double) * D);
        else if (t->kind == ORC_FUNNEL)
            orc_funnel_init(D, seed, chain, x);
        else
            orc_normal_init(D, seed, chain, x);
        double lx = orc_logpdf(t, x);
        if (!use_fsm) {
            for (int i = 0; i < n; ++i) {
                int s = orc_drsym_sample(t, sp->n_stages, sp->scales[0], seed, chain, (uint32_t)i, x, &lx,
                                         work);
                if (counts) counts[i] = s;
                memcpy(out + (size_t)i * D, x, sizeof(double) * D);
            }
        } else {
            drsym_fsm f;
            f.s = 0;
            f.t = 0;
            f.lx = lx;
            f.lstar = -INFINITY;
            f.x = x;
            f.c = work;
            f.y = work + D;
            memcpy(f.c, x, sizeof(double) * D);
            while ((int)f.t < n) {
                int is_sample = drsym_fsm_step(t, sp->n_stages, sp->scales[0], seed, chain, &f);
                ++nsteps;
                if (edges) edges[2 * 4 + 2]++; /* PROPOSE -> PROPOSE (INIT and DONE bundled) */
                if (is_sample) {
                    if (counts) counts[f.t] = f.s;
                    memcpy(out + (size_t)f.t * D, f.x, sizeof(double) * D);
                    f.t++;
                    f.s = 0;
                }
            }
        }
        free(buf);
    } else if (sp->kind == ORC_NUTS) {
        if (sp->max_depth < 1 || sp->max_depth > ORC_NUTS_MAXJ) return -1;
        double* buf = (double*)malloc(sizeof(double) * ((size_t)D * 2 + nuts_ws_len(D)));
        double *th = buf, *g = buf + D, *wsb = buf + 2 * D;
        if (x0)
            memcpy(th, x0, sizeof(double) * D);
        else if (t->kind == ORC_FUNNEL)
            orc_funnel_init(D, seed, chain, th);
        else
            orc_normal_init(D, seed, chain, th);
        double U = orc_potential(t, th, g);
        if (!use_fsm) {
            for (int i = 0; i < n; ++i) {
                orc_nuts_info info;
                orc_nuts_sample(t, sp->step_size, sp->max_depth, seed, chain, (uint32_t)i, th, &U, g,
                                wsb, &info);
                if (counts) counts[i] = info.n_leapfrog;
                memcpy(out + (size_t)i * D, th, sizeof(double) * D);
            }
        } else {
            nuts_fsm f;
            memset(&f, 0, sizeof(f));
            f.k = NUTS_INIT;
            f.th = th;
            f.g = g;
            f.U = U;
            nuts_ws_bind(&f.w, wsb, D);
            while ((int)f.t < n) {
                int k0 = f.k;
                int is_sample = nuts_fsm_step(t, sp->step_size, sp->max_depth, seed, chain, &f);
                ++nsteps;
                if (edges) edges[k0 * 6 + f.k]++;
                if (is_sample) {
                    if (counts) counts[f.t] = f.nleap;
                    memcpy(out + (size_t)f.t * D, f.th, sizeof(double) * D);
                    f.t++;
                }
            }
        }
        free(buf);
    } else {
        return -1;
    }
    if (steps) *steps = nsteps;
    return guards;
}

/*
 * One draw of any sampler from the state x (in/out), with its branch
 * decisions recorded into (margin, scale) arrays of capacity cap and, if
 * flip_at >= 0, decision number flip_at inverted.  The cached quantities
 * (log L(x), or U and grad U) are recomputed from x.  Returns the loop count
 * of the draw (ESS: evaluations, negative if the guard tripped; NUTS:
 * leapfrogs; DR: stages), or 0 on a bad argument; *n_dec is the number of
 * decisions taken.
 */
int orc_draw_traced(const orc_target* t, const orc_sampler* sp, uint64_t seed, uint32_t chain,
                    uint32_t draw, double* x, double* margin, double* scale, int32_t cap,
                    int32_t* n_dec, int32_t flip_at)
{
    int D = t->dim;
    if (D <= 0) return 0;
    orc_trace tr = {margin, scale, cap, 0, flip_at};
    int r = 0;
    g_trace = &tr;
    if (sp->kind == ORC_ESS) {
        double* work = (double*)calloc((size_t)D * 3, sizeof(double));
        double lx = orc_gp_loglik(t, x);
        r = orc_ess_sample(t, sp->chol_L, seed, chain, draw, x, &lx, work);
        free(work);
    } else if (sp->kind == ORC_DRMH) {
        double* work = (double*)calloc((size_t)D * 3, sizeof(double));
        double lx = orc_logpdf(t, x);
        r = orc_dr_sample(t, sp->n_stages, sp->scales, seed, chain, draw, x, &lx, work);
        free(work);
    } else if (sp->kind == ORC_SLICE && sp->scales[0] > 0.0) {
        double* work = (double*)calloc((size_t)D * 3, sizeof(double));
        double lx = orc_logpdf(t, x);
        r = orc_slice_sample(t, sp->scales[0], seed, chain, draw, x, &lx, work);
        if (r < 0) r = -r;
        free(work);
    } else if (sp->kind == ORC_DRSYM && sp->n_stages >= 1) {
        double* work = (double*)calloc((size_t)D * 2, sizeof(double));
        double lx = orc_logpdf(t, x);
        r = orc_drsym_sample(t, sp->n_stages, sp->scales[0], seed, chain, draw, x, &lx, work);
        free(work);
    } else if (sp->kind == ORC_NUTS && sp->max_depth >= 1 && sp->max_depth <= ORC_NUTS_MAXJ) {
        /* zeroed: a replay with an inverted decision may read a slot that the
         * uninverted draw always writes first */
        double* buf = (double*)calloc((size_t)D + nuts_ws_len(D), sizeof(double));
        double *g = buf, *wsb = buf + D;
        double U = orc_potential(t, x, g);
        orc_nuts_info info;
        r = orc_nuts_sample(t, sp->step_size, sp->max_depth, seed, chain, draw, x, &U, g, wsb, &info);
        free(buf);
    }
    g_trace = NULL;
    *n_dec = tr.n;
    return r;
}
