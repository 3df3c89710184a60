/*
 * ns_oracle.c -- plain, slow, FP64 reference implementation of gradient-guided
 * nested sampling (GGNS) with the batched Hamiltonian slice sampling (HSS) walk.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file.  The GPU engine shares no code,
 * header, table or constant with it; both sides only read the same seeded
 * inputs (positions, likelihood parameters, run settings and the 64-bit seed)
 * and each implements the two published random-number generators on its own.
 *
 * What it follows (paper: Lemos et al., "Improving Gradient-guided Nested
 * Sampling for Posterior Inference", arXiv:2312.03911):
 *   - Appendix A, Algorithm "simple nested sampling" and Eqs. (cum_prior_mass),
 *     (ns_sum), (delta_x), (importance_weight), (shell_volume): kill the lowest
 *     point, add X*L/(n+1) to Z, shrink X by n/(n+1).
 *   - Appendix H, Algorithm "GGNS": kill n_live//2 per iteration, start walkers
 *     from surviving live points, run the HSS walk, adapt dt from out_frac
 *     (x0.9 above 0.15, x1.1 below 0.05), add the new points, final sweep.
 *   - Appendix H, Algorithm "GGNS HSS": drift x += p dt, evaluate L and grad L,
 *     mark points outside the slice, reflect p -= 2 (p.n) n with n the unit
 *     gradient, multiply p by (1 + delta_p * eps), count reflections, keep
 *     in-slice points after min_ref reflections, return a uniform pick and the
 *     fraction of outside steps.
 *   - Section 2.3, Eq. (reflection) and the outside-point scheme; Section 3
 *     (adaptive dt, trajectory preservation, pruning, parallel evolution,
 *     termination); Appendix C table of defaults.
 *   - Appendix H, Eqs. (ini0)-(ini11) and (update0)-(update9), single cluster:
 *     the moments Zbar, Z2bar, ZXbar, Xbar, X2bar, updated one killed point at
 *     a time with n_p decreasing while the batch is removed.
 *   - Section 2.1, Eq. (logZ_error): sigma(log Z) ~ sqrt(D_KL / n_live).
 *
 * Readings where the paper is silent or garbled (each one is also taken by the
 * GPU engine):
 *   R1  k walkers per iteration (default n_live//2); starts drawn uniformly,
 *       with replacement, from the survivors listed in ascending slot order.
 *   R2  L* is the largest killed log-likelihood; a point is outside the slice
 *       when log L <= L* (strict constraint), compared in FP64.
 *   R3  kill order: ascending (log L, slot index).
 *   R4  the reflection normal is taken at the current (outside) position.
 *   R5  a zero or non-finite gradient reflects p -> -p.
 *   R6  leaving the prior box counts as outside and takes precedence; the
 *       momentum component of every violated axis is negated.
 *   R7  the noise eps of p *= (1 + delta_p eps): one normal per walker and
 *       step scaling all components alike (noise_mode 1, the default; two
 *       words of the walker's first block stream per step, the first normal
 *       of their Box-Muller pair); per component
 *       (noise_mode 0); or, as an option that is not the paper's formula, an
 *       isotropic vector p += delta_p (|p| / sqrt d) eps (noise_mode 2).
 *       Applied to every walker at every step, after any reflection.
 *   R8  a point is saved when it is inside the slice and the batch minimum
 *       of num_reflections has reached min_ref (save_mode 1, the algorithm's
 *       condition with its "<" read as ">=", as the text of Section 3 and the
 *       Appendix C table say); save_mode 0 uses the walker's own count.
 *   R9  x_saved is sampled per walker: one uniform pick from the walker's
 *       own saved points by a size-one reservoir (Vitter's Algorithm R;
 *       draw_mode 0, the default), or the batch's saved points are pooled and
 *       k points drawn uniformly with replacement (draw_mode 1).
 *   R10 empty saved set: output the last in-slice point, else the start point.
 *   R11 the walk loops while the batch minimum of num_reflections is below
 *       max_ref (stop_mode 1, the algorithm's loop condition), for at most
 *       n_steps_max steps; stop_mode 0 stops each walker at its own max_ref
 *       (the Appendix C wording); max_ref = 0 selects a fixed number of steps
 *       (n_steps_max) for every walker.
 *   R12 pruning: prune_streak consecutive outside steps reset the walker to its
 *       start point with fresh momentum; the reflection count is kept under
 *       the batch-minimum loop (it never decreases) and restarts from zero
 *       when each walker stops on its own.
 *   R13 one dt per run, updated once per iteration from that run's out_frac.
 *   R14 dt_init is in units of the prior width.
 *   R16 batch kill with n_p = n, n-1, ..., n-k+1 (the Xbar convention).
 *   R17 final sweep with n_p = n, ..., 1.
 *   R18 termination: remaining-evidence test Xbar * max L < tol * Zbar, or the
 *       X*L peak test of the paper (skipped at the first iteration) in one of
 *       its two forms: L the largest live likelihood (Algorithm GGNS, loop
 *       end), or L the likelihood of the current dead point, read as the
 *       highest point killed in the previous iteration, with the volume left
 *       after that kill (the tol entry of the Appendix C table).
 *   R19 sigma_mom^2 = log Z2bar - 2 log Zbar from the moment recursion, every
 *       right-hand side using pre-update values and X2bar initialised to 1.
 *   R22 random streams: Philox4x32-10 (counter based) for prior draws, start
 *       indices, initial and pruning momenta and for seeding; xoshiro128++ per
 *       (walker, block of four coordinates) for the per-step noise and one per
 *       walker for the reservoir; Box-Muller normals from 24-bit uniforms.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Random numbers (reading R22).                                       */
/* ------------------------------------------------------------------ */

/* Philox4x32 with 10 rounds, as defined by Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3" (SC'11): each round multiplies
 * words 0 and 2 by two fixed odd constants, swaps the high/low halves across
 * the lanes and xors in the key; the key is bumped by two Weyl constants
 * between rounds. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

enum { TAG_INIT = 1, TAG_START = 2, TAG_P0 = 3, TAG_EPS = 4, TAG_RES = 5 };

static void stream_draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                        uint32_t tag, uint32_t sub, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, (tag << 24) | (sub & 0xFFFFFFu)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox(ctr, key, out);
}

/* xoshiro128++ of Blackman and Vigna, "Scrambled linear pseudorandom number
 * generators" (2018): output rotl(s0 + s3, 7) + s0, then the xor-shift state
 * update with shift 9 and rotation 11. */
static inline uint32_t rotl32(uint32_t v, int k) { return (v << k) | (v >> (32 - k)); }

uint32_t orc_xoshiro_next(uint32_t s[4])
{
    uint32_t result = rotl32(s[0] + s[3], 7) + s[0];
    uint32_t t = s[1] << 9;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl32(s[3], 11);
    return result;
}

static void xoshiro_seed(uint32_t s[4], const uint32_t w[4])
{
    s[0] = w[0]; s[1] = w[1]; s[2] = w[2]; s[3] = w[3];
    if ((s[0] | s[1] | s[2] | s[3]) == 0u) s[0] = 1u;   /* the all-zero state is a fixed point */
}

/* Uniforms from the top 24 bits: open interval for the logarithm, half-open
 * for the angle. */
static inline double u24_open(uint32_t a) { return ((double)(a >> 8) + 0.5) * (1.0 / 16777216.0); }
static inline double u24_half(uint32_t a) { return (double)(a >> 8) * (1.0 / 16777216.0); }

/* Box-Muller: four 32-bit words give four standard normals. */
void orc_box_muller4(const uint32_t w[4], double z[4])
{
    for (int pair = 0; pair < 2; ++pair) {
        double u1 = u24_open(w[2 * pair]);
        double u2 = u24_half(w[2 * pair + 1]);
        double r = sqrt(-2.0 * log(u1));
        double ang = 2.0 * M_PI * u2;
        z[2 * pair] = r * cos(ang);
        z[2 * pair + 1] = r * sin(ang);
    }
}

/* d standard normals for one walker from the counter-based stream `tag`. */
static void normals_philox(uint64_t seed, uint32_t walker, uint32_t iter, uint32_t tag,
                           uint32_t sub, int d, double *z)
{
    for (int b = 0; 4 * b < d; ++b) {
        uint32_t w[4];
        double zz[4];
        stream_draw(seed, (uint32_t)b, walker, iter, tag, sub, w);
        orc_box_muller4(w, zz);
        for (int j = 0; j < 4 && 4 * b + j < d; ++j) z[4 * b + j] = zz[j];
    }
}

/* ------------------------------------------------------------------ */
/* Likelihoods (FP64).  All are normalised densities in theta, so log Z  */
/* under the uniform box prior has a closed form.                        */
/* ------------------------------------------------------------------ */

enum { LIK_GAUSS_DIAG = 0, LIK_GAUSS_FULL = 1, LIK_SHELLS = 2, LIK_GMM_DIAG = 3, LIK_TORUS = 4 };

static double logaddexp(double a, double b)
{
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    double m = a > b ? a : b;
    return m + log(exp(a - m) + exp(b - m));
}

/* Round to bfloat16 (round to nearest, ties to even) after rounding to FP32:
 * the operand rounding of a BF16 matrix-core product. */
static double round_bf16(double v)
{
    float f = (float)v;
    uint32_t bits;
    memcpy(&bits, &f, 4);
    uint32_t lsb = (bits >> 16) & 1u;
    bits += 0x7FFFu + lsb;
    bits &= 0xFFFF0000u;
    memcpy(&f, &bits, 4);
    return (double)f;
}

/* Parameter blocks (raw, FP64):
 *   GAUSS_DIAG: mu[d], sigma[d]
 *   GAUSS_FULL: mu[d], P[d*d] (precision, row-major), log det P
 *   SHELLS:     K times { c[d], r, w }
 *   GMM_DIAG:   K times { mu[d], sigma[d] }, equal weights 1/K
 *   TORUS:      alpha, beta, c: the reward of Eq. (torus),
 *               L = (sum_{i even} sin(alpha x_i) + sum_{j odd} cos(beta x_j) + c)^3
 *               with the paper's 1-based indices i, j = 1 .. d (x[i-1] in C)
 * Writes log L to *logl and grad log L to g[d] (when g is not NULL). */
int orc_loglike(int kind, int n_comp, const double *prm, int d, const double *x,
                double *logl, double *g, int bf16)
{
    const double log2pi = log(2.0 * M_PI);
    if (kind == LIK_GAUSS_DIAG) {
        const double *mu = prm, *sg = prm + d;
        double l = 0.0;
        for (int a = 0; a < d; ++a) {
            double r = x[a] - mu[a];
            double iv = 1.0 / (sg[a] * sg[a]);
            l += -0.5 * (log2pi + 2.0 * log(sg[a])) - 0.5 * r * r * iv;
            if (g) g[a] = -r * iv;
        }
        *logl = l;
        return 0;
    }
    if (kind == LIK_GAUSS_FULL) {
        const double *mu = prm, *P = prm + d;
        double logdet = prm[d + (int64_t)d * d];
        double *r = (double *)malloc(sizeof(double) * d);
        double *rr = (double *)malloc(sizeof(double) * d);
        for (int a = 0; a < d; ++a) {
            r[a] = x[a] - mu[a];
            rr[a] = bf16 ? round_bf16(r[a]) : r[a];
        }
        double q = 0.0;
        for (int i = 0; i < d; ++i) {
            double y = 0.0;
            for (int j = 0; j < d; ++j) {
                double pij = P[(int64_t)i * d + j];
                if (bf16) pij = round_bf16(pij);
                y += pij * rr[j];
            }
            q += r[i] * y;
            if (g) g[i] = -y;
        }
        *logl = -0.5 * d * log2pi + 0.5 * logdet - 0.5 * q;
        free(r);
        free(rr);
        return 0;
    }
    if (kind == LIK_SHELLS) {
        int K = n_comp;
        double lp[64], rho[64];
        if (K > 64) return -1;
        double l = -INFINITY;
        for (int k = 0; k < K; ++k) {
            const double *c = prm + (int64_t)k * (d + 2);
            double rad = c[d], w = c[d + 1];
            double s = 0.0;
            for (int a = 0; a < d; ++a) s += (x[a] - c[a]) * (x[a] - c[a]);
            rho[k] = sqrt(s);
            double e = rho[k] - rad;
            lp[k] = -0.5 * (log2pi + 2.0 * log(w)) - 0.5 * e * e / (w * w);
            l = logaddexp(l, lp[k]);
        }
        *logl = l;
        if (g) {
            for (int a = 0; a < d; ++a) g[a] = 0.0;
            for (int k = 0; k < K; ++k) {
                const double *c = prm + (int64_t)k * (d + 2);
                double rad = c[d], w = c[d + 1];
                if (!(rho[k] > 0.0)) continue;
                double resp = exp(lp[k] - l);
                double coef = -resp * (rho[k] - rad) / (w * w) / rho[k];
                for (int a = 0; a < d; ++a) g[a] += coef * (x[a] - c[a]);
            }
        }
        return 0;
    }
    if (kind == LIK_TORUS) {
        const double alpha = prm[0], beta = prm[1], c = prm[2];
        double s = c;
        for (int i = 1; i <= d; ++i)
            s += (i % 2 == 0) ? sin(alpha * x[i - 1]) : cos(beta * x[i - 1]);
        *logl = 3.0 * log(s);
        if (g)
            for (int i = 1; i <= d; ++i)
                g[i - 1] = 3.0 * ((i % 2 == 0) ? alpha * cos(alpha * x[i - 1])
                                                : -beta * sin(beta * x[i - 1])) / s;
        return 0;
    }
    if (kind == LIK_GMM_DIAG) {
        int K = n_comp;
        double lp[64];
        if (K > 64) return -1;
        double l = -INFINITY;
        for (int k = 0; k < K; ++k) {
            const double *mu = prm + (int64_t)k * 2 * d, *sg = mu + d;
            double s = -log((double)K);
            for (int a = 0; a < d; ++a) {
                double r = x[a] - mu[a];
                s += -0.5 * (log2pi + 2.0 * log(sg[a])) - 0.5 * r * r / (sg[a] * sg[a]);
            }
            lp[k] = s;
            l = logaddexp(l, s);
        }
        *logl = l;
        if (g) {
            for (int a = 0; a < d; ++a) g[a] = 0.0;
            for (int k = 0; k < K; ++k) {
                const double *mu = prm + (int64_t)k * 2 * d, *sg = mu + d;
                double resp = exp(lp[k] - l);
                for (int a = 0; a < d; ++a) g[a] += -resp * (x[a] - mu[a]) / (sg[a] * sg[a]);
            }
        }
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* Run settings and state (plain structs filled by the Python wrapper). */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t d, n_live, n_kill, kind, n_comp, bf16;
    double lo, hi, dt_init;
    int32_t n_steps_max, min_ref, max_ref, prune_streak;
    double delta_p, out_hi, out_lo, dt_down, dt_up;
    int32_t term_kind, max_iter;
    double term_tol;
    uint64_t seed;
    int32_t noise_mode;         /* R7: 0 per component, 1 one normal per walker */
    int32_t cluster_mode;       /* C1-C10: 0 one cluster, 1 cluster recognition and spawning */
    int32_t cluster_kmax;       /* C2: largest neighbour count tried */
    int32_t stop_mode;          /* R11: 0 each walker at its own max_ref, 1 batch minimum */
    int32_t save_mode;          /* R8: 0 the walker's own count, 1 the batch minimum */
    int32_t draw_mode;          /* R9: 0 one pick per walker, 1 pooled x_saved */
    int32_t pad_desc;
} orc_desc;

enum { ST_ACTIVE = 0, ST_DONE = 1, ST_MAXITER = 2, ST_NONFINITE = 3 };

typedef struct {
    double *live_x;       /* [n_live * d], point-major */
    double *live_logl;    /* [n_live] */
    double *dead_logl;    /* [dead_cap] */
    double *dead_logw;    /* [dead_cap]: log of the prior-volume shell w_i */
    int64_t dead_cap, n_dead;
    int32_t *killed;      /* [n_kill], ascending (log L, slot) */
    int32_t *surv;        /* [n_live - n_kill], ascending slot */
    int32_t *start;       /* [n_kill], start slot of each walker */
    double *out_x;        /* [n_kill * d] walker outputs */
    double *out_logl;     /* [n_kill] */
    double lz, lx, lz2, lzx, lx2; /* log of the moments Zbar, Z2bar, ZXbar, Xbar, X2bar */
    double lxl_max, dt, lstar;
    int64_t iter, evals, steps_out, steps_in, prunes, nosave, it_outs, it_steps;
    int32_t state, pad;
    double h, sigma_kl, sigma_mom;
    /* optional per-step trace of the first trace_steps steps of each walker */
    double *trace_x;      /* [trace_steps * n_kill * d] */
    double *trace_logl;   /* [trace_steps * n_kill] */
    int32_t *trace_out;   /* [trace_steps * n_kill] */
    int32_t trace_steps, pad2;
    /* clusters (cluster_mode 1): label of each live slot; per cluster its
     * log Xbar_p and live count; survivors grouped by cluster with offsets */
    int32_t *label;        /* [n_live] */
    double *clx;           /* [ORC_CL_MAX] */
    int32_t *cn;           /* [ORC_CL_MAX] */
    int32_t *surv_off;     /* [ORC_CL_MAX + 1] */
    int32_t *start_cl;     /* [n_kill] cluster of each walker */
    int32_t n_clusters, n_splits;
    int32_t split_kmax;    /* the largest neighbour count at which a split was made */
    int32_t kstop_max;     /* the largest neighbour count the loop reached (stop or end) */
    /* cluster moments (cluster_mode 1), logs of: Zbar_p, Z2bar_p, (Z X_p)bar,
     * (Z_p X_p)bar, (X_p^2)bar [ORC_CL_MAX each], then (X_p X_q)bar
     * [ORC_CL_MAX x ORC_CL_MAX]; see ORC_CM_* */
    double *cm;
} orc_state;

static void moments_init(orc_state *S);

/* Step 1 of the outer loop: n_live uniform prior draws and their likelihoods
 * (Algorithm GGNS, first three lines); moments as in Eqs. (ini0)-(ini11). */
int orc_init(const orc_desc *D, const double *prm, orc_state *S)
{
    int d = D->d, n = D->n_live;
    double w = D->hi - D->lo;
    for (int i = 0; i < n; ++i) {
        double *x = S->live_x + (int64_t)i * d;
        for (int b = 0; 4 * b < d; ++b) {
            uint32_t u[4];
            stream_draw(D->seed, (uint32_t)b, (uint32_t)i, 0u, TAG_INIT, 0u, u);
            for (int j = 0; j < 4 && 4 * b + j < d; ++j) x[4 * b + j] = D->lo + w * u24_open(u[j]);
        }
        orc_loglike(D->kind, D->n_comp, prm, d, x, &S->live_logl[i], NULL, D->bf16);
    }
    S->lz = -INFINITY; S->lz2 = -INFINITY; S->lzx = -INFINITY;
    S->lx = 0.0; S->lx2 = 0.0;
    S->lxl_max = -INFINITY;
    S->dt = D->dt_init * w;
    S->lstar = -INFINITY;
    S->iter = 0; S->evals = n; S->n_dead = 0;
    S->steps_out = S->steps_in = S->prunes = S->nosave = 0;
    S->it_outs = S->it_steps = 0;
    S->state = ST_ACTIVE;
    /* the torus reward is positive everywhere only for c > d */
    if (D->kind == LIK_TORUS && !(prm[2] > (double)d)) S->state = ST_NONFINITE;
    S->h = S->sigma_kl = S->sigma_mom = 0.0;
    if (D->cluster_mode) {
        for (int i = 0; i < n; ++i) S->label[i] = 0;
        S->n_clusters = 1;
        S->n_splits = 0;
        S->split_kmax = 0;
        moments_init(S);
        S->kstop_max = 0;
        S->clx[0] = 0.0;
        S->cn[0] = n;
    }
    return 0;
}

/* Kill one point with n_p live points before the removal: record the dead
 * point with its shell volume and apply the single-cluster moment updates
 * (update0), (update2), (update3), (update5) and (update8); every right-hand
 * side uses the values before this update. */
static void kill_one(orc_state *S, double l, int64_t n_p)
{
    double ln = log((double)n_p), ln1 = log((double)n_p + 1.0), ln2 = log((double)n_p + 2.0);
    double lz = S->lz, lz2 = S->lz2, lzx = S->lzx, lx = S->lx, lx2 = S->lx2;
    double logw = lx - ln1;                       /* E[X_{i-1} - X_i] = Xbar/(n_p+1) */
    if (S->n_dead < S->dead_cap) {
        S->dead_logl[S->n_dead] = l;
        S->dead_logw[S->n_dead] = logw;
    }
    S->n_dead += 1;
    S->lz = logaddexp(lz, lx + l - ln1);
    S->lz2 = logaddexp(lz2, logaddexp(log(2.0) + lzx + l - ln1,
                                      log(2.0) + lx2 + 2.0 * l - ln1 - ln2));
    S->lzx = logaddexp(ln + lzx - ln1, ln + lx2 + l - ln1 - ln2);
    S->lx = lx + ln - ln1;
    S->lx2 = lx2 + ln - ln2;
}

static int cmp_lslot(const double *logl, int a, int b)
{
    if (logl[a] < logl[b]) return -1;
    if (logl[a] > logl[b]) return 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* Order slots by ascending (log L, slot) with a bottom-up merge sort. */
static void sort_slots(const double *logl, int n, int32_t *order)
{
    for (int i = 0; i < n; ++i) order[i] = i;
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    for (int width = 1; width < n; width *= 2) {
        for (int lo = 0; lo < n; lo += 2 * width) {
            int mid = lo + width < n ? lo + width : n;
            int hi = lo + 2 * width < n ? lo + 2 * width : n;
            int i = lo, j = mid, k = lo;
            while (i < mid && j < hi) tmp[k++] = (cmp_lslot(logl, order[i], order[j]) <= 0) ? order[i++] : order[j++];
            while (i < mid) tmp[k++] = order[i++];
            while (j < hi) tmp[k++] = order[j++];
        }
        memcpy(order, tmp, sizeof(int32_t) * n);
    }
    free(tmp);
}

static void kill_one_cluster(orc_state *S, double l, int p);
static double log_sum_clusters(const orc_state *S);

/* Final sweep (Algorithm GGNS, closing loop; reading R17) and the run
 * summary: posterior weights p_i = L_i w_i / Z, H = sum p_i log(L_i / Z),
 * sigma_KL = sqrt(H / n_live), sigma_mom from the moments. */
static void final_sweep(const orc_desc *D, orc_state *S)
{
    int n = D->n_live;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * n);
    sort_slots(S->live_logl, n, order);
    for (int j = 0; j < n; ++j) {
        if (D->cluster_mode)
            kill_one_cluster(S, S->live_logl[order[j]], S->label[order[j]]);
        else
            kill_one(S, S->live_logl[order[j]], (int64_t)n - j);
    }
    free(order);
    if (D->cluster_mode) S->lx = log_sum_clusters(S);
    int64_t nd = S->n_dead < S->dead_cap ? S->n_dead : S->dead_cap;
    double h = 0.0;
    for (int64_t i = 0; i < nd; ++i) {
        double lp = S->dead_logl[i] + S->dead_logw[i] - S->lz;
        h += exp(lp) * (S->dead_logl[i] - S->lz);
    }
    S->h = h;
    S->sigma_kl = sqrt(h > 0.0 ? h / n : 0.0);
    double v = S->lz2 - 2.0 * S->lz;
    S->sigma_mom = sqrt(v > 0.0 ? v : 0.0);
}

/* ------------------------------------------------------------------------
 * Clusters (cluster_mode 1): recognition by k-nearest neighbours, per-cluster
 * prior volumes, spawning in proportion to them (Section 3, mode collapse
 * mitigation; Algorithm GGNS with its cluster-finding algorithm; Eqs. new0,
 * new4 for the split of the volume).  Readings:
 *   C1  cluster finding runs at the start of every iteration that goes on,
 *       once for each existing cluster (clusters created in this iteration
 *       are not re-examined in it);
 *   C2  for k = 2, 3, ..., m - 1 (m points in the cluster): link every point
 *       to its k nearest other points of the cluster (FP64 Euclidean
 *       distance, ties by slot), take the connected components of the
 *       undirected graph and their sizes; stop at the first k whose sorted
 *       sizes equal those of k - 1 and use that k's components.  If it never
 *       stops, or m < 3, the cluster stays whole.  cluster_kmax > 0 caps k
 *       (an option; 0 runs the loop as the algorithm writes it);
 *   C3  the components, ordered by their smallest slot, become clusters: the
 *       first keeps the old index, the others take new indices (at most
 *       ORC_CL_MAX clusters; a split that would exceed it is not made); the
 *       volume splits as Xbar_i = (n_i / n) Xbar_p (Eq. new0);
 *   C4  a killed point of cluster p with n_p live points before its removal
 *       has weight Xbar_p / (n_p + 1) and Xbar_p <- n_p Xbar_p / (n_p + 1)
 *       (Eqs. update0, update2); a cluster left without points is removed;
 *       the run's Xbar is the sum over clusters;
 *   C5  each walker draws its cluster p with probability Xbar_p / sum_q Xbar_q
 *       over the clusters with survivors (start stream word 1, inverse CDF in
 *       cluster order), then a start uniformly among that cluster's survivors
 *       (word 0); the new point joins that cluster;
 *   C6  the second moments follow the cluster recursion, Eqs. (update0)-
 *       (update9) per killed point and (new0)-(new6) per split (see
 *       moments_kill, moments_split); sigma_mom from log Z2bar and log Zbar
 *       as in the single-cluster case.
 * ------------------------------------------------------------------------ */
#define ORC_CL_MAX 64

/* The moments of the cluster recursion (Eqs. ini0-ini11, update0-update9,
 * new0-new6), all kept as logarithms (every moment is >= 0):
 *   lzp[p]   log Zbar_p          evidence of cluster p
 *   lz2p[p]  log (Z_p^2)bar
 *   lzx[p]   log (Z X_p)bar      run evidence times the cluster's volume
 *   lzpx[p]  log (Z_p X_p)bar
 *   lx2[p]   log (X_p^2)bar
 *   lxx[p][q] log (X_p X_q)bar   (p != q; symmetric)
 * beside log Zbar, log Z2bar (the run's) and log Xbar_p (clx). */
#define ORC_CM_LZP 0
#define ORC_CM_LZ2P (ORC_CL_MAX)
#define ORC_CM_LZX (2 * ORC_CL_MAX)
#define ORC_CM_LZPX (3 * ORC_CL_MAX)
#define ORC_CM_LX2 (4 * ORC_CL_MAX)
#define ORC_CM_LXX (5 * ORC_CL_MAX)
#define ORC_CM_SIZE (5 * ORC_CL_MAX + ORC_CL_MAX * ORC_CL_MAX)

/* Eqs. (ini0)-(ini11): one cluster holding the whole prior, Xbar = 1,
 * (X^2)bar = 1 (its value for the volume before any kill), no evidence. */
static void moments_init(orc_state *S)
{
    double *cm = S->cm;
    for (int i = 0; i < ORC_CM_SIZE; ++i) cm[i] = -INFINITY;
    cm[ORC_CM_LX2 + 0] = 0.0;
    S->lz = -INFINITY;
    S->lz2 = -INFINITY;
}

/* Kill a point of log-likelihood l from cluster p, which holds n_p live
 * points before the removal: the dead record with weight Xbar_p / (n_p + 1),
 * then Eqs. (update0)-(update9), every right-hand side taking the values
 * before this kill.  In (update3) the likelihood is the killed point's (the
 * subscript of the printed L_p is read as a typo), and in (update6) the
 * cross moment added to is (Z X_q)bar, the right-hand side's (Z X_p)bar read
 * as a typo for it. */
static void moments_kill(orc_state *S, double l, int p)
{
    double *cm = S->cm;
    const int nq = S->n_clusters;
    const int n_p = S->cn[p];
    const double ln = log((double)n_p), ln1 = log((double)n_p + 1.0), ln2 = log((double)n_p + 2.0);
    const double lx = S->clx[p], lzx = cm[ORC_CM_LZX + p], lx2 = cm[ORC_CM_LX2 + p];
    const double lzp = cm[ORC_CM_LZP + p], lz2p = cm[ORC_CM_LZ2P + p], lzpx = cm[ORC_CM_LZPX + p];
    const double l2 = log(2.0);
    const double logw = lx - ln1;
    if (S->n_dead < S->dead_cap) {
        S->dead_logl[S->n_dead] = l;
        S->dead_logw[S->n_dead] = logw;
    }
    S->n_dead += 1;
    S->lz = logaddexp(S->lz, lx + l - ln1);                                        /* update0 */
    cm[ORC_CM_LZP + p] = logaddexp(lzp, lx + l - ln1);                           /* update1 */
    S->clx[p] = lx + ln - ln1;                                                    /* update2 */
    S->lz2 = logaddexp(S->lz2, logaddexp(l2 + lzx + l - ln1,
                                         l2 + lx2 + 2.0 * l - ln1 - ln2));       /* update3 */
    cm[ORC_CM_LZ2P + p] = logaddexp(lz2p, logaddexp(l2 + lzpx + l - ln1,
                                                    l2 + lx2 + 2.0 * l - ln1 - ln2)); /* update4 */
    cm[ORC_CM_LZX + p] = logaddexp(ln + lzx - ln1, ln + lx2 + l - ln1 - ln2);    /* update5 */
    for (int q = 0; q < nq; ++q)                                                  /* update6 */
        if (q != p) cm[ORC_CM_LZX + q] = logaddexp(cm[ORC_CM_LZX + q],
                                                   cm[ORC_CM_LXX + p * ORC_CL_MAX + q] + l - ln1);
    cm[ORC_CM_LZPX + p] = logaddexp(ln + lzpx - ln1, ln + lx2 + l - ln1 - ln2);  /* update7 */
    cm[ORC_CM_LX2 + p] = lx2 + ln - ln2;                                          /* update8 */
    for (int q = 0; q < nq; ++q) {                                                /* update9 */
        if (q == p) continue;
        const double v = cm[ORC_CM_LXX + p * ORC_CL_MAX + q] + ln - ln1;
        cm[ORC_CM_LXX + p * ORC_CL_MAX + q] = v;
        cm[ORC_CM_LXX + q * ORC_CL_MAX + p] = v;
    }
    S->cn[p] = n_p - 1;
    if (S->cn[p] == 0) S->clx[p] = -INFINITY;
}

/* Split cluster p of m points into nc clusters of cnt[c] points, component c
 * taking index q[c] (q[0] = p): Eqs. (new0)-(new6) from the values of p
 * before the split.  (new3) with Y = X_r applies to every other existing
 * cluster r; (new2) gives the cross moments between the new clusters. */
static void moments_split(orc_state *S, int p, int m, int nc, const int32_t *cnt, const int *q)
{
    double *cm = S->cm;
    const double lx = S->clx[p], lx2 = cm[ORC_CM_LX2 + p], lzx = cm[ORC_CM_LZX + p];
    const double lzp = cm[ORC_CM_LZP + p], lz2p = cm[ORC_CM_LZ2P + p], lzpx = cm[ORC_CM_LZPX + p];
    const double lm = log((double)m), lmm = log((double)m * (m + 1.0));
    const int n_before = S->n_clusters;
    double lxr[ORC_CL_MAX];
    for (int r = 0; r < n_before; ++r) lxr[r] = cm[ORC_CM_LXX + p * ORC_CL_MAX + r];
    for (int c = 0; c < nc; ++c) {
        const int qc = q[c];
        const double ln = log((double)cnt[c]), lnn = log((double)cnt[c] * (cnt[c] + 1.0));
        S->clx[qc] = lx + ln - lm;                                   /* new0 */
        cm[ORC_CM_LX2 + qc] = lx2 + lnn - lmm;                       /* new1 */
        cm[ORC_CM_LZX + qc] = lzx + ln - lm;                         /* new3, Y = Z */
        cm[ORC_CM_LZP + qc] = lzp + ln - lm;                         /* new4 */
        cm[ORC_CM_LZPX + qc] = lzpx + lnn - lmm;                     /* new5 */
        cm[ORC_CM_LZ2P + qc] = lz2p + lnn - lmm;                     /* new6 */
        for (int r = 0; r < n_before; ++r) {                         /* new3, Y = X_r */
            if (r == p) continue;
            const double v = lxr[r] + ln - lm;
            cm[ORC_CM_LXX + qc * ORC_CL_MAX + r] = v;
            cm[ORC_CM_LXX + r * ORC_CL_MAX + qc] = v;
        }
        S->cn[qc] = cnt[c];
    }
    for (int a = 0; a < nc; ++a)                                     /* new2 */
        for (int b = 0; b < nc; ++b) {
            if (a == b) continue;
            cm[ORC_CM_LXX + q[a] * ORC_CL_MAX + q[b]] =
                lx2 + log((double)cnt[a] * (double)cnt[b]) - lmm;
        }
}

/* The cluster recursion over a given event sequence (test hook for the
 * Monte Carlo pin of the moments): type 0 kills a point of log L l[e] from
 * cluster cl[e]; type 1 adds a live point to cluster cl[e]; type 2 splits
 * cluster cl[e] into ncomp[e] clusters whose point counts follow in counts[]
 * (consumed in order; the new ones take the next free indices).  Starts from
 * one cluster of n0 points.  Writes log Zbar, log Z2bar, then per cluster
 * log Zbar_p, log (Z_p^2)bar, log Xbar_p (ORC_CL_MAX each) to out. */
int orc_moment_sequence(int n0, int n_events, const int32_t *type, const int32_t *cl,
                        const double *l, const int32_t *ncomp, const int32_t *counts, double *out)
{
    orc_state S;
    memset(&S, 0, sizeof(S));
    double cm[ORC_CM_SIZE], clx[ORC_CL_MAX], dl[1], dw[1];
    int32_t cn[ORC_CL_MAX];
    S.cm = cm;
    S.clx = clx;
    S.cn = cn;
    S.dead_logl = dl;
    S.dead_logw = dw;
    S.dead_cap = 0;
    for (int p = 0; p < ORC_CL_MAX; ++p) { clx[p] = -INFINITY; cn[p] = 0; }
    clx[0] = 0.0;
    cn[0] = n0;
    S.n_clusters = 1;
    moments_init(&S);
    int ci = 0;
    for (int e = 0; e < n_events; ++e) {
        if (type[e] == 0) {
            if (cn[cl[e]] < 1) return -1;
            moments_kill(&S, l[e], cl[e]);
        } else if (type[e] == 1) {
            cn[cl[e]] += 1;
        } else {
            int nc = ncomp[e], p = cl[e], q[ORC_CL_MAX], m = 0;
            if (nc < 2 || S.n_clusters + nc - 1 > ORC_CL_MAX) return -1;
            for (int c = 0; c < nc; ++c) {
                q[c] = (c == 0) ? p : S.n_clusters + c - 1;
                m += counts[ci + c];
            }
            if (m != cn[p]) return -1;
            moments_split(&S, p, m, nc, counts + ci, q);
            S.n_clusters += nc - 1;
            ci += nc;
        }
    }
    out[0] = S.lz;
    out[1] = S.lz2;
    for (int p = 0; p < ORC_CL_MAX; ++p) {
        out[2 + p] = cm[ORC_CM_LZP + p];
        out[2 + ORC_CL_MAX + p] = cm[ORC_CM_LZ2P + p];
        out[2 + 2 * ORC_CL_MAX + p] = clx[p];
    }
    return 0;
}

/* Squared Euclidean distance (FP64). */
static double dist2(const double *a, const double *b, int d)
{
    double s = 0.0;
    for (int i = 0; i < d; ++i) {
        double t = a[i] - b[i];
        s += t * t;
    }
    return s;
}

/* the K nearest other points of each of the m points idx[0..m) (local
 * indices into idx), ordered by (squared distance, slot) */
static void knn_lists(const double *X, int d, const int32_t *idx, int m, int K, int32_t *nb)
{
    double *bd = (double *)malloc(sizeof(double) * (K > 0 ? K : 1));
    int32_t *bi = (int32_t *)malloc(sizeof(int32_t) * (K > 0 ? K : 1));
    for (int i = 0; i < m; ++i) {
        int cnt = 0;
        const double *xi = X + (int64_t)idx[i] * d;
        for (int j = 0; j < m; ++j) {
            if (j == i) continue;
            double dd = dist2(xi, X + (int64_t)idx[j] * d, d);
            /* insertion into the sorted list of the best K so far */
            int pos = cnt;
            while (pos > 0 && (dd < bd[pos - 1] || (dd == bd[pos - 1] && idx[j] < idx[bi[pos - 1]])))
                --pos;
            if (pos >= K) continue;
            int last = cnt < K ? cnt : K - 1;
            for (int t = last; t > pos; --t) { bd[t] = bd[t - 1]; bi[t] = bi[t - 1]; }
            bd[pos] = dd;
            bi[pos] = j;
            if (cnt < K) ++cnt;
        }
        for (int t = 0; t < K; ++t) nb[(int64_t)i * K + t] = bi[t];
    }
    free(bd);
    free(bi);
}

static int uf_find(int32_t *par, int i)
{
    while (par[i] != i) i = par[i];
    return i;
}

/* connected components of the graph linking each point to its first k
 * neighbours; root[i] = smallest local index of i's component; the sizes,
 * sorted in decreasing order, go to sizes[0..returned count) */
static int components(int m, int k, int K, const int32_t *nb, int32_t *root, int32_t *sizes)
{
    int32_t *par = (int32_t *)malloc(sizeof(int32_t) * m);
    for (int i = 0; i < m; ++i) par[i] = i;
    for (int i = 0; i < m; ++i)
        for (int t = 0; t < k; ++t) {
            int a = uf_find(par, i), b = uf_find(par, nb[(int64_t)i * K + t]);
            if (a != b) { if (a < b) par[b] = a; else par[a] = b; }
        }
    int nc = 0;
    int32_t *count = (int32_t *)calloc((size_t)m, sizeof(int32_t));
    for (int i = 0; i < m; ++i) { root[i] = uf_find(par, i); count[root[i]] += 1; }
    for (int i = 0; i < m; ++i)
        if (count[i] > 0) sizes[nc++] = count[i];
    /* decreasing order (insertion sort; nc is small in practice) */
    for (int a = 1; a < nc; ++a) {
        int v = sizes[a], b = a;
        while (b > 0 && sizes[b - 1] < v) { sizes[b] = sizes[b - 1]; --b; }
        sizes[b] = v;
    }
    free(par);
    free(count);
    return nc;
}

/* Cluster finding for every cluster that exists now (C1-C3). */
static void find_clusters(const orc_desc *D, orc_state *S)
{
    int n = D->n_live, d = D->d;
    int n_before = S->n_clusters;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *root = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *best = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *sz = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * n);
    for (int p = 0; p < n_before; ++p) {
        int m = 0;
        for (int i = 0; i < n; ++i)
            if (S->label[i] == p) idx[m++] = i;
        if (m < 3) continue;
        int kend = m - 1;
        if (D->cluster_kmax > 0 && D->cluster_kmax < kend) kend = D->cluster_kmax;
        if (kend < 2) continue;
        /* the neighbour lists are computed for the first K neighbours and
         * extended (K doubled) when k passes K: a list for K is a prefix of
         * the list for any larger K, the order (distance, slot) being total */
        int K = kend < 8 ? kend : 8;
        int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * K);
        knn_lists(S->live_x, d, idx, m, K, nb);
        int nprev = -1, found = 0, nc = 0;
        int k;
        for (k = 2; k <= kend; ++k) {
            if (k > K) {
                K = 2 * K < kend ? 2 * K : kend;
                free(nb);
                nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * K);
                knn_lists(S->live_x, d, idx, m, K, nb);
            }
            nc = components(m, k, K, nb, root, sz);
            int same = (nc == nprev);
            for (int t = 0; same && t < nc; ++t) same = (sz[t] == prev[t]);
            if (same) { found = 1; break; }
            memcpy(prev, sz, sizeof(int32_t) * nc);
            nprev = nc;
        }
        free(nb);
        if ((found ? k : kend) > S->kstop_max) S->kstop_max = found ? k : kend;
        if (!found || nc < 2 || S->n_clusters + nc - 1 > ORC_CL_MAX) continue;
        /* components in order of their smallest slot (= their root, local) */
        for (int i = 0; i < m; ++i) best[i] = -1;
        int next = 0;
        for (int i = 0; i < m; ++i)
            if (root[i] == i) best[i] = next++;
        int32_t *cnt = (int32_t *)calloc((size_t)nc, sizeof(int32_t));
        int qs[ORC_CL_MAX];
        for (int i = 0; i < m; ++i) cnt[best[root[i]]] += 1;
        for (int c = 0; c < nc; ++c) qs[c] = (c == 0) ? p : S->n_clusters + c - 1;
        moments_split(S, p, m, nc, cnt, qs);
        for (int i = 0; i < m; ++i) {
            int c = best[root[i]];
            S->label[idx[i]] = (c == 0) ? p : S->n_clusters + c - 1;
        }
        S->n_clusters += nc - 1;
        S->n_splits += 1;
        if (k > S->split_kmax) S->split_kmax = k;
        free(cnt);
    }
    free(idx); free(root); free(best); free(sz); free(prev);
}

static double log_sum_clusters(const orc_state *S)
{
    double r = -INFINITY;
    for (int p = 0; p < S->n_clusters; ++p)
        if (S->cn[p] > 0) r = logaddexp(r, S->clx[p]);
    return r;
}

/* Kill one point of cluster p (C4): dead record, evidence, volume and the
 * moments of the cluster recursion. */
static void kill_one_cluster(orc_state *S, double l, int p)
{
    moments_kill(S, l, p);
}

/* Termination test, kill step and evidence update of one iteration
 * (Algorithm GGNS, loop head and the kill loop; readings R16, R18). */
int orc_evidence_update(const orc_desc *D, orc_state *S, int force_final)
{
    if (S->state != ST_ACTIVE) return 0;
    int n = D->n_live, k = D->n_kill;
    double lmax = -INFINITY;
    for (int i = 0; i < n; ++i) {
        if (isnan(S->live_logl[i])) { S->state = ST_NONFINITE; return 0; }
        if (S->live_logl[i] > lmax) lmax = S->live_logl[i];
    }
    int stop = force_final != 0;
    if (D->term_kind == 0) {
        if (S->lx + lmax < log(D->term_tol) + S->lz) stop = 1;
    } else {
        double r = S->lx + (D->term_kind == 1 ? lmax : S->lstar);
        if (r > S->lxl_max) S->lxl_max = r;
        if (S->iter > 0 && r - S->lxl_max < log(D->term_tol)) stop = 1;
    }
    if (!stop && S->iter >= D->max_iter) { final_sweep(D, S); S->state = ST_MAXITER; return 0; }
    if (stop) { final_sweep(D, S); S->state = ST_DONE; return 0; }

    if (D->cluster_mode) find_clusters(D, S);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * n);
    sort_slots(S->live_logl, n, order);
    for (int j = 0; j < k; ++j) {
        S->killed[j] = order[j];
        if (D->cluster_mode)
            kill_one_cluster(S, S->live_logl[order[j]], S->label[order[j]]);
        else
            kill_one(S, S->live_logl[order[j]], (int64_t)n - j);
    }
    S->lstar = S->live_logl[order[k - 1]];
    char *dead = (char *)calloc((size_t)n, 1);
    for (int j = 0; j < k; ++j) dead[order[j]] = 1;
    int m = 0;
    if (D->cluster_mode) {
        /* survivors grouped by cluster, ascending slot within each */
        for (int p = 0; p < S->n_clusters; ++p) {
            S->surv_off[p] = m;
            for (int i = 0; i < n; ++i)
                if (!dead[i] && S->label[i] == p) S->surv[m++] = i;
        }
        S->surv_off[S->n_clusters] = m;
        S->lx = log_sum_clusters(S);
    } else {
        for (int i = 0; i < n; ++i)
            if (!dead[i]) S->surv[m++] = i;
    }
    free(dead);
    free(order);
    return 0;
}

/* One walker of the batched HSS walk (Algorithm GGNS HSS; Eq. reflection;
 * readings R4-R12): its position, start, momentum, streams and counters. */
typedef struct {
    int m, s;
    double *x, *x0, *p, *g, *eps, *out;
    uint32_t *xs;          /* one xoshiro state per block of four coordinates (EPS) */
    uint32_t xr[4];        /* reservoir stream (RES) */
    double l0, l, out_l;   /* start log L, current log L, log L of the kept point */
    int nref, streak, steps, outs, n_prune, outside, done;
    int64_t nsave;
} orc_walker;

/* Start walker m: its start slot (uniform over the survivors, or cluster
 * first, C5), x = x0, p ~ N(0, I) from stream P0, and its stream states. */
static void walker_start(const orc_desc *D, orc_state *S, int m, orc_walker *W)
{
    int d = D->d, nsurv = D->n_live - D->n_kill;
    uint32_t it = (uint32_t)S->iter;
    uint32_t u[4];
    stream_draw(D->seed, 0u, (uint32_t)m, it, TAG_START, 0u, u);
    int s;
    if (D->cluster_mode) {
        /* C5: the walker's cluster in proportion to Xbar_p, then a survivor of it */
        double cmax = -INFINITY, tot = 0.0;
        for (int p = 0; p < S->n_clusters; ++p)
            if (S->surv_off[p + 1] > S->surv_off[p] && S->clx[p] > cmax) cmax = S->clx[p];
        for (int p = 0; p < S->n_clusters; ++p)
            if (S->surv_off[p + 1] > S->surv_off[p]) tot += exp(S->clx[p] - cmax);
        double target = ((double)u[1] + 0.5) * 0x1p-32 * tot, cum = 0.0;
        int pc = -1;
        for (int p = 0; p < S->n_clusters; ++p) {
            if (S->surv_off[p + 1] == S->surv_off[p]) continue;
            cum += exp(S->clx[p] - cmax);
            pc = p;
            if (target < cum) break;
        }
        int cnt = S->surv_off[pc + 1] - S->surv_off[pc];
        s = S->surv[S->surv_off[pc] + (int)(((uint64_t)u[0] * (uint64_t)cnt) >> 32)];
        S->start_cl[m] = pc;
    } else {
        s = S->surv[(int)(((uint64_t)u[0] * (uint64_t)nsurv) >> 32)];
    }
    S->start[m] = s;
    memset(W, 0, sizeof(*W));
    W->m = m;
    W->s = s;
    W->x = (double *)malloc(sizeof(double) * d);
    W->x0 = (double *)malloc(sizeof(double) * d);
    W->p = (double *)malloc(sizeof(double) * d);
    W->g = (double *)malloc(sizeof(double) * d);
    W->eps = (double *)malloc(sizeof(double) * (d + 4));
    int nb = (d + 3) / 4;
    W->xs = (uint32_t *)malloc(sizeof(uint32_t) * 4 * nb);
    memcpy(W->x0, S->live_x + (int64_t)s * d, sizeof(double) * d);
    memcpy(W->x, W->x0, sizeof(double) * d);
    W->l0 = S->live_logl[s];
    normals_philox(D->seed, (uint32_t)m, it, TAG_P0, 0u, d, W->p);
    for (int b = 0; b < nb; ++b) {
        stream_draw(D->seed, (uint32_t)b, (uint32_t)m, it, TAG_EPS, 0u, u);
        xoshiro_seed(W->xs + 4 * b, u);
    }
    stream_draw(D->seed, 0u, (uint32_t)m, it, TAG_RES, 0u, u);
    xoshiro_seed(W->xr, u);
    /* the output starts as the start point (reading R10's last fallback) */
    W->out = S->out_x + (int64_t)m * d;
    memcpy(W->out, W->x0, sizeof(double) * d);
    W->out_l = W->l0;
}

static void walker_free(orc_walker *W)
{
    free(W->x); free(W->x0); free(W->p); free(W->g); free(W->eps); free(W->xs);
}

/* One step of Algorithm GGNS HSS for one walker: x += p dt; log L and its
 * gradient; outside test (box first, R6; then log L <= L*, R2); reflection
 * (Eq. reflection with the normal at the outside point, R4/R5; box faces
 * flip their axes, R6); noise p *= (1 + delta_p eps) (R7); reflection count,
 * outside streak and pruning (R12: back to the start with fresh momentum;
 * the reflection count restarts only when walkers stop one by one, so that
 * the batch minimum of a whole-batch stop never decreases).  Returns the
 * reservoir word of this step. */
static uint32_t walker_step(const orc_desc *D, const double *prm, orc_state *S, orc_walker *W)
{
    int d = D->d, k = D->n_kill, m = W->m;
    double dt = S->dt, lstar = S->lstar;
    double *x = W->x, *p = W->p, *g = W->g;
    for (int a = 0; a < d; ++a) x[a] = x[a] + dt * p[a];
    orc_loglike(D->kind, D->n_comp, prm, d, x, &W->l, g, D->bf16);
    int box = 0;
    for (int a = 0; a < d; ++a)
        if (x[a] < D->lo || x[a] > D->hi) box = 1;
    int outside = box || (W->l <= lstar);
    if (S->trace_x && W->steps < S->trace_steps) {
        int64_t row = (int64_t)W->steps * k + m;
        memcpy(S->trace_x + row * d, x, sizeof(double) * d);
        S->trace_logl[row] = W->l;
        S->trace_out[row] = outside;
    }
    W->steps += 1;
    if (outside) {
        if (box) {
            for (int a = 0; a < d; ++a)
                if (x[a] < D->lo || x[a] > D->hi) p[a] = -p[a];
        } else {
            double pg = 0.0, gg = 0.0;
            for (int a = 0; a < d; ++a) { pg += p[a] * g[a]; gg += g[a] * g[a]; }
            if (isfinite(gg) && gg > 0.0) {
                /* p' = p - 2 (p.n) n with n = g / |g| */
                double f = 2.0 * pg / gg;
                for (int a = 0; a < d; ++a) p[a] = p[a] - f * g[a];
            } else {
                for (int a = 0; a < d; ++a) p[a] = -p[a];
            }
        }
    }
    if (D->noise_mode == 1) {
        /* one normal per walker and step: two words of the walker's first
         * block stream, the first normal of their Box-Muller pair */
        uint32_t w0 = orc_xoshiro_next(W->xs), w1 = orc_xoshiro_next(W->xs);
        W->eps[0] = sqrt(-2.0 * log(u24_open(w0))) * cos(2.0 * M_PI * u24_half(w1));
    } else {
        int nb = (d + 3) / 4;
        for (int b = 0; b < nb; ++b) {
            uint32_t w[4];
            for (int j = 0; j < 4; ++j) w[j] = orc_xoshiro_next(W->xs + 4 * b);
            orc_box_muller4(w, W->eps + 4 * b);
        }
    }
    if (D->noise_mode == 2) {
        /* isotropic: p += delta_p (|p| / sqrt d) eps, eps ~ N(0, I_d) */
        double pp = 0.0;
        for (int a = 0; a < d; ++a) pp += p[a] * p[a];
        double sc = D->delta_p * sqrt(pp / d);
        for (int a = 0; a < d; ++a) p[a] = p[a] + sc * W->eps[a];
    } else {
        for (int a = 0; a < d; ++a)
            p[a] = p[a] * (1.0 + D->delta_p * (D->noise_mode ? W->eps[0] : W->eps[a]));
    }
    uint32_t ures = orc_xoshiro_next(W->xr);
    W->outside = outside;
    W->nref += outside;
    W->outs += outside;
    W->streak = outside ? W->streak + 1 : 0;
    if (D->prune_streak > 0 && W->streak >= D->prune_streak) {
        memcpy(x, W->x0, sizeof(double) * d);
        W->n_prune += 1;
        normals_philox(D->seed, (uint32_t)m, (uint32_t)S->iter, TAG_P0, (uint32_t)W->n_prune, d, p);
        if (D->stop_mode == 0) W->nref = 0;
        W->streak = 0;
    }
    return ures;
}

/* Keep the point of this step (trajectory preservation, R8-R10): an
 * in-slice point that may be saved enters the walker's size-one reservoir
 * with probability 1/nsave (Vitter's Algorithm R, decided on the integer
 * word: keep iff word * nsave < 2^32); before the first saved point the
 * output tracks the last in-slice point. */
static void walker_keep(const orc_desc *D, orc_walker *W, int may_save, uint32_t ures)
{
    if (W->outside) return;
    if (may_save) {
        W->nsave += 1;
        if ((uint64_t)ures * (uint64_t)W->nsave < ((uint64_t)1 << 32)) {
            memcpy(W->out, W->x, sizeof(double) * D->d);
            W->out_l = W->l;
        }
    } else if (W->nsave == 0) {
        memcpy(W->out, W->x, sizeof(double) * D->d);
        W->out_l = W->l;
    }
}

/* A walker on its own, stopping at its own max_ref-th reflection (R11, the
 * per-walker reading of the loop condition) or after n_steps_max steps. */
static void walk_one(const orc_desc *D, const double *prm, orc_state *S, orc_walker *W)
{
    while (W->steps < D->n_steps_max && (D->max_ref == 0 || W->nref < D->max_ref)) {
        uint32_t ures = walker_step(D, prm, S, W);
        walker_keep(D, W, W->nref >= D->min_ref, ures);
    }
    S->out_logl[W->m] = W->out_l;
}

/* The saved trajectory points of the whole batch, in the order the
 * algorithm appends them (step by step, walkers in index order). */
typedef struct {
    double *x, *l;
    int64_t n, cap;
} orc_pool;

static void pool_add(orc_pool *P, const double *x, double l, int d)
{
    if (P->n == P->cap) {
        P->cap = P->cap ? 2 * P->cap : 1024;
        P->x = (double *)realloc(P->x, sizeof(double) * (size_t)P->cap * d);
        P->l = (double *)realloc(P->l, sizeof(double) * (size_t)P->cap);
    }
    memcpy(P->x + P->n * d, x, sizeof(double) * d);
    P->l[P->n] = l;
    P->n += 1;
}

/* All k walkers in lockstep, as Algorithm GGNS HSS writes the loop: every
 * step moves every walker that is still going; the loop runs while the
 * batch minimum of num_reflections is below max_ref (stop_mode 1) or while
 * any walker is below it (stop_mode 0: each walker stops at its own
 * max_ref), for at most n_steps_max steps.  A point is saved when it is
 * in-slice and either the batch minimum (save_mode 1) or the walker's own
 * count (save_mode 0) has reached min_ref.  The new points are one pick per
 * walker from its own saved points (draw_mode 0) or k uniform draws with
 * replacement from the pooled x_saved of the whole batch (draw_mode 1,
 * stream RES with sub 1, word 0 of walker slot j: index floor(u * N / 2^32)). */
static void walk_lockstep(const orc_desc *D, const double *prm, orc_state *S, orc_walker *W)
{
    int k = D->n_kill, d = D->d;
    uint32_t *ures = (uint32_t *)malloc(sizeof(uint32_t) * k);
    orc_pool pool = {NULL, NULL, 0, 0};
    for (int t = 0; t < D->n_steps_max; ++t) {
        int minref = W[0].nref, going = 0;
        for (int m = 0; m < k; ++m) {
            if (W[m].nref < minref) minref = W[m].nref;
            going += !W[m].done;
        }
        if (D->max_ref > 0 && (D->stop_mode == 1 ? minref >= D->max_ref : going == 0)) break;
#pragma omp parallel for schedule(static)
        for (int m = 0; m < k; ++m)
            if (!W[m].done) ures[m] = walker_step(D, prm, S, &W[m]);
        minref = W[0].nref;
        for (int m = 1; m < k; ++m)
            if (W[m].nref < minref) minref = W[m].nref;
        for (int m = 0; m < k; ++m) {
            if (W[m].done) continue;
            int may_save = D->save_mode == 1 ? minref >= D->min_ref : W[m].nref >= D->min_ref;
            if (D->draw_mode == 1) {
                if (!W[m].outside && may_save) pool_add(&pool, W[m].x, W[m].l, d);
                else walker_keep(D, &W[m], 0, 0u);   /* the fallback point only */
            } else {
                walker_keep(D, &W[m], may_save, ures[m]);
            }
            if (D->stop_mode == 0 && D->max_ref > 0 && W[m].nref >= D->max_ref) W[m].done = 1;
        }
    }
    if (D->draw_mode == 1) {
        for (int j = 0; j < k; ++j) {
            if (pool.n == 0) continue;
            uint32_t u[4];
            stream_draw(D->seed, 0u, (uint32_t)j, (uint32_t)S->iter, TAG_RES, 1u, u);
            int64_t idx = (int64_t)(((uint64_t)u[0] * (uint64_t)pool.n) >> 32);
            memcpy(W[j].out, pool.x + idx * d, sizeof(double) * d);
            W[j].out_l = pool.l[idx];
            W[j].nsave = 1;
        }
    }
    for (int m = 0; m < k; ++m) S->out_logl[m] = W[m].out_l;
    free(pool.x);
    free(pool.l);
    free(ures);
}

int orc_hss_walk(const orc_desc *D, const double *prm, orc_state *S)
{
    if (S->state != ST_ACTIVE) return 0;
    int k = D->n_kill;
    orc_walker *W = (orc_walker *)malloc(sizeof(orc_walker) * k);
    for (int m = 0; m < k; ++m) walker_start(D, S, m, &W[m]);
    if (D->stop_mode == 0 && D->save_mode == 0 && D->draw_mode == 0) {
        /* every walker is independent of the others */
#pragma omp parallel for schedule(dynamic, 4)
        for (int m = 0; m < k; ++m) walk_one(D, prm, S, &W[m]);
    } else {
        walk_lockstep(D, prm, S, W);
    }
    int64_t outs = 0, steps = 0, prunes = 0, nosave = 0;
    for (int m = 0; m < k; ++m) {
        outs += W[m].outs;
        steps += W[m].steps;
        prunes += W[m].n_prune;
        nosave += (W[m].nsave == 0);
        walker_free(&W[m]);
    }
    free(W);
    S->it_outs = outs;
    S->it_steps = steps;
    S->steps_out += outs;
    S->steps_in += steps - outs;
    S->prunes += prunes;
    S->nosave += nosave;
    S->evals += steps;
    return 0;
}

/* Add the new points into the killed slots and adapt dt from out_frac
 * (Algorithm GGNS, dt update and "add theta_new"). */
int orc_replace_dead(const orc_desc *D, orc_state *S)
{
    if (S->state != ST_ACTIVE) return 0;
    int d = D->d, k = D->n_kill;
    for (int m = 0; m < k; ++m) {
        int slot = S->killed[m];
        memcpy(S->live_x + (int64_t)slot * d, S->out_x + (int64_t)m * d, sizeof(double) * d);
        S->live_logl[slot] = S->out_logl[m];
        if (D->cluster_mode) {
            int p = S->start_cl[m];
            S->label[slot] = p;
            S->cn[p] += 1;
        }
    }
    if (S->it_steps > 0) {
        double out_frac = (double)S->it_outs / (double)S->it_steps;
        if (out_frac > D->out_hi) S->dt *= D->dt_down;
        else if (out_frac < D->out_lo) S->dt *= D->dt_up;
    }
    S->iter += 1;
    return 0;
}

/* Whole run: init, iterate until termination, final sweep. */
int orc_run(const orc_desc *D, const double *prm, orc_state *S)
{
    orc_init(D, prm, S);
    while (S->state == ST_ACTIVE) {
        orc_evidence_update(D, S, 0);
        if (S->state != ST_ACTIVE) break;
        orc_hss_walk(D, prm, S);
        orc_replace_dead(D, S);
    }
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Raw stream access for the generator tests. */
void orc_stream_words(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag,
                      uint32_t sub, uint32_t out[4])
{
    stream_draw(seed, c0, c1, c2, tag, sub, out);
}

double orc_round_bf16(double v) { return round_bf16(v); }
