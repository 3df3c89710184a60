/*
 * ggns.h -- C ABI of the MI355X engine for the data-parallel hot path of
 * gradient-guided nested sampling (GGNS; Lemos et al., arXiv:2312.03911).
 *
 * The engine advances many independent nested-sampling runs at once.  Per run
 * and per iteration the caller enqueues, on one stream and in this order:
 *
 *   ggns_evidence_update  termination test, kill of the n_kill lowest live
 *                         points, evidence and prior-volume bookkeeping
 *                         (Appendix A Eqs. ns_sum / delta_x / importance_weight
 *                         / shell_volume; Algorithm GGNS kill loop; Eqs.
 *                         update0-update9), and the final sweep when the run
 *                         stops (Algorithm GGNS closing loop);
 *   ggns_hss_walk         the batched Hamiltonian slice sampling walk that
 *                         moves every walker at once (Algorithm GGNS HSS;
 *                         Eq. reflection; Section 3: adaptive dt, trajectory
 *                         preservation, pruning, parallel evolution);
 *   ggns_replace_dead     the walk outputs replace the killed points and dt
 *                         is adapted from the fraction of outside steps
 *                         (Algorithm GGNS, dt update and "add theta_new").
 *
 * Memory.  The library never allocates device memory.  The caller allocates
 * one device "arena" of ggns_arena_bytes(...) bytes and hands it to
 * ggns_init; every per-run array (live set, dead records, walker outputs,
 * accumulators, the parameter blocks converted to the run's precision) lives
 * inside it at the byte offsets reported by ggns_run_layout.  The arena and
 * the raw parameter buffer stay owned by the caller and must outlive the
 * context.  All calls taking `stream` (a hipStream_t; NULL = the default
 * stream) enqueue asynchronous work and return at once, except
 * ggns_read_stats, which synchronises the stream.
 *
 * Errors.  Return codes below zero (GGNS_E*) mean that nothing was enqueued
 * (argument or state errors) or that a launch failed (GGNS_EHIP).  Numerical
 * trouble inside the kernels is reported per run through
 * ggns_run_stats.state (GGNS_RUN_*); kernels skip runs that are not ACTIVE, so
 * enqueuing further iterations after a run ended is harmless.
 *
 * Layout conventions.  Positions are point-major, [n_live][d] per run, in the
 * run's precision (double for GGNS_FP64, float otherwise).  Log-likelihoods,
 * log-weights and every evidence quantity are double.
 */
#ifndef GGNS_H
#define GGNS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
enum {
    GGNS_OK = 0,
    GGNS_EINVAL = -1,        /* bad argument (sizes, kinds, null pointers, arena too small) */
    GGNS_EHIP = -2,          /* a HIP call or kernel launch failed */
    GGNS_EUNSUPPORTED = -3,  /* a size or combination this build does not implement */
    GGNS_ESTATE = -4,        /* call out of order (e.g. no context) */
    GGNS_ESCRATCH = -5       /* a run needs more scratch than the library's fixed device buffer
                                (GGNS_STATIC_SCRATCH_BYTES) holds: ggns_hss_walk_plain_static */
};

/* Per-run states (ggns_run_stats.state). */
enum {
    GGNS_RUN_ACTIVE = 0,
    GGNS_RUN_DONE = 1,       /* terminated by its criterion; final sweep done */
    GGNS_RUN_MAXITER = 2,    /* stopped at max_iter; final sweep done */
    GGNS_RUN_NONFINITE = 3   /* a live log-likelihood was NaN; the run stopped */
};

/* Likelihood families.  Raw FP64 parameter blocks, at param_offset:
 *   GAUSS_DIAG: mu[d], sigma[d]                        N(mu, diag sigma^2)
 *   GAUSS_FULL: mu[d], P[d*d] (row-major), log det P   N(mu, P^-1)
 *   SHELLS:     n_comp x { c[d], r, w }   sum_k (2 pi w^2)^-1/2 exp(-(|x-c_k|-r)^2 / 2w^2)
 *   GMM_DIAG:   n_comp x { mu[d], sigma[d] }           equal-weight diagonal mixture
 *   TORUS:      { alpha, beta, c }   the reward of Eq. (torus), L = (S + c)^3 with
 *               S = sum over coordinates a = 0 .. d-1 of cos(beta x_a) for even a
 *               (the paper's odd 1-based indices) and sin(alpha x_a) for odd a; meant
 *               for the prior box [0, 2 pi)^d; c > d is required (L > 0): a run
 *               with c <= d starts stopped, in state GGNS_RUN_NONFINITE.  With alpha, beta nonzero integers the normalisation
 *               over the box is (2 pi)^d (c^3 + 3 d c / 2) (Appendix F). */
enum { GGNS_LIK_GAUSS_DIAG = 0, GGNS_LIK_GAUSS_FULL = 1, GGNS_LIK_SHELLS = 2, GGNS_LIK_GMM_DIAG = 3,
       GGNS_LIK_TORUS = 4 };

/* Arithmetic of the walk.  The threshold compare, the evidence, the weights and
 * the log prior volume are FP64 in every mode. */
enum {
    GGNS_FP64 = 0,           /* positions, momenta, likelihood in double */
    GGNS_FP32 = 1,           /* positions, momenta, likelihood in float */
    GGNS_FP32_BF16MMA = 2    /* GAUSS_FULL only: P r on BF16 matrix cores, FP32 accumulate */
};

/* Termination (paper: Appendix A loop test and the X*L peak criterion of
 * Section 3 / Appendix I).  All three are tested at the head of an iteration,
 * with Xbar the expected prior volume left; the peak tests are skipped at the
 * first iteration.
 *   REMAINING_Z:   Xbar * max live L < tol * Zbar.
 *   XL_PEAK:       Xbar * max live L below tol times its running maximum
 *                  (L as in the loop end of Algorithm GGNS).
 *   XL_PEAK_DEAD:  the same test with L the likelihood of the highest point
 *                  killed in the previous iteration, i.e. L_i X_i of the
 *                  current dead point (the tol entry of the Appendix C table).
 *                  A lucky live point far above the rest can hold the largest
 *                  live L high for several iterations, long enough for
 *                  XL_PEAK to fire before the bulk of the evidence; the dead
 *                  point's L is a quantile of the live set and does not jump. */
enum { GGNS_TERM_REMAINING_Z = 0, GGNS_TERM_XL_PEAK = 1, GGNS_TERM_XL_PEAK_DEAD = 2 };

/* One run.  Defaults from the paper: min_ref 1, max_ref 3, delta_p 0.05
 * (Appendix C table), dt_init 0.1 (Appendix G), out_frac band 0.05 / 0.15 with
 * factors 1.1 / 0.9 (Algorithm GGNS). */
typedef struct {
    int32_t d;               /* dimension, 1..256 */
    int32_t n_live;          /* live points, 2..4096 */
    int32_t n_kill;          /* killed and re-walked per iteration, 1..n_live-1 (paper: n_live/2) */
    int32_t lik_kind;        /* GGNS_LIK_* */
    int32_t precision;       /* GGNS_FP64 / GGNS_FP32 / GGNS_FP32_BF16MMA */
    int32_t n_comp;          /* components for SHELLS / GMM_DIAG (1..8), else 1 */
    int64_t param_offset;    /* index (in doubles) of this run's raw block in params_dev */
    double prior_lo, prior_hi;  /* uniform prior on [lo, hi]^d */
    double dt_init;          /* initial step in units of (hi - lo) */
    int32_t n_steps_max;     /* fixed walk length when max_ref == 0, else a cap */
    int32_t min_ref;         /* keep in-slice points once a walker has this many reflections */
    int32_t max_ref;         /* a walker stops at this many reflections; 0 = fixed steps */
    int32_t prune_streak;    /* consecutive outside steps that reset a walker; 0 = never */
    double delta_p;          /* momentum noise p *= 1 + delta_p * eps */
    double out_hi, out_lo;   /* out_frac band */
    double dt_down, dt_up;   /* dt factors above / below the band */
    int32_t term_kind;       /* GGNS_TERM_* */
    int32_t max_iter;        /* iteration cap; the dead-record capacity is n_kill*max_iter+n_live */
    double term_tol;         /* remaining evidence fraction, or the X*L fraction */
    uint64_t seed;           /* key of every random stream of the run */
    int32_t tile_c;          /* walk tile shape, 0 = library choice.  Vector-ALU runs: coordinates
                                per lane (1,2,4,8).  GGNS_FP32_BF16MMA runs: wavefronts sharing a
                                group of 16 walkers, W, with d_pad = d rounded up to 32 and
                                d_pad / (4W) in {4, 8, 16} (d_pad 256: 8, 16; 96, 160, 192,
                                224: 8 only); default
                                d_pad / 32.  Other values: GGNS_EUNSUPPORTED. */
    int32_t noise_mode;      /* the eps of p <- p (1 + delta_p eps) (Algorithm GGNS HSS):
                                1 = one normal per walker and step (default reading): two
                                words of the walker's first block stream per step, the first
                                normal of their Box-Muller pair; 0 = one normal per
                                coordinate, four words of each block stream per step */
    int32_t cluster_mode;    /* 1: cluster recognition and spawning in proportion to the clusters'
                                prior volumes (Section 3, mode collapse mitigation; Algorithm GGNS
                                with its cluster-finding algorithm; Eqs. update0-update9 and
                                new0-new6 for the volumes and moments); 0: one cluster. */
    int32_t cluster_kmax;    /* largest neighbour count the cluster finding tries, 2..32 (the
                                neighbours are found in passes of eight, a pass only for the
                                clusters whose loop has not stopped; a cluster still going at
                                cluster_kmax stays whole, counted in the table's n_cut) */
    int32_t walk_mode;       /* reflection-mode walks (max_ref > 0), Algorithm GGNS HSS:
                                1 = the loop runs while the minimum of num_reflections over the
                                run's n_kill walkers is below max_ref (every walker moves until the
                                last one reaches it, at most n_steps_max steps), and a point is
                                saved once that minimum has reached min_ref; each walker returns a
                                uniform pick of its own saved points.  Enqueued as two launches: a
                                first walk of each walker to its own max_ref-th reflection, then
                                its continuation to the run's stopping step (a walker whose first
                                walk reached the saving window is walked again from its start).
                                0 = each walker stops at its own max_ref-th reflection and saves
                                after its own min_ref-th.  Must be 0 when max_ref == 0. */
    int32_t reserved0;       /* 0 */
} ggns_run_desc;

/* Byte offsets (from the arena base) of one run's arrays. */
typedef struct {
    int64_t live_x;          /* [n_live][d] run precision */
    int64_t live_logl;       /* [n_live] double */
    int64_t killed;          /* [n_kill] int32, slots in ascending (log L, slot) order */
    int64_t survivors;       /* [n_live - n_kill] int32, ascending slot */
    int64_t start;           /* [n_kill] int32, start slot of each walker */
    int64_t walk_x;          /* [n_kill][d] run precision, walker outputs */
    int64_t walk_logl;       /* [n_kill] double */
    int64_t dead_logl;       /* [dead_cap] double, in kill order */
    int64_t dead_logw;       /* [dead_cap] double, log prior-volume shell of each dead point */
    int64_t dead_cap;        /* capacity (elements) */
    int32_t elem_bytes;      /* 8 (FP64) or 4 */
    int32_t reserved;
    int64_t label;           /* cluster mode: [n_live] int32 cluster of each live slot; else -1 */
    int64_t cluster_table;   /* cluster mode: double log_xbar[64], double spawn_cdf[64],
                                int32 n_live[64], int32 survivor_offsets[65],
                                int32 member_offsets[65], int32 n_clusters, n_splits, stopping,
                                pad, int32 need[64], cc_done, n_cut, pad[2], then the logs of the
                                cluster moments double Zbar_p[64], Z2bar_p[64], ZXbar_p[64],
                                ZpXpbar_p[64], X2bar_p[64], XpXqbar[64][64]; survivors are
                                grouped by cluster; else -1 */
    int64_t knn;             /* cluster mode: [n_live][32] int32 neighbour slots of each live
                                slot within its cluster, nearest first; else -1 */
    int64_t knn_dist;        /* cluster mode: [n_live][32] double, their squared distances */
} ggns_layout;

/* Per-run results and counters. */
typedef struct {
    double log_z;            /* log Zbar (batched kills, Xbar convention) */
    double log_x;            /* log Xbar */
    double log_z2;           /* log of the second moment of Z (Eqs. update3, update5, update8):
                                after ggns_finalize with one cluster; in cluster mode (the
                                cluster recursion, Eqs. update3-update9, new0-new6) kept
                                after every kill */
    double dt;               /* current step (prior units) */
    double lstar;            /* current threshold log L* */
    double log_xl_max;       /* running max of log(X * L_max) (X*L peak criterion) */
    double h;                /* information H = sum p_i log(L_i / Z), after ggns_finalize */
    double sigma_kl;         /* sqrt(H / n_live) (Eq. logZ_error) */
    double sigma_mom;        /* sqrt(log Z2bar - 2 log Zbar), after ggns_finalize */
    int64_t iter;            /* iterations done */
    int64_t evals;           /* likelihood+gradient evaluations (n_live + walker steps) */
    int64_t n_dead;          /* dead records written */
    int64_t steps_out, steps_in;  /* walker steps outside / inside the slice */
    int64_t prunes;          /* pruning resets */
    int64_t nosave;          /* walks that saved no point (fell back to the last in-slice point) */
    int64_t it_outs, it_steps;    /* counters of the last walk (out_frac) */
    int64_t replayed;        /* walk_mode 1: walker steps walked a second time (a walker whose first
                                walk reached the saving window is walked again from its start);
                                not counted in evals */
    int32_t state;           /* GGNS_RUN_* */
    int32_t n_clusters;      /* cluster mode: cluster indices in use (removed ones included); else 0 */
} ggns_run_stats;

/* Values a caller may load into a run (tests, checkpoint/resume). */
typedef struct {
    double log_z, log_x, dt;
    int64_t iter;
} ggns_run_vars;

typedef struct ggns_ctx ggns_ctx;

/* Bytes of device arena needed for these runs (< 0 on invalid descriptors). */
int64_t ggns_arena_bytes(const ggns_run_desc *runs, int32_t n_runs);

/* Build a context over a zero-based arena and enqueue the start of every run:
 * convert parameters, draw n_live points uniformly in the prior box, evaluate
 * their log-likelihoods, set log Zbar = -inf, log Xbar = 0, dt = dt_init (in
 * prior units) (Algorithm GGNS, initialisation).  `runs` is copied; params_dev
 * (n_params doubles, device) must stay valid while the context is used. */
int ggns_init(ggns_ctx **out, const ggns_run_desc *runs, int32_t n_runs,
              const double *params_dev, int64_t n_params, void *arena_dev,
              int64_t arena_bytes, void *stream);

/* As ggns_init, but over an arena that already holds the state of these runs
 * (checkpoint/resume): converts parameters only. */
int ggns_attach(ggns_ctx **out, const ggns_run_desc *runs, int32_t n_runs,
                const double *params_dev, int64_t n_params, void *arena_dev,
                int64_t arena_bytes, void *stream);

/* Termination test, kill and evidence update for every ACTIVE run; a run that
 * meets its criterion (or max_iter, or final_sweep != 0) gets the final sweep
 * (its remaining live points become dead records and enter log Z) and leaves
 * the ACTIVE state. */
int ggns_evidence_update(ggns_ctx *ctx, int32_t final_sweep, void *stream);

/* Summary of every run whose final sweep is done and not yet summarised: the
 * information H, sigma_KL = sqrt(H / n_live) (Eq. logZ_error) and sigma_mom
 * from the second moment of Z (Eqs. update0-update9, single cluster), over the
 * whole dead sequence.  One launch for all runs; call it once they stopped. */
int ggns_finalize(ggns_ctx *ctx, void *stream);

/* The batched HSS walk for every ACTIVE run (Algorithm GGNS HSS, with the
 * trajectory preservation, pruning and parallel evolution of Section 3):
 * n_kill walkers per run, started from survivors drawn uniformly, write their
 * outputs to walk_x / walk_logl and the step counters dt adaptation uses.
 * Runs are grouped into kernel classes (precision, tile shape, family); when
 * there are several, the classes after the first run on side streams of the
 * context that wait on `stream` and are joined back into it, so the call is
 * ordered on `stream` like a single launch and can be graph-captured. */
int ggns_hss_walk(ggns_ctx *ctx, void *stream);

/* Scatter walker outputs into the killed slots, adapt dt, advance the
 * iteration counter. */
int ggns_replace_dead(ggns_ctx *ctx, void *stream);

/* n_iter iterations of the nested sampling loop (Algorithm GGNS: the evidence
 * update, the kill of the n_kill lowest points, the walk and the replacement),
 * each the same work per run as ggns_evidence_update(final_sweep = 0),
 * ggns_hss_walk and ggns_replace_dead called in that order, with bitwise the
 * same results.  Each kernel class walks its own chain of iterations over its
 * own runs, on the side streams ggns_hss_walk uses: a class does not wait for
 * the slowest class at every iteration, only at the end of the call.  The call
 * is ordered on `stream` like a single launch and can be graph-captured.
 * n_iter < 0 is GGNS_EINVAL; 0 does nothing. */
int ggns_iterate(ggns_ctx *ctx, int32_t n_iter, void *stream);

/* log L (and grad log L if grad_dev is not NULL) of run `run` at n points
 * x_dev [n][d] (run precision); logl_dev [n] double, grad_dev [n][d] run
 * precision.  The likelihood the walk uses, callable on its own. */
int ggns_loglike_grad(ggns_ctx *ctx, int32_t run, const void *x_dev, int64_t n,
                      double *logl_dev, void *grad_dev, void *stream);

/* Adjoint (vector-Jacobian product) of log L: gx[i] = gout[i] * grad log L(x[i]). */
int ggns_loglike_vjp(ggns_ctx *ctx, int32_t run, const void *x_dev, int64_t n,
                     const double *gout_dev, void *gx_dev, void *stream);

/* The plain FP64 walk, the speed baseline of the fused walk: the same method,
 * random streams and outputs as ggns_hss_walk (Algorithm GGNS HSS; the readings
 * of the fused walk), executed as a per-step array program -- one thread per
 * walker, the walk state in the caller's device workspace, one kernel launch
 * per step, the number of active walkers read back by the host every 8 steps,
 * runs walked one after another.  Every run of the context must be GGNS_FP64
 * (else GGNS_EUNSUPPORTED).  `workspace_dev` (device, 256-byte aligned, caller
 * owned, at least ggns_plain_workspace_bytes(ctx) bytes, contents need not be
 * initialised) is scratch for the duration of the call.  Synchronises `stream`
 * (it polls), so it cannot be captured in a graph. */
int64_t ggns_plain_workspace_bytes(const ggns_ctx *ctx);

/* The walk with a likelihood the caller evaluates (for likelihoods written in a
 * framework with automatic differentiation, the setting Section 3 describes:
 * the gradient comes from differentiable programming).  Same method, streams,
 * readings and outputs as ggns_hss_walk_plain, for one FP64 run, with every
 * step split at the likelihood:
 *   ggns_ext_begin    gathers the starts, draws the momenta and stream seeds
 *                     and drifts every walker once (x = x_start + dt p0);
 *   the caller        evaluates, for every walker m, log L and its gradient
 *                     at x[:, m] into logl[m] and grad[:, m];
 *   ggns_ext_step(t)  takes step t (outside test, reflection, noise, kept
 *                     point, pruning, stop) and drifts the walkers that go on;
 *                     active[t] counts them;
 * until active[t] is 0 or t reaches n_steps_max - 1.  A walk_mode 1 run (the
 * batch-minimum loop) takes one call more, t = n_steps_max, that applies the
 * save rule of the last step (each call applies the one of the step before it,
 * once the run's minimum reflection count after that step is known); its
 * log L and gradient inputs are not read.  The walker outputs then
 * sit where ggns_replace_dead reads them.  Buffers live in the caller's device
 * workspace (256-byte aligned, at least ggns_ext_workspace_bytes(ctx, run),
 * contents need not be initialised; the same workspace for the whole walk):
 * ggns_ext_buffers returns x [d][n_kill] and grad [d][n_kill] (component-major,
 * walker m in column m), logl [n_kill] and active [n_steps_max + 1], all double
 * but active (int32).  The live set's log L must come from the same likelihood
 * (write it over the live_logl section after ggns_init); the run's likelihood
 * family in its descriptor is then unused.  A run that is not GGNS_FP64 gives
 * GGNS_EUNSUPPORTED.  All calls are asynchronous on `stream`. */
int64_t ggns_ext_workspace_bytes(const ggns_ctx *ctx, int32_t run);
int ggns_ext_buffers(const ggns_ctx *ctx, int32_t run, void *workspace_dev, int64_t workspace_bytes,
                     double **x_dev, double **logl_dev, double **grad_dev, int32_t **active_dev);
int ggns_ext_begin(ggns_ctx *ctx, int32_t run, void *workspace_dev, int64_t workspace_bytes,
                   void *stream);
int ggns_ext_step(ggns_ctx *ctx, int32_t run, void *workspace_dev, int64_t workspace_bytes,
                  int32_t step, void *stream);
int ggns_hss_walk_plain(ggns_ctx *ctx, void *workspace_dev, int64_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under graph capture
 * of the surrounding work, serving loops, harnesses that forbid hipMalloc):
 * ggns_hss_walk_plain with its workspace taken from a fixed device buffer that
 * the library holds, GGNS_STATIC_SCRATCH_BYTES (16 MiB) on each GPU it runs on
 * until the process ends.  The call allocates nothing: no hipMalloc, no
 * hipFree, no allocating library routine.  Same walk, streams, outputs and
 * synchronisation as ggns_hss_walk_plain (so not capturable itself).  A
 * context any of whose runs needs more than that buffer
 * (ggns_plain_workspace_bytes(ctx) > GGNS_STATIC_SCRATCH_BYTES) gets
 * GGNS_ESCRATCH and nothing is enqueued; a run that is not GGNS_FP64 gets
 * GGNS_EUNSUPPORTED.  Every call on one GPU shares that GPU's buffer, which
 * keeps the last call's contents (the walk initialises what it reads):
 * calls that overlap in time on one GPU, from any context or stream, race. */
#define GGNS_STATIC_SCRATCH_BYTES (16ll << 20)
int ggns_hss_walk_plain_static(ggns_ctx *ctx, void *stream);

int ggns_run_layout(const ggns_ctx *ctx, int32_t run, ggns_layout *out);

/* Copy every run's stats to host memory `out` (n_runs entries); synchronises `stream`. */
int ggns_read_stats(ggns_ctx *ctx, ggns_run_stats *out, void *stream);

/* The same copy, enqueued on `stream` without waiting: a small gather kernel
 * packs the records inside the arena, then one device-to-host copy fills
 * `out` (n_runs entries, caller owned).  `out` should be pinned host memory
 * (hipHostMalloc, or a pinned torch tensor) for the copy to run
 * asynchronously; it is valid once the stream (or an event recorded on it
 * after this call) has completed, and must not be read or reused before.  A
 * driver loop can so poll the runs' states one block of iterations behind
 * without draining the stream between blocks (a stopped run's launches are
 * no-ops, so the extra block enqueued meanwhile changes nothing).  Not for
 * graph capture. */
int ggns_read_stats_async(ggns_ctx *ctx, ggns_run_stats *out, void *stream);

/* Load log Zbar, log Xbar, dt and the iteration counter of one run. */
int ggns_write_vars(ggns_ctx *ctx, int32_t run, const ggns_run_vars *vars, void *stream);

/* Record the first trace_steps steps of each walker of `run` during later walks:
 * trace_x [trace_steps][n_kill][d] run precision, trace_logl [..][n_kill] double,
 * trace_out [..][n_kill] int32 (1 = outside).  NULL trace_x switches it off. */
int ggns_set_trace(ggns_ctx *ctx, int32_t run, void *trace_x, double *trace_logl,
                   int32_t *trace_out, int32_t trace_steps);

/* Keep the positions of a run's dead points (the weighted posterior samples
 * of Appendix A's importance weights) from now on: every later
 * ggns_evidence_update writes the position of each dead point it records to
 * row n_dead of dead_x_dev ([capacity_rows][d], the run's precision, device,
 * caller-owned; rows beyond capacity_rows are not written), in the order of the
 * dead records (log L, log w).  NULL or capacity 0 switches it off.
 * Synchronous with respect to the host. */
int ggns_set_dead_x(ggns_ctx *ctx, int32_t run, void *dead_x_dev, int64_t capacity_rows);

/* The walk tile of a run after defaults: coordinates per lane and lanes per
 * walker (matrix-core runs: dimensions per lane and 4 W lanes per walker). */
int ggns_tile_shape(const ggns_ctx *ctx, int32_t run, int32_t *coords_per_lane,
                    int32_t *lanes_per_walker);

/* The walk's momentum-noise stream (the eps of p <- p (1 + delta_p eps),
 * Algorithm GGNS HSS) on its own, for checking the stream and timing the
 * generator.  Walker m's coordinate block b at iteration `iteration` seeds
 * xoshiro128++ from Philox4x32-10(key seed; counter b, m, iteration,
 * EPS << 24) and draws four words per step, turned into four normals by
 * Box-Muller on 24-bit uniforms in FP32, as the walk does with per-component
 * noise (noise_mode 0; with one normal per walker the walk takes two words of
 * block 0 per step and the first normal of their pair).  With
 * i = ((t * n_walkers + m) * n_blocks + b) * 4 + j for step t < steps, j < 4:
 *   normals_dev[i] (float) and words_dev[i] (uint32), each nullable;
 *   checksum_dev[m * n_blocks + b] = sum of the thread's normals (nullable).
 * Device pointers, caller-owned; enqueued on `stream`.  GGNS_EINVAL for
 * negative sizes or more than 2^30 (walker, block) pairs. */
int ggns_noise_normals(uint64_t seed, int32_t iteration, int32_t n_walkers, int32_t n_blocks,
                       int32_t steps, float *normals_dev, uint32_t *words_dev, float *checksum_dev,
                       void *stream);

/* Device-rate probes, for the roofline: the rates this build reaches on the
 * vector ALU and on the matrix cores, beside the published peaks.  `blocks`
 * workgroups of 256 threads, each thread running `iters` rounds.
 * ggns_probe_valu: eight independent FP32 chains v <- fma(v, a, b) per
 * thread, started at v = (lane mod 64) / 64 + chain (16 iters FLOP per
 * thread; the walk's compilation: one FMA per lane and instruction).
 * ggns_probe_mfma: four independent v_mfma_f32_16x16x32_bf16 accumulations
 * per wavefront with every A entry a and every B entry b rounded to BF16
 * (16384 iters FLOP per accumulator and wavefront); each accumulator entry
 * gains 32 a b per round.
 * out_dev[thread] = the sum of the thread's chains or accumulator entries;
 * out_dev holds blocks * 256 floats, caller-owned device memory.  Enqueued on
 * `stream`.  GGNS_EINVAL for blocks outside [1, 2^20], iters < 0 or a null
 * out_dev. */
int ggns_probe_valu(int32_t blocks, int32_t iters, float a, float b, float *out_dev, void *stream);
int ggns_probe_mfma(int32_t blocks, int32_t iters, float a, float b, float *out_dev, void *stream);

void ggns_free(ggns_ctx *ctx);

const char *ggns_status_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* GGNS_H */
