// The plain FP64 form of the same walk, kept as the speed baseline: the
// execution model of a per-step tensor program (Algorithm GGNS HSS written as
// whole-batch array operations).  One thread per walker, the walk state (x, p,
// the score, the random-stream states and the counters) lives in HBM and is
// read and written back by one kernel launch per step, the host polls the
// number of active walkers between launches, and runs are walked one after
// the other.  It draws the same random streams and takes the same decisions as
// the fused walk (readings as there), so for FP64 runs the two agree up to the
// order of floating-point sums.  The batch-minimum loop (walk_mode 1) is the
// algorithm's lockstep loop as written: every walker steps in every launch,
// each launch records the run's minimum reflection count after its step, and
// the next launch (one more follows the last step) applies that step's save
// rule and stops every walker once the minimum has reached max_ref.
#include "ggns_device.h"

namespace ggns {

namespace {

// Walk state of one run, carved from the caller's workspace.  Component-major
// ([component][walker]) like the arrays of a batched tensor program, so that
// consecutive threads touch consecutive addresses.
struct PlainState {
    double *x, *p, *g, *out_l;  // x, p, g: [d][k]
    double *l;      // [k] log L at x (external-likelihood walk: written by the caller)
    uint32_t *eps;  // [nb * 4][k] xoshiro states, nb = ceil(d / 4)
    uint32_t *res;  // [4][k]
    int32_t *s, *nref, *streak, *steps, *outs, *nprune, *nsave, *done;
    int32_t *active;  // [n_steps_max + 1] walkers still walking after step t
    // batch-minimum loop: the run's minimum reflection count after step t,
    // and each walker's in-slice point of its last step awaiting the save rule
    int32_t *minref;  // [n_steps_max + 1]
    int32_t *pend;    // [k] 1: the last step was in-slice
    uint32_t *pures;  // [k] its reservoir word
    double *xc, *lc;  // [d][k], [k] its position and log L
};

__host__ __device__ inline int64_t plain_align(int64_t v) { return (v + 255) / 256 * 256; }

__host__ __device__ inline int64_t plain_bytes(int k, int d, int n_steps_max, PlainState *st,
                                               unsigned char *base) {
    const int nb = (d + 3) / 4;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        unsigned char *p = base ? base + off : nullptr;
        off = plain_align(off + bytes);
        return p;
    };
    double *x = (double *)take((int64_t)k * d * 8);
    double *p = (double *)take((int64_t)k * d * 8);
    double *g = (double *)take((int64_t)k * d * 8);
    double *ol = (double *)take((int64_t)k * 8);
    double *lx = (double *)take((int64_t)k * 8);
    uint32_t *eps = (uint32_t *)take((int64_t)k * nb * 16);
    uint32_t *res = (uint32_t *)take((int64_t)k * 16);
    int32_t *ints[9];
    for (int i = 0; i < 9; ++i) ints[i] = (int32_t *)take((int64_t)k * 4);
    int32_t *act = (int32_t *)take((int64_t)(n_steps_max + 1) * 4);
    int32_t *mref = (int32_t *)take((int64_t)(n_steps_max + 1) * 4);
    uint32_t *pu = (uint32_t *)take((int64_t)k * 4);
    double *xc = (double *)take((int64_t)k * d * 8);
    double *lc = (double *)take((int64_t)k * 8);
    if (st) {
        st->x = x; st->p = p; st->g = g; st->out_l = ol; st->l = lx; st->eps = eps; st->res = res;
        st->s = ints[0]; st->nref = ints[1]; st->streak = ints[2]; st->steps = ints[3];
        st->outs = ints[4]; st->nprune = ints[5]; st->nsave = ints[6]; st->done = ints[7];
        st->pend = ints[8];
        st->active = act;
        st->minref = mref;
        st->pures = pu;
        st->xc = xc;
        st->lc = lc;
    }
    return off;
}

__device__ void plain_momentum(uint64_t seed, uint32_t m, uint32_t it, uint32_t sub, int d, int64_t k,
                               double *p) {
    for (int b = 0; b * 4 < d; ++b) {
        uint32_t w[4];
        draw4(seed, (uint32_t)b, m, it, TAG_P0, sub, w);
        double z[4];
        normals2(w[0], w[1], z[0], z[1]);
        normals2(w[2], w[3], z[2], z[3]);
        for (int j = 0; j < 4 && 4 * b + j < d; ++j) p[(4 * b + j) * k + m] = z[j];
    }
}

// log L and its score at x (FP64, plain loops over the run's converted
// parameters; padding entries are never read).  x and g have stride k.
__device__ double plain_loglike(const RunDev &R, const double *prm, const double *xm, double *gm,
                                int64_t k) {
    const int d = R.d, dp = R.dp;
    auto x = [&](int a) { return xm[a * k]; };
    auto gset = [&](int a, double v) { gm[a * k] = v; };
    auto gadd = [&](int a, double v) { gm[a * k] += v; };
    if (R.kind == GGNS_LIK_GAUSS_DIAG) {
        double q = 0.0;
        for (int a = 0; a < d; ++a) {
            const double r = x(a) - prm[a];
            q += prm[dp + a] * r * r;
            gset(a, -prm[dp + a] * r);
        }
        return prm[2 * dp] - 0.5 * q;
    }
    if (R.kind == GGNS_LIK_TORUS) {
        double q = prm[2 * dp];
        for (int a = 0; a < d; ++a) q += sin(prm[a] * x(a) + prm[dp + a]);
        for (int a = 0; a < d; ++a) gset(a, 3.0 * prm[a] * cos(prm[a] * x(a) + prm[dp + a]) / q);
        return 3.0 * log(q);
    }
    if (R.kind == GGNS_LIK_GAUSS_FULL) {
        const double *P = prm + d + 1;
        double q = 0.0;
        for (int i = 0; i < d; ++i) {
            double y = 0.0;
            for (int j = 0; j < d; ++j) y += P[(int64_t)i * d + j] * (x(j) - prm[j]);
            q += (x(i) - prm[i]) * y;
            gset(i, -y);
        }
        return prm[d] - 0.5 * q;
    }
    const int K = R.n_comp;
    double lp[kMaxComp], aux[kMaxComp];
    double l = -INFINITY;
    if (R.kind == GGNS_LIK_SHELLS) {
        for (int c = 0; c < K; ++c) {
            const double *o = prm + c * (dp + 3);
            double s = 0.0;
            for (int a = 0; a < d; ++a) s += (x(a) - o[a]) * (x(a) - o[a]);
            aux[c] = sqrt(s);
            const double e = aux[c] - o[dp];
            lp[c] = o[dp + 2] - 0.5 * e * e * o[dp + 1];
            const double hi = fmax(l, lp[c]);
            l = (hi == -INFINITY) ? hi : hi + log(exp(l - hi) + exp(lp[c] - hi));
        }
        for (int a = 0; a < d; ++a) gset(a, 0.0);
        for (int c = 0; c < K; ++c) {
            const double *o = prm + c * (dp + 3);
            if (!(aux[c] > 0.0)) continue;
            const double coef = -exp(lp[c] - l) * (aux[c] - o[dp]) * o[dp + 1] / aux[c];
            for (int a = 0; a < d; ++a) gadd(a, coef * (x(a) - o[a]));
        }
        return l;
    }
    for (int c = 0; c < K; ++c) {
        const double *o = prm + c * gmm_stride(dp);
        double q = 0.0;
        for (int a = 0; a < d; ++a) q += o[dp + a] * (x(a) - o[a]) * (x(a) - o[a]);
        lp[c] = o[2 * dp] - 0.5 * q;
        const double hi = fmax(l, lp[c]);
        l = (hi == -INFINITY) ? hi : hi + log(exp(l - hi) + exp(lp[c] - hi));
    }
    for (int a = 0; a < d; ++a) gset(a, 0.0);
    for (int c = 0; c < K; ++c) {
        const double *o = prm + c * gmm_stride(dp);
        const double resp = exp(lp[c] - l);
        for (int a = 0; a < d; ++a) gadd(a, -resp * o[dp + a] * (x(a) - o[a]));
    }
    return l;
}

__global__ void plain_start_kernel(void *arena, const RunDev *__restrict__ runs, int run,
                                   unsigned char *ws) {
    const RunDev &R = runs[run];
    const Acc *acc = at<Acc>(arena, R.off_acc);
    PlainState S;
    plain_bytes(R.n_kill, R.d, R.n_steps_max, &S, ws);
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    for (int t = m; t <= R.n_steps_max; t += gridDim.x * blockDim.x) {
        S.active[t] = 0;
        S.minref[t] = INT_MAX;
    }
    if (acc->state != GGNS_RUN_ACTIVE || m >= R.n_kill) return;
    const int d = R.d, nsurv = R.n_live - R.n_kill, nb = (d + 3) / 4;
    const int64_t k = R.n_kill;
    const uint32_t it = (uint32_t)acc->iter;
    uint32_t w[4];
    draw4(R.seed, 0u, (uint32_t)m, it, TAG_START, 0u, w);
    int cl;
    const int s = pick_start(R, arena, w, &cl);
    at<int32_t>(arena, R.off_start)[m] = s;
    if (R.cluster_mode) at<int32_t>(arena, R.off_start_cl)[m] = cl;
    const double *xs = at<double>(arena, R.off_live_x) + (int64_t)s * d;
    double *wo = at<double>(arena, R.off_walk_x) + (int64_t)m * d;
    for (int a = 0; a < d; ++a) S.x[a * k + m] = wo[a] = xs[a];
    S.out_l[m] = at<double>(arena, R.off_live_logl)[s];
    plain_momentum(R.seed, (uint32_t)m, it, 0u, d, k, S.p);
    for (int b = 0; b < nb; ++b) {
        draw4(R.seed, (uint32_t)b, (uint32_t)m, it, TAG_EPS, 0u, w);
        Xoshiro e;
        e.seed(w);
        uint32_t *st = S.eps + (int64_t)(4 * b) * k + m;
        st[0] = e.s0; st[k] = e.s1; st[2 * k] = e.s2; st[3 * k] = e.s3;
    }
    draw4(R.seed, 0u, (uint32_t)m, it, TAG_RES, 0u, w);
    Xoshiro r;
    r.seed(w);
    S.res[m] = r.s0; S.res[k + m] = r.s1; S.res[2 * k + m] = r.s2; S.res[3 * k + m] = r.s3;
    S.s[m] = s;
    S.nref[m] = S.streak[m] = S.steps[m] = S.outs[m] = S.nprune[m] = S.nsave[m] = S.done[m] = 0;
    S.pend[m] = 0;
}

// One step of every walker of the run.  EXT = false: drift, then log L and the
// score from the run's own family.  EXT = true (external likelihood): the
// caller has evaluated log L and the score at the already drifted positions
// into the workspace; after the step the walkers that go on drift for the
// next one, so the caller always evaluates at the current positions.
template <bool EXT>
__global__ void plain_step_kernel(void *arena, const RunDev *__restrict__ runs, int run,
                                  unsigned char *ws, int t) {
    const RunDev &R = runs[run];
    Acc *acc = at<Acc>(arena, R.off_acc);
    if (acc->state != GGNS_RUN_ACTIVE) return;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= R.n_kill) return;
    PlainState S;
    plain_bytes(R.n_kill, R.d, R.n_steps_max, &S, ws);
    if (S.done[m]) return;
    const int d = R.d, nb = (d + 3) / 4;
    const int64_t k = R.n_kill;
    const double dt = acc->dt, lstar = acc->lstar, dpn = R.delta_p;
    const uint32_t it = (uint32_t)acc->iter;
    double *x = S.x + m, *p = S.p + m, *g = S.g + m;  // component a at [a * k]
    const double *prm = at<double>(arena, R.off_prm);
    const bool batch = R.walk_mode == 1;
    auto finish = [&]() {
        S.done[m] = 1;
        const int steps = S.steps[m], outs = S.outs[m];
        at<double>(arena, R.off_walk_logl)[m] = S.out_l[m];
        atomicAdd(&acc->it_outs, (unsigned long long)outs);
        atomicAdd(&acc->it_steps, (unsigned long long)steps);
        atomicAdd(reinterpret_cast<unsigned long long *>(&acc->steps_out), (unsigned long long)outs);
        atomicAdd(reinterpret_cast<unsigned long long *>(&acc->steps_in),
                  (unsigned long long)(steps - outs));
        atomicAdd(reinterpret_cast<unsigned long long *>(&acc->evals), (unsigned long long)steps);
        atomicAdd(reinterpret_cast<unsigned long long *>(&acc->prunes),
                  (unsigned long long)S.nprune[m]);
        atomicAdd(reinterpret_cast<unsigned long long *>(&acc->nosave),
                  (unsigned long long)(S.nsave[m] == 0 ? 1 : 0));
    };
    if (batch && t > 0) {
        // the save rule of the previous step, now that the run's minimum
        // reflection count after it is known; then the loop condition
        const int mr = S.minref[t - 1];
        if (S.pend[m]) {
            const bool keep = mr >= R.min_ref;
            const int nsave = S.nsave[m] + (keep ? 1 : 0);
            const bool take =
                keep ? ((uint64_t)S.pures[m] * (uint64_t)nsave < (1ull << 32)) : (nsave == 0);
            if (take) {
                double *wo = at<double>(arena, R.off_walk_x) + (int64_t)m * d;
                for (int a = 0; a < d; ++a) wo[a] = S.xc[a * k + m];
                S.out_l[m] = S.lc[m];
            }
            S.nsave[m] = nsave;
            S.pend[m] = 0;
        }
        if (mr >= R.max_ref || t >= R.n_steps_max) {
            finish();
            return;
        }
    }

    // drift, log L and the score
    double l;
    if constexpr (EXT) {
        l = S.l[m];
    } else {
        for (int a = 0; a < d; ++a) x[a * k] += dt * p[a * k];
        l = plain_loglike(R, prm, x, g, k);
    }
    bool viol = false;
    for (int a = 0; a < d; ++a) viol = viol || x[a * k] < R.lo || x[a * k] > R.hi;
    const bool out = viol || l <= lstar;
    const int steps = S.steps[m] + 1;
    // reflection and the componentwise momentum noise of this step
    double pg = 0.0, gg = 0.0;
    for (int a = 0; a < d; ++a) {
        pg += p[a * k] * g[a * k];
        gg += g[a * k] * g[a * k];
    }
    const bool use_g = out && !viol && isfinite(gg) && gg > 0.0;
    const bool flip_all = out && !viol && !use_g;
    const double f = use_g ? 2.0 * pg / gg : 0.0;
    // noise_mode 1: one normal per walker, two words of block 0's stream and
    // the first normal of their pair; noise_mode 0: four words per block
    double e0 = 0.0;
    if (R.noise_mode) {
        uint32_t *st = S.eps + m;
        Xoshiro e{st[0], st[k], st[2 * k], st[3 * k]};
        const uint32_t w0 = e.next(), w1 = e.next();
        st[0] = e.s0; st[k] = e.s1; st[2 * k] = e.s2; st[3 * k] = e.s3;
        e0 = normal_first(w0, w1, e0);
    }
    for (int b = 0; b < nb; ++b) {
        double z[4];
        if (R.noise_mode) {
            for (int j = 0; j < 4; ++j) z[j] = e0;
        } else {
            uint32_t *st = S.eps + (int64_t)(4 * b) * k + m;
            Xoshiro e{st[0], st[k], st[2 * k], st[3 * k]};
            uint32_t w[4];
            for (int j = 0; j < 4; ++j) w[j] = e.next();
            st[0] = e.s0; st[k] = e.s1; st[2 * k] = e.s2; st[3 * k] = e.s3;
            normals2(w[0], w[1], z[0], z[1]);
            normals2(w[2], w[3], z[2], z[3]);
        }
        for (int j = 0; j < 4 && 4 * b + j < d; ++j) {
            const int64_t a = (4 * b + j) * k;
            const bool flip = flip_all || (out && (x[a] < R.lo || x[a] > R.hi));
            const double pr = (flip ? -p[a] : p[a]) - f * g[a];
            p[a] = pr * (1.0 + dpn * z[j]);
        }
    }
    Xoshiro rs{S.res[m], S.res[k + m], S.res[2 * k + m], S.res[3 * k + m]};
    const uint32_t ures = rs.next();
    S.res[m] = rs.s0; S.res[k + m] = rs.s1; S.res[2 * k + m] = rs.s2; S.res[3 * k + m] = rs.s3;
    // bookkeeping: reflections, the kept-point reservoir, pruning, the stop
    int nref = S.nref[m] + (out ? 1 : 0);
    const int outs = S.outs[m] + (out ? 1 : 0);
    int streak = out ? S.streak[m] + 1 : 0;
    int nsave = S.nsave[m];
    if (batch) {
        // the save rule waits for the run's minimum after this step
        S.pend[m] = out ? 0 : 1;
        if (!out) {
            for (int a = 0; a < d; ++a) S.xc[a * k + m] = x[a * k];
            S.lc[m] = l;
            S.pures[m] = ures;
        }
    } else {
        const bool keep = !out && nref >= R.min_ref;
        nsave += keep ? 1 : 0;
        const bool take = !out && (keep ? ((uint64_t)ures * (uint64_t)nsave < (1ull << 32)) : (nsave == 0));
        if (take) {
            double *wo = at<double>(arena, R.off_walk_x) + (int64_t)m * d;
            for (int a = 0; a < d; ++a) wo[a] = x[a * k];
            S.out_l[m] = l;
        }
    }
    int nprune = S.nprune[m];
    if (R.prune_streak > 0 && streak >= R.prune_streak) {
        const double *xs = at<double>(arena, R.off_live_x) + (int64_t)S.s[m] * d;
        for (int a = 0; a < d; ++a) x[a * k] = xs[a];
        nprune += 1;
        plain_momentum(R.seed, (uint32_t)m, it, (uint32_t)nprune, d, k, S.p);
        // the batch minimum never decreases: its count is kept
        nref = batch ? nref : 0;
        streak = 0;
    }
    S.nref[m] = nref; S.outs[m] = outs; S.streak[m] = streak; S.steps[m] = steps;
    S.nsave[m] = nsave; S.nprune[m] = nprune;
    if (batch) {
        atomicMin(&S.minref[t], nref);
        atomicAdd(&S.active[t], 1);
        if constexpr (EXT)
            for (int a = 0; a < d; ++a) x[a * k] += dt * p[a * k];
        return;
    }
    const bool done = !(steps < R.n_steps_max && (R.max_ref == 0 || nref < R.max_ref));
    if (done) {
        finish();
    } else {
        atomicAdd(&S.active[t], 1);
        if constexpr (EXT)
            for (int a = 0; a < d; ++a) x[a * k] += dt * p[a * k];
    }
}

// External-likelihood walk, first step's positions: the starts drifted once.
__global__ void ext_drift_kernel(void *arena, const RunDev *__restrict__ runs, int run,
                                 unsigned char *ws) {
    const RunDev &R = runs[run];
    const Acc *acc = at<Acc>(arena, R.off_acc);
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (acc->state != GGNS_RUN_ACTIVE || m >= R.n_kill) return;
    PlainState S;
    plain_bytes(R.n_kill, R.d, R.n_steps_max, &S, ws);
    const int64_t k = R.n_kill;
    const double dt = acc->dt;
    for (int a = 0; a < R.d; ++a) S.x[a * k + m] += dt * S.p[a * k + m];
}

}  // namespace

int64_t plain_workspace_bytes(const RunDev &R) {
    return plain_bytes(R.n_kill, R.d, R.n_steps_max, nullptr, nullptr);
}

int launch_walk_plain(void *arena, const RunDev *runs_dev, int run, const RunDev &R, void *ws,
                      int poll_every, hipStream_t s) {
    const int threads = 256, blocks = (R.n_kill + threads - 1) / threads;
    unsigned char *w = reinterpret_cast<unsigned char *>(ws);
    hipLaunchKernelGGL(plain_start_kernel, dim3(blocks), dim3(threads), 0, s, arena, runs_dev, run, w);
    if (hipGetLastError() != hipSuccess) return GGNS_EHIP;
    PlainState S;
    plain_bytes(R.n_kill, R.d, R.n_steps_max, &S, w);
    // the batch-minimum loop takes one launch more: the save rule of the last step
    const int n_launch = R.n_steps_max + (R.walk_mode == 1 ? 1 : 0);
    for (int t = 0; t < n_launch; ++t) {
        hipLaunchKernelGGL(plain_step_kernel<false>, dim3(blocks), dim3(threads), 0, s, arena, runs_dev,
                           run, w, t);
        if (hipGetLastError() != hipSuccess) return GGNS_EHIP;
        if ((t + 1) % poll_every == 0 && t + 1 < n_launch) {
            int32_t n_active = 0;
            if (hipMemcpyAsync(&n_active, S.active + t, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return GGNS_EHIP;
            if (n_active == 0) break;
        }
    }
    return GGNS_OK;
}

int launch_ext_begin(void *arena, const RunDev *runs_dev, int run, const RunDev &R, void *ws,
                     hipStream_t s) {
    const int threads = 256, blocks = (R.n_kill + threads - 1) / threads;
    unsigned char *w = reinterpret_cast<unsigned char *>(ws);
    hipLaunchKernelGGL(plain_start_kernel, dim3(blocks), dim3(threads), 0, s, arena, runs_dev, run, w);
    hipLaunchKernelGGL(ext_drift_kernel, dim3(blocks), dim3(threads), 0, s, arena, runs_dev, run, w);
    return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

int launch_ext_step(void *arena, const RunDev *runs_dev, int run, const RunDev &R, void *ws, int t,
                    hipStream_t s) {
    const int threads = 256, blocks = (R.n_kill + threads - 1) / threads;
    hipLaunchKernelGGL(plain_step_kernel<true>, dim3(blocks), dim3(threads), 0, s, arena, runs_dev, run,
                       reinterpret_cast<unsigned char *>(ws), t);
    return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

void ext_buffers(const RunDev &R, void *ws, double **x, double **logl, double **grad,
                 int32_t **active) {
    PlainState S;
    plain_bytes(R.n_kill, R.d, R.n_steps_max, &S, reinterpret_cast<unsigned char *>(ws));
    *x = S.x;
    *logl = S.l;
    *grad = S.g;
    *active = S.active;
}

}  // namespace ggns
