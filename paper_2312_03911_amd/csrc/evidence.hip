// Termination test, kill, evidence and prior-volume bookkeeping, final sweep
// and run summary; one workgroup of 1024 threads per run.
//
// Paper: Appendix A (Z = sum L_i w_i with w_i the prior-volume shell, X shrinks
// by n/(n+1) per kill), Algorithm GGNS (kill n_kill points per iteration, the
// X*L peak test, final sweep of the live points) and Eqs. (update0)-(update9)
// for the moments.  Batch form used here: killing k of n points one by one
// with n_p = n, n-1, ..., n-k+1 gives every killed point the same expected
// shell Xbar/(n+1) and leaves Xbar (n+1-k)/(n+1) (the per-kill factors
// telescope), so one iteration needs a sort, one log-sum-exp and one update.
// The final sweep uses n_p = n, ..., 1, which gives every remaining point
// Xbar/(n+1).  All of it is FP64.
#include "ggns_device.h"

namespace ggns {

namespace {

constexpr int kEvThreads = 1024;

// Order-preserving 64-bit key of a log L.  -0 and +0 compare equal (a tie,
// broken by slot like any other), so -0 takes the key of +0.
__device__ __forceinline__ unsigned long long order_key(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v == 0.0 ? 0.0 : v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double key_value(unsigned long long k) {
    const unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return __longlong_as_double((long long)b);
}

// Running log-sum-exp accumulator: (m, s) represents m + log(s).
__device__ __forceinline__ void lse_push(double v, double &m, double &s) {
    if (v == -INFINITY) return;
    if (v > m) {
        s = (m == -INFINITY) ? 1.0 : s * exp(m - v) + 1.0;
        m = v;
    } else {
        s += exp(v - m);
    }
}

__device__ __forceinline__ double lae(double a, double b) {
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    const double m = a > b ? a : b;
    return m + log(exp(a - m) + exp(b - m));
}

// Block reductions over 1024 threads (16 waves).
__device__ double block_max(double v, double *scratch) {
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(v, o, 64);
        v = t > v ? t : v;
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    double r = scratch[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = scratch[i] > r ? scratch[i] : r;
    __syncthreads();
    return r;
}

__device__ double block_sum(double v, double *scratch) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += scratch[i];
    __syncthreads();
    return r;
}

// log-sum-exp over the block of per-thread partial (max, sum exp(v - max)).
__device__ double block_lse(double lmax_local, double sum_local, double *scratch) {
    const double gmax = block_max(lmax_local, scratch);
    if (gmax == -INFINITY) return -INFINITY;
    const double part = (lmax_local == -INFINITY) ? 0.0 : sum_local * exp(lmax_local - gmax);
    return gmax + log(block_sum(part, scratch));
}

// Exclusive scans over the block's per-thread values: an inclusive scan
// inside each wavefront with lane shuffles, the wavefront totals through LDS
// (one barrier), each thread adding the totals of the wavefronts before it.
template <typename T, typename Op>
__device__ __forceinline__ T block_exscan(T v, T ident, Op op, T *wtot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T a = __shfl_up(incl, o, 64);
        if (lane >= o) incl = op(a, incl);
    }
    T excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = ident;
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    T pre = ident;
    for (int i = 0; i < w; ++i) pre = op(pre, wtot[i]);
    __syncthreads();   // wtot may be reused by the next scan
    return op(pre, excl);
}

__device__ double block_exscan_lae(double v, double *buf) {
    return block_exscan<double>(v, -INFINITY, [](double a, double b) { return lae(a, b); }, buf);
}

__device__ int block_exscan_int(int v, int *buf) {
    return block_exscan<int>(v, 0, [](int a, int b) { return a + b; }, buf);
}


// Block-wide maximum and sum with one barrier each: DPP and lane permutes
// inside the wavefront, the 16 wavefront results through LDS.  Every call
// takes its own 16 slots of scratch, so none needs a trailing barrier.
__device__ __forceinline__ double wave_max_d(double v) {
    v = fmax(v, dpp_mov<kDppXor1>(v));
    v = fmax(v, dpp_mov<kDppXor2>(v));
    v = fmax(v, dpp_mov<kDppHalfMirror>(v));
    v = fmax(v, dpp_mov<kDppMirror>(v));
    v = fmax(v, __shfl_xor(v, 16, 64));
    return fmax(v, __shfl_xor(v, 32, 64));
}
__device__ __forceinline__ double wave_sum_d(double v) {
    v += dpp_mov<kDppXor1>(v);
    v += dpp_mov<kDppXor2>(v);
    v += dpp_mov<kDppHalfMirror>(v);
    v += dpp_mov<kDppMirror>(v);
    v += __shfl_xor(v, 16, 64);
    return v + __shfl_xor(v, 32, 64);
}
__device__ double block_max_once(double v, double *sc) {
    v = wave_max_d(v);
    if ((threadIdx.x & 63) == 0) sc[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sc[0];
    for (int i = 1; i < kEvThreads / 64; ++i) r = fmax(r, sc[i]);
    return r;
}
__device__ double block_sum_once(double v, double *sc) {
    v = wave_sum_d(v);
    if ((threadIdx.x & 63) == 0) sc[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < kEvThreads / 64; ++i) r += sc[i];
    return r;
}

// One iteration of one run (Algorithm GGNS, the kill loop, and Eqs. update0 to
// update9 in batch form), with its n log L held E per thread: termination
// test, kill order, dead records and evidence, volumes, survivors.  The run's
// accumulators are read once, at the start, next to the log L loads.
// The n log L of a run in slot order as (key, slot) pairs, E per thread.
template <int E>
__device__ __forceinline__ void load_pairs(const double *ll, int n, unsigned long long (&kk)[E],
                                           int (&ss)[E], double &vmax, bool &bad) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = E * threadIdx.x + e;
        if (i < n) {
            const double v = ll[i];
            bad = bad | isnan(v);
            vmax = v > vmax ? v : vmax;
            kk[e] = order_key(v);
            ss[e] = i;
        } else {
            kk[e] = ~0ull;
            ss[e] = 0x7FFFFFFF;
        }
    }
}

// Pairs (log L key, slot) of the list entries slots[i], i < m, H per thread.
template <int H>
__device__ __forceinline__ void gather_pairs(const double *ll, const int32_t *slots, int m,
                                             unsigned long long (&kk)[H], int (&ss)[H],
                                             double &vmax, bool &bad) {
#pragma unroll
    for (int e = 0; e < H; ++e) {
        const int i = H * threadIdx.x + e;
        if (i < m) {
            const int sl = slots[i];
            const double v = ll[sl];
            bad = bad | isnan(v);
            vmax = v > vmax ? v : vmax;
            kk[e] = order_key(v);
            ss[e] = sl;
        } else {
            kk[e] = ~0ull;
            ss[e] = 0x7FFFFFFF;
        }
    }
}

// Entries of the ascending (key, slot) list lk/ls[0, m) smaller than (kv, sv)
// (m <= 4095; the pairs are distinct, so no entry equals it).
__device__ __forceinline__ int count_below(const unsigned long long *lk, const int *ls, int m,
                                           unsigned long long kv, int sv) {
    int pos = 0;
#pragma unroll
    for (int step = 2048; step > 0; step >>= 1) {
        const int q = pos + step;
        if (q <= m && kv_greater(kv, sv, lk[q - 1], ls[q - 1])) pos = q;
    }
    return pos;
}

// Cluster mode: the moments of the cluster recursion (Eqs. update1, update3-
// update9) over one batch of kills, in kill order (ascending log L, then
// slot).  Within a batch the per-kill factors telescope: the r-th kill of
// cluster q, which held n0 points at the batch start, sees
//   Xbar_q = Xbar_q0 (n0+1-r)/(n0+1),
//   (X_q^2)bar = (X_q^2)bar_0 (n0+1-r)(n0+2-r)/((n0+1)(n0+2)),
//   (X_a X_q)bar = (X_a X_q)bar_0 f_a f_q,   f = (n0+1-r)/(n0+1) per cluster.
// With G_q = (Z X_q)bar / f_q and H_q = (Z_q X_q)bar / f_q every update
// becomes a sum over earlier kills with coefficients fixed at the batch start:
// a kill of log L l in cluster a adds to G_q
//   (a == q) (X_q^2)bar_0 L / (n0_q+2),   (a != q) (X_a X_q)bar_0 L / (n0_a+1),
// and to H_a the first of these; the kill itself adds to Z2bar
//   2 L G_a / (n0_a+1) + 2 (X_a^2)bar_0 L^2 / ((n0_a+1)(n0_a+2))
// (G_a before it), to (Z_a^2)bar the same with H_a, and to Zbar_a
// Xbar_a0 L / (n0_a+1).  The sums run in linear space, scaled per cluster
// (kill values by the cluster's largest log L, G and H by their largest
// term), as an exclusive scan over chunks of the kill list for every target
// cluster at once: thread t takes target q = t mod Q and chunk t / Q.  Called
// by every thread of the block, before the volumes are updated.
__device__ void cluster_moments(ClusterTab *tab, const int32_t *label, const unsigned long long *key,
                                const int *slot, int nkill, const int *kcount, Acc *acc) {
    __shared__ double ev[kMaxLive];               // exp(log L_j - lam[cluster of j])
    __shared__ unsigned char kc[kMaxLive];        // cluster of kill j
    __shared__ double kap[kClMax * kClMax];       // [a][q] G coefficient, scaled
    __shared__ double bg[kEvThreads], bh[kEvThreads];   // per (chunk, target) partials
    double *b3 = ev, *b4 = ev + kEvThreads;       // ev is free once the chunks are walked
    __shared__ double lam[kClMax], mq[kClMax], nq[kClMax], g0[kClMax], h0[kClMax], rho[kClMax];
    __shared__ double gfin[kClMax], hfin[kClMax], lf[kClMax], zq[kClMax];
    __shared__ int lastj[kClMax];
    const int t = threadIdx.x, T = blockDim.x;
    const int nc = tab->n_clusters;
    for (int q = t; q < kClMax; q += T) lastj[q] = -1;
    __syncthreads();
    for (int j = t; j < nkill; j += T) {
        const int a = label[slot[j]];
        kc[j] = (unsigned char)a;
        atomicMax(&lastj[a], j);
    }
    __syncthreads();
    // per cluster: its largest killed log L, log f after the batch, and the
    // scales of G and H
    for (int q = t; q < nc; q += T) {
        lam[q] = (lastj[q] >= 0) ? key_value(key[lastj[q]]) : -INFINITY;
        const int n0 = tab->cn[q], kq = kcount[q];
        lf[q] = (kq > 0) ? log((double)(n0 + 1 - kq)) - log((double)n0 + 1.0) : 0.0;
    }
    __syncthreads();
    for (int q = t; q < nc; q += T) {
        const int n0 = tab->cn[q];
        double m = tab->lzx[q];
        for (int a = 0; a < nc; ++a) {
            if (lastj[a] < 0) continue;
            const double lc = (a == q) ? tab->lx2[q] - log((double)n0 + 2.0)
                                       : tab->lxx[a * kClMax + q] - log((double)tab->cn[a] + 1.0);
            const double v = lc + lam[a];
            m = v > m ? v : m;
        }
        mq[q] = m;
        g0[q] = (m == -INFINITY || tab->lzx[q] == -INFINITY) ? 0.0 : exp(tab->lzx[q] - m);
        double nh = tab->lzpx[q];
        const double hv = (lastj[q] >= 0) ? tab->lx2[q] - log((double)n0 + 2.0) + lam[q] : -INFINITY;
        nh = hv > nh ? hv : nh;
        nq[q] = nh;
        h0[q] = (nh == -INFINITY || tab->lzpx[q] == -INFINITY) ? 0.0 : exp(tab->lzpx[q] - nh);
        rho[q] = (nh == -INFINITY || hv == -INFINITY) ? 0.0 : exp(hv - nh);
    }
    __syncthreads();
    for (int e = t; e < nc * nc; e += T) {
        const int a = e / nc, q = e % nc;
        double v = 0.0;
        if (lastj[a] >= 0 && mq[q] != -INFINITY) {
            const double lc = (a == q) ? tab->lx2[q] - log((double)tab->cn[q] + 2.0)
                                       : tab->lxx[a * kClMax + q] - log((double)tab->cn[a] + 1.0);
            if (lc != -INFINITY) v = exp(lc + lam[a] - mq[q]);
        }
        kap[a * kClMax + q] = v;
    }
    for (int j = t; j < nkill; j += T) ev[j] = exp(key_value(key[j]) - lam[kc[j]]);
    __syncthreads();
    // targets Q (a power of two >= nc) by chunks C
    int Q = 1;
    while (Q < nc) Q <<= 1;
    const int C = T / Q, q = t & (Q - 1), c = t / Q;
    const int csz = (nkill + C - 1) / C, j0 = c * csz, j1 = (j0 + csz < nkill) ? j0 + csz : nkill;
    const bool on = q < nc;
    double sg = 0.0, sh = 0.0;
    if (on)
        for (int j = j0; j < j1; ++j) {
            const int a = kc[j];
            sg += kap[a * kClMax + q] * ev[j];
            if (a == q) sh += rho[q] * ev[j];
        }
    // exclusive scan over the chunks of each target (Hillis-Steele on the
    // partials shifted by one chunk)
    if (c + 1 < C) { bg[(c + 1) * Q + q] = sg; bh[(c + 1) * Q + q] = sh; }
    if (c == 0) { bg[q] = 0.0; bh[q] = 0.0; }
    __syncthreads();
    for (int off = 1; off < C; off <<= 1) {
        const double vg = (c >= off) ? bg[(c - off) * Q + q] : 0.0;
        const double vh = (c >= off) ? bh[(c - off) * Q + q] : 0.0;
        __syncthreads();
        bg[c * Q + q] += vg;
        bh[c * Q + q] += vh;
        __syncthreads();
    }
    double g = on ? g0[q] + bg[c * Q + q] : 0.0, h = on ? h0[q] + bh[c * Q + q] : 0.0;
    double cross = 0.0, own = 0.0, sq = 0.0, zp = 0.0;
    if (on)
        for (int j = j0; j < j1; ++j) {
            const int a = kc[j];
            const double e = ev[j];
            if (a == q) {
                cross += e * g;
                own += e * h;
                sq += e * e;
                zp += e;
                h += rho[q] * e;
            }
            g += kap[a * kClMax + q] * e;
        }
    if (on && c == C - 1) { gfin[q] = g; hfin[q] = h; }
    __syncthreads();
    // sums over the chunks of each target
    bg[c * Q + q] = cross;
    bh[c * Q + q] = own;
    b3[c * Q + q] = sq;
    b4[c * Q + q] = zp;
    __syncthreads();
    for (int s = C >> 1; s > 0; s >>= 1) {
        if (c < s) {
            bg[c * Q + q] += bg[(c + s) * Q + q];
            bh[c * Q + q] += bh[(c + s) * Q + q];
            b3[c * Q + q] += b3[(c + s) * Q + q];
            b4[c * Q + q] += b4[(c + s) * Q + q];
        }
        __syncthreads();
    }
    const double l2 = 0.69314718055994530942;
    if (t < nc) {
        const int p = t, n0 = tab->cn[p], kp = kcount[p];
        const double ln1 = log((double)n0 + 1.0), ln2 = log((double)n0 + 2.0);
        double z2 = -INFINITY;
        if (kp > 0) {
            const double lcr = (bg[p] > 0.0) ? l2 + lam[p] + mq[p] - ln1 + log(bg[p]) : -INFINITY;
            const double lsq = l2 + tab->lx2[p] - ln1 - ln2 + 2.0 * lam[p] + log(b3[p]);
            const double lown = (bh[p] > 0.0) ? l2 + nq[p] + lam[p] - ln1 + log(bh[p]) : -INFINITY;
            z2 = lae(lcr, lsq);
            tab->lz2p[p] = lae(tab->lz2p[p], lae(lown, lsq));                           // update4
            tab->lzp[p] = lae(tab->lzp[p], tab->clx[p] - ln1 + lam[p] + log(b4[p]));     // update1
            tab->lzpx[p] = (hfin[p] > 0.0) ? lf[p] + nq[p] + log(hfin[p]) : -INFINITY;  // update7
            tab->lx2[p] += log((double)(n0 + 1 - kp) * (double)(n0 + 2 - kp)) - ln1 - ln2;  // update8
        }
        // update5, update6 (every cluster, killed from or not)
        tab->lzx[p] = (gfin[p] > 0.0) ? lf[p] + mq[p] + log(gfin[p]) : -INFINITY;
        zq[p] = z2;
    }
    __syncthreads();
    // update9 on every pair, then the run's Z2bar (update3)
    for (int e = t; e < nc * nc; e += T) {
        const int a = e / nc, b = e % nc;
        if (a != b) tab->lxx[a * kClMax + b] += lf[a] + lf[b];
    }
    if (t == 0) {
        double s = acc->log_z2;
        for (int p = 0; p < nc; ++p) s = lae(s, zq[p]);
        acc->log_z2 = s;
    }
    __syncthreads();
}

template <int E>
__device__ void evidence_body(void *arena, const RunDev &R, Acc *acc, int final_sweep,
                              unsigned long long *key, int *slot, unsigned char *dead_flag,
                              int *kcount, int *ibuf, double *scratch, int *flags) {
    const int n = R.n_live, k = R.n_kill;
    const int t = threadIdx.x, T = blockDim.x;
    const double *ll = at<double>(arena, R.off_live_logl);
    unsigned long long kk[E];
    int ss[E];
    double vmax = -INFINITY;
    bool bad = false;
    // Runs of more than 1024 live points (E = 2, 4) whose previous kill left
    // its order behind: the k new points are the only unsorted ones (the
    // survivors' log L are unchanged since that kill), so they are sorted alone
    // (512 E entries) and merged with the survivors' list; the result is the
    // same total order as the full sort
    constexpr int H = (E >= 2) ? E / 2 : 1;   // pairs per thread of each list
    constexpr int SN = 1024 * H;                // entries of the new points' sort
    unsigned long long ka[H], kb[H];
    int sa[H], sb[H];
    bool merge = false;
    if constexpr (E >= 2)
        merge = R.cluster_mode == 0 && acc->order_ok != 0 && k <= SN && n - k <= SN;
    if (merge) {
        gather_pairs<H>(ll, at<int32_t>(arena, R.off_killed), k, ka, sa, vmax, bad);
        gather_pairs<H>(ll, at<int32_t>(arena, R.off_surv_sorted), n - k, kb, sb, vmax, bad);
    } else {
        load_pairs<E>(ll, n, kk, ss, vmax, bad);
    }
    // the accumulator fields this launch reads (the termination test's and the
    // kill's), loaded once
    Acc a;
    a.state = acc->state;
    a.log_x = acc->log_x;
    a.log_z = acc->log_z;
    a.lstar = acc->lstar;
    a.log_xl_max = acc->log_xl_max;
    a.iter = acc->iter;
    a.n_dead = acc->n_dead;
    if (a.state != GGNS_RUN_ACTIVE) return;
    for (int i = t; i < E * 1024; i += T) dead_flag[i] = 0;
    for (int p = t; p < kClMax; p += T) kcount[p] = 0;
    // the largest log L and, through the same barrier, whether any is NaN
    {
        const double wm = wave_max_d(vmax);
        const bool wbad = __ballot(bad) != 0ull;
        if ((t & 63) == 0) {
            scratch[t >> 6] = wm;
            flags[t >> 6] = wbad ? 1 : 0;
        }
    }
    __syncthreads();
    double lmax = scratch[0];
    int anybad = flags[0];
    for (int i = 1; i < kEvThreads / 64; ++i) {
        lmax = fmax(lmax, scratch[i]);
        anybad |= flags[i];
    }
    if (anybad) {
        if (t == 0) acc->state = GGNS_RUN_NONFINITE;
        return;
    }
    double xl = a.log_xl_max;
    const int stop = termination_decision(R, &a, lmax, final_sweep, &xl);
    if (t == 0) acc->log_xl_max = xl;
    if (merge) {
        // the survivors' list above the range the new points sort in; it must
        // still be in order (no log L of a survivor changed), else the whole
        // set is sorted after all
        const int nb = n - k;
        unsigned long long *bk = key + SN;
        int *bs = slot + SN;
#pragma unroll
        for (int e = 0; e < H; ++e) {
            const int i = H * t + e;
            if (i < nb) {
                bk[i] = kb[e];
                bs[i] = sb[e];
            }
        }
        __syncthreads();
        bool unsorted = false;
#pragma unroll
        for (int e = 0; e < H; ++e) {
            const int i = H * t + e;
            if (i + 1 < nb) unsorted = unsorted | kv_greater(bk[i], bs[i], bk[i + 1], bs[i + 1]);
        }
        merge = __syncthreads_or(unsorted) == 0;
        if (merge) {
            sort_pairs<H>(ka, sa, key, slot);   // the new points, ascending in [0, k)
            int pa[H], pb[H];
#pragma unroll
            for (int e = 0; e < H; ++e) {
                const int i = H * t + e;
                pa[e] = (i < k) ? i + count_below(bk, bs, nb, ka[e], sa[e]) : -1;
                pb[e] = (i < nb) ? i + count_below(key, slot, k, kb[e], sb[e]) : -1;
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < H; ++e) {
                if (pa[e] >= 0) {
                    key[pa[e]] = ka[e];
                    slot[pa[e]] = sa[e];
                }
                if (pb[e] >= 0) {
                    key[pb[e]] = kb[e];
                    slot[pb[e]] = sb[e];
                }
            }
            __syncthreads();
        } else {
            double vm2 = -INFINITY;
            bool bad2 = false;
            load_pairs<E>(ll, n, kk, ss, vm2, bad2);
        }
    }
    if (!merge) sort_pairs<E>(kk, ss, key, slot);   // ends with a barrier

    const bool clm = R.cluster_mode != 0;
    ClusterTab *tab = clm ? at<ClusterTab>(arena, R.off_cltab) : nullptr;
    int32_t *label = clm ? at<int32_t>(arena, R.off_label) : nullptr;
    double *dead_l = at<double>(arena, R.off_dead_logl);
    double *dead_w = at<double>(arena, R.off_dead_logw);
    const long long nd = a.n_dead;
    const double lw = a.log_x - log((double)n + 1.0);
    const int nkill = stop ? n : k;

    // dead records and the log-sum-exp of the killed log L.  With clusters a
    // killed point of cluster p weighs Xbar_p / (n_p + 1) with n_p its live
    // count before the batch: the per-point updates Xbar_p <- n Xbar_p/(n+1)
    // within the batch telescope to that (Eqs. update0, update2)
    double m_loc = -INFINITY, s_loc = 0.0;
    for (int j = t; j < nkill; j += T) {
        const double v = key_value(key[j]);
        double wj = lw;
        if (clm) {
            const int p = label[slot[j]];
            wj = tab->clx[p] - log((double)tab->cn[p] + 1.0);
            atomicAdd(&kcount[p], 1);
        }
        if (nd + j < R.dead_cap) {
            dead_l[nd + j] = v;
            dead_w[nd + j] = wj;
        }
        lse_push(clm ? v + wj : v, m_loc, s_loc);
    }
    // positions of the dead points in the same order (posterior samples)
    if (R.dead_x != nullptr) {
        const int d = R.d;
        const int es = (R.prec == GGNS_FP64) ? 8 : 4;
        const unsigned char *lx = at<unsigned char>(arena, R.off_live_x);
        unsigned char *dx = reinterpret_cast<unsigned char *>(R.dead_x);
        const long long rows = (nd + nkill <= R.dead_x_cap) ? nkill
                               : (nd < R.dead_x_cap ? R.dead_x_cap - nd : 0);
        for (long long e = t; e < rows * d; e += T) {
            const long long j = e / d, c = e % d;
            const long long src = ((long long)slot[j] * d + c) * es, dst = ((nd + j) * d + c) * es;
            if (es == 8)
                *reinterpret_cast<double *>(dx + dst) = *reinterpret_cast<const double *>(lx + src);
            else
                *reinterpret_cast<float *>(dx + dst) = *reinterpret_cast<const float *>(lx + src);
        }
    }
    const double gmax = block_max_once(m_loc, scratch + 16);
    double lse = -INFINITY;
    if (gmax != -INFINITY) {
        const double part = (m_loc == -INFINITY) ? 0.0 : s_loc * exp(m_loc - gmax);
        lse = gmax + log(block_sum_once(part, scratch + 32));
    }
    if (t == 0) {
        acc->log_z = lae(a.log_z, clm ? lse : lse + lw);
        acc->n_dead = nd + nkill;
    }
    if (clm) {
        __syncthreads();   // kcount complete
        cluster_moments(tab, label, key, slot, nkill, kcount, acc);
        if (t == 0) {
            // volumes after the batch: Xbar_p (n_p - k_p + 1) / (n_p + 1); a
            // cluster left without points is removed; Xbar = sum over clusters
            double lsum = -INFINITY;
            for (int p = 0; p < tab->n_clusters; ++p) {
                const int kp = kcount[p], np = tab->cn[p];
                if (kp > 0) {
                    tab->clx[p] = (np - kp > 0)
                        ? tab->clx[p] + (log((double)(np - kp + 1)) - log((double)np + 1.0))
                        : -INFINITY;
                    tab->cn[p] = np - kp;
                }
                if (tab->cn[p] > 0) lsum = lae(lsum, tab->clx[p]);
            }
            acc->log_x = lsum;
            acc->n_clusters = tab->n_clusters;
        }
    }
    if (t == 0) {
        if (stop) {
            if (!clm) acc->log_x = lw;
        } else {
            if (!clm) acc->log_x = a.log_x + (log((double)(n + 1 - k)) - log((double)n + 1.0));
            acc->lstar = key_value(key[k - 1]);
            acc->it_outs = 0ull;
            acc->it_steps = 0ull;
            acc->win_a = 0;
            acc->win_b = 0;
        }
    }
    if (stop) {
        // the summary (H, sigma_KL, sigma_mom) is left to the finalize launch,
        // so runs that stop at different iterations do not serialise on it
        if (t == 0) {
            acc->summary_pending = 1;
            acc->state = stop;
        }
        return;
    }
    // killed slots in kill order; survivors in ascending slot order
    int32_t *killed = at<int32_t>(arena, R.off_killed);
    int32_t *surv = at<int32_t>(arena, R.off_surv);
    for (int j = t; j < k; j += T) {
        killed[j] = slot[j];
        dead_flag[slot[j]] = 1;
    }
    if constexpr (E >= 2) {
        // the survivors in kill order, for the next iteration's merge
        if (!clm && k <= SN && n - k <= SN) {
            int32_t *so = at<int32_t>(arena, R.off_surv_sorted);
            for (int j = t; j < n - k; j += T) so[j] = slot[k + j];
            if (t == 0) acc->order_ok = 1;
        }
    }
    if (clm) return;   // cluster mode: cluster_group_kernel groups the survivors
    __syncthreads();
    // each thread owns a contiguous range of slots
    const int per = (n + T - 1) / T;
    const int s0 = t * per, s1 = (s0 + per < n) ? s0 + per : n;
    int cnt = 0;
    for (int i = s0; i < s1; ++i) cnt += dead_flag[i] ? 0 : 1;
    int pos = block_exscan_int(cnt, ibuf);
    for (int i = s0; i < s1; ++i)
        if (!dead_flag[i]) surv[pos++] = i;
}

// Cluster mode, after the kill: survivors grouped by cluster (ascending slot
// within each) by a sort of (label, slot) keys, the survivor offsets of every
// cluster and the spawning CDF over the clusters (Algorithm GGNS, the cluster
// labels of the new points drawn in proportion to Xbar_p).  A launch of its
// own, so that the evidence kernel's registers do not carry a second sort.
template <int E>
__device__ void cluster_group_body(void *arena, const RunDev &R, unsigned long long *key, int *slot,
                                   unsigned char *dead_flag) {
    const int n = R.n_live, k = R.n_kill, t = threadIdx.x, T = blockDim.x;
    const int32_t *killed = at<int32_t>(arena, R.off_killed);
    const int32_t *label = at<int32_t>(arena, R.off_label);
    int32_t *surv = at<int32_t>(arena, R.off_surv);
    ClusterTab *tab = at<ClusterTab>(arena, R.off_cltab);
    for (int i = t; i < E * 1024; i += T) dead_flag[i] = 0;
    __syncthreads();
    for (int j = t; j < k; j += T) dead_flag[killed[j]] = 1;
    __syncthreads();
    {
        unsigned long long ck[E];
        int cs[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = E * t + e;
            ck[e] = (i < n && !dead_flag[i])
                        ? (((unsigned long long)label[i] << 12) | (unsigned long long)i) : ~0ull;
            cs[e] = 0;
        }
        sort_pairs<E>(ck, cs, key, slot);
    }
    const int nsurv = n - k;
    for (int i = t; i < nsurv; i += T) surv[i] = (int32_t)(key[i] & 0xFFFull);
    const int ncl = tab->n_clusters;
    for (int p = t; p <= ncl; p += T) {
        int lo = 0, hi = nsurv;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((int)(key[mid] >> 12) < p) lo = mid + 1; else hi = mid;
        }
        tab->soff[p] = lo;
    }
    __syncthreads();
    if (t == 0) {
        double cmax = -INFINITY, cum = 0.0;
        for (int p = 0; p < ncl; ++p)
            if (tab->soff[p + 1] > tab->soff[p] && tab->clx[p] > cmax) cmax = tab->clx[p];
        for (int p = 0; p < ncl; ++p) {
            if (tab->soff[p + 1] > tab->soff[p]) cum += exp(tab->clx[p] - cmax);
            tab->cum[p] = cum;
        }
    }
}

__global__ void __launch_bounds__(kEvThreads)
cluster_group_kernel(void *arena, const RunDev *__restrict__ runs) {
    const RunDev &R = runs[blockIdx.x];
    const Acc *acc = at<Acc>(arena, R.off_acc);
    if (!R.cluster_mode || acc->state != GGNS_RUN_ACTIVE) return;
    __shared__ unsigned long long key[kMaxLive];
    __shared__ int slot[kMaxLive];
    __shared__ unsigned char dead_flag[kMaxLive];
    const int n = R.n_live;
    if (n <= 1024) cluster_group_body<1>(arena, R, key, slot, dead_flag);
    else if (n <= 2048) cluster_group_body<2>(arena, R, key, slot, dead_flag);
    else cluster_group_body<4>(arena, R, key, slot, dead_flag);
}

__global__ void __launch_bounds__(kEvThreads)
evidence_kernel(void *arena, const RunDev *__restrict__ runs, int final_sweep) {
    const RunDev &R = runs[blockIdx.x];
    Acc *acc = at<Acc>(arena, R.off_acc);
    __shared__ unsigned long long key[kMaxLive];
    __shared__ int slot[kMaxLive];
    __shared__ unsigned char dead_flag[kMaxLive];
    __shared__ int kcount[kClMax];
    __shared__ int ibuf[kEvThreads / 64];
    __shared__ double scratch[48];
    __shared__ int flags[kEvThreads / 64];
    const int n = R.n_live;
    if (n <= 1024)
        evidence_body<1>(arena, R, acc, final_sweep, key, slot, dead_flag, kcount, ibuf, scratch, flags);
    else if (n <= 2048)
        evidence_body<2>(arena, R, acc, final_sweep, key, slot, dead_flag, kcount, ibuf, scratch, flags);
    else
        evidence_body<4>(arena, R, acc, final_sweep, key, slot, dead_flag, kcount, ibuf, scratch, flags);
}

// ---------------------------------------------------------------------------
// Run summary after the final sweep: information H and the second moment of Z
// from the single-cluster recursion (Eqs. update0, update2, update3, update5,
// update8), over the dead sequence in chunks of kFinChunk records, one
// workgroup per chunk and run.  Written as scans: with X_i = prod n_p/(n_p+1)
// and Y_i = prod n_p/(n_p+2) over the records before i, and
// S_i = sum_{j<i} c_j, c_j = Y_j L_j / ((n_j+2) X_j):
//   Z2 = sum_i 2 X_i S_i L_i/(n_i+1) + 2 Y_i L_i^2 / ((n_i+1)(n_i+2)),
//   Zr = sum_i X_i L_i/(n_i+1)  (the recursion's own Z).
// The live count n_p of record i follows from the kill pattern (iterations
// kill k points with n_p = n, ..., n-k+1; the final sweep n points with
// n_p = n, ..., 1), so X_i and Y_i telescope to closed forms:
//   r kills into a pattern give n+1-r over n+1 for X and
//   (n+1-r)(n+2-r) over (n+1)(n+2) for Y; a whole iteration r = k.
// Four launches: chunk totals of H and of the log-sum of c; a per-run scan of
// the c totals; the chunk totals of Z2 and Zr from each chunk's start S; the
// per-run sums.  Every partial lives in the run's `fin` section:
//   [0][chunk] H part, [1][chunk] log-sum of c, [2][chunk] exclusive scan of [1],
//   [3][chunk] log Z2 part, [4][chunk] log Zr part.
// ---------------------------------------------------------------------------
struct FinRun {
    int n, k;
    long long N, n_batch;
    double lk_x, lk_y;   // log X and log Y factors of one whole iteration
};

__device__ __forceinline__ FinRun fin_run(const RunDev &R, const Acc *acc) {
    FinRun f;
    f.n = R.n_live;
    f.k = R.n_kill;
    const long long nd = acc->n_dead;
    f.N = (nd < R.dead_cap) ? nd : R.dead_cap;
    f.n_batch = nd - R.n_live;
    const double n1 = f.n + 1.0, n2 = f.n + 2.0;
    f.lk_x = log((f.n - f.k + 1.0) / n1);
    f.lk_y = log((f.n - f.k + 1.0) * (f.n - f.k + 2.0) / (n1 * n2));
    return f;
}

// live count, log X and log Y before record i (lg[v] = log v)
__device__ __forceinline__ void fin_record(const FinRun &f, long long i, const double *lg, int &np,
                                           double &lx, double &ly) {
    long long q;
    int r;
    if (i < f.n_batch) {
        q = i / f.k;
        r = (int)(i % f.k);
    } else {
        q = f.n_batch / f.k;
        r = (int)(i - f.n_batch);
    }
    np = f.n - r;
    lx = (double)q * f.lk_x + (lg[f.n + 1 - r] - lg[f.n + 1]);
    ly = (double)q * f.lk_y + (lg[f.n + 1 - r] + lg[f.n + 2 - r] - lg[f.n + 1] - lg[f.n + 2]);
}

__device__ __forceinline__ void fin_log_table(int n, double *lg) {
    for (int v = threadIdx.x; v <= n + 2; v += blockDim.x) lg[v] = (v > 0) ? log((double)v) : -INFINITY;
    __syncthreads();
}

// chunk totals of H and of the log-sum of c
__global__ void __launch_bounds__(kFinThreads)
fin_chunk_kernel(void *arena, const RunDev *__restrict__ runs) {
    const RunDev &R = runs[blockIdx.y];
    const Acc *acc = at<Acc>(arena, R.off_acc);
    if (!acc->summary_pending) return;
    const FinRun f = fin_run(R, acc);
    const long long c0 = (long long)blockIdx.x * kFinChunk;
    if (c0 >= f.N) return;
    __shared__ double lg[kMaxLive + 3];
    __shared__ double scratch[32];
    fin_log_table(f.n, lg);
    const double *dl = at<double>(arena, R.off_dead_logl);
    const double *dw = at<double>(arena, R.off_dead_logw);
    const double lz = acc->log_z;
    const long long i0 = c0 + (long long)threadIdx.x * kFinPerThread;
    double hpart = 0.0, cm = -INFINITY, cs = 0.0;
    for (long long i = i0; i < i0 + kFinPerThread && i < f.N; ++i) {
        const double lp = dl[i] + dw[i] - lz;
        hpart += exp(lp) * (dl[i] - lz);
        int np;
        double lx, ly;
        fin_record(f, i, lg, np, lx, ly);
        lse_push(ly + dl[i] - lg[np + 2] - lx, cm, cs);
    }
    double *fin = at<double>(arena, R.off_fin);
    const int nc = R.fin_chunks;
    const double h = block_sum(hpart, scratch);
    const double lc = block_lse(cm, cs, scratch);
    if (threadIdx.x == 0) {
        fin[blockIdx.x] = h;
        fin[nc + blockIdx.x] = lc;
    }
}

// per run: H, sigma_KL, and the exclusive log-sum-exp scan of the chunk totals
__global__ void __launch_bounds__(kFinThreads)
fin_scan_kernel(void *arena, const RunDev *__restrict__ runs) {
    const RunDev &R = runs[blockIdx.x];
    Acc *acc = at<Acc>(arena, R.off_acc);
    if (!acc->summary_pending) return;
    const FinRun f = fin_run(R, acc);
    const int used = (int)((f.N + kFinChunk - 1) / kFinChunk);
    const int nc = R.fin_chunks;
    double *fin = at<double>(arena, R.off_fin);
    __shared__ double scratch[32];
    __shared__ double buf[kFinThreads];
    const int per = (used + kFinThreads - 1) / kFinThreads;
    const int b0 = threadIdx.x * per, b1 = (b0 + per < used) ? b0 + per : used;
    double h = 0.0, lc = -INFINITY;
    for (int b = b0; b < b1; ++b) {
        h += fin[b];
        lc = lae(lc, fin[nc + b]);
    }
    const double H = block_sum(h, scratch);
    double run_lc = block_exscan_lae(lc, buf);
    for (int b = b0; b < b1; ++b) {
        fin[2 * nc + b] = run_lc;
        run_lc = lae(run_lc, fin[nc + b]);
    }
    if (threadIdx.x == 0) {
        acc->h = H;
        acc->sigma_kl = sqrt(H > 0.0 ? H / f.n : 0.0);
    }
}

// chunk totals of Z2 and Zr, each thread starting from its exclusive S
__global__ void __launch_bounds__(kFinThreads)
fin_moment_kernel(void *arena, const RunDev *__restrict__ runs) {
    const RunDev &R = runs[blockIdx.y];
    const Acc *acc = at<Acc>(arena, R.off_acc);
    if (!acc->summary_pending) return;
    const FinRun f = fin_run(R, acc);
    const long long c0 = (long long)blockIdx.x * kFinChunk;
    if (c0 >= f.N) return;
    __shared__ double lg[kMaxLive + 3];
    __shared__ double scratch[32];
    __shared__ double buf[kFinThreads];
    fin_log_table(f.n, lg);
    const double *dl = at<double>(arena, R.off_dead_logl);
    const long long i0 = c0 + (long long)threadIdx.x * kFinPerThread;
    const long long i1 = (i0 + kFinPerThread < f.N) ? i0 + kFinPerThread : f.N;
    // this thread's log-sum of c, then its exclusive prefix within the run
    double cm = -INFINITY, cs = 0.0;
    for (long long i = i0; i < i1; ++i) {
        int np;
        double lx, ly;
        fin_record(f, i, lg, np, lx, ly);
        lse_push(ly + dl[i] - lg[np + 2] - lx, cm, cs);
    }
    const double lc_local = (cm == -INFINITY) ? -INFINITY : cm + log(cs);
    const double *fin_c = at<double>(arena, R.off_fin);
    const int nc = R.fin_chunks;
    const double lsum = lae(fin_c[2 * nc + blockIdx.x], block_exscan_lae(lc_local, buf));
    double am = -INFINITY, as = 0.0, zm = -INFINITY, zs = 0.0;
    double sm = lsum, ss = (lsum == -INFINITY) ? 0.0 : 1.0;   // running S as (sm, ss)
    const double l2 = 0.69314718055994530942;
    for (long long i = i0; i < i1; ++i) {
        int np;
        double x, y;
        fin_record(f, i, lg, np, x, y);
        const double ln1 = lg[np + 1], ln2 = lg[np + 2];
        const double ls = (sm == -INFINITY) ? -INFINITY : sm + log(ss);
        lse_push(l2 + x + ls + dl[i] - ln1, am, as);
        lse_push(l2 + y + 2.0 * dl[i] - ln1 - ln2, am, as);
        lse_push(x + dl[i] - ln1, zm, zs);
        lse_push(y + dl[i] - ln2 - x, sm, ss);
    }
    const double lz2 = block_lse(am, as, scratch);
    const double lzr = block_lse(zm, zs, scratch);
    if (threadIdx.x == 0) {
        double *fin = at<double>(arena, R.off_fin);
        fin[3 * nc + blockIdx.x] = lz2;
        fin[4 * nc + blockIdx.x] = lzr;
    }
}

// per run: log Z2 and sigma_mom from the chunk totals; the summary is done
__global__ void __launch_bounds__(kFinThreads)
fin_total_kernel(void *arena, const RunDev *__restrict__ runs) {
    const RunDev &R = runs[blockIdx.x];
    Acc *acc = at<Acc>(arena, R.off_acc);
    if (!acc->summary_pending) return;
    const FinRun f = fin_run(R, acc);
    const int used = (int)((f.N + kFinChunk - 1) / kFinChunk);
    const int nc = R.fin_chunks;
    const double *fin = at<double>(arena, R.off_fin);
    __shared__ double scratch[32];
    double m2 = -INFINITY, s2 = 0.0, mr = -INFINITY, sr = 0.0;
    for (int b = threadIdx.x; b < used; b += blockDim.x) {
        lse_push(fin[3 * nc + b], m2, s2);
        lse_push(fin[4 * nc + b], mr, sr);
    }
    const double lz2 = block_lse(m2, s2, scratch);
    const double lzr = block_lse(mr, sr, scratch);
    if (threadIdx.x == 0) {
        // cluster mode keeps Z2bar from the cluster recursion, run per batch
        if (!R.cluster_mode) acc->log_z2 = lz2;
        const double v = R.cluster_mode ? acc->log_z2 - 2.0 * acc->log_z : lz2 - 2.0 * lzr;
        acc->sigma_mom = sqrt(v > 0.0 ? v : 0.0);
        acc->summary_pending = 0;
    }
}

}  // namespace

void launch_finalize(void *arena, const RunDev *runs_dev, int n_runs, int max_chunks, hipStream_t s) {
    const dim3 chunks((unsigned)max_chunks, (unsigned)n_runs);
    hipLaunchKernelGGL(fin_chunk_kernel, chunks, dim3(kFinThreads), 0, s, arena, runs_dev);
    hipLaunchKernelGGL(fin_scan_kernel, dim3(n_runs), dim3(kFinThreads), 0, s, arena, runs_dev);
    hipLaunchKernelGGL(fin_moment_kernel, chunks, dim3(kFinThreads), 0, s, arena, runs_dev);
    hipLaunchKernelGGL(fin_total_kernel, dim3(n_runs), dim3(kFinThreads), 0, s, arena, runs_dev);
}

void launch_evidence(void *arena, const RunDev *runs_dev, int n_runs, int final_sweep,
                     int any_cluster, hipStream_t s) {
    hipLaunchKernelGGL(evidence_kernel, dim3(n_runs), dim3(kEvThreads), 0, s, arena, runs_dev,
                       final_sweep);
    if (any_cluster)
        hipLaunchKernelGGL(cluster_group_kernel, dim3(n_runs), dim3(kEvThreads), 0, s, arena, runs_dev);
}

}  // namespace ggns
