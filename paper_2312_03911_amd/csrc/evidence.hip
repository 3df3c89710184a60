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

__device__ __forceinline__ unsigned long long order_key(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
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

__device__ double block_exscan_sum(double v, double *buf) {
    return block_exscan<double>(v, 0.0, [](double a, double b) { return a + b; }, buf);
}

__device__ double block_exscan_lae(double v, double *buf) {
    return block_exscan<double>(v, -INFINITY, [](double a, double b) { return lae(a, b); }, buf);
}

__device__ int block_exscan_int(int v, int *buf) {
    return block_exscan<int>(v, 0, [](int a, int b) { return a + b; }, buf);
}

// Bitonic sort of 1024 E (key, slot) pairs, E per thread (element i = E t + e
// of thread t), ascending by key and then slot.  Compare-exchange stages of
// stride below E stay inside the thread; strides E .. 32 E pair lanes
// stride / E apart in the same wavefront (DPP for 1 and 2 lanes, ds_swizzle
// up to 16, a lane permute for 32); strides of 64 E and more cross wavefronts
// through LDS between two barriers.  The order is total (slots are distinct;
// the padding entries are all equal), so the sorted sequence is unique.
template <int X>
__device__ __forceinline__ int xor_lanes(int v) {
    if constexpr (X == 1) return __builtin_amdgcn_update_dpp(0, v, kDppXor1, 0xF, 0xF, false);
    else if constexpr (X == 2) return __builtin_amdgcn_update_dpp(0, v, kDppXor2, 0xF, 0xF, false);
    else if constexpr (X <= 16) return __builtin_amdgcn_ds_swizzle(v, (X << 10) | 0x1F);
    else return __shfl_xor(v, X, 64);
}

__device__ __forceinline__ bool kv_greater(unsigned long long ka, int sa, unsigned long long kb,
                                           int sb) {
    return (ka > kb) | ((ka == kb) & (sa > sb));
}

// This lane's pair against the lane X away: keep the smaller when keep_min.
template <int X>
__device__ __forceinline__ void lane_cas(unsigned long long &k, int &s, bool keep_min) {
    const int lo = xor_lanes<X>((int)(unsigned)k);
    const int hi = xor_lanes<X>((int)(unsigned)(k >> 32));
    const int so = xor_lanes<X>(s);
    const unsigned long long ko = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
    const bool gt = kv_greater(k, s, ko, so);
    const bool take = keep_min ? gt : !gt;
    k = take ? ko : k;
    s = take ? so : s;
}

template <int E>
__device__ void sort_pairs(unsigned long long (&k)[E], int (&s)[E], unsigned long long *lk, int *ls) {
    constexpr int N = 1024 * E;
    const int t = threadIdx.x;
#pragma unroll
    for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= 64 * E) {
                __syncthreads();
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    lk[E * t + e] = k[e];
                    ls[E * t + e] = s[e];
                }
                __syncthreads();
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int i = E * t + e, j = i ^ stride;
                    const unsigned long long kb = lk[j];
                    const int sb = ls[j];
                    const bool keep_min = ((i & size) == 0) == ((i & stride) == 0);
                    const bool gt = kv_greater(k[e], s[e], kb, sb);
                    const bool take = keep_min ? gt : !gt;
                    k[e] = take ? kb : k[e];
                    s[e] = take ? sb : s[e];
                }
            } else if (stride >= E) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int i = E * t + e;
                    const bool keep_min = ((i & size) == 0) == ((i & stride) == 0);
                    switch (stride / E) {
                        case 1: lane_cas<1>(k[e], s[e], keep_min); break;
                        case 2: lane_cas<2>(k[e], s[e], keep_min); break;
                        case 4: lane_cas<4>(k[e], s[e], keep_min); break;
                        case 8: lane_cas<8>(k[e], s[e], keep_min); break;
                        case 16: lane_cas<16>(k[e], s[e], keep_min); break;
                        default: lane_cas<32>(k[e], s[e], keep_min); break;
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if (e & stride) continue;
                    const int f = e | stride;
                    const bool asc = ((E * t + e) & size) == 0;
                    const bool sw = kv_greater(k[e], s[e], k[f], s[f]) == asc;
                    const unsigned long long ka = k[e];
                    const int sa = s[e];
                    k[e] = sw ? k[f] : k[e];
                    s[e] = sw ? s[f] : s[e];
                    k[f] = sw ? ka : k[f];
                    s[f] = sw ? sa : s[f];
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        lk[E * t + e] = k[e];
        ls[E * t + e] = s[e];
    }
    __syncthreads();
}

// Run summary over the whole dead sequence: information H, and the second
// moment of Z from the single-cluster recursion (update0, update2, update3,
// update5, update8).  Written as scans: with X_i = prod n_p/(n_p+1) and
// Y_i = prod n_p/(n_p+2) over the records before i, ZX_i = X_i sum_{j<i}
// Y_j L_j / ((n_j+2) X_j), and Z2 = sum_i 2 ZX_i L_i/(n_i+1) + 2 Y_i L_i^2 /
// ((n_i+1)(n_i+2)).  The live count n_p of record i follows from the kill
// pattern (iterations kill k points with n_p = n, ..., n-k+1; the final sweep
// n points with n_p = n, ..., 1), so log n_p, log(n_p+1), log(n_p+2) come from a
// table of log v, v = 0 .. n+2, held in LDS.
__device__ void run_summary(const RunDev &R, Acc *acc, const double *dl, const double *dw,
                            long long N, long long n_batch, double *lg, double *buf,
                            double *scratch) {
    const int n = R.n_live, k = R.n_kill;
    const int T = blockDim.x, t = threadIdx.x;
    for (int v = t; v <= n + 2; v += T) lg[v] = (v > 0) ? log((double)v) : -INFINITY;
    __syncthreads();
    const long long chunk = (N + T - 1) / T;
    const long long i0 = (long long)t * chunk;
    const long long i1 = (i0 + chunk < N) ? i0 + chunk : N;
    const double lz = acc->log_z;
    // position of record i0 in its kill pattern
    auto np_at = [&](long long i) -> int {
        return (i < n_batch) ? n - (int)(i % k) : n - (int)(i - n_batch);
    };

    // H = sum p_i (log L_i - log Z), p_i = L_i w_i / Z; prefix sums of log X, log Y
    double hpart = 0.0, sx = 0.0, sy = 0.0;
    {
        int np = (i0 < N) ? np_at(i0) : n;
        for (long long i = i0; i < i1; ++i) {
            const double lp = dl[i] + dw[i] - lz;
            hpart += exp(lp) * (dl[i] - lz);
            sx += lg[np] - lg[np + 1];
            sy += lg[np] - lg[np + 2];
            --np;
            if (i + 1 == n_batch || (i + 1 < n_batch && np == n - k)) np = n;
        }
    }
    const double h = block_sum(hpart, scratch);
    const double lx0 = block_exscan_sum(sx, buf);
    const double ly0 = block_exscan_sum(sy, buf);
    // local log-sum of c_j = Y_j L_j / ((n_j+2) X_j)
    double cm = -INFINITY, cs = 0.0;
    {
        double x = lx0, y = ly0;
        int np = (i0 < N) ? np_at(i0) : n;
        for (long long i = i0; i < i1; ++i) {
            lse_push(y + dl[i] - lg[np + 2] - x, cm, cs);
            x += lg[np] - lg[np + 1];
            y += lg[np] - lg[np + 2];
            --np;
            if (i + 1 == n_batch || (i + 1 < n_batch && np == n - k)) np = n;
        }
    }
    const double lc_local = (cm == -INFINITY) ? -INFINITY : cm + log(cs);
    const double lsum = block_exscan_lae(lc_local, buf);
    // terms of Z2 and of the recursion's own Z
    double am = -INFINITY, as = 0.0, zm = -INFINITY, zs = 0.0;
    {
        double x = lx0, y = ly0;
        double sm = lsum, ss = (lsum == -INFINITY) ? 0.0 : 1.0;   // running S_j as (sm, ss)
        const double l2 = 0.69314718055994530942;
        int np = (i0 < N) ? np_at(i0) : n;
        for (long long i = i0; i < i1; ++i) {
            const double ln1 = lg[np + 1], ln2 = lg[np + 2];
            const double ls = (sm == -INFINITY) ? -INFINITY : sm + log(ss);
            lse_push(l2 + x + ls + dl[i] - ln1, am, as);
            lse_push(l2 + y + 2.0 * dl[i] - ln1 - ln2, am, as);
            lse_push(x + dl[i] - ln1, zm, zs);
            lse_push(y + dl[i] - ln2 - x, sm, ss);
            x += lg[np] - ln1;
            y += lg[np] - ln2;
            --np;
            if (i + 1 == n_batch || (i + 1 < n_batch && np == n - k)) np = n;
        }
    }
    const double lz2 = block_lse(am, as, scratch);
    const double lzr = block_lse(zm, zs, scratch);
    if (t == 0) {
        acc->h = h;
        acc->sigma_kl = sqrt(h > 0.0 ? h / n : 0.0);
        acc->log_z2 = R.cluster_mode ? -INFINITY : lz2;
        const double v = lz2 - 2.0 * lzr;
        acc->sigma_mom = R.cluster_mode ? 0.0 : sqrt(v > 0.0 ? v : 0.0);
    }
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
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = E * t + e;
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
    sort_pairs<E>(kk, ss, key, slot);   // ends with a barrier

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
    __syncthreads();
    if (!clm) {
        // each thread owns a contiguous range of slots
        const int per = (n + T - 1) / T;
        const int s0 = t * per, s1 = (s0 + per < n) ? s0 + per : n;
        int cnt = 0;
        for (int i = s0; i < s1; ++i) cnt += dead_flag[i] ? 0 : 1;
        int pos = block_exscan_int(cnt, ibuf);
        for (int i = s0; i < s1; ++i)
            if (!dead_flag[i]) surv[pos++] = i;
        return;
    }
    // cluster mode: survivors grouped by cluster (ascending slot within each),
    // by a sort of (label, slot) keys; the spawning CDF over the clusters
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

__global__ void __launch_bounds__(kEvThreads)
finalize_kernel(void *arena, const RunDev *__restrict__ runs) {
    const RunDev &R = runs[blockIdx.x];
    Acc *acc = at<Acc>(arena, R.off_acc);
    if (!acc->summary_pending) return;
    __shared__ double lg[kMaxLive + 3];
    __shared__ double buf[kEvThreads];
    __shared__ double scratch[32];
    const long long nd = acc->n_dead;
    const long long N = (nd < R.dead_cap) ? nd : R.dead_cap;
    const long long n_batch = nd - R.n_live;
    run_summary(R, acc, at<double>(arena, R.off_dead_logl), at<double>(arena, R.off_dead_logw), N,
                n_batch, lg, buf, scratch);
    if (threadIdx.x == 0) acc->summary_pending = 0;
}

}  // namespace

void launch_finalize(void *arena, const RunDev *runs_dev, int n_runs, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(n_runs), dim3(kEvThreads), 0, s, arena, runs_dev);
}

void launch_evidence(void *arena, const RunDev *runs_dev, int n_runs, int final_sweep,
                     hipStream_t s) {
    hipLaunchKernelGGL(evidence_kernel, dim3(n_runs), dim3(kEvThreads), 0, s, arena, runs_dev,
                       final_sweep);
}

}  // namespace ggns
