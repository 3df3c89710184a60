// Cluster recognition for runs in cluster mode (Section 3, mode collapse
// mitigation; Algorithm GGNS with its cluster-finding algorithm; Eq. new0
// for the split of a cluster's prior volume).  Readings: cluster finding
// runs at the start of every iteration that goes on, once for every cluster
// that exists then; for k = 2, 3, ... every point of a cluster is linked to
// its k nearest other points of the cluster (squared Euclidean distance,
// ties by slot) and the connected components of the undirected graph are
// taken; the first k whose component sizes equal those of k - 1 gives the
// clustering (k up to min(cluster_kmax, m - 1), cluster_kmax <= 32, else the
// cluster stays whole); components ordered by their smallest slot become
// clusters, the first keeping the old index, at most kClMax in all;
// Xbar_i = (n_i/n) Xbar_p.
//
// Launches per iteration: cluster_pre (termination decision; the live slots
// grouped by cluster), then up to four passes of knn (the next kKnnPass
// nearest neighbours of every point within its cluster, beyond the last one
// of the previous pass in (distance, slot) order) and cluster_cc (one
// workgroup per run: over the neighbours found so far; a cluster whose loop
// is still going when they run out asks for the next pass, the others wait;
// union-find over the k-th neighbour edges for k = 1, 2, ...; since the graph
// for k contains the graph for k - 1, its partition is a coarsening, and equal
// component sizes are equal component counts, which is what is compared).
#include "ggns_device.h"

namespace ggns {

namespace {

constexpr int kClThreads = 1024;

template <typename T>
__device__ __forceinline__ bool lex_less(T a, int sa, T b, int sb) {
    return a < b || (a == b && sa < sb);
}

}  // namespace

// (label << 12 | slot) of the n live slots, E per thread, sorted into key[]
template <int E>
__device__ void group_members(int n, const int32_t *label, unsigned long long *key, int *slot) {
    unsigned long long k[E];
    int s[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = E * threadIdx.x + e;
        k[e] = (i < n) ? (((unsigned long long)label[i] << 12) | (unsigned long long)i) : ~0ull;
        s[e] = 0;
    }
    sort_pairs<E>(k, s, key, slot);
}

// Termination decision and members grouped by cluster.
__global__ void __launch_bounds__(kClThreads)
cluster_pre_kernel(void *arena, const RunDev *__restrict__ runs, int final_sweep) {
    const RunDev &R = runs[blockIdx.x];
    if (!R.cluster_mode) return;
    Acc *acc = at<Acc>(arena, R.off_acc);
    if (acc->state != GGNS_RUN_ACTIVE) return;
    ClusterTab *tab = at<ClusterTab>(arena, R.off_cltab);
    __shared__ unsigned long long key[kMaxLive];
    __shared__ int slot_s[kMaxLive];
    __shared__ double scratch[32];
    __shared__ int nanflag;
    const int n = R.n_live, t = threadIdx.x, T = blockDim.x;
    const double *ll = at<double>(arena, R.off_live_logl);
    const int32_t *label = at<int32_t>(arena, R.off_label);
    if (t == 0) nanflag = 0;
    __syncthreads();
    double lmax = -INFINITY;
    for (int i = t; i < n; i += T) {
        const double v = ll[i];
        if (isnan(v)) nanflag = 1;
        lmax = v > lmax ? v : lmax;
    }
    lmax = block_max_d(lmax, scratch);
    const int stop = nanflag ? 1 : termination_decision(R, acc, lmax, final_sweep, nullptr);
    if (t == 0) {
        tab->stopping = stop;
        tab->cc_done = 0;
    }
    for (int p = t; p < kClMax; p += T) tab->need[p] = 0;
    if (stop) return;
    // live slots grouped by cluster: sort of (label << 12 | slot) keys
    if (n <= 1024) group_members<1>(n, label, key, slot_s);
    else if (n <= 2048) group_members<2>(n, label, key, slot_s);
    else group_members<4>(n, label, key, slot_s);
    int32_t *members = at<int32_t>(arena, R.off_members);
    for (int i = t; i < n; i += T) members[i] = (int32_t)(key[i] & 0xFFFu);
    const int nc = tab->n_clusters;
    for (int p = t; p <= nc; p += T) {
        // first position whose label is >= p
        int lo = 0, hi = n;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((int)(key[mid] >> 12) < p) lo = mid + 1; else hi = mid;
        }
        tab->moff[p] = lo;
    }
}

// Nearest neighbours within clusters, in two launches.  knn_part: a
// workgroup of 4 wavefronts takes 64 consecutive entries of the cluster-grouped
// member list as queries (one per lane) and one of kKnnSplit shares of the
// candidate range of their clusters, split again between its wavefronts; a
// candidate is the same for every lane of a wavefront, so its coordinates
// arrive through scalar loads; each lane keeps the KN best of its share
// (squared distance accumulated with fused multiply-adds in coordinate order,
// in the run's precision; ties by slot); the wavefronts' lists merge in LDS
// and go to a partial-list buffer.  knn_merge: one thread per query merges its
// kKnnSplit partial lists into its neighbour list.
constexpr int kKnnWaves = 4;

// What one wavefront's share of the candidate scan needs.
template <typename T>
struct KnnScan {
    const T *X;
    const int32_t *members, *label;
    int u0, u1, d, qi, qc;
    bool qvalid;
    T thr_d;
    int thr_s;
};

// Candidate j (the same for every lane) into this lane's sorted list of the KN
// best, if it belongs to the query's cluster, is not the query and comes after
// the previous passes' last neighbour.
template <typename T, int KN>
__device__ __forceinline__ void knn_insert(const KnnScan<T> &sc, T dist, int j, T (&bd)[KN], int (&bs)[KN]) {
    const bool ok = sc.qvalid && sc.label[j] == sc.qc && j != sc.qi && lex_less(sc.thr_d, sc.thr_s, dist, j) &&
                    lex_less(dist, j, bd[KN - 1], bs[KN - 1]);
    if (ok) {
        bd[KN - 1] = dist;
        bs[KN - 1] = j;
#pragma unroll
        for (int q = KN - 1; q > 0; --q) {
            const bool sw = lex_less(bd[q], bs[q], bd[q - 1], bs[q - 1]);
            const T td = bd[q];
            const int ts = bs[q];
            bd[q] = sw ? bd[q - 1] : bd[q];
            bs[q] = sw ? bs[q - 1] : bs[q];
            bd[q - 1] = sw ? td : bd[q - 1];
            bs[q - 1] = sw ? ts : bs[q - 1];
        }
    }
}

// The scan over candidates [u0, u1) of the cluster-grouped member list, TILE at
// a time; squared distances accumulated with fused multiply-adds in coordinate
// order from zero.  D > 0: d == D, the query's D coordinates in registers and
// each candidate row read as 16-byte vectors through scalar loads (rows start
// on 16-byte boundaries: the arena is aligned and D is a multiple of four).
// D == 0: any d, the query re-read in chunks for each tile.
template <typename T, int KN, int D>
__device__ __forceinline__ void knn_scan(const KnnScan<T> &sc, const T *xq, T (&bd)[KN], int (&bs)[KN]) {
    constexpr int TILE = 8;
    if constexpr (D > 0) {
        constexpr int V = 16 / sizeof(T);   // elements per 16-byte vector
        typedef T vec __attribute__((ext_vector_type(V)));
        T qv[D];
#pragma unroll
        for (int a = 0; a < D; ++a) qv[a] = xq[a];
        for (int ub = sc.u0; ub < sc.u1; ub += TILE) {
            int cj[TILE];
            T acc2[TILE];
#pragma unroll
            for (int t = 0; t < TILE; ++t) {
                cj[t] = __builtin_amdgcn_readfirstlane((ub + t < sc.u1) ? sc.members[ub + t] : -1);
                acc2[t] = (T)0;
            }
#pragma unroll
            for (int t = 0; t < TILE; ++t) {
                if (cj[t] < 0) continue;
                const vec *xc = reinterpret_cast<const vec *>(sc.X + (int64_t)cj[t] * D);
#pragma unroll
                for (int v = 0; v < D / V; ++v) {
                    const vec c = xc[v];
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        const T df = qv[V * v + e] - c[e];
                        acc2[t] = fma(df, df, acc2[t]);
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < TILE; ++t)
                if (cj[t] >= 0) knn_insert<T, KN>(sc, acc2[t], cj[t], bd, bs);
        }
    } else {
        constexpr int CHUNK = (sizeof(T) == 8) ? 16 : 32;
        const int d = sc.d;
        for (int ub = sc.u0; ub < sc.u1; ub += TILE) {
            int cj[TILE];
            T acc2[TILE];
#pragma unroll
            for (int t = 0; t < TILE; ++t) {
                // the same candidate for every lane: make that explicit so that its
                // coordinates come through scalar loads
                cj[t] = __builtin_amdgcn_readfirstlane((ub + t < sc.u1) ? sc.members[ub + t] : -1);
                acc2[t] = (T)0;
            }
            for (int c0 = 0; c0 < d; c0 += CHUNK) {
                const int cn = (d - c0 < CHUNK) ? d - c0 : CHUNK;
                T qv[CHUNK];
#pragma unroll
                for (int a = 0; a < CHUNK; ++a) qv[a] = (a < cn) ? xq[c0 + a] : (T)0;
#pragma unroll
                for (int t = 0; t < TILE; ++t) {
                    if (cj[t] < 0) continue;
                    const T *xc = sc.X + (int64_t)cj[t] * d + c0;
#pragma unroll
                    for (int a = 0; a < CHUNK; ++a) {
                        if (a < cn) {
                            const T e = qv[a] - xc[a];
                            acc2[t] = fma(e, e, acc2[t]);
                        }
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < TILE; ++t)
                if (cj[t] >= 0) knn_insert<T, KN>(sc, acc2[t], cj[t], bd, bs);
        }
    }
}

template <typename T, int KN>
__global__ void __launch_bounds__(64 * kKnnWaves)
knn_part_kernel(void *arena, const RunDev *__restrict__ runs, int pass) {
    const RunDev &R = runs[blockIdx.y];
    if (!R.cluster_mode || (R.prec == GGNS_FP64) != (sizeof(T) == 8)) return;
    const Acc *acc = at<Acc>(arena, R.off_acc);
    if (acc->state != GGNS_RUN_ACTIVE) return;
    const ClusterTab *tab = at<ClusterTab>(arena, R.off_cltab);
    if (tab->stopping || tab->cc_done) return;
    const int n = R.n_live;
    const int qb = blockIdx.x / kKnnSplit, split = blockIdx.x % kKnnSplit;
    const int q0 = qb * 64;
    if (q0 >= n) return;
    __shared__ T lst_d[kKnnWaves][KN][64];
    __shared__ int lst_s[kKnnWaves][KN][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t *label = at<int32_t>(arena, R.off_label);
    const int32_t *members = at<int32_t>(arena, R.off_members);
    const int qn = (n - q0 < 64) ? n - q0 : 64;
    const int qi = members[q0 + (lane < qn ? lane : 0)];
    const int qc = label[qi];
    // after the first pass only the points of clusters whose loop goes on;
    // the same queries in every wavefront of the block
    const bool qvalid = lane < qn && (pass == 0 || tab->need[qc] != 0);
    if (!__any(qvalid)) return;
    // candidates must come after the last neighbour found by the passes before
    T thr_d = (T)(-INFINITY);
    int thr_s = -1;
    if (pass > 0 && qvalid) {
        const int64_t at_ = (int64_t)qi * kKnnMax + kKnnPass * pass - 1;
        thr_d = (T)at<double>(arena, R.off_knn_d)[at_];
        thr_s = at<int32_t>(arena, R.off_knn)[at_];
    }
    // candidate range: the clusters of the first and the last query; this
    // block's share of it, and this wavefront's share of that
    const int c_lo = label[members[q0]], c_hi = label[members[q0 + qn - 1]];
    const int lo = tab->moff[c_lo], hi = tab->moff[c_hi + 1];
    const int parts = kKnnSplit * kKnnWaves, part = split * kKnnWaves + wave;
    const int per = (hi - lo + parts - 1) / parts;
    const int u0 = lo + part * per, u1 = (u0 + per < hi) ? u0 + per : hi;
    const int d = R.d;
    const T *__restrict__ X = at<T>(arena, R.off_live_x);
    const T *xq = X + (int64_t)qi * d;
    T bd[KN];
    int bs[KN];
#pragma unroll
    for (int q = 0; q < KN; ++q) { bd[q] = (T)INFINITY; bs[q] = 0x7FFFFFFF; }
    // dimensions 8, 16, 32 and 64 (FP64: up to 32): the query in registers for
    // the whole scan and each candidate row in 16-byte scalar loads; any other d
    // in chunks of the query
    const KnnScan<T> sc{X, members, label, u0, u1, d, qi, qc, qvalid, thr_d, thr_s};
    switch (d) {
        case 8: knn_scan<T, KN, 8>(sc, xq, bd, bs); break;
        case 16: knn_scan<T, KN, 16>(sc, xq, bd, bs); break;
        case 32: knn_scan<T, KN, 32>(sc, xq, bd, bs); break;
        case 64:
            if constexpr (sizeof(T) == 4) knn_scan<T, KN, 64>(sc, xq, bd, bs);
            else knn_scan<T, KN, 0>(sc, xq, bd, bs);
            break;
        default: knn_scan<T, KN, 0>(sc, xq, bd, bs); break;
    }
#pragma unroll
    for (int q = 0; q < KN; ++q) {
        lst_d[wave][q][lane] = bd[q];
        lst_s[wave][q][lane] = bs[q];
    }
    __syncthreads();
    if (wave == 0 && qvalid) {
        int head[kKnnWaves];
#pragma unroll
        for (int w = 0; w < kKnnWaves; ++w) head[w] = 0;
        double *pd = at<double>(arena, R.off_knn_part) + ((int64_t)(q0 + lane) * kKnnSplit + split) * kKnnPass;
        int32_t *ps = at<int32_t>(arena, R.off_knn_part_s) + ((int64_t)(q0 + lane) * kKnnSplit + split) * kKnnPass;
        for (int r = 0; r < KN; ++r) {
            int bw = 0;
            T dmin = (T)INFINITY;
            int smin = 0x7FFFFFFF;
#pragma unroll
            for (int w = 0; w < kKnnWaves; ++w) {
                if (head[w] >= KN) continue;
                const T dv = lst_d[w][head[w]][lane];
                const int sv = lst_s[w][head[w]][lane];
                if (lex_less(dv, sv, dmin, smin)) { dmin = dv; smin = sv; bw = w; }
            }
            pd[r] = (double)dmin;
            ps[r] = smin;
            head[bw] += 1;
        }
    }
}

__global__ void knn_merge_kernel(void *arena, const RunDev *__restrict__ runs, int pass) {
    const RunDev &R = runs[blockIdx.y];
    if (!R.cluster_mode) return;
    const Acc *acc = at<Acc>(arena, R.off_acc);
    if (acc->state != GGNS_RUN_ACTIVE) return;
    const ClusterTab *tab = at<ClusterTab>(arena, R.off_cltab);
    if (tab->stopping || tab->cc_done) return;
    const int qpos = blockIdx.x * blockDim.x + threadIdx.x;
    if (qpos >= R.n_live) return;
    const int qi = at<int32_t>(arena, R.off_members)[qpos];
    const int qc = at<int32_t>(arena, R.off_label)[qi];
    if (pass > 0 && !tab->need[qc]) return;
    const int m = tab->moff[qc + 1] - tab->moff[qc];
    if (m < 3) return;
    const int keff = (R.cluster_kmax < m - 1) ? R.cluster_kmax : m - 1;
    const int r0 = kKnnPass * pass;
    const int nr = (keff - r0 < kKnnPass) ? keff - r0 : kKnnPass;
    const double *pd = at<double>(arena, R.off_knn_part) + (int64_t)qpos * kKnnSplit * kKnnPass;
    const int32_t *ps = at<int32_t>(arena, R.off_knn_part_s) + (int64_t)qpos * kKnnSplit * kKnnPass;
    int head[kKnnSplit];
#pragma unroll
    for (int w = 0; w < kKnnSplit; ++w) head[w] = 0;
    int32_t *knn = at<int32_t>(arena, R.off_knn) + (int64_t)qi * kKnnMax + r0;
    double *knn_d = at<double>(arena, R.off_knn_d) + (int64_t)qi * kKnnMax + r0;
    for (int r = 0; r < nr; ++r) {
        int bw = 0;
        double dmin = INFINITY;
        int smin = 0x7FFFFFFF;
#pragma unroll
        for (int w = 0; w < kKnnSplit; ++w) {
            if (head[w] >= kKnnPass) continue;
            const double dv = pd[w * kKnnPass + head[w]];
            const int sv = ps[w * kKnnPass + head[w]];
            if (lex_less(dv, sv, dmin, smin)) { dmin = dv; smin = sv; bw = w; }
        }
        knn[r] = smin;
        knn_d[r] = dmin;
        head[bw] += 1;
    }
}

namespace {

__device__ __forceinline__ int uf_root(volatile int *par, int i) {
    int r = i;
    while (par[r] != r) r = par[r];
    return r;
}

}  // namespace

// (cluster << 12 | slot) of the component roots of stopped clusters, the rest
// above every key, sorted into key[] (1024 E entries)
template <int E>
__device__ void sort_roots(int n, const int *label, const int *par, const int *stopped,
                           unsigned long long *key, int *slot) {
    unsigned long long k[E];
    int s[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = E * threadIdx.x + e;
        k[e] = (i < n && stopped[label[i]] && par[i] == i)
                   ? (((unsigned long long)label[i] << 12) | (unsigned long long)i) : ~0ull;
        s[e] = 0;
    }
    sort_pairs<E>(k, s, key, slot);
}

// One workgroup per run: components for k = 1, 2, ... neighbours, the stop
// rule per cluster, and the splits.
__global__ void __launch_bounds__(kClThreads)
cluster_cc_kernel(void *arena, const RunDev *__restrict__ runs, int pass) {
    const RunDev &R = runs[blockIdx.x];
    if (!R.cluster_mode) return;
    Acc *acc = at<Acc>(arena, R.off_acc);
    if (acc->state != GGNS_RUN_ACTIVE) return;
    ClusterTab *tab = at<ClusterTab>(arena, R.off_cltab);
    if (tab->stopping || tab->cc_done) return;
    // neighbours available after this pass
    const int kav = (kKnnPass * (pass + 1) < R.cluster_kmax) ? kKnnPass * (pass + 1) : R.cluster_kmax;
    __shared__ int any_need;
    __shared__ int par[kMaxLive];
    __shared__ int keff[kClMax], stopped[kClMax], cnt_prev[kClMax], cnt_cur[kClMax];
    __shared__ int nroot[kClMax], roots[kClMax][kClMax], newid_base[kClMax];
    __shared__ int ccount[kClMax];
    __shared__ int changed;
    __shared__ int label[kMaxLive];
    __shared__ unsigned long long rkey[kMaxLive];
    __shared__ int rslot[kMaxLive];
    __shared__ int fpos[kClMax];
    __shared__ double lxr[kClMax];
    const int n = R.n_live, t = threadIdx.x, T = blockDim.x;
    int32_t *label_g = at<int32_t>(arena, R.off_label);
    for (int i = t; i < n; i += T) label[i] = label_g[i];
    const int32_t *knn = at<int32_t>(arena, R.off_knn);
    const int nc0 = tab->n_clusters;
    for (int p = t; p < kClMax; p += T) {
        const int m = (p < nc0) ? tab->moff[p + 1] - tab->moff[p] : 0;
        const int ke = (R.cluster_kmax < m - 1) ? R.cluster_kmax : m - 1;
        keff[p] = (m >= 3 && ke >= 2) ? ke : 0;
        stopped[p] = 0;
        cnt_prev[p] = -1;
        nroot[p] = 0;
        ccount[p] = 0;
    }
    for (int i = t; i < n; i += T) par[i] = i;
    __syncthreads();
    for (int k = 1; k <= kav; ++k) {
        // add the edges to each point's k-th nearest neighbour, merge roots
        do {
            __syncthreads();
            if (t == 0) changed = 0;
            __syncthreads();
            for (int i = t; i < n; i += T) {
                const int p = label[i];
                if (k > keff[p] || stopped[p]) continue;
                const int a = uf_root(par, i), b = uf_root(par, knn[(int64_t)i * kKnnMax + k - 1]);
                if (a != b) {
                    atomicMin(&par[a > b ? a : b], a > b ? b : a);
                    changed = 1;
                }
            }
            __syncthreads();
            for (int i = t; i < n; i += T) par[i] = uf_root(par, i);
        } while (changed);
        __syncthreads();
        if (k < 2) continue;
        for (int p = t; p < kClMax; p += T) cnt_cur[p] = 0;
        __syncthreads();
        for (int i = t; i < n; i += T) {
            const int p = label[i];
            if (keff[p] && !stopped[p] && k <= keff[p] && par[i] == i) atomicAdd(&cnt_cur[p], 1);
        }
        __syncthreads();
        if (t == 0) changed = 0;
        __syncthreads();
        for (int p = t; p < kClMax; p += T) {
            if (!keff[p] || stopped[p] || k > keff[p]) continue;
            if (k >= 3 && cnt_cur[p] == cnt_prev[p]) stopped[p] = k;
            cnt_prev[p] = cnt_cur[p];
            if (!stopped[p] && k < keff[p]) changed = 1;   // some cluster still grows its graph
        }
        __syncthreads();
        if (!changed) break;
    }
    // a cluster still going when the neighbours found so far run out takes
    // the next pass (the run's splits wait for it); at the last pass it stays
    // whole (counted in n_cut)
    if (t == 0) any_need = 0;
    __syncthreads();
    for (int p = t; p < nc0; p += T) {
        const int nd = (keff[p] && !stopped[p] && keff[p] > kav) ? 1 : 0;
        tab->need[p] = nd;
        if (nd) any_need = 1;
    }
    __syncthreads();
    if (any_need && pass + 1 < kKnnPasses) return;
    if (t == 0) {
        tab->cc_done = 1;
        if (any_need)
            for (int p = 0; p < nc0; ++p) tab->n_cut += tab->need[p];
    }
    // roots of the stopped clusters in ascending slot order: a sort of
    // (cluster << 12 | slot) keys of the roots, then per-cluster runs
    {
        const int NP = (n <= 1024) ? 1024 : (n <= 2048 ? 2048 : 4096);   // entries sorted
        if (n <= 1024) sort_roots<1>(n, label, par, stopped, rkey, rslot);
        else if (n <= 2048) sort_roots<2>(n, label, par, stopped, rkey, rslot);
        else sort_roots<4>(n, label, par, stopped, rkey, rslot);
        for (int j = t; j < n; j += T) {
            const unsigned long long kj = rkey[j];
            if (kj == ~0ull) continue;
            const int p = (int)(kj >> 12);
            if (j == 0 || (int)(rkey[j - 1] >> 12) != p) fpos[p] = j;
            if (j + 1 == NP || (int)(rkey[j + 1] >> 12) != p) nroot[p] = j + 1;   // end, for now
        }
        __syncthreads();
        for (int j = t; j < n; j += T) {
            const unsigned long long kj = rkey[j];
            if (kj == ~0ull) continue;
            const int p = (int)(kj >> 12), r = j - fpos[p];
            if (r < kClMax) roots[p][r] = (int)(kj & 0xFFFu);
        }
        __syncthreads();
        for (int p = t; p < kClMax; p += T)
            if (nroot[p] > 0) nroot[p] -= fpos[p];
        __syncthreads();
    }
    if (t == 0) {
        int ncl = nc0, splits = tab->n_splits;
        for (int p = 0; p < nc0; ++p) {
            newid_base[p] = -1;
            const int c = nroot[p];
            if (!stopped[p] || c < 2 || ncl + c - 1 > kClMax) continue;
            newid_base[p] = ncl;       // component r > 0 of p becomes ncl + r - 1
            ncl += c - 1;
            splits += 1;
        }
        tab->n_clusters = ncl;
        tab->n_splits = splits;
        acc->n_clusters = ncl;
    }
    __syncthreads();
    // relabel the points of split clusters and count the new clusters
    for (int i = t; i < n; i += T) {
        const int p = label[i];
        if (p >= nc0 || newid_base[p] < 0) continue;
        const int r = par[i];
        int rank = 0;
        while (rank < kClMax - 1 && roots[p][rank] != r) ++rank;
        const int q = (rank == 0) ? p : newid_base[p] + rank - 1;
        label_g[i] = q;
        atomicAdd(&ccount[q], 1);
    }
    __syncthreads();
    // volumes and moments of the new clusters (Eqs. new0-new6), split by split
    // in ascending order of the split cluster, each from the values before it:
    // the clusters that exist before a split (those of earlier splits
    // included) take the cross moments of (new3) with Y = X_r, the new
    // clusters among themselves those of (new2)
    if (t == 0) {
        int nb = nc0;
        for (int p = 0; p < nc0; ++p) {
            if (newid_base[p] < 0) continue;
            const int m = tab->moff[p + 1] - tab->moff[p];
            const double lxp = tab->clx[p], lm = log((double)m), lmm = log((double)m * (m + 1.0));
            const double lx2 = tab->lx2[p], lzx = tab->lzx[p], lzp = tab->lzp[p];
            const double lzpx = tab->lzpx[p], lz2p = tab->lz2p[p];
            for (int r = 0; r < nb; ++r) lxr[r] = tab->lxx[p * kClMax + r];
            const int c = nroot[p];
            for (int r = 0; r < c; ++r) {
                const int q = (r == 0) ? p : newid_base[p] + r - 1;
                const double ln = log((double)ccount[q]);
                const double lnn = log((double)ccount[q] * (ccount[q] + 1.0));
                tab->clx[q] = lxp + ln - lm;              // new0
                tab->cn[q] = ccount[q];
                tab->lx2[q] = lx2 + lnn - lmm;            // new1
                tab->lzx[q] = lzx + ln - lm;              // new3, Y = Z
                tab->lzp[q] = lzp + ln - lm;              // new4
                tab->lzpx[q] = lzpx + lnn - lmm;          // new5
                tab->lz2p[q] = lz2p + lnn - lmm;          // new6
                for (int o = 0; o < nb; ++o) {            // new3, Y = X_o
                    if (o == p) continue;
                    const double v = lxr[o] + ln - lm;
                    tab->lxx[q * kClMax + o] = v;
                    tab->lxx[o * kClMax + q] = v;
                }
            }
            for (int a = 0; a < c; ++a)                   // new2
                for (int b = 0; b < c; ++b) {
                    if (a == b) continue;
                    const int qa = (a == 0) ? p : newid_base[p] + a - 1;
                    const int qb = (b == 0) ? p : newid_base[p] + b - 1;
                    tab->lxx[qa * kClMax + qb] =
                        lx2 + log((double)ccount[qa] * (double)ccount[qb]) - lmm;
                }
            nb += c - 1;
        }
    }
}

int launch_clusters(void *arena, const RunDev *runs_dev, int n_runs, int max_live, int final_sweep,
                    bool any_fp64, bool any_fp32, hipStream_t s) {
    hipLaunchKernelGGL(cluster_pre_kernel, dim3(n_runs), dim3(kClThreads), 0, s, arena, runs_dev,
                       final_sweep);
    const dim3 grid((max_live + 63) / 64 * kKnnSplit, n_runs);
    // every pass is enqueued; a pass nobody needs returns at once
    for (int pass = 0; pass < kKnnPasses; ++pass) {
        if (any_fp64)
            hipLaunchKernelGGL((knn_part_kernel<double, kKnnPass>), grid, dim3(64 * kKnnWaves), 0, s,
                               arena, runs_dev, pass);
        if (any_fp32)
            hipLaunchKernelGGL((knn_part_kernel<float, kKnnPass>), grid, dim3(64 * kKnnWaves), 0, s,
                               arena, runs_dev, pass);
        hipLaunchKernelGGL(knn_merge_kernel, dim3((max_live + 255) / 256, n_runs), dim3(256), 0, s,
                           arena, runs_dev, pass);
        hipLaunchKernelGGL(cluster_cc_kernel, dim3(n_runs), dim3(kClThreads), 0, s, arena, runs_dev,
                           pass);
    }
    return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

}  // namespace ggns
