// Cluster recognition for runs in cluster mode (Section 3, mode collapse
// mitigation; Algorithm GGNS with its cluster-finding algorithm; Eq. new0
// for the split of a cluster's prior volume).  Readings: cluster finding
// runs at the start of every iteration that goes on, once for every cluster
// that exists then; for k = 2, 3, ... every point of a cluster is linked to
// its k nearest other points of the cluster (squared Euclidean distance,
// ties by slot) and the connected components of the undirected graph are
// taken; the first k whose component sizes equal those of k - 1 gives the
// clustering (k up to min(cluster_kmax, m - 1), else the cluster stays
// whole); components ordered by their smallest slot become clusters, the
// first keeping the old index, at most kClMax in all; Xbar_i = (n_i/n) Xbar_p.
//
// Three launches per iteration: cluster_pre (termination decision; the live
// slots grouped by cluster), knn (one wavefront per point: its nearest
// neighbours within its cluster, distances summed in FP64 in coordinate order
// so that neighbour ranks are exact), cluster_cc (one workgroup per run:
// union-find over the k-th neighbour edges for k = 1, 2, ...; since the graph
// for k contains the graph for k - 1, its partition is a coarsening, and equal
// component sizes are equal component counts, which is what is compared).
#include "ggns_device.h"

namespace ggns {

namespace {

constexpr int kClThreads = 1024;

__device__ __forceinline__ bool lex_less(double a, int sa, double b, int sb) {
    return a < b || (a == b && sa < sb);
}

}  // namespace

// Termination decision and members grouped by cluster.
__global__ void __launch_bounds__(kClThreads)
cluster_pre_kernel(void *arena, const RunDev *__restrict__ runs, int final_sweep) {
    const RunDev &R = runs[blockIdx.x];
    if (!R.cluster_mode) return;
    Acc *acc = at<Acc>(arena, R.off_acc);
    if (acc->state != GGNS_RUN_ACTIVE) return;
    ClusterTab *tab = at<ClusterTab>(arena, R.off_cltab);
    __shared__ uint32_t key[kMaxLive];
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
    if (t == 0) tab->stopping = stop;
    if (stop) return;
    // live slots grouped by cluster: sort of (label << 12 | slot)
    int NP = 1;
    while (NP < n) NP <<= 1;
    for (int i = t; i < NP; i += T) key[i] = (i < n) ? ((uint32_t)label[i] << 12) | (uint32_t)i : 0xFFFFFFFFu;
    for (int size = 2; size <= NP; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int i = t; i < (NP >> 1); i += T) {
                const int lo = 2 * stride * (i / stride) + (i % stride), hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint32_t a = key[lo], b = key[hi];
                if ((a > b) == asc) { key[lo] = b; key[hi] = a; }
            }
        }
    }
    __syncthreads();
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

// One wavefront per live point: its kKnnMax nearest other points of its cluster.
template <typename T>
__global__ void __launch_bounds__(256)
knn_kernel(void *arena, const RunDev *__restrict__ runs) {
    const RunDev &R = runs[blockIdx.y];
    if (!R.cluster_mode || (R.prec == GGNS_FP64) != (sizeof(T) == 8)) return;
    const Acc *acc = at<Acc>(arena, R.off_acc);
    if (acc->state != GGNS_RUN_ACTIVE) return;
    const ClusterTab *tab = at<ClusterTab>(arena, R.off_cltab);
    if (tab->stopping) return;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= R.n_live) return;
    const int32_t *label = at<int32_t>(arena, R.off_label);
    const int c = label[i];
    const int m0 = tab->moff[c], m = tab->moff[c + 1] - m0;
    if (m < 3) return;
    const int keff = (R.cluster_kmax < m - 1) ? R.cluster_kmax : m - 1;
    const int d = R.d;
    const T *X = at<T>(arena, R.off_live_x);
    const T *xi = X + (int64_t)i * d;
    const int32_t *members = at<int32_t>(arena, R.off_members);
    double bd[kKnnMax];
    int bs[kKnnMax];
#pragma unroll
    for (int q = 0; q < kKnnMax; ++q) { bd[q] = INFINITY; bs[q] = 0x7FFFFFFF; }
    for (int u = lane; u < m; u += 64) {
        const int j = members[m0 + u];
        if (j == i) continue;
        const T *xj = X + (int64_t)j * d;
        double s = 0.0;
        {
#pragma clang fp contract(off)
            for (int a = 0; a < d; ++a) {
                const double e = (double)xi[a] - (double)xj[a];
                s = s + e * e;
            }
        }
        if (lex_less(s, j, bd[kKnnMax - 1], bs[kKnnMax - 1])) {
            bd[kKnnMax - 1] = s;
            bs[kKnnMax - 1] = j;
#pragma unroll
            for (int q = kKnnMax - 1; q > 0; --q) {
                const bool sw = lex_less(bd[q], bs[q], bd[q - 1], bs[q - 1]);
                const double td = bd[q];
                const int ts = bs[q];
                bd[q] = sw ? bd[q - 1] : bd[q];
                bs[q] = sw ? bs[q - 1] : bs[q];
                bd[q - 1] = sw ? td : bd[q - 1];
                bs[q - 1] = sw ? ts : bs[q - 1];
            }
        }
    }
    // merge the 64 lane lists: keff rounds of a wavefront arg-min of the heads
    int32_t *knn = at<int32_t>(arena, R.off_knn) + (int64_t)i * kKnnMax;
    for (int r = 0; r < keff; ++r) {
        double hd = bd[0];
        int hs = bs[0];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double od = __shfl_xor(hd, o, 64);
            const int os = __shfl_xor(hs, o, 64);
            const bool take = lex_less(od, os, hd, hs);
            hd = take ? od : hd;
            hs = take ? os : hs;
        }
        if (lane == 0) knn[r] = hs;
        if (bs[0] == hs) {
#pragma unroll
            for (int q = 0; q < kKnnMax - 1; ++q) { bd[q] = bd[q + 1]; bs[q] = bs[q + 1]; }
            bd[kKnnMax - 1] = INFINITY;
            bs[kKnnMax - 1] = 0x7FFFFFFF;
        }
    }
}

namespace {

__device__ __forceinline__ int uf_root(volatile int *par, int i) {
    int r = i;
    while (par[r] != r) r = par[r];
    return r;
}

}  // namespace

// One workgroup per run: components for k = 1, 2, ... neighbours, the stop
// rule per cluster, and the splits.
__global__ void __launch_bounds__(kClThreads)
cluster_cc_kernel(void *arena, const RunDev *__restrict__ runs) {
    const RunDev &R = runs[blockIdx.x];
    if (!R.cluster_mode) return;
    Acc *acc = at<Acc>(arena, R.off_acc);
    if (acc->state != GGNS_RUN_ACTIVE) return;
    ClusterTab *tab = at<ClusterTab>(arena, R.off_cltab);
    if (tab->stopping) return;
    __shared__ int par[kMaxLive];
    __shared__ int keff[kClMax], stopped[kClMax], cnt_prev[kClMax], cnt_cur[kClMax];
    __shared__ int nroot[kClMax], roots[kClMax][kClMax], newid_base[kClMax];
    __shared__ int ccount[kClMax];
    __shared__ int changed;
    const int n = R.n_live, t = threadIdx.x, T = blockDim.x;
    int32_t *label = at<int32_t>(arena, R.off_label);
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
    for (int k = 1; k <= R.cluster_kmax && k <= kKnnMax; ++k) {
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
        for (int p = t; p < kClMax; p += T) {
            if (!keff[p] || stopped[p] || k > keff[p]) continue;
            if (k >= 3 && cnt_cur[p] == cnt_prev[p]) stopped[p] = k;
            cnt_prev[p] = cnt_cur[p];
        }
        __syncthreads();
    }
    // roots of the stopped clusters in ascending slot order
    if (t == 0) {
        for (int i = 0; i < n; ++i) {
            const int p = label[i];
            if (stopped[p] && par[i] == i) {
                if (nroot[p] < kClMax) roots[p][nroot[p]] = i;
                nroot[p] += 1;
            }
        }
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
        label[i] = q;
        atomicAdd(&ccount[q], 1);
    }
    __syncthreads();
    if (t == 0) {
        for (int p = 0; p < nc0; ++p) {
            if (newid_base[p] < 0) continue;
            const double lxp = tab->clx[p], lm = log((double)(tab->moff[p + 1] - tab->moff[p]));
            const int c = nroot[p];
            for (int r = 0; r < c; ++r) {
                const int q = (r == 0) ? p : newid_base[p] + r - 1;
                tab->clx[q] = lxp + log((double)ccount[q]) - lm;
                tab->cn[q] = ccount[q];
            }
        }
    }
}

int launch_clusters(void *arena, const RunDev *runs_dev, int n_runs, int max_live, int final_sweep,
                    bool any_fp64, bool any_fp32, hipStream_t s) {
    hipLaunchKernelGGL(cluster_pre_kernel, dim3(n_runs), dim3(kClThreads), 0, s, arena, runs_dev,
                       final_sweep);
    const dim3 grid((max_live + 3) / 4, n_runs);
    if (any_fp64)
        hipLaunchKernelGGL(knn_kernel<double>, grid, dim3(256), 0, s, arena, runs_dev);
    if (any_fp32)
        hipLaunchKernelGGL(knn_kernel<float>, grid, dim3(256), 0, s, arena, runs_dev);
    hipLaunchKernelGGL(cluster_cc_kernel, dim3(n_runs), dim3(kClThreads), 0, s, arena, runs_dev);
    return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

}  // namespace ggns
