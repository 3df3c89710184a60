// Run start (parameter conversion, prior draws, first log-likelihoods),
// replacement of the killed points with dt adaptation, and the stand-alone
// log-likelihood / adjoint kernels.
#include "ggns_device.h"

namespace ggns {

namespace {

constexpr double kLog2Pi = 1.83787706640934548356;

// Converted parameters in the run's precision over the padded layout (padding
// coordinates zero, padding components with lognorm = -inf); constants in
// FP64 first.
template <typename T>
__device__ void convert_params(const RunDev &R, const double *raw, T *out) {
    const int d = R.d, dp = R.dp, K = R.n_comp, t = threadIdx.x, nt = blockDim.x;
    const int slots = variant_slots(R.var);
    if (R.kind == GGNS_LIK_GAUSS_DIAG) {
        const double *mu = raw, *sg = raw + d;
        for (int a = t; a < dp; a += nt) {
            out[a] = (a < d) ? (T)mu[a] : T(0);
            out[dp + a] = (a < d) ? (T)(1.0 / (sg[a] * sg[a])) : T(0);
        }
        if (t == 0) {
            double c = 0.0;
            for (int a = 0; a < d; ++a) c += -0.5 * kLog2Pi - log(sg[a]);
            out[2 * dp] = (T)c;
        }
    } else if (R.kind == GGNS_LIK_GAUSS_FULL) {
        // BF16 runs keep P rounded to BF16 (held in FP32) for their vector-ALU paths
        const bool bf = R.prec == GGNS_FP32_BF16MMA;
        for (int a = t; a < d; a += nt) out[a] = (T)raw[a];
        for (int64_t e = t; e < (int64_t)d * d; e += nt)
            out[d + 1 + e] = bf ? (T)round_bf16((float)raw[d + e]) : (T)raw[d + e];
        if (t == 0) out[d] = (T)(-0.5 * d * kLog2Pi + 0.5 * raw[d + (int64_t)d * d]);
    } else if (R.kind == GGNS_LIK_TORUS) {
        // the even coordinates (the paper's odd 1-based indices) carry cos(beta x),
        // written sin(beta x + pi/2); the odd ones sin(alpha x)
        const double half_pi = 1.57079632679489661923;
        for (int a = t; a < dp; a += nt) {
            const bool on = a < d;
            out[a] = on ? (T)((a & 1) ? raw[0] : raw[1]) : T(0);
            out[dp + a] = (on && !(a & 1)) ? (T)half_pi : T(0);
        }
        if (t == 0) out[2 * dp] = (T)raw[2];
    } else if (R.kind == GGNS_LIK_SHELLS) {
        for (int kk = 0; kk < slots; ++kk) {
            const double *blk = raw + kk * (d + 2);
            T *o = out + kk * (dp + 3);
            for (int a = t; a < dp; a += nt) o[a] = (kk < K && a < d) ? (T)blk[a] : T(0);
            if (t == 0) {
                if (kk < K) {
                    const double w = blk[d + 1];
                    o[dp] = (T)blk[d];
                    o[dp + 1] = (T)(1.0 / (w * w));
                    o[dp + 2] = (T)(-0.5 * kLog2Pi - log(w));
                } else {
                    o[dp] = T(0);
                    o[dp + 1] = T(0);
                    o[dp + 2] = (T)(-INFINITY);
                }
            }
        }
    } else {
        for (int kk = 0; kk < slots; ++kk) {
            const double *mu = raw + kk * 2 * d, *sg = mu + d;
            T *o = out + kk * gmm_stride(dp);
            for (int a = t; a < dp; a += nt) {
                const bool on = kk < K && a < d;
                o[a] = on ? (T)mu[a] : T(0);
                o[dp + a] = on ? (T)(1.0 / (sg[a] * sg[a])) : T(0);
            }
            if (t == 0) {
                if (kk < K) {
                    double c = -log((double)K);
                    for (int a = 0; a < d; ++a) c += -0.5 * kLog2Pi - log(sg[a]);
                    o[2 * dp] = (T)c;
                } else {
                    o[2 * dp] = (T)(-INFINITY);
                }
                for (int a = 2 * dp + 1; a < gmm_stride(dp); ++a) o[a] = T(0);
            }
        }
    }
}

__global__ void prepare_kernel(void *arena, const RunDev *__restrict__ runs, const double *params,
                               int init_state) {
    const RunDev &R = runs[blockIdx.x];
    const double *raw = params + R.param_offset;
    if (R.prec == GGNS_FP64)
        convert_params<double>(R, raw, at<double>(arena, R.off_prm));
    else
        convert_params<float>(R, raw, at<float>(arena, R.off_prm));
    if (R.prec == GGNS_FP32_BF16MMA && R.off_prm_bf16 >= 0) {
        // P rounded to BF16 (round to nearest even, via FP32) as the A operands
        // of the matrix-core walk: tiles (gmb, kb) of 64 lanes x 8 values, lane
        // l holding row l%16 and columns 8(l/16)+j of the tile.  M-block gmb is
        // block mb of wavefront w (gmb = w MBW + mb) and its row 4q+j is
        // dimension w dp/W + q L + 4 mb + j (L = dp / 4W dimensions per lane,
        // MBW = L / 4); column 8q+j of K-block kb is dimension 32 kb + 8q + j.
        // Padding entries are zero.
        const int d = R.d, dp = (d + 31) & ~31, W = R.mw, L = dp / (4 * W), MBW = L / 4;
        const int KB = dp / 32;
        uint16_t *pb = at<uint16_t>(arena, R.off_prm_bf16);
        const double *P = raw + d;
        for (int64_t e = threadIdx.x; e < (int64_t)dp * dp; e += blockDim.x) {
            const int t = (int)(e / 512), lane = (int)((e / 8) % 64), j = (int)(e % 8);
            const int gmb = t / KB, kb = t % KB;
            const int w = gmb / MBW, mb = gmb % MBW;
            const int ro = lane % 16, qk = lane / 16;
            const int o = w * (dp / W) + (ro / 4) * L + 4 * mb + (ro % 4);
            const int i = 32 * kb + 8 * qk + j;
            const float f = (o < d && i < d) ? (float)P[(int64_t)o * d + i] : 0.0f;
            uint32_t b = __float_as_uint(f);
            b += 0x7FFFu + ((b >> 16) & 1u);
            pb[e] = (uint16_t)(b >> 16);
        }
    }
    if (init_state && threadIdx.x == 0) {
        Acc *acc = at<Acc>(arena, R.off_acc);
        acc->log_z = -INFINITY;
        acc->log_x = 0.0;
        acc->log_z2 = -INFINITY;
        acc->dt = R.dt_init * (R.hi - R.lo);
        acc->lstar = -INFINITY;
        acc->log_xl_max = -INFINITY;
        acc->h = acc->sigma_kl = acc->sigma_mom = 0.0;
        acc->iter = 0;
        acc->evals = R.n_live;
        acc->n_dead = 0;
        acc->steps_out = acc->steps_in = acc->prunes = acc->nosave = 0;
        acc->it_outs = acc->it_steps = 0ull;
        acc->win_a = acc->win_b = 0;
        acc->replayed = 0ull;
        acc->state = GGNS_RUN_ACTIVE;
        // the torus reward is a likelihood only where S + c > 0 for every x: c > d
        if (R.kind == GGNS_LIK_TORUS && !(raw[2] > (double)R.d)) acc->state = GGNS_RUN_NONFINITE;
        acc->n_clusters = R.cluster_mode ? 1 : 0;
        acc->order_ok = 0;
        acc->summary_pending = 0;
        if (R.cluster_mode) {
            ClusterTab *tab = at<ClusterTab>(arena, R.off_cltab);
            for (int p = 0; p < kClMax; ++p) {
                tab->clx[p] = (p == 0) ? 0.0 : -INFINITY;
                tab->cn[p] = (p == 0) ? R.n_live : 0;
                tab->cum[p] = 0.0;
            }
            for (int p = 0; p <= kClMax; ++p) tab->soff[p] = tab->moff[p] = 0;
            tab->n_clusters = 1;
            tab->n_splits = 0;
            tab->stopping = 0;
            tab->cc_done = 0;
            tab->n_cut = 0;
            // Eqs. (ini0)-(ini11): one cluster, Xbar = 1, (X^2)bar = 1, no evidence
            for (int p = 0; p < kClMax; ++p) {
                tab->need[p] = 0;
                tab->lzp[p] = tab->lz2p[p] = tab->lzx[p] = tab->lzpx[p] = -INFINITY;
                tab->lx2[p] = (p == 0) ? 0.0 : -INFINITY;
            }
            for (int i = 0; i < kClMax * kClMax; ++i) tab->lxx[i] = -INFINITY;
        }
    }
    if (init_state && R.cluster_mode) {
        int32_t *label = at<int32_t>(arena, R.off_label);
        for (int i = threadIdx.x; i < R.n_live; i += blockDim.x) label[i] = 0;
    }
}

// Prior draws: coordinate a of point i is lo + (hi - lo) u with u the 24-bit
// open uniform of word (a & 3) of the INIT stream block (a >> 2); then the
// log-likelihood of the point.  Lane-group layout as in the walk.
template <typename T, int C, int KIND>
__global__ void __launch_bounds__(kWalkThreads)
init_points_kernel(void *arena, const RunDev *__restrict__ runs, const Tile *__restrict__ tiles) {
    const Tile tile = tiles[blockIdx.x];
    const RunDev &R = runs[tile.run];
    extern __shared__ __align__(16) unsigned char smem[];
    const int d = R.d, G = R.G;
    const int lane = threadIdx.x & 63, gl = lane & (G - 1), grp = threadIdx.x / G;
    const int a0 = gl * C;
    const int i = tile.m_begin + grp;
    const bool valid = i < tile.m_end;
    T *xch = reinterpret_cast<T *>(smem) + grp * (G * C);
    const T *prm = at<T>(arena, R.off_prm);
    const double w = R.hi - R.lo;
    T x[C], g[C], p0[C];
    uint32_t u[4];
    int last_b = -1;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int a = a0 + c;
        x[c] = T(0);
        if (a < d && valid) {
            if ((a >> 2) != last_b) {
                last_b = a >> 2;
                draw4(R.seed, (uint32_t)last_b, (uint32_t)i, 0u, TAG_INIT, 0u, u);
            }
            const uint32_t word = (a & 3) == 0 ? u[0] : ((a & 3) == 1 ? u[1] : ((a & 3) == 2 ? u[2] : u[3]));
            x[c] = (T)(R.lo + w * u24_open(word));
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) p0[c] = T(0);
    typename ParamsOf<T, C, KIND>::type P;
    P.load(prm, R.dp, a0);
    const T l = lik_step<T, C, KIND>(P, d, a0, G, x, p0, g, xch).l;
    if (valid) {
        T *xo = at<T>(arena, R.off_live_x) + (int64_t)i * d;
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (a0 + c < d) xo[a0 + c] = x[c];
        if (gl == 0) at<double>(arena, R.off_live_logl)[i] = (double)l;
    }
}

// Walker outputs into the killed slots; dt update from out_frac; next iteration.
// A work item is four consecutive coordinates of one walker's row (and, for the
// row's first item, its log L and cluster label): the killed slot is read once
// per item, the four loads of the row issue together, and the index arithmetic
// stays in 32 bits.
template <typename T>
__device__ __forceinline__ void scatter_item(const RunDev &R, const int32_t *killed, const T *wx,
                                             T *lx, int m, int c0) {
    const int d = R.d;
    const int slot = killed[m];
    const T *src = wx + (int64_t)m * d + c0;
    T v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = (c0 + j < d) ? src[j] : T(0);
    T *dst = lx + (int64_t)slot * d + c0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (c0 + j < d) dst[j] = v[j];
}

__global__ void replace_kernel(void *arena, const RunDev *__restrict__ runs) {
    const RunDev &R = runs[blockIdx.y];
    Acc *acc = at<Acc>(arena, R.off_acc);
    if (acc->state != GGNS_RUN_ACTIVE) return;
    const int k = R.n_kill, nchunk = (R.d + 3) >> 2;
    const int items = k * nchunk;
    const int i0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    const int32_t *killed = at<int32_t>(arena, R.off_killed);
    const double *wl = at<double>(arena, R.off_walk_logl);
    double *ll = at<double>(arena, R.off_live_logl);
    const bool f64 = R.prec == GGNS_FP64;
    for (int it = i0; it < items; it += stride) {
        const int m = it / nchunk, c0 = (it - m * nchunk) << 2;
        if (f64)
            scatter_item<double>(R, killed, at<double>(arena, R.off_walk_x),
                                 at<double>(arena, R.off_live_x), m, c0);
        else
            scatter_item<float>(R, killed, at<float>(arena, R.off_walk_x),
                                at<float>(arena, R.off_live_x), m, c0);
        if (c0 == 0) ll[killed[m]] = wl[m];
    }
    if (R.cluster_mode) {
        // the new point joins the cluster its walker was spawned in; the
        // workgroup counts its joins in LDS and adds them with one atomic per
        // cluster
        __shared__ int joins[kClMax];
        int32_t *label = at<int32_t>(arena, R.off_label);
        const int32_t *scl = at<int32_t>(arena, R.off_start_cl);
        ClusterTab *tab = at<ClusterTab>(arena, R.off_cltab);
        for (int p = threadIdx.x; p < kClMax; p += blockDim.x) joins[p] = 0;
        __syncthreads();
        for (int m = i0; m < k; m += stride) {
            label[killed[m]] = scl[m];
            atomicAdd(&joins[scl[m]], 1);
        }
        __syncthreads();
        for (int p = threadIdx.x; p < kClMax; p += blockDim.x)
            if (joins[p] != 0) atomicAdd(&tab->cn[p], joins[p]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned long long st = acc->it_steps;
        if (st > 0) {
            const double out_frac = (double)acc->it_outs / (double)st;
            if (out_frac > R.out_hi)
                acc->dt *= R.dt_down;
            else if (out_frac < R.out_lo)
                acc->dt *= R.dt_up;
        }
        acc->iter += 1;
    }
}

// Stand-alone log L, score or adjoint at caller-provided points.
template <typename T, int C, int KIND>
__global__ void __launch_bounds__(kWalkThreads)
loglike_kernel(void *arena, const RunDev *__restrict__ run, const T *__restrict__ xs, int64_t n,
               double *logl, T *grad, const double *gout) {
    const RunDev &R = *run;
    extern __shared__ __align__(16) unsigned char smem[];
    const int d = R.d, G = R.G;
    const int lane = threadIdx.x & 63, gl = lane & (G - 1), grp = threadIdx.x / G;
    const int a0 = gl * C;
    const int ngroups = blockDim.x / G;
    const int64_t i = (int64_t)blockIdx.x * ngroups + grp;
    const bool valid = i < n;
    T *xch = reinterpret_cast<T *>(smem) + grp * (G * C);
    const T *prm = at<T>(arena, R.off_prm);
    T x[C], g[C], p0[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        x[c] = (valid && a0 + c < d) ? xs[i * d + a0 + c] : T(0);
        p0[c] = T(0);
    }
    typename ParamsOf<T, C, KIND>::type P;
    P.load(prm, R.dp, a0);
    const T l = lik_step<T, C, KIND>(P, d, a0, G, x, p0, g, xch).l;
    if (!valid) return;
    if (logl != nullptr && gl == 0) logl[i] = (double)l;
    if (grad != nullptr) {
        const T s = (gout != nullptr) ? (T)gout[i] : T(1);
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (a0 + c < d) grad[i * d + a0 + c] = s * g[c];
    }
}

__global__ void set_vars_kernel(void *arena, const RunDev *__restrict__ run, double log_z,
                                double log_x, double dt, long long iter) {
    Acc *acc = at<Acc>(arena, run->off_acc);
    acc->log_z = log_z;
    acc->log_x = log_x;
    acc->dt = dt;
    acc->iter = iter;
}

template <typename T, int C>
hipError_t init_t(void *arena, const RunDev *runs, const Tile *tiles, int n_tiles, int kind,
                  size_t lds, hipStream_t s) {
    GGNS_DISPATCH_KIND(kind, hipLaunchKernelGGL((init_points_kernel<T, C, KIND_>), dim3(n_tiles),
                                                dim3(kWalkThreads), lds, s, arena, runs, tiles));
    return hipGetLastError();
}

template <typename T, int C>
hipError_t loglike_t(void *arena, const RunDev *run, const void *x, int64_t n, double *logl,
                     void *grad, const double *gout, int G, int kind, hipStream_t s) {
    const int ngroups = kWalkThreads / G;
    const int64_t blocks = (n + ngroups - 1) / ngroups;
    const size_t lds = (size_t)kWalkThreads * C * sizeof(T);
    GGNS_DISPATCH_KIND(kind, hipLaunchKernelGGL((loglike_kernel<T, C, KIND_>), dim3((unsigned)blocks),
                                                dim3(kWalkThreads), lds, s, arena, run,
                                                reinterpret_cast<const T *>(x), n, logl,
                                                reinterpret_cast<T *>(grad), gout));
    return hipGetLastError();
}

}  // namespace

void launch_prepare(void *arena, const RunDev *runs_dev, int n_runs, const double *params,
                    hipStream_t s, int init_state) {
    hipLaunchKernelGGL(prepare_kernel, dim3(n_runs), dim3(256), 0, s, arena, runs_dev, params,
                       init_state);
}

int launch_init_class(void *arena, const RunDev *runs_dev, const Tile *tiles, int n_tiles, int prec,
                      int C, int kind, hipStream_t s) {
    hipError_t e = hipErrorInvalidValue;
    const size_t lds = (size_t)kWalkThreads * C * (prec == GGNS_FP64 ? 8 : 4);
    if (prec == GGNS_FP64) {
        switch (C) {
            case 1: e = init_t<double, 1>(arena, runs_dev, tiles, n_tiles, kind, lds, s); break;
            case 2: e = init_t<double, 2>(arena, runs_dev, tiles, n_tiles, kind, lds, s); break;
            case 4: e = init_t<double, 4>(arena, runs_dev, tiles, n_tiles, kind, lds, s); break;
        }
    } else {
        switch (C) {
            case 1: e = init_t<float, 1>(arena, runs_dev, tiles, n_tiles, kind, lds, s); break;
            case 2: e = init_t<float, 2>(arena, runs_dev, tiles, n_tiles, kind, lds, s); break;
            case 4: e = init_t<float, 4>(arena, runs_dev, tiles, n_tiles, kind, lds, s); break;
            case 8: e = init_t<float, 8>(arena, runs_dev, tiles, n_tiles, kind, lds, s); break;
        }
    }
    return e == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

void launch_replace(void *arena, const RunDev *runs_dev, int n_runs, int max_kd, hipStream_t s) {
    // about one four-coordinate item per thread for the largest run
    int bx = (max_kd / 4 + 255) / 256;
    if (bx < 1) bx = 1;
    if (bx > 1024) bx = 1024;
    hipLaunchKernelGGL(replace_kernel, dim3(bx, n_runs), dim3(256), 0, s, arena, runs_dev);
}

int launch_loglike(void *arena, const RunDev *run_dev, const RunDev &run_host, const void *x,
                   int64_t n, double *logl, void *grad, const double *gout, hipStream_t s) {
    hipError_t e = hipErrorInvalidValue;
    const int C = run_host.C, G = run_host.G;
    if (run_host.prec == GGNS_FP64) {
        switch (C) {
            case 1: e = loglike_t<double, 1>(arena, run_dev, x, n, logl, grad, gout, G, run_host.var, s); break;
            case 2: e = loglike_t<double, 2>(arena, run_dev, x, n, logl, grad, gout, G, run_host.var, s); break;
            case 4: e = loglike_t<double, 4>(arena, run_dev, x, n, logl, grad, gout, G, run_host.var, s); break;
        }
    } else {
        switch (C) {
            case 1: e = loglike_t<float, 1>(arena, run_dev, x, n, logl, grad, gout, G, run_host.var, s); break;
            case 2: e = loglike_t<float, 2>(arena, run_dev, x, n, logl, grad, gout, G, run_host.var, s); break;
            case 4: e = loglike_t<float, 4>(arena, run_dev, x, n, logl, grad, gout, G, run_host.var, s); break;
            case 8: e = loglike_t<float, 8>(arena, run_dev, x, n, logl, grad, gout, G, run_host.var, s); break;
        }
    }
    return e == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

// The walk's momentum-noise stream on its own: thread (m, b) seeds the
// xoshiro128++ state of walker m's coordinate block b exactly as the walk does
// and draws four words and four FP32 normals per step.
__global__ void noise_normals_kernel(uint64_t seed, uint32_t it, int n_walkers, int n_blocks,
                                     int steps, float *normals, uint32_t *words, float *checksum) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n_walkers * n_blocks;
    if (gid >= total) return;
    const int m = (int)(gid / n_blocks), b = (int)(gid % n_blocks);
    uint32_t w[4];
    draw4(seed, (uint32_t)b, (uint32_t)m, it, TAG_EPS, 0u, w);
    Xoshiro e;
    e.seed(w);
    float acc = 0.0f;
    for (int t = 0; t < steps; ++t) {
        w[0] = e.next();
        w[1] = e.next();
        w[2] = e.next();
        w[3] = e.next();
        float z[4];
        normals2(w[0], w[1], z[0], z[1]);
        normals2(w[2], w[3], z[2], z[3]);
        const int64_t row = ((int64_t)t * total + gid) * 4;
        if (normals != nullptr)
            for (int j = 0; j < 4; ++j) normals[row + j] = z[j];
        if (words != nullptr)
            for (int j = 0; j < 4; ++j) words[row + j] = w[j];
        acc += (z[0] + z[1]) + (z[2] + z[3]);
    }
    if (checksum != nullptr) checksum[gid] = acc;
}

int launch_noise_normals(uint64_t seed, int iteration, int n_walkers, int n_blocks, int steps,
                         float *normals, uint32_t *words, float *checksum, hipStream_t s) {
    const int64_t total = (int64_t)n_walkers * n_blocks;
    if (total == 0) return GGNS_OK;
    const int threads = 256;
    const int64_t blocks = (total + threads - 1) / threads;
    hipLaunchKernelGGL(noise_normals_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, seed,
                       (uint32_t)iteration, n_walkers, n_blocks, steps, normals, words, checksum);
    return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

// Every run's accumulators as the public stats record, packed for one copy.
__global__ void gather_acc_kernel(void *arena, const RunDev *__restrict__ runs, int n_runs,
                                  ggns_run_stats *mirror) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_runs) return;
    const Acc &a = *at<Acc>(arena, runs[r].off_acc);
    ggns_run_stats o;
    o.log_z = a.log_z; o.log_x = a.log_x; o.log_z2 = a.log_z2; o.dt = a.dt; o.lstar = a.lstar;
    o.log_xl_max = a.log_xl_max; o.h = a.h; o.sigma_kl = a.sigma_kl; o.sigma_mom = a.sigma_mom;
    o.iter = a.iter; o.evals = a.evals; o.n_dead = a.n_dead; o.steps_out = a.steps_out;
    o.steps_in = a.steps_in; o.prunes = a.prunes; o.nosave = a.nosave;
    o.it_outs = (int64_t)a.it_outs; o.it_steps = (int64_t)a.it_steps;
    o.replayed = (int64_t)a.replayed;
    o.state = a.state; o.n_clusters = a.n_clusters;
    mirror[r] = o;
}

int launch_gather_acc(void *arena, const RunDev *runs_dev, int n_runs, ggns_run_stats *mirror,
                      hipStream_t s) {
    if (n_runs <= 0) return GGNS_OK;
    hipLaunchKernelGGL(gather_acc_kernel, dim3((n_runs + 63) / 64), dim3(64), 0, s, arena, runs_dev,
                       n_runs, mirror);
    return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

void launch_set_vars(void *arena, const RunDev *run_dev, double log_z, double log_x, double dt,
                     long long iter, hipStream_t s) {
    hipLaunchKernelGGL(set_vars_kernel, dim3(1), dim3(1), 0, s, arena, run_dev, log_z, log_x, dt,
                       iter);
}

}  // namespace ggns
