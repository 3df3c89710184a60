// The batched HSS walk for correlated Gaussians on the BF16 matrix cores.
//
// Same walk as the vector-ALU kernel (Algorithm GGNS HSS; Eq. reflection;
// Section 3), specialised to log L = c - r.P r / 2 with r = x - mu and score
// -P r: the product Y^T = P R^T of the precision matrix with the residuals of
// 16 walkers is a dense contraction and runs as v_mfma_f32_16x16x32_bf16 (BF16
// operands rounded to nearest even, FP32 accumulation); r.y, p.y and y.y and
// everything else stay FP32 on the vector ALUs, the threshold compare FP64.
//
// Layout.  A wavefront advances 16 walkers; lane l serves walker slot l % 16
// and owns the quarter q = l / 16 of its dimensions, [q*Q, q*Q + Q) with
// Q = dp / 4 (dp = d padded to a multiple of 32), holding x, p and y = P r for
// them in registers.  The MFMA's B operand (K rows of R^T for one walker
// column, 8 per lane quarter) and its accumulator (4 output rows per lane
// quarter) both land on a lane's own dimensions once the rows and columns of P
// are relabelled: output row 4q'+j of M-block mb is dimension q'Q + 4mb + j and
// K row 8q'+j of K-block kb is dimension q'Q + 8kb + j.  The prepare kernel
// stores P in that relabelled, MFMA-tiled order (one 1 KB tile of 64 lanes x 8
// BF16 per (mb, kb)), so every A operand is one contiguous 16-byte LDS read and
// no data moves between lanes around the contraction.  Reductions over a
// walker's dimensions are lane-local sums plus two cross-row exchanges
// (lanes l, l^16, l^32, l^48).
#include "ggns_device.h"

namespace ggns {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaThreads = 256;   // 4 wavefronts, 64 walker slots

__device__ __forceinline__ float sum4(float v) {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

template <int Q>
__device__ __forceinline__ void momentum_quarter(uint64_t seed, uint32_t m, uint32_t it,
                                                 uint32_t sub, int a0, int d, float (&p)[Q]) {
#pragma unroll
    for (int i = 0; i < Q / 4; ++i) {
        uint32_t w[4];
        draw4(seed, (uint32_t)((a0 >> 2) + i), m, it, TAG_P0, sub, w);
        normals2(w[0], w[1], p[4 * i], p[4 * i + 1]);
        normals2(w[2], w[3], p[4 * i + 2], p[4 * i + 3]);
    }
#pragma unroll
    for (int c = 0; c < Q; ++c) p[c] = (a0 + c < d) ? p[c] : 0.0f;
}

}  // namespace

// dp = 4Q; tiles: (dp/16) x (dp/32) of 512 BF16 each, then mu[dp] (FP32).
template <int Q>
__global__ void __launch_bounds__(kMfmaThreads)
walk_mfma_kernel(void *arena, const RunDev *__restrict__ runs, const Tile *__restrict__ tiles) {
    constexpr int DP = 4 * Q, MB = DP / 16, KB = DP / 32;
    const Tile tile = tiles[blockIdx.x];
    const RunDev &R = runs[tile.run];
    Acc *acc = at<Acc>(arena, R.off_acc);
    if (acc->state != GGNS_RUN_ACTIVE) return;

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int next_walker;
    __shared__ unsigned long long blk_cnt[4];
    bf16x8 *ptile = reinterpret_cast<bf16x8 *>(smem);
    float *mu_s = reinterpret_cast<float *>(smem + (size_t)MB * KB * 64 * 16);
    {
        const uint4 *src = at<uint4>(arena, R.off_prm_bf16);
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        for (int i = threadIdx.x; i < MB * KB * 64; i += blockDim.x) dst[i] = src[i];
        const float *prm = at<float>(arena, R.off_prm);
        for (int i = threadIdx.x; i < DP; i += blockDim.x) mu_s[i] = (i < R.d) ? prm[i] : 0.0f;
    }
    if (threadIdx.x == 0) {
        next_walker = tile.m_begin + kMfmaThreads / 4;
        blk_cnt[0] = blk_cnt[1] = blk_cnt[2] = blk_cnt[3] = 0ull;
    }
    __syncthreads();

    const int d = R.d;
    const int lane = threadIdx.x & 63;
    const int slot = lane & 15, quarter = lane >> 4;
    const int a0 = quarter * Q;
    const float cst = at<float>(arena, R.off_prm)[d];
    // padding coordinates (a >= d) hold zero position and momentum
#define VALID(c) (a0 + (c) < d)

    const double lstar = acc->lstar;
    const float dt = (float)acc->dt;
    const uint32_t it = (uint32_t)acc->iter;
    const float lo = (float)R.lo, hi = (float)R.hi, dpn = (float)R.delta_p;
    const uint64_t seed = R.seed;
    const int nsurv = R.n_live - R.n_kill;
    const int min_ref = R.min_ref, max_ref = R.max_ref, n_steps_max = R.n_steps_max;
    const int prune_streak = R.prune_streak;
    const int32_t *surv = at<int32_t>(arena, R.off_surv);
    int32_t *start_arr = at<int32_t>(arena, R.off_start);
    const float *live_x = at<float>(arena, R.off_live_x);
    const double *live_logl = at<double>(arena, R.off_live_logl);
    float *walk_x = at<float>(arena, R.off_walk_x);
    double *walk_logl = at<double>(arena, R.off_walk_logl);
    float *trace_x = reinterpret_cast<float *>(R.trace_x);
    const int k = R.n_kill;
    const unsigned long long gmask = 0x0001000100010001ull << slot;

    float x[Q], p[Q], y[Q];
    Xoshiro eps[Q / 4];
    Xoshiro res;
    int m = tile.m_begin + (threadIdx.x >> 6) * 16 + slot;
    bool active = m < tile.m_end;
    int s = 0, nref = 0, streak = 0, steps = 0, outs = 0, nprune = 0, nsave = 0;
    double out_l = 0.0;
    unsigned long long c_outs = 0, c_steps = 0, c_prunes = 0, c_nosave = 0;

    auto start_walker = [&](int mm) {
        uint32_t w[4];
        draw4(seed, 0u, (uint32_t)mm, it, TAG_START, 0u, w);
        s = surv[(int)(((uint64_t)w[0] * (uint64_t)nsurv) >> 32)];
        if (quarter == 0) start_arr[mm] = s;
        const float *xs = live_x + (int64_t)s * d;
        float *wo = walk_x + (int64_t)mm * d;
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            x[c] = VALID(c) ? xs[a0 + c] : 0.0f;
            if (VALID(c)) wo[a0 + c] = x[c];
        }
        out_l = live_logl[s];
        momentum_quarter<Q>(seed, (uint32_t)mm, it, 0u, a0, d, p);
#pragma unroll
        for (int i = 0; i < Q / 4; ++i) {
            draw4(seed, (uint32_t)((a0 >> 2) + i), (uint32_t)mm, it, TAG_EPS, 0u, w);
            eps[i].seed(w);
        }
        draw4(seed, 0u, (uint32_t)mm, it, TAG_RES, 0u, w);
        res.seed(w);
        nref = streak = steps = outs = nprune = nsave = 0;
    };

    if (active) start_walker(m);

    while (__any(active)) {
        const uint32_t ures = res.next();
        // drift and residuals; BF16 B operands of R^T straight from registers
        bf16x8 bop[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int c = 8 * kb + j;
                x[c] = x[c] + dt * p[c];
                bop[kb][j] = (__bf16)(x[c] - mu_s[a0 + c]);
            }
        // Y^T = P R^T on the matrix cores, one 16x16 block of output rows at a time
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            floatx4 c4 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                c4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ptile[(mb * KB + kb) * 64 + lane],
                                                             bop[kb], c4, 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j) y[4 * mb + j] = c4[j];
        }
        // r.y, p.g and g.g with g = -y
        float qv = 0.0f, pg = 0.0f, gg = 0.0f;
        bool vany = false;
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            qv += (x[c] - mu_s[a0 + c]) * y[c];
            pg -= p[c] * y[c];
            gg += y[c] * y[c];
            vany = vany || (VALID(c) && (x[c] < lo || x[c] > hi));
        }
        qv = sum4(qv);
        pg = sum4(pg);
        gg = sum4(gg);
        const float l = cst - 0.5f * qv;
        const bool viol = (__ballot(vany) & gmask) != 0ull;
        const bool out = viol || ((double)l <= lstar);
        if (trace_x != nullptr) {
            if (active && steps < R.trace_steps) {
                const int64_t row = (int64_t)steps * k + m;
#pragma unroll
                for (int c = 0; c < Q; ++c)
                    if (VALID(c)) trace_x[row * d + a0 + c] = x[c];
                if (quarter == 0) {
                    R.trace_logl[row] = (double)l;
                    R.trace_out[row] = out ? 1 : 0;
                }
            }
        }
        steps += 1;
        const bool use_g = out && !viol && isfinite(gg) && gg > 0.0f;
        const bool flip_all = out && !viol && !use_g;
        const float f = use_g ? m_div(2.0f * pg, gg) : 0.0f;
#pragma unroll
        for (int i = 0; i < Q / 4; ++i) {
            // this step's noise for the block of four coordinates 4i..4i+3
            float z[4];
            const uint32_t w0 = eps[i].next(), w1 = eps[i].next(), w2 = eps[i].next(),
                           w3 = eps[i].next();
            normals2(w0, w1, z[0], z[1]);
            normals2(w2, w3, z[2], z[3]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * i + j;
                const bool vm = VALID(c) && (x[c] < lo || x[c] > hi);
                const bool flip = flip_all || (out && vm);
                const float pr = (flip ? -p[c] : p[c]) + f * y[c];   // p - f g with g = -y
                p[c] = pr * (1.0f + dpn * z[j]);
            }
        }
        nref += out ? 1 : 0;
        outs += out ? 1 : 0;
        streak = out ? streak + 1 : 0;
        const bool keep = !out && nref >= min_ref;
        nsave += keep ? 1 : 0;
        const bool take = !out && (keep ? ((uint64_t)ures * (uint64_t)nsave < (1ull << 32))
                                        : (nsave == 0));
        if (take && active) {
            float *wo = walk_x + (int64_t)m * d;
#pragma unroll
            for (int c = 0; c < Q; ++c)
                if (VALID(c)) wo[a0 + c] = x[c];
            out_l = (double)l;
        }
        if (prune_streak > 0 && streak >= prune_streak) {
            if (active) {
                const float *xs = live_x + (int64_t)s * d;
#pragma unroll
                for (int c = 0; c < Q; ++c) x[c] = VALID(c) ? xs[a0 + c] : 0.0f;
            }
            nprune += 1;
            momentum_quarter<Q>(seed, (uint32_t)m, it, (uint32_t)nprune, a0, d, p);
            nref = 0;
            streak = 0;
        }
        const bool done = !(steps < n_steps_max && (max_ref == 0 || nref < max_ref));
        const bool need = active && done;
        if (need && quarter == 0) {
            walk_logl[m] = out_l;
            c_outs += outs;
            c_steps += steps;
            c_prunes += nprune;
            c_nosave += (nsave == 0) ? 1 : 0;
        }
        int nm = 0;
        if (need && quarter == 0) nm = atomicAdd(&next_walker, 1);
        nm = __shfl(nm, slot, 64);
        if (need) {
            m = nm;
            active = m < tile.m_end;
            if (active) start_walker(m);
        }
    }

#undef VALID
    if (quarter == 0 && c_steps > 0) {
        atomicAdd(&blk_cnt[0], c_outs);
        atomicAdd(&blk_cnt[1], c_steps);
        atomicAdd(&blk_cnt[2], c_prunes);
        atomicAdd(&blk_cnt[3], c_nosave);
    }
    __syncthreads();
    if (threadIdx.x == 0 && blk_cnt[1] > 0) {
        atomicAdd(&acc->it_outs, blk_cnt[0]);
        atomicAdd(&acc->it_steps, blk_cnt[1]);
        atomicAdd(reinterpret_cast<unsigned long long *>(&acc->steps_out), blk_cnt[0]);
        atomicAdd(reinterpret_cast<unsigned long long *>(&acc->steps_in), blk_cnt[1] - blk_cnt[0]);
        atomicAdd(reinterpret_cast<unsigned long long *>(&acc->evals), blk_cnt[1]);
        atomicAdd(reinterpret_cast<unsigned long long *>(&acc->prunes), blk_cnt[2]);
        atomicAdd(reinterpret_cast<unsigned long long *>(&acc->nosave), blk_cnt[3]);
    }
}

size_t mfma_lds_bytes(int dp) {
    return (size_t)(dp / 16) * (dp / 32) * 64 * 16 + (size_t)dp * 4;
}

template <int Q>
static hipError_t launch_mfma_t(void *arena, const RunDev *runs, const Tile *tiles, int n_tiles,
                                hipStream_t s) {
    const size_t lds = mfma_lds_bytes(4 * Q);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&walk_mfma_kernel<Q>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr_set = true;
    }
    hipLaunchKernelGGL((walk_mfma_kernel<Q>), dim3(n_tiles), dim3(kMfmaThreads), lds, s, arena, runs,
                       tiles);
    return hipGetLastError();
}

int launch_walk_mfma(void *arena, const RunDev *runs_dev, const Tile *tiles, int n_tiles, int d_pad,
                     hipStream_t s) {
    hipError_t e = hipErrorInvalidValue;
    switch (d_pad) {
        case 32: e = launch_mfma_t<8>(arena, runs_dev, tiles, n_tiles, s); break;
        case 64: e = launch_mfma_t<16>(arena, runs_dev, tiles, n_tiles, s); break;
        case 128: e = launch_mfma_t<32>(arena, runs_dev, tiles, n_tiles, s); break;
        case 256: e = launch_mfma_t<64>(arena, runs_dev, tiles, n_tiles, s); break;
        default: return GGNS_EUNSUPPORTED;
    }
    return e == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

}  // namespace ggns
