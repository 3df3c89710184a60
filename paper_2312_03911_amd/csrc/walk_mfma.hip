// The batched HSS walk for correlated Gaussians on the BF16 matrix cores.
//
// Same walk as the vector-ALU kernel (Algorithm GGNS HSS; Eq. reflection;
// Section 3), specialised to log L = c - r.P r / 2 with r = x - mu and score
// -P r: the product Y^T = P R^T of the precision matrix with the residuals of
// 16 walkers is a dense contraction and runs as v_mfma_f32_16x16x32_bf16 (BF16
// operands rounded to nearest even, FP32 accumulation); r.y, p.y and y.y and
// everything else stay FP32 on the vector ALUs, the threshold compare FP64.
//
// Layout.  A workgroup of W wavefronts advances 16 walker slots together and
// splits the output rows of P between its wavefronts: wavefront w owns the
// dimensions [w dp/W, (w+1) dp/W) (dp = d padded to a multiple of 32) and holds
// its dp/W rows of P, as ready-made BF16 A operands, in registers for the whole
// walk.  Within a wavefront lane l serves walker slot l % 16 and owns the
// L = dp / (4W) consecutive dimensions a0 = w dp/W + (l/16) L ... of it,
// holding x, p, mu, y = P r and the reservoir point for them in registers.  With the output rows
// relabelled (row 4q+j of the wavefront's M-block mb is dimension
// w dp/W + q L + 4 mb + j) the accumulator lands on the lane that owns those
// dimensions.  Per step each lane writes its BF16 residuals to LDS, every
// wavefront reads the 16 walkers' residuals back as B operands (16-byte reads,
// rows padded against bank conflicts), and the per-wavefront partial sums of
// r.y, p.y, y.y and the box test meet in LDS; two workgroup barriers a step.
// All wavefronts take the same decisions for a walker from the same sums, and
// refill finished slots from the tile in slot order, so the refill needs no
// atomics.  The batch-minimum loop (walk_mode 1) runs as the vector-ALU walk
// runs it: a first walk of each walker to its own max_ref-th reflection that
// leaves its state and the run's saving window, then the continuation to the
// window's end.
#include "ggns_device.h"

namespace ggns {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// sum over the four lane quarters (lanes l, l^16, l^32, l^48), by row swaps
__device__ __forceinline__ float sum4(float v) { return xor32_sum(xor16_sum(v)); }

template <int L>
__device__ __forceinline__ void momentum_lane(uint64_t seed, uint32_t m, uint32_t it, uint32_t sub,
                                              int a0, int d, float (&p)[L]) {
#pragma unroll
    for (int i = 0; i < L / 4; ++i) {
        uint32_t w[4];
        draw4(seed, (uint32_t)((a0 >> 2) + i), m, it, TAG_P0, sub, w);
        normals2(w[0], w[1], p[4 * i], p[4 * i + 1]);
        normals2(w[2], w[3], p[4 * i + 2], p[4 * i + 3]);
    }
#pragma unroll
    for (int c = 0; c < L; ++c) p[c] = (a0 + c < d) ? p[c] : 0.0f;
}

}  // namespace

// L dimensions per lane, W wavefronts per group of 16 walkers; dp = 4 L W.
// NZ = 1: one noise normal per walker and step (one stream per lane, one noise
// factor per walker); NZ = 0: one per dimension (a stream per block of four).
template <int L, int W, int NZ>
__global__ void __launch_bounds__(64 * W, 1)
walk_mfma_kernel(void *arena, const RunDev *__restrict__ runs, const Tile *__restrict__ tiles,
                 int phase) {
    constexpr int DP = 4 * L * W, MBW = L / 4, KB = DP / 32, RS = DP + 8;
    constexpr int NE = NZ ? 1 : L / 4;   // noise streams per lane
    const Tile tile = tiles[blockIdx.x];
    const RunDev &R = runs[tile.run];
    Acc *acc = at<Acc>(arena, R.off_acc);
    if (acc->state != GGNS_RUN_ACTIVE) return;
    // phase 1: first walk of the batch-minimum loop (walk_mode 1 runs only);
    // phase 2: its continuation, or the whole per-walker walk (walk_mode 0)
    const bool batch = R.walk_mode == 1;
    if (phase == 1 && !batch) return;
    const bool first = phase == 1, cont = phase == 2 && batch;

    __shared__ __align__(16) __bf16 rbuf[16 * RS];       // residuals of the 16 slots
    __shared__ __align__(16) floatx4 part[W * 16];       // per-wavefront partial sums
    __shared__ unsigned long long blk_cnt[5];

    const int d = R.d;
    constexpr bool scalar_noise = NZ != 0;   // one noise normal per walker and step
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane & 15, quarter = lane >> 4;
    const int a0 = wave * (DP / W) + quarter * L;
    const bool lead = wave == 0 && quarter == 0;   // the lane that writes per-walker results
#define VALID(c) (a0 + (c) < d)

    // this wavefront's rows of P as A operands, and mu for the lane's dimensions
    bf16x8 amat[MBW][KB];
    {
        const bf16x8 *src = at<bf16x8>(arena, R.off_prm_bf16);
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                amat[mb][kb] = src[((wave * MBW + mb) * KB + kb) * 64 + lane];
    }
    const float *prm = at<float>(arena, R.off_prm);
    float mu[L];
#pragma unroll
    for (int c = 0; c < L; ++c) mu[c] = VALID(c) ? prm[a0 + c] : 0.0f;
    const float cst = prm[d];
    if (threadIdx.x < 5) blk_cnt[threadIdx.x] = 0ull;

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
    // stop and save rules of this launch (as in the vector-ALU walk)
    const int never = n_steps_max + 1;
    const int win_a = cont ? acc->win_a : 0, win_b = cont ? acc->win_b : 0;
    const int keep_ref = batch ? (first ? INT_MAX : 0) : min_ref;
    const int keep_step = cont ? win_a : 0;
    const int end_steps = cont ? win_b : n_steps_max;
    const int end_ref = cont ? 0 : max_ref;
    unsigned char *wst = batch ? at<unsigned char>(arena, R.off_wstate) : nullptr;

    float x[L], p[L], y[L], xo[L];   // xo: the walker's reservoir point, written when it ends
    Xoshiro eps[NE];
    Xoshiro res;
    int m = tile.m_begin + slot;
    int next = tile.m_begin + 16;      // same in every lane: slots refill in slot order
    bool active = m < tile.m_end;
    int s = 0, nref = 0, streak = 0, steps = 0, outs = 0, nprune = 0, nsave = 0, a_step = never;
    double out_l = 0.0;
    // padding dimensions sit at x = lo (inside the box, and without effect on
    // log L or the score: their rows and columns of P and their mu are zero),
    // so the box test needs no per-dimension bounds
    const float xpad = lo;

    auto start_walker = [&](int mm) __attribute__((always_inline)) {
        uint32_t w[4];
        draw4(seed, 0u, (uint32_t)mm, it, TAG_START, 0u, w);
        int cl;
        s = pick_start(R, arena, w, &cl);
        if (lead) {
            start_arr[mm] = s;
            if (R.cluster_mode) at<int32_t>(arena, R.off_start_cl)[mm] = cl;
        }
        const float *xs = live_x + (int64_t)s * d;
#pragma unroll
        for (int c = 0; c < L; ++c) {
            x[c] = VALID(c) ? xs[a0 + c] : xpad;
            xo[c] = x[c];
        }
        out_l = live_logl[s];
        momentum_lane<L>(seed, (uint32_t)mm, it, 0u, a0, d, p);
        // one normal per walker: every lane carries block 0's stream
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            draw4(seed, scalar_noise ? 0u : (uint32_t)((a0 >> 2) + i), (uint32_t)mm, it, TAG_EPS, 0u, w);
            eps[i].seed(w);
        }
        draw4(seed, 0u, (uint32_t)mm, it, TAG_RES, 0u, w);
        res.seed(w);
        nref = streak = steps = outs = nprune = nsave = 0;
        a_step = never;
    };

    // walker state between the two launches (layout as in the vector-ALU walk)
    auto wrow = [&](int mm) __attribute__((always_inline)) { return wst + (int64_t)mm * R.wstate_stride; };
    auto save_walker = [&]() __attribute__((always_inline)) {
        unsigned char *row = wrow(m);
        float *sx = reinterpret_cast<float *>(row), *sp = sx + DP, *so = sp + DP;
        uint32_t *se = reinterpret_cast<uint32_t *>(so + DP);
#pragma unroll
        for (int c = 0; c < L; ++c) {
            sx[a0 + c] = x[c];
            sp[a0 + c] = p[c];
            so[a0 + c] = xo[c];
        }
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            uint32_t *e = se + 4 * ((a0 >> 2) + i);
            e[0] = eps[i].s0; e[1] = eps[i].s1; e[2] = eps[i].s2; e[3] = eps[i].s3;
        }
        if (lead) {
            uint32_t *sr = se + DP;
            sr[0] = res.s0; sr[1] = res.s1; sr[2] = res.s2; sr[3] = res.s3;
            int32_t *si = reinterpret_cast<int32_t *>(sr + 4);
            si[0] = nref; si[1] = streak; si[2] = nprune; si[3] = outs; si[4] = steps;
            *reinterpret_cast<double *>(si + 6) = out_l;
            atomicMax(&acc->win_a, a_step);
            atomicMax(&acc->win_b, steps);
        }
    };
    auto acquire = [&](int mm) __attribute__((always_inline)) {
        if (cont) {
            const unsigned char *row = wrow(mm);
            const float *sx = reinterpret_cast<const float *>(row), *sp = sx + DP, *so = sp + DP;
            const uint32_t *se = reinterpret_cast<const uint32_t *>(so + DP);
            const uint32_t *sr = se + DP;
            const int32_t *si = reinterpret_cast<const int32_t *>(sr + 4);
            const int b = si[4];
            if (b < win_a) {
                s = at<int32_t>(arena, R.off_start)[mm];
#pragma unroll
                for (int c = 0; c < L; ++c) {
                    x[c] = sx[a0 + c];
                    p[c] = sp[a0 + c];
                    xo[c] = so[a0 + c];
                }
#pragma unroll
                for (int i = 0; i < NE; ++i) {
                    const uint32_t *e = se + 4 * ((a0 >> 2) + i);
                    eps[i].s0 = e[0]; eps[i].s1 = e[1]; eps[i].s2 = e[2]; eps[i].s3 = e[3];
                }
                res.s0 = sr[0]; res.s1 = sr[1]; res.s2 = sr[2]; res.s3 = sr[3];
                nref = si[0]; streak = si[1]; nprune = si[2]; outs = si[3]; steps = b;
                nsave = 0;
                out_l = *reinterpret_cast<const double *>(si + 6);
                return;
            }
            start_walker(mm);
            if (lead) atomicAdd(&blk_cnt[4], (unsigned long long)b);
            return;
        }
        start_walker(mm);
    };
    auto emit = [&]() __attribute__((always_inline)) {
        if (first) {
            save_walker();
            return;
        }
        float *wo = walk_x + (int64_t)m * d;
#pragma unroll
        for (int c = 0; c < L; ++c)
            if (VALID(c)) wo[a0 + c] = xo[c];
        if (lead) {
            walk_logl[m] = out_l;
            // the walker's counts go straight to the block's totals (LDS)
            atomicAdd(&blk_cnt[0], (unsigned long long)outs);
            atomicAdd(&blk_cnt[1], (unsigned long long)steps);
            atomicAdd(&blk_cnt[2], (unsigned long long)nprune);
            if (nsave == 0) atomicAdd(&blk_cnt[3], 1ull);
        }
    };
    // slots whose walker is done emit it and take the next walkers of the tile
    // in slot order, until each has a walker with steps to go (or none is
    // left); every lane of every wavefront sees the same masks
    auto retire = [&](bool need) __attribute__((always_inline)) {
        while (__any(need)) {
            if (need) emit();
            const uint32_t fin = (uint32_t)(__ballot(need) & 0xFFFFull);
            if (need) {
                m = next + __popc(fin & ((1u << slot) - 1u));
                active = m < tile.m_end;
                if (active) acquire(m);
            }
            next += __popc(fin);
            need = need && active && steps >= end_steps;
        }
    };

    if (active) acquire(m);
    retire(active && steps >= end_steps);
    __syncthreads();

    // slots can only end inside the rare-event branch, so whether any walker
    // is left is a uniform flag updated there (the same in every wavefront)
    bool any_left = __any(active);
    while (any_left) {
        const uint32_t ures = res.next();
        // drift; BF16 residuals of the lane's dimensions to LDS
        bool vany = false;
        {
            __bf16 rb[L];
#pragma unroll
            for (int c = 0; c < L; ++c) {
                x[c] = x[c] + dt * p[c];
                rb[c] = (__bf16)(x[c] - mu[c]);
                vany = vany | (x[c] < lo) | (x[c] > hi);
            }
            __bf16 *dst = rbuf + slot * RS + a0;
#pragma unroll
            for (int c = 0; c < L; c += 4)
                *reinterpret_cast<bf16x4 *>(dst + c) = bf16x4{rb[c], rb[c + 1], rb[c + 2], rb[c + 3]};
        }
        __syncthreads();
        // Y^T = P R^T for this wavefront's rows; B operands: K rows 8q..8q+7 of each K-block
        // (K-blocks outer: one B operand is live at a time; each M-block still
        // accumulates its K-blocks in order)
        {
            floatx4 c4[MBW];
#pragma unroll
            for (int mb = 0; mb < MBW; ++mb) c4[mb] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                const bf16x8 bop =
                    *reinterpret_cast<const bf16x8 *>(rbuf + slot * RS + 32 * kb + 8 * quarter);
#pragma unroll
                for (int mb = 0; mb < MBW; ++mb)
                    c4[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(amat[mb][kb], bop, c4[mb], 0, 0, 0);
            }
#pragma unroll
            for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
                for (int j = 0; j < 4; ++j) y[4 * mb + j] = c4[mb][j];
        }
        // r.y, p.g and g.g (g = -y) and the box test: lane sums, quarters, then wavefronts
        {
            float qv = 0.0f, pg = 0.0f, gg = 0.0f;
#pragma unroll
            for (int c = 0; c < L; ++c) {
                qv += (x[c] - mu[c]) * y[c];
                pg -= p[c] * y[c];
                gg += y[c] * y[c];
            }
            qv = sum4(qv);
            pg = sum4(pg);
            gg = sum4(gg);
            const bool vw = (__ballot(vany) & (0x0001000100010001ull << slot)) != 0ull;
            if (quarter == 0) part[wave * 16 + slot] = floatx4{qv, pg, gg, vw ? 1.0f : 0.0f};
        }
        // this step's noise: with one normal per walker, two words of block 0's
        // stream and the first normal of their pair (every lane alike), else
        // the four normals of each block (those of block 0 here, the others
        // where they are used)
        float zb0[4], nf0 = 1.0f;
        if constexpr (NZ) {
            const uint32_t w0 = eps[0].next(), w1 = eps[0].next();
            nf0 = 1.0f + dpn * normal_first(w0, w1, 0.0f);
        } else {
            const uint32_t w0 = eps[0].next(), w1 = eps[0].next(), w2 = eps[0].next(),
                           w3 = eps[0].next();
            normals2(w0, w1, zb0[0], zb0[1]);
            normals2(w2, w3, zb0[2], zb0[3]);
        }
        __syncthreads();
        floatx4 tot = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int w = 0; w < W; ++w) tot += part[w * 16 + slot];
        const float l = cst - 0.5f * tot[0];
        const float pg = tot[1], gg = tot[2];
        const bool viol = tot[3] > 0.0f;
        const bool out = viol || ((double)l <= lstar);
        if (trace_x != nullptr) {
            if (active && steps < R.trace_steps) {
                const int64_t row = (int64_t)steps * k + m;
#pragma unroll
                for (int c = 0; c < L; ++c)
                    if (VALID(c)) trace_x[row * d + a0 + c] = x[c];
                if (lead) {
                    R.trace_logl[row] = (double)l;
                    R.trace_out[row] = out ? 1 : 0;
                }
            }
        }
        steps += 1;
        const bool use_g = out && !viol && isfinite(gg) && gg > 0.0f;
        const bool flip_all = out && !viol && !use_g;
        const float f = use_g ? m_div(2.0f * pg, gg) : 0.0f;
        // box faces: a walker outside the box flips the momentum of each
        // violated dimension (rare; f is 0 and flip_all false for it)
        if (__builtin_expect(__any(vany), 0)) {
#pragma unroll
            for (int c = 0; c < L; ++c) p[c] = ((x[c] < lo) | (x[c] > hi)) ? -p[c] : p[c];
        }
#pragma unroll
        for (int i = 0; i < L / 4; ++i) {
            // this step's noise factors for the block of four dimensions 4i..4i+3
            float nf[4];
            if constexpr (NZ) {
                nf[0] = nf[1] = nf[2] = nf[3] = nf0;
            } else {
                float z[4];
                if (i == 0) {
                    z[0] = zb0[0]; z[1] = zb0[1]; z[2] = zb0[2]; z[3] = zb0[3];
                } else {
                    const uint32_t w0 = eps[i].next(), w1 = eps[i].next(), w2 = eps[i].next(),
                                   w3 = eps[i].next();
                    normals2(w0, w1, z[0], z[1]);
                    normals2(w2, w3, z[2], z[3]);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) nf[j] = 1.0f + dpn * z[j];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * i + j;
                const float pr = (flip_all ? -p[c] : p[c]) + f * y[c];   // p - f g with g = -y
                p[c] = pr * nf[j];
            }
        }
        nref += out ? 1 : 0;
        outs += out ? 1 : 0;
        streak = out ? streak + 1 : 0;
        a_step = (a_step == never && nref >= min_ref) ? steps : a_step;
        const bool keep = !out && nref >= keep_ref && steps >= keep_step;
        nsave += keep ? 1 : 0;
        const bool take = !out && (keep ? ((uint64_t)ures * (uint64_t)nsave < (1ull << 32))
                                        : (nsave == 0));
#pragma unroll
        for (int c = 0; c < L; ++c) xo[c] = take ? x[c] : xo[c];
        out_l = take ? (double)l : out_l;
        // rare events, one branch: a prune (back to the start with fresh
        // momentum), then the end of walkers (kept point to HBM, the slot takes
        // the next walker of the tile).  Slot states are the same in every lane
        // of a slot and every wavefront, so all wavefronts take the branch together
        const bool pruning = prune_streak > 0 && streak >= prune_streak;
        const bool ends = !(steps < end_steps && (end_ref == 0 || nref < end_ref));
        if (__builtin_expect(__any(active & (pruning | ends)), 0)) {
            if (active & pruning) {
                const float *xs = live_x + (int64_t)s * d;
#pragma unroll
                for (int c = 0; c < L; ++c) x[c] = VALID(c) ? xs[a0 + c] : xpad;
                nprune += 1;
                momentum_lane<L>(seed, (uint32_t)m, it, (uint32_t)nprune, a0, d, p);
                // the batch minimum never decreases: its count is kept
                nref = batch ? nref : 0;
                streak = 0;
            }
            retire(active && !(steps < end_steps && (end_ref == 0 || nref < end_ref)));
            any_left = __any(active);
        }
    }

#undef VALID
    __syncthreads();
    if (threadIdx.x == 0 && blk_cnt[4] > 0)
        atomicAdd(&acc->replayed, blk_cnt[4]);
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

template <int L, int W>
static hipError_t launch_mfma_t(void *arena, const RunDev *runs, const Tile *tiles, int n_tiles,
                                int nz, int phase, hipStream_t s) {
    if (nz)
        hipLaunchKernelGGL((walk_mfma_kernel<L, W, 1>), dim3(n_tiles), dim3(64 * W), 0, s, arena,
                           runs, tiles, phase);
    else
        hipLaunchKernelGGL((walk_mfma_kernel<L, W, 0>), dim3(n_tiles), dim3(64 * W), 0, s, arena,
                           runs, tiles, phase);
    return hipGetLastError();
}

bool mfma_shape_ok(int d_pad, int waves) {
    if (waves < 1 || d_pad % (16 * waves) != 0) return false;
    const int L = d_pad / (4 * waves);
    switch (d_pad) {
        case 32: return L == 8 || L == 4;
        case 64: case 128: return L == 16 || L == 8 || L == 4;
        case 256: return L == 16 || L == 8;
        case 96: case 160: case 192: case 224: return L == 8;
        default: return false;
    }
}

int launch_walk_mfma(void *arena, const RunDev *runs_dev, const Tile *tiles, int n_tiles, int d_pad,
                     int waves, int nz, int phase, hipStream_t s) {
    if (!mfma_shape_ok(d_pad, waves)) return GGNS_EUNSUPPORTED;
    const int L = d_pad / (4 * waves);
    hipError_t e = hipErrorInvalidValue;
#define GGNS_MFMA_CASE(LL, WW) \
    if (L == LL && waves == WW) e = launch_mfma_t<LL, WW>(arena, runs_dev, tiles, n_tiles, nz, phase, s);
    GGNS_MFMA_CASE(8, 1) GGNS_MFMA_CASE(4, 2)                          // dp 32
    GGNS_MFMA_CASE(16, 1) GGNS_MFMA_CASE(8, 2) GGNS_MFMA_CASE(4, 4)    // dp 64
    GGNS_MFMA_CASE(8, 3)                                               // dp 96
    GGNS_MFMA_CASE(16, 2) GGNS_MFMA_CASE(8, 4) GGNS_MFMA_CASE(4, 8)    // dp 128
    GGNS_MFMA_CASE(8, 5)                                               // dp 160
    GGNS_MFMA_CASE(8, 6)                                               // dp 192
    GGNS_MFMA_CASE(8, 7)                                               // dp 224
    GGNS_MFMA_CASE(16, 4) GGNS_MFMA_CASE(8, 8)                         // dp 256
#undef GGNS_MFMA_CASE
    return e == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

}  // namespace ggns
