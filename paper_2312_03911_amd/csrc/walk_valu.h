// The batched Hamiltonian slice sampling walk on the vector ALUs.
//
// Paper: Algorithm GGNS HSS (drift x += p dt, log L and its gradient, outside
// mask, reflection p -= 2 (p.n) n with n the unit score (Eq. reflection),
// momentum noise p *= 1 + delta_p eps, reflection count, kept in-slice points,
// out_frac) and Section 3 (trajectory preservation, pruning, parallel
// evolution of the killed points).  Readings: the loop runs while the minimum
// of num_reflections over the run's walkers is below max_ref and points are
// saved once that minimum has reached min_ref (walk_mode 1; walk_mode 0: each
// walker stops and saves by its own count), or every walker runs n_steps_max
// steps (max_ref == 0); the prior box
// counts as outside and flips the violated momentum components; a zero or
// non-finite score reflects p -> -p; a walker keeps its in-slice points once it
// has min_ref reflections and returns a uniform pick through a size-one
// reservoir, else its last in-slice point, else its start; prune_streak outside
// steps in a row reset it to its start with fresh momentum.
//
// The batch-minimum loop is two launches.  The first (phase 1) walks each
// walker to its own max_ref-th reflection (or the cap), saving nothing, and
// leaves its state in the arena together with the run's window: win_b = the
// largest of those step counts (the step at which the minimum reaches
// max_ref) and win_a = the largest step at which a walker reached min_ref
// (the first step of the saving window).  The second (phase 2) continues each
// walker to win_b with the reservoir over its in-slice steps >= win_a; a
// walker whose first walk already reached win_a is walked again from its
// start (same streams, same steps), so that its steps inside the window are
// seen.  The walkers are independent given the window, so this is the
// lockstep loop of the algorithm step for step.
//
// Layout: one walker per group of G lanes (G = 1..64, power of two), lane g
// owning C consecutive coordinates [g*C, g*C + C) of x, p and the score in
// registers for the whole walk.  The run's converted parameters (zero-padded
// to G*C coordinates) are staged in LDS once per block.  A step is branch-free
// apart from the rare events (a reservoir write, a prune, the end of a walker):
// one fused xor-butterfly reduction round in DPP, selects for the reflection
// and the reservoir, and the noise generated first so that it overlaps the
// reduction latency.  The reservoir point lives in registers and is written
// once, when the walker ends: the only HBM traffic of a walk is the gather of
// its start point and that one row.
#pragma once

#include <type_traits>

#include "ggns_device.h"

#ifndef GGNS_WALK_WAVES
#define GGNS_WALK_WAVES 1
#endif

namespace ggns {

namespace {

__device__ __forceinline__ float pick4(const float (&z)[4], int i) {
    return i == 0 ? z[0] : (i == 1 ? z[1] : (i == 2 ? z[2] : z[3]));
}
__device__ __forceinline__ double pick4(const double (&z)[4], int i) {
    return i == 0 ? z[0] : (i == 1 ? z[1] : (i == 2 ? z[2] : z[3]));
}

// Four normals from four stream words.
template <typename T>
__device__ __forceinline__ void normals4(const uint32_t (&w)[4], T (&z)[4]) {
    normals2(w[0], w[1], z[0], z[1]);
    normals2(w[2], w[3], z[2], z[3]);
}

// Scatter the normals of this lane's stream blocks onto its C coordinates.
// With C a multiple of four every lane starts on a block boundary and the
// mapping is static; with C < 4 the lane takes words (a0 & 3) ... of its block.
template <typename T, int C>
__device__ __forceinline__ void take_block(const T (&z)[4], int i, int a0, T (&out)[C]) {
    if constexpr (C >= 4) {
#pragma unroll
        for (int j = 0; j < 4; ++j) out[4 * i + j] = z[j];
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) out[c] = pick4(z, (a0 & 3) + c);
    }
}

// d standard normals of walker `m` from the counter-based stream (initial and
// pruning momenta); this lane computes its own coordinates, zero on padding.
template <typename T, int C>
__device__ __forceinline__ void momentum_draw(uint64_t seed, uint32_t m, uint32_t it, uint32_t sub,
                                              int a0, int d, T (&p)[C]) {
    constexpr int NB = (C + 3) / 4;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        uint32_t w[4];
        draw4(seed, (uint32_t)((a0 >> 2) + i), m, it, TAG_P0, sub, w);
        T z[4];
        normals4(w, z);
        take_block<T, C>(z, i, a0, p);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) p[c] = (a0 + c < d) ? p[c] : T(0);
}

}  // namespace

// GF: the group size when fixed at compile time (4, 8, 16 or 32), else 0 (read from the run).
// A fixed size folds the group-size branches of the reductions and the
// broadcast away, so the step's common path has no branch taken.
template <typename T, int C, int VAR, int GF>
__global__ void __launch_bounds__(kWalkThreads, GGNS_WALK_WAVES)
walk_valu_kernel(void *arena, const RunDev *__restrict__ runs, const Tile *__restrict__ tiles,
                 int phase) {
    constexpr int NB = (C + 3) / 4;
    const Tile tile = tiles[blockIdx.x];
    const RunDev &R = runs[tile.run];
    Acc *acc = at<Acc>(arena, R.off_acc);
    if (acc->state != GGNS_RUN_ACTIVE) return;
    // phase 1: first walk of the batch-minimum loop (walk_mode 1 runs only);
    // phase 2: its continuation, or the whole per-walker walk (walk_mode 0)
    const bool batch = R.walk_mode == 1;
    if (phase == 1 && !batch) return;
    const bool first = phase == 1, cont = phase == 2 && batch;

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int next_walker;
    __shared__ unsigned long long blk_cnt[5];

    const int d = R.d, dp = R.dp, G = GF ? GF : R.G;
    const int ngroups = blockDim.x / G;
    const T *prm = at<T>(arena, R.off_prm);
    if (R.nprm_bytes_lds > 0) {
        T *sp = reinterpret_cast<T *>(smem);
        for (int i = threadIdx.x; i < R.nprm; i += blockDim.x) sp[i] = prm[i];
        prm = sp;
    }
    T *xch_all = reinterpret_cast<T *>(smem + ((R.nprm_bytes_lds + 15) & ~15));
    if (threadIdx.x == 0) {
        next_walker = tile.m_begin + ngroups;
        blk_cnt[0] = blk_cnt[1] = blk_cnt[2] = blk_cnt[3] = blk_cnt[4] = 0ull;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int grp = threadIdx.x / G;
    const int gbase = lane & ~(G - 1);
    const int a0 = gl * C;
    // the lanes of this lane's group, as a wavefront mask
    const unsigned long long gmask = (G >= 64) ? ~0ull : (((1ull << G) - 1ull) << gbase);
    T *xch = xch_all + grp * (G * C);
    bool valid[C];
#pragma unroll
    for (int c = 0; c < C; ++c) valid[c] = a0 + c < d;
    typename ParamsOf<T, C, VAR>::type P;
    if constexpr (VAR == VAR_GMM_STAGED)
        P.load(reinterpret_cast<const T *>(smem), dp, a0);   // always staged (checked on the host)
    else
        P.load(prm, dp, a0);

    const double lstar = acc->lstar;
    const T dt = (T)acc->dt;
    const uint32_t it = (uint32_t)acc->iter;
    const T lo = (T)R.lo, hi = (T)R.hi, dpn = (T)R.delta_p;
    // the prior box per coordinate; padding coordinates get an unbounded one,
    // so the outside test needs no validity mask
    T blo[C], bhi[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        blo[c] = valid[c] ? lo : T(-INFINITY);
        bhi[c] = valid[c] ? hi : T(INFINITY);
    }
    const uint64_t seed = R.seed;
    const int nsurv = R.n_live - R.n_kill;
    const int min_ref = R.min_ref, max_ref = R.max_ref, n_steps_max = R.n_steps_max;
    const int prune_streak = R.prune_streak;
    const int32_t *surv = at<int32_t>(arena, R.off_surv);
    int32_t *start_arr = at<int32_t>(arena, R.off_start);
    const T *live_x = at<T>(arena, R.off_live_x);
    const double *live_logl = at<double>(arena, R.off_live_logl);
    T *walk_x = at<T>(arena, R.off_walk_x);
    double *walk_logl = at<double>(arena, R.off_walk_logl);
    T *trace_x = reinterpret_cast<T *>(R.trace_x);
    const int k = R.n_kill;
    // stop and save rules of this launch: a point is kept when it is in-slice,
    // nref >= keep_ref and its step >= keep_step; a walker ends after end_steps
    // steps or at end_ref reflections (0: never)
    const int never = n_steps_max + 1;
    const int win_a = cont ? acc->win_a : 0, win_b = cont ? acc->win_b : 0;
    const int keep_ref = batch ? (first ? INT_MAX : 0) : min_ref;
    const int keep_step = cont ? win_a : 0;
    const int end_steps = cont ? win_b : n_steps_max;
    const int end_ref = cont ? 0 : max_ref;
    unsigned char *wst = batch ? at<unsigned char>(arena, R.off_wstate) : nullptr;

    const bool walker_noise = R.noise_mode != 0;
    T x[C], p[C], g[C], xo[C];
    Xoshiro eps[NB];
    Xoshiro res;
    int m = tile.m_begin + grp;
    bool active = m < tile.m_end;
    int s = 0, nref = 0, streak = 0, steps = 0, outs = 0, nprune = 0, nsave = 0, a_step = never;
    double out_l = 0.0;

    auto start_walker = [&](int mm) __attribute__((always_inline)) {
        uint32_t w[4];
        draw4(seed, 0u, (uint32_t)mm, it, TAG_START, 0u, w);
        int cl;
        s = pick_start(R, arena, w, &cl);
        if (gl == 0) {
            start_arr[mm] = s;
            if (R.cluster_mode) at<int32_t>(arena, R.off_start_cl)[mm] = cl;
        }
        const T *xs = live_x + (int64_t)s * d;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            x[c] = valid[c] ? xs[a0 + c] : T(0);
            xo[c] = x[c];
        }
        out_l = live_logl[s];
        momentum_draw<T, C>(seed, (uint32_t)mm, it, 0u, a0, d, p);
        // one normal per walker: every lane of the group carries block 0's
        // stream, so each computes the walker's normal itself
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            draw4(seed, walker_noise ? 0u : (uint32_t)((a0 >> 2) + i), (uint32_t)mm, it, TAG_EPS, 0u, w);
            eps[i].seed(w);
        }
        draw4(seed, 0u, (uint32_t)mm, it, TAG_RES, 0u, w);
        res.seed(w);
        nref = streak = steps = outs = nprune = nsave = 0;
        a_step = never;
    };

    // walker state between the two launches of the batch-minimum loop: x, p,
    // the fallback point (T), the noise stream states (one per block of four
    // coordinates), the reservoir stream, the counters and the fallback log L
    const int wdp = (int)((R.wstate_stride - 80) / (3 * (int64_t)sizeof(T) + 4));
    auto wrow = [&](int mm) __attribute__((always_inline)) { return wst + (int64_t)mm * R.wstate_stride; };
    auto save_walker = [&]() __attribute__((always_inline)) {
        unsigned char *row = wrow(m);
        T *sx = reinterpret_cast<T *>(row), *sp = sx + wdp, *so = sp + wdp;
        uint32_t *se = reinterpret_cast<uint32_t *>(so + wdp);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            sx[a0 + c] = x[c];
            sp[a0 + c] = p[c];
            so[a0 + c] = xo[c];
        }
        if ((a0 & 3) == 0) {
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                uint32_t *e = se + 4 * ((a0 >> 2) + i);
                e[0] = eps[i].s0; e[1] = eps[i].s1; e[2] = eps[i].s2; e[3] = eps[i].s3;
            }
        }
        if (gl == 0) {
            uint32_t *sr = se + wdp;
            sr[0] = res.s0; sr[1] = res.s1; sr[2] = res.s2; sr[3] = res.s3;
            int32_t *si = reinterpret_cast<int32_t *>(sr + 4);
            si[0] = nref; si[1] = streak; si[2] = nprune; si[3] = outs; si[4] = steps;
            *reinterpret_cast<double *>(si + 6) = out_l;
            atomicMax(&acc->win_a, a_step);
            atomicMax(&acc->win_b, steps);
        }
    };
    // the continuation takes a walker up where its first walk left it, unless
    // that walk reached the saving window: then it walks again from its start
    auto acquire = [&](int mm) __attribute__((always_inline)) {
        if (cont) {
            const unsigned char *row = wrow(mm);
            const T *sx = reinterpret_cast<const T *>(row), *sp = sx + wdp, *so = sp + wdp;
            const uint32_t *se = reinterpret_cast<const uint32_t *>(so + wdp);
            const uint32_t *sr = se + wdp;
            const int32_t *si = reinterpret_cast<const int32_t *>(sr + 4);
            const int b = si[4];
            if (b < win_a) {
                s = at<int32_t>(arena, R.off_start)[mm];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    x[c] = sx[a0 + c];
                    p[c] = sp[a0 + c];
                    xo[c] = so[a0 + c];
                }
#pragma unroll
                for (int i = 0; i < NB; ++i) {
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
            if (gl == 0) atomicAdd(&blk_cnt[4], (unsigned long long)b);
            return;
        }
        start_walker(mm);
    };
    // a walker ends: its state (first walk), or its kept point and counts
    auto emit = [&]() __attribute__((always_inline)) {
        if (first) {
            save_walker();
            return;
        }
        T *wo = walk_x + (int64_t)m * d;
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (valid[c]) wo[a0 + c] = xo[c];
        if (gl == 0) {
            walk_logl[m] = out_l;
            // the walker's counts go straight to the block's totals (LDS),
            // so no per-lane counter rides through the step loop
            atomicAdd(&blk_cnt[0], (unsigned long long)outs);
            atomicAdd(&blk_cnt[1], (unsigned long long)steps);
            atomicAdd(&blk_cnt[2], (unsigned long long)nprune);
            if (nsave == 0) atomicAdd(&blk_cnt[3], 1ull);
        }
    };
    // the group's walker is done (groups enter whole): emit it and take the
    // next walkers of the tile until one has steps to go
    auto retire = [&]() __attribute__((always_inline)) {
        bool need = true;
        while (need) {
            emit();
            int nm = 0;
            if (gl == 0) nm = atomicAdd(&next_walker, 1);
            m = __shfl(nm, gbase, 64);
            active = m < tile.m_end;
            if (active) acquire(m);
            need = active && steps >= end_steps;
        }
    };

    if (active) {
        acquire(m);
        if (steps >= end_steps) retire();
    }

    // the wavefront's walkers can only end inside the rare-event branch, so
    // whether any is left is a uniform flag updated there, not a vote per step
    bool any_left = __any(active);
    while (any_left) {
        // this step's noise and reservoir draw do not depend on the step, so
        // they are generated first and overlap the reduction latency; nf is
        // the noise factor 1 + delta_p eps of each coordinate
        T nf[C];
        if (walker_noise) {
            // one normal per walker and step: two words of block 0's stream,
            // the first normal of their Box-Muller pair (every lane alike)
            const uint32_t w0 = eps[0].next(), w1 = eps[0].next();
            const T f = T(1) + dpn * normal_first(w0, w1, T(0));
#pragma unroll
            for (int c = 0; c < C; ++c) nf[c] = f;
        } else {
            T eps_c[C];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                uint32_t w[4];
                w[0] = eps[i].next();
                w[1] = eps[i].next();
                w[2] = eps[i].next();
                w[3] = eps[i].next();
                if constexpr (C >= 4) {
                    T z[4];
                    normals4(w, z);
                    take_block<T, C>(z, i, a0, eps_c);
                } else {
                    // a lane owning one or two coordinates of the block transforms
                    // only the Box-Muller pair they come from
                    const bool upper = (a0 & 2) != 0;
                    T z0, z1;
                    normals2(upper ? w[2] : w[0], upper ? w[3] : w[1], z0, z1);
                    if constexpr (C == 2) {
                        eps_c[0] = z0;
                        eps_c[1] = z1;
                    } else {
                        eps_c[0] = (a0 & 1) ? z1 : z0;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) nf[c] = T(1) + dpn * eps_c[c];
        }
        const uint32_t ures = res.next();
        // drift (Algorithm GGNS HSS: x += p dt)
#pragma unroll
        for (int c = 0; c < C; ++c) x[c] = x[c] + dt * p[c];
        // log L, the score at the new position and the reflection dot products
        const LikOut<T> lk = lik_step<T, C, VAR>(P, d, a0, G, x, p, g, xch);
        // outside the slice: out of the prior box, or log L <= L* (compared in
        // FP64); the box test as one wavefront mask of lanes with a coordinate
        // outside, masked to the group
        unsigned long long bm = 0ull;
#pragma unroll
        for (int c = 0; c < C; ++c) bm |= __ballot(x[c] < blo[c]) | __ballot(x[c] > bhi[c]);
        const bool viol = (bm & gmask) != 0ull;
        const bool out = viol || ((double)lk.l <= lstar);
        if (__builtin_expect(trace_x != nullptr, 0)) {
            if (active && steps < R.trace_steps) {
                const int64_t row = (int64_t)steps * k + m;
#pragma unroll
                for (int c = 0; c < C; ++c)
                    if (valid[c]) trace_x[row * d + a0 + c] = x[c];
                if (gl == 0) {
                    R.trace_logl[row] = (double)lk.l;
                    R.trace_out[row] = out ? 1 : 0;
                }
            }
        }
        steps += 1;
        // reflection (Eq. reflection with n = g / |g|; box faces flip their
        // axis; a zero or non-finite score flips the whole momentum), as selects
        const bool use_g = out && !viol && isfinite(lk.gg) && lk.gg > T(0);
        const bool flip_all = out && !viol && !use_g;
        const T f = use_g ? m_div(T(2) * lk.pg, lk.gg) : T(0);
        // box faces: a walker outside the box flips the momentum of each
        // violated axis (rare; f is 0 and flip_all false for such a walker)
        if (__builtin_expect(bm != 0ull, 0)) {
#pragma unroll
            for (int c = 0; c < C; ++c) p[c] = ((x[c] < blo[c]) | (x[c] > bhi[c])) ? -p[c] : p[c];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const T pr = (flip_all ? -p[c] : p[c]) - f * g[c];
            // momentum noise: p *= 1 + delta_p * eps
            p[c] = pr * nf[c];
        }
        nref += out ? 1 : 0;
        outs += out ? 1 : 0;
        streak = out ? streak + 1 : 0;
        a_step = (a_step == never && nref >= min_ref) ? steps : a_step;
        // trajectory preservation: size-one reservoir over the kept points
        const bool keep = !out && nref >= keep_ref && steps >= keep_step;
        nsave += keep ? 1 : 0;
        // the reservoir's test u * nsave < 2^32 is a zero high word of the product;
        // bitwise on purpose: the decision costs no branch
        const bool hit = __umulhi(ures, (uint32_t)nsave) == 0u;
        const bool take = !out & (keep ? hit : (nsave == 0));
#pragma unroll
        for (int c = 0; c < C; ++c) xo[c] = take ? x[c] : xo[c];
        out_l = take ? (double)lk.l : out_l;
        // rare events, one branch: a prune (back to the start with fresh
        // momentum), then the end of the walker (its kept point to HBM, the
        // group takes the next walker of the tile); streak, nref and steps are
        // the same on every lane of a group, so groups enter whole
        const bool pruning = prune_streak > 0 && streak >= prune_streak;
        const bool ends = !(steps < end_steps && (end_ref == 0 || nref < end_ref));
        const bool rare = active & (pruning | ends);
        if (__builtin_expect(__any(rare), 0)) {
          if (rare) {
            if (pruning) {
                const T *xs = live_x + (int64_t)s * d;
#pragma unroll
                for (int c = 0; c < C; ++c) x[c] = valid[c] ? xs[a0 + c] : T(0);
                nprune += 1;
                momentum_draw<T, C>(seed, (uint32_t)m, it, (uint32_t)nprune, a0, d, p);
                // the batch minimum never decreases: its count is kept
                nref = batch ? nref : 0;
                streak = 0;
            }
            if (!(steps < end_steps && (end_ref == 0 || nref < end_ref))) retire();
          }
          any_left = __any(active);
        }
    }

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

// FP32 classes whose runs all have groups of 4, 8, 16 or 32 lanes take the
// kernel with the group size fixed; every other class reads it from the run.
template <typename T, int C, int VAR>
static void launch_gf(int gf, int n_tiles, size_t lds, hipStream_t s, void *arena,
                      const RunDev *runs, const Tile *tiles, int phase) {
    const dim3 grid(n_tiles), block(kWalkThreads);
    if constexpr (std::is_same<T, float>::value) {
        if (gf == 4)
            hipLaunchKernelGGL((walk_valu_kernel<T, C, VAR, 4>), grid, block, lds, s, arena, runs, tiles, phase);
        else if (gf == 8)
            hipLaunchKernelGGL((walk_valu_kernel<T, C, VAR, 8>), grid, block, lds, s, arena, runs, tiles, phase);
        else if (gf == 16)
            hipLaunchKernelGGL((walk_valu_kernel<T, C, VAR, 16>), grid, block, lds, s, arena, runs, tiles, phase);
        else if (gf == 32)
            hipLaunchKernelGGL((walk_valu_kernel<T, C, VAR, 32>), grid, block, lds, s, arena, runs, tiles, phase);
        else
            hipLaunchKernelGGL((walk_valu_kernel<T, C, VAR, 0>), grid, block, lds, s, arena, runs, tiles, phase);
    } else {
        hipLaunchKernelGGL((walk_valu_kernel<T, C, VAR, 0>), grid, block, lds, s, arena, runs, tiles, phase);
    }
}

template <typename T, int C>
inline hipError_t launch_walk_t(void *arena, const RunDev *runs, const Tile *tiles, int n_tiles,
                                int var, int gf, size_t lds, int phase, hipStream_t s) {
    if (var == VAR_GMM_STAGED)
        launch_gf<T, C, VAR_GMM_STAGED>(gf, n_tiles, lds, s, arena, runs, tiles, phase);
    else
        GGNS_DISPATCH_KIND(var, (launch_gf<T, C, KIND_>(gf, n_tiles, lds, s, arena, runs, tiles, phase)));
    return hipGetLastError();
}

}  // namespace ggns
