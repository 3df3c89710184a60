// Device building blocks of the engine: random streams, lane-group
// reductions and the log-likelihood + score of each family in the lane-group
// layout used by the walk (one walker per group of G lanes, C consecutive
// coordinates per lane: lane g of a group owns coordinates [g*C, g*C + C)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ggns_common.h"

namespace ggns {

// ---------------------------------------------------------------------------
// Random streams.
// ---------------------------------------------------------------------------

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// -> 64-bit products on words 0 and 2, cross-lane swap, key xor; the two key
// words advance by Weyl increments between rounds.
__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Counter layout: (c0 = block / aux, c1 = walker or point, c2 = iteration,
// c3 = tag << 24 | sub), key = the run's 64-bit seed.
__device__ __forceinline__ void draw4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                      uint32_t tag, uint32_t sub, uint32_t out[4]) {
    philox10(c0, c1, c2, (tag << 24) | (sub & 0xFFFFFFu), (uint32_t)seed, (uint32_t)(seed >> 32), out);
}

// xoshiro128++ (Blackman & Vigna 2018).
struct Xoshiro {
    uint32_t s0, s1, s2, s3;
    __device__ __forceinline__ void seed(const uint32_t w[4]) {
        s0 = w[0]; s1 = w[1]; s2 = w[2]; s3 = w[3];
        if ((s0 | s1 | s2 | s3) == 0u) s0 = 1u;
    }
    __device__ __forceinline__ uint32_t next() {
        const uint32_t sum = s0 + s3;
        const uint32_t out = ((sum << 7) | (sum >> 25)) + s0;
        const uint32_t t = s1 << 9;
        s2 ^= s0;
        s3 ^= s1;
        s1 ^= s2;
        s0 ^= s3;
        s2 ^= t;
        s3 = (s3 << 11) | (s3 >> 21);
        return out;
    }
};

// Box-Muller on 24-bit uniforms: (w0, w1) -> (z0, z1), (w2, w3) -> (z2, z3).
__device__ __forceinline__ void normals2(uint32_t a, uint32_t b, float &z0, float &z1) {
    const float u1 = ((float)(a >> 8) + 0.5f) * 0x1p-24f;
    const float u2 = (float)(b >> 8) * 0x1p-24f;
    // v_log_f32 is log2; v_sin_f32 / v_cos_f32 take revolutions.
    const float r = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u1));
    z0 = r * __builtin_amdgcn_cosf(u2);
    z1 = r * __builtin_amdgcn_sinf(u2);
}

__device__ __forceinline__ void normals2(uint32_t a, uint32_t b, double &z0, double &z1) {
    const double u1 = ((double)(a >> 8) + 0.5) * 0x1p-24;
    const double u2 = (double)(b >> 8) * 0x1p-24;
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// The first normal of the Box-Muller pair of (a, b), r cos(2 pi u2): the one
// noise normal per walker and step (the third argument only picks the type).
__device__ __forceinline__ float normal_first(uint32_t a, uint32_t b, float) {
    const float u1 = ((float)(a >> 8) + 0.5f) * 0x1p-24f;
    const float u2 = (float)(b >> 8) * 0x1p-24f;
    return __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u1)) *
           __builtin_amdgcn_cosf(u2);
}
__device__ __forceinline__ double normal_first(uint32_t a, uint32_t b, double) {
    const double u1 = ((double)(a >> 8) + 0.5) * 0x1p-24;
    const double u2 = (double)(b >> 8) * 0x1p-24;
    return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

// Uniform in (0,1) from the top 24 bits (prior draws), in double.
__device__ __forceinline__ double u24_open(uint32_t a) {
    return ((double)(a >> 8) + 0.5) * 0x1p-24;
}

// ---------------------------------------------------------------------------
// Lane-group reductions (group of G lanes, G a power of two <= 64, aligned).
// Offsets 1, 2, 4, 8 use DPP lane swizzles (quad permutes, half-row and row
// mirrors), offsets 16 and 32 the row swaps of gfx950 (v_permlane16_swap,
// v_permlane32_swap), so every level stays in the vector ALU.  The butterfly
// leaves the same, bitwise identical sum in every lane of the group (each
// step adds a pair in either order).
// ---------------------------------------------------------------------------

// Every pattern used here reads a lane inside the same row, so each lane gets
// its source's value; bound_ctrl marks the destination's old contents as unused.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, true);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// v + (v of lane l ^ 16) and v + (v of lane l ^ 32): swapping a register with
// itself leaves the row pair's first row in the first result and its second
// row in the second, in both rows of the pair (or both halves of the wave)
__device__ __forceinline__ float xor16_sum(float v) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xor32_sum(float v) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double xor16_sum(double v) {
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ double xor32_sum(double v) {
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}

constexpr int kDppQuad0 = 0x00;       // quad_perm [0,0,0,0]
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7-i within 8
constexpr int kDppMirror = 0x140;     // lane i <-> 15-i within 16

// Sum N values over the group at once (independent chains interleave).  Groups
// of 8 or more lanes take the three in-row levels every group needs without
// selects, the fourth in-row level and the two cross-row levels behind uniform
// branches; groups of 1, 2 or 4 lanes issue the two quad levels and keep or
// drop each by a select on the uniform group size.  The additions, and their
// order, are the same for every path.
template <typename T, int N>
__device__ __forceinline__ void group_sum_n(T (&v)[N], int G) {
    if (G >= 8) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_mov<kDppXor1>(v[i]);
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_mov<kDppXor2>(v[i]);
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_mov<kDppHalfMirror>(v[i]);
        if (G > 8) {
#pragma unroll
            for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_mov<kDppMirror>(v[i]);
            if (G > 16) {
#pragma unroll
                for (int i = 0; i < N; ++i) v[i] = xor16_sum(v[i]);
                if (G > 32) {
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i] = xor32_sum(v[i]);
                }
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const T a1 = v[i] + dpp_mov<kDppXor1>(v[i]);
            v[i] = (G > 1) ? a1 : v[i];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const T a2 = v[i] + dpp_mov<kDppXor2>(v[i]);
            v[i] = (G > 2) ? a2 : v[i];
        }
    }
}

__device__ __forceinline__ bool group_any(bool pred, int G) {
    const unsigned long long b = __ballot(pred);
    const int lane = threadIdx.x & 63;
    const unsigned long long m = (G >= 64) ? ~0ull : (((1ull << G) - 1ull) << (lane & ~(G - 1)));
    return (b & m) != 0ull;
}

// Scalar math per precision: hardware approximations in FP32 (v_exp, v_log,
// v_sqrt, v_rcp; about one ulp), correctly rounded library calls in FP64.
__device__ __forceinline__ float m_exp(float v) { return __expf(v); }
__device__ __forceinline__ double m_exp(double v) { return exp(v); }
// natural log on v_log_f32 without the denormal rescaling: every caller passes
// a log-sum-exp sum, which is at least one
__device__ __forceinline__ float m_log(float v) {
    return __builtin_amdgcn_logf(v) * 0.693147180559945309417f;
}
__device__ __forceinline__ double m_log(double v) { return log(v); }
__device__ __forceinline__ float m_sqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ double m_sqrt(double v) { return sqrt(v); }
__device__ __forceinline__ float m_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double m_div(double a, double b) { return a / b; }
__device__ __forceinline__ float m_rsqrt(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double m_rsqrt(double v) { return 1.0 / sqrt(v); }

// ---------------------------------------------------------------------------
// Log-likelihood, score and the two reflection dot products p.g and g.g, in the
// lane-group layout.
//
// Converted parameter blocks (run precision T), laid out over the padded
// dimension dp = G*C and, for mixtures, over KM component slots:
//   GAUSS_DIAG: mu[dp], iv[dp] = 1/sigma^2, cst = sum(-log(2 pi)/2 - log sigma)
//   GAUSS_FULL: mu[d], cst = -d log(2 pi)/2 + log det P / 2, P[d*d]   (unpadded)
//   SHELLS:     KM blocks {c[dp], r, iw2 = 1/w^2, lognorm = -log(2 pi w^2)/2}
//   GMM_DIAG:   KM blocks {mu[dp], iv[dp], lognorm = -log K + sum(-log(2 pi)/2 - log sigma)}
//   TORUS:      f[dp] (beta on even coordinates, alpha on odd ones), ph[dp] (pi/2 on even
//               coordinates, 0 on odd ones: cos y = sin(y + pi/2)), c
// Padding coordinates hold zeros (positions and momenta are zero there too) and
// padding components have lognorm = -inf, so both contribute exactly nothing
// and the arithmetic needs no per-coordinate or per-component branch.
// Every lane returns the same log L, p.g and g.g; g[] receives the score of the
// lane's own coordinates.  Where the score is a combination of per-component
// vectors, p.g and g.g are assembled from per-component dot products reduced in
// the same round as the likelihood sums, so each step needs a single reduction
// round (two for the mixture).
// ---------------------------------------------------------------------------

template <typename T>
struct LikOut {
    T l, pg, gg;
};

// Each lane keeps its own slice of the converted parameters in registers for
// the whole walk (they never change inside a launch); load() reads it from the
// staged block once.
template <typename T, int C>
struct DiagParams {
    T mu[C], iv[C], cst;
    __device__ __forceinline__ void load(const T *prm, int dp, int a0) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            mu[c] = prm[a0 + c];
            iv[c] = prm[dp + a0 + c];
        }
        cst = prm[2 * dp];
    }
};

template <typename T, int C, int KM>
struct ShellParams {
    T cen[KM][C], rad[KM], iw2[KM], lnrm[KM];
    __device__ __forceinline__ void load(const T *prm, int dp, int a0) {
        const int stride = dp + 3;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
#pragma unroll
            for (int c = 0; c < C; ++c) cen[k][c] = prm[k * stride + a0 + c];
            rad[k] = prm[k * stride + dp];
            iw2[k] = prm[k * stride + dp + 1];
            lnrm[k] = prm[k * stride + dp + 2];
        }
    }
};

// Mixture block: per component mu[dp], 1/sigma^2[dp], the log normaliser, padded
// to a multiple of four elements.
__host__ __device__ inline int gmm_stride(int dp) { return (2 * dp + 4) & ~3; }

template <typename T, int C, int KM>
struct GmmParams {
    T mu[KM][C], iv[KM][C], lnrm[KM];
    __device__ __forceinline__ void load(const T *prm, int dp, int a0) {
        const int stride = gmm_stride(dp);
#pragma unroll
        for (int k = 0; k < KM; ++k) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                mu[k][c] = prm[k * stride + a0 + c];
                iv[k][c] = prm[k * stride + dp + a0 + c];
            }
            lnrm[k] = prm[k * stride + 2 * dp];
        }
    }
    __device__ __forceinline__ void row(int k, T (&m)[C], T (&v)[C]) const {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            m[c] = mu[k][c];
            v[c] = iv[k][c];
        }
    }
};

template <typename T, int C>
__device__ __forceinline__ void load_row(const T *p, T (&out)[C]);

// The same block left where the walk staged it (LDS) and read at every
// evaluation: 2 KM C fewer registers per lane, for walk classes with more
// wavefronts than the chip has SIMDs, where occupancy decides the rate.
template <typename T, int C, int KM>
struct GmmParamsStaged {
    const T *lane;   // component 0's mu at this lane's first coordinate
    int stride, dp;
    T lnrm[KM];
    __device__ __forceinline__ void load(const T *prm, int dp_, int a0) {
        dp = dp_;
        stride = gmm_stride(dp_);
        lane = prm + a0;
#pragma unroll
        for (int k = 0; k < KM; ++k) lnrm[k] = prm[k * stride + 2 * dp_];
    }
    __device__ __forceinline__ void row(int k, T (&m)[C], T (&v)[C]) const {
        load_row<T, C>(lane + k * stride, m);
        load_row<T, C>(lane + k * stride + dp, v);
    }
};

// C consecutive values from p, with 16-byte loads where C allows (the mixture
// block's rows start on 16-byte boundaries for C a multiple of 4 in FP32 and
// of 2 in FP64: its stride is a multiple of four elements and a0, dp are
// multiples of C).
template <typename T, int C>
__device__ __forceinline__ void load_row(const T *p, T (&out)[C]) {
    if constexpr (sizeof(T) == 4 && C % 4 == 0) {
#pragma unroll
        for (int c = 0; c < C; c += 4) {
            const float4 v = *reinterpret_cast<const float4 *>(p + c);
            out[c] = v.x; out[c + 1] = v.y; out[c + 2] = v.z; out[c + 3] = v.w;
        }
    } else if constexpr (sizeof(T) == 8 && C % 2 == 0) {
#pragma unroll
        for (int c = 0; c < C; c += 2) {
            const double2 v = *reinterpret_cast<const double2 *>(p + c);
            out[c] = v.x; out[c + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) out[c] = p[c];
    }
}

template <typename T, int C>
struct TorusParams {
    T f[C], ph[C], c;
    __device__ __forceinline__ void load(const T *prm, int dp, int a0) {
#pragma unroll
        for (int j = 0; j < C; ++j) {
            f[j] = prm[a0 + j];
            ph[j] = prm[dp + a0 + j];
        }
        c = prm[2 * dp];
    }
};

// The correlated Gaussian keeps P where it was staged (LDS or global) and
// reads rows of it every step.
template <typename T>
struct FullParams {
    const T *prm;
    __device__ __forceinline__ void load(const T *p, int, int) { prm = p; }
};

template <typename T, int C>
__device__ __forceinline__ LikOut<T> lik_gauss_diag(const DiagParams<T, C> &P, int G,
                                                    const T (&x)[C], const T (&p)[C], T (&g)[C]) {
    T acc[3] = {T(0), T(0), T(0)};   // r.iv.r, p.g, g.g
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const T r = x[c] - P.mu[c];
        const T t = r * P.iv[c];
        acc[0] += r * t;
        acc[1] -= p[c] * t;
        acc[2] += t * t;
        g[c] = -t;
    }
    group_sum_n<T, 3>(acc, G);
    return {P.cst - T(0.5) * acc[0], acc[1], acc[2]};
}

// sin and cos of one argument: hardware v_sin / v_cos (they take revolutions)
// in FP32, the library in FP64.
__device__ __forceinline__ void m_sincos(float v, float &s, float &c) {
    const float r = v * 0.159154943091895335769f;
    s = __builtin_amdgcn_sinf(r);
    c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ void m_sincos(double v, double &s, double &c) { sincos(v, &s, &c); }

// Torus reward (Eq. torus): log L = 3 log(S + c), S = sum_a sin(f_a x_a + ph_a),
// score g_a = 3 f_a cos(f_a x_a + ph_a) / (S + c).  Padding coordinates have
// f = ph = 0 and add sin(0) = 0.  One reduction round: S, sum p_a f_a cos_a and
// sum (f_a cos_a)^2.
template <typename T, int C>
__device__ __forceinline__ LikOut<T> lik_torus(const TorusParams<T, C> &P, int G,
                                               const T (&x)[C], const T (&p)[C], T (&g)[C]) {
    T acc[3] = {T(0), T(0), T(0)};   // S, p.(f cos), |f cos|^2
    T fc[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
        T sn, cs;
        m_sincos(P.f[j] * x[j] + P.ph[j], sn, cs);
        fc[j] = P.f[j] * cs;
        acc[0] += sn;
        acc[1] += p[j] * fc[j];
        acc[2] += fc[j] * fc[j];
    }
    group_sum_n<T, 3>(acc, G);
    const T q = acc[0] + P.c;
    const T inv = m_div(T(3), q);
#pragma unroll
    for (int j = 0; j < C; ++j) g[j] = inv * fc[j];
    return {T(3) * m_log(q), inv * acc[1], inv * inv * acc[2]};
}

// Shells: with u_k = x - c_k, the score is g = sum_k coef_k u_k, so
// p.g = sum_k coef_k (p.u_k) and g.g = sum_kl coef_k coef_l (u_k.u_l).
template <typename T, int C, int KM>
__device__ __forceinline__ LikOut<T> lik_shells(const ShellParams<T, C, KM> &P, int G,
                                                const T (&x)[C], const T (&p)[C], T (&g)[C]) {
    constexpr int NB = KM * (KM - 1) / 2;
    T v[2 * KM + NB];   // |u_k|^2, p.u_k, u_k.u_l (k < l)
#pragma unroll
    for (int i = 0; i < 2 * KM + NB; ++i) v[i] = T(0);
    T u[KM][C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            u[k][c] = x[c] - P.cen[k][c];
            v[k] += u[k][c] * u[k][c];
            v[KM + k] += p[c] * u[k][c];
        }
        int q = 2 * KM;
#pragma unroll
        for (int k = 0; k < KM; ++k)
#pragma unroll
            for (int l = k + 1; l < KM; ++l) v[q++] += u[k][c] * u[l][c];
    }
    group_sum_n<T, 2 * KM + NB>(v, G);
    // rho_k = |u_k| and 1/rho_k from one reciprocal square root (0 at rho = 0,
    // where the component's score term vanishes); the responsibilities
    // exp(lp_k - l) are the log-sum-exp terms over their sum
    T lp[KM], rho[KM], rinv[KM], ek[KM], coef[KM];
    T lmax = T(-INFINITY);
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        rinv[k] = (v[k] > T(0)) ? m_rsqrt(v[k]) : T(0);
        rho[k] = v[k] * rinv[k];
        const T e = rho[k] - P.rad[k];
        lp[k] = P.lnrm[k] - T(0.5) * e * e * P.iw2[k];
        lmax = lp[k] > lmax ? lp[k] : lmax;
    }
    if constexpr (KM == 2) {
        // the larger component's term is exp(0) = 1: one exponential, of
        // -|lp0 - lp1| (= the smaller one's lp - lmax, exactly)
        const T dl = lp[0] - lp[1];
        const T e = m_exp(-fabs(dl));
        ek[0] = (dl >= T(0)) ? T(1) : e;
        ek[1] = (dl >= T(0)) ? e : T(1);
    } else {
#pragma unroll
        for (int k = 0; k < KM; ++k) ek[k] = m_exp(lp[k] - lmax);
    }
    // the terms are >= 0, so starting from the first equals adding it to zero
    T sum = ek[0];
#pragma unroll
    for (int k = 1; k < KM; ++k) sum += ek[k];
    const T l = lmax + m_log(sum);
    const T isum = m_div(T(1), sum);
#pragma unroll
    for (int k = 0; k < KM; ++k) coef[k] = -(ek[k] * isum) * (rho[k] - P.rad[k]) * P.iw2[k] * rinv[k];
    T pg = T(0), gg = T(0);
    int q = 2 * KM;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        pg += coef[k] * v[KM + k];
        gg += coef[k] * coef[k] * v[k];
#pragma unroll
        for (int l = k + 1; l < KM; ++l) gg += T(2) * coef[k] * coef[l] * v[q++];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        T s = T(0);
#pragma unroll
        for (int k = 0; k < KM; ++k) s += coef[k] * u[k][c];
        g[c] = s;
    }
    return {l, pg, gg};
}

template <typename T, int C, int KM, typename PT>
__device__ __forceinline__ LikOut<T> lik_gmm(const PT &P, int G, const T (&x)[C], const T (&p)[C],
                                             T (&g)[C]) {
    T q[KM];
    T u[KM][C];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        T mu[C], iv[C];
        P.row(k, mu, iv);
        q[k] = T(0);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const T r = x[c] - mu[c];
            u[k][c] = r * iv[c];
            q[k] += r * u[k][c];
        }
    }
    group_sum_n<T, KM>(q, G);
    T lmax = T(-INFINITY);
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        q[k] = P.lnrm[k] - T(0.5) * q[k];   // log of component k
        lmax = q[k] > lmax ? q[k] : lmax;
    }
    // the responsibilities exp(q_k - l) are the log-sum-exp terms over their sum
    T resp[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) resp[k] = m_exp(q[k] - lmax);
    T sum = resp[0];   // terms >= 0: the same as adding the first to zero
#pragma unroll
    for (int k = 1; k < KM; ++k) sum += resp[k];
    const T l = lmax + m_log(sum);
    const T isum = m_div(T(1), sum);
#pragma unroll
    for (int k = 0; k < KM; ++k) resp[k] *= isum;
    T acc[2] = {T(0), T(0)};
#pragma unroll
    for (int c = 0; c < C; ++c) {
        T s = T(0);
#pragma unroll
        for (int k = 0; k < KM; ++k) s -= resp[k] * u[k][c];
        g[c] = s;
        acc[0] += p[c] * s;
        acc[1] += s * s;
    }
    group_sum_n<T, 2>(acc, G);
    return {l, acc[0], acc[1]};
}

// Correlated Gaussian on the vector ALUs: r goes through the group's LDS slot
// xch[d] so that every lane can form its rows of P r.  With BF16 set, the
// product uses r rounded to BF16 (P was rounded when converted): the
// arithmetic of the matrix-core walk, for the prior draws and stand-alone
// evaluations of a BF16 run.
__device__ __forceinline__ float round_bf16(float v) { return (float)(__bf16)v; }

template <typename T, int C, bool BF16 = false>
__device__ __forceinline__ LikOut<T> lik_gauss_full(const T *prm, int d, int a0, int G,
                                                    const T (&x)[C], const T (&p)[C], T (&g)[C],
                                                    T *xch) {
    const T *mu = prm;
    const T cst = prm[d];
    const T *P = prm + d + 1;
    T r[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int a = a0 + c;
        r[c] = (a < d) ? x[c] - mu[a] : T(0);
        if constexpr (BF16) {
            if (a < d) xch[a] = round_bf16(r[c]);
        } else {
            if (a < d) xch[a] = r[c];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    T acc[3] = {T(0), T(0), T(0)};   // r.y, p.g, g.g with g = -y
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int a = a0 + c;
        T y = T(0);
        if (a < d) {
            const T *row = P + (int64_t)a * d;
            for (int j = 0; j < d; ++j) y += row[j] * xch[j];
        }
        acc[0] += r[c] * y;
        acc[1] -= p[c] * y;
        acc[2] += y * y;
        g[c] = -y;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    group_sum_n<T, 3>(acc, G);
    return {cst - T(0.5) * acc[0], acc[1], acc[2]};
}

// Kernel variants: the five families, with shells split by component count
// (two or fewer, else up to kMaxComp) so the fused reduction carries only the
// dot products it needs.
enum {
    VAR_GAUSS_DIAG = 0,
    VAR_GAUSS_FULL = 1,
    VAR_SHELLS2 = 2,
    VAR_GMM = 3,
    VAR_SHELLS8 = 4,
    VAR_GAUSS_FULL_BF16 = 5,
    VAR_TORUS = 6,
    // walk kernels only: the mixture with its block read from LDS every step
    // (chosen per walk class, never a run's own variant)
    VAR_GMM_STAGED = 7
};

__host__ __device__ inline int lik_variant(int kind, int K, int prec) {
    if (kind == GGNS_LIK_SHELLS) return K <= 2 ? VAR_SHELLS2 : VAR_SHELLS8;
    if (kind == GGNS_LIK_GAUSS_FULL && prec == GGNS_FP32_BF16MMA) return VAR_GAUSS_FULL_BF16;
    if (kind == GGNS_LIK_TORUS) return VAR_TORUS;
    return kind;
}

// Family chosen at compile time so that each kernel instance only carries the
// registers of its own likelihood.
template <typename T, int C, int VAR>
struct ParamsOf;
template <typename T, int C>
struct ParamsOf<T, C, VAR_GAUSS_DIAG> { using type = DiagParams<T, C>; };
template <typename T, int C>
struct ParamsOf<T, C, VAR_GAUSS_FULL> { using type = FullParams<T>; };
template <typename T, int C>
struct ParamsOf<T, C, VAR_GAUSS_FULL_BF16> { using type = FullParams<T>; };
template <typename T, int C>
struct ParamsOf<T, C, VAR_SHELLS2> { using type = ShellParams<T, C, 2>; };
template <typename T, int C>
struct ParamsOf<T, C, VAR_SHELLS8> { using type = ShellParams<T, C, kMaxComp>; };
template <typename T, int C>
struct ParamsOf<T, C, VAR_GMM> { using type = GmmParams<T, C, kMaxComp>; };
template <typename T, int C>
struct ParamsOf<T, C, VAR_TORUS> { using type = TorusParams<T, C>; };
template <typename T, int C>
struct ParamsOf<T, C, VAR_GMM_STAGED> { using type = GmmParamsStaged<T, C, kMaxComp>; };

template <typename T, int C, int VAR>
__device__ __forceinline__ LikOut<T> lik_step(const typename ParamsOf<T, C, VAR>::type &P, int d,
                                              int a0, int G, const T (&x)[C], const T (&p)[C],
                                              T (&g)[C], T *xch) {
    if constexpr (VAR == VAR_GAUSS_DIAG) return lik_gauss_diag<T, C>(P, G, x, p, g);
    else if constexpr (VAR == VAR_SHELLS2) return lik_shells<T, C, 2>(P, G, x, p, g);
    else if constexpr (VAR == VAR_SHELLS8) return lik_shells<T, C, kMaxComp>(P, G, x, p, g);
    else if constexpr (VAR == VAR_GMM || VAR == VAR_GMM_STAGED) return lik_gmm<T, C, kMaxComp>(P, G, x, p, g);
    else if constexpr (VAR == VAR_TORUS) return lik_torus<T, C>(P, G, x, p, g);
    else if constexpr (VAR == VAR_GAUSS_FULL_BF16)
        return lik_gauss_full<T, C, true>(P.prm, d, a0, G, x, p, g, xch);
    else return lik_gauss_full<T, C>(P.prm, d, a0, G, x, p, g, xch);
}

// Component slots of a variant's converted block.
__host__ __device__ inline int variant_slots(int var) {
    return var == VAR_SHELLS2 ? 2
                              : ((var == VAR_SHELLS8 || var == VAR_GMM || var == VAR_GMM_STAGED) ? kMaxComp : 1);
}

// Elements of the converted parameter block (run precision) for a variant.
__host__ __device__ inline int64_t converted_size(int var, int d, int dp) {
    switch (var) {
        case VAR_GAUSS_DIAG:
        case VAR_TORUS: return 2 * (int64_t)dp + 1;
        case VAR_GAUSS_FULL:
        case VAR_GAUSS_FULL_BF16: return (int64_t)d + 1 + (int64_t)d * d;
        case VAR_SHELLS2: return 2 * ((int64_t)dp + 3);
        case VAR_SHELLS8: return kMaxComp * ((int64_t)dp + 3);
        default: return kMaxComp * (int64_t)gmm_stride(dp);
    }
}

// ---------------------------------------------------------------------------
// Run-level helpers shared by the evidence and cluster kernels.
// ---------------------------------------------------------------------------

// Bitonic sort of 1024 E (key, slot) pairs by a workgroup of 1024 threads, E
// per thread (element i = E t + e of thread t), ascending by key and then slot.  Compare-exchange stages of
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
__device__ inline void sort_pairs(unsigned long long (&k)[E], int (&s)[E], unsigned long long *lk, int *ls) {
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

// Maximum over a workgroup of up to 1024 threads (barriers inside).
__device__ inline double block_max_d(double v, double *scratch) {
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

// Termination test at the head of an iteration (remaining evidence, or the
// X L peak), or max_iter: 0 to go on, else the run's final state.  The new
// running maximum of X L goes to *xl_max when it is not null.
__device__ inline int termination_decision(const RunDev &R, const Acc *acc, double lmax,
                                           int final_sweep, double *xl_max) {
    int stop = final_sweep ? GGNS_RUN_DONE : 0;
    const double ltol = log(R.term_tol);
    if (R.term_kind == GGNS_TERM_REMAINING_Z) {
        if (acc->log_x + lmax < ltol + acc->log_z) stop = GGNS_RUN_DONE;
    } else {
        const double r = acc->log_x + (R.term_kind == GGNS_TERM_XL_PEAK ? lmax : acc->lstar);
        const double xl = r > acc->log_xl_max ? r : acc->log_xl_max;
        if (xl_max) *xl_max = xl;
        if (acc->iter > 0 && r - xl < ltol) stop = GGNS_RUN_DONE;
    }
    if (!stop && acc->iter >= R.max_iter) stop = GGNS_RUN_MAXITER;
    return stop;
}

// A walker's start: without clusters a survivor picked by word 0; with
// clusters first the cluster, in proportion to its prior volume over the
// clusters with survivors (word 1 against the spawning CDF), then one of its
// survivors (word 0).  Writes the cluster to *cl.
__device__ inline int pick_start(const RunDev &R, void *arena, const uint32_t (&w)[4], int *cl) {
    const int32_t *surv = at<int32_t>(arena, R.off_surv);
    if (!R.cluster_mode) {
        *cl = 0;
        const int nsurv = R.n_live - R.n_kill;
        return surv[(int)(((uint64_t)w[0] * (uint64_t)nsurv) >> 32)];
    }
    const ClusterTab *tab = at<ClusterTab>(arena, R.off_cltab);
    const int nc = tab->n_clusters;
    double tot = 0.0;
    for (int p = 0; p < nc; ++p)
        if (tab->soff[p + 1] > tab->soff[p]) tot = tab->cum[p];
    const double target = ((double)w[1] + 0.5) * 0x1p-32 * tot;
    int pc = 0;
    for (int p = 0; p < nc; ++p) {
        if (tab->soff[p + 1] == tab->soff[p]) continue;
        pc = p;
        if (target < tab->cum[p]) break;
    }
    const int cnt = tab->soff[pc + 1] - tab->soff[pc];
    *cl = pc;
    return surv[tab->soff[pc] + (int)(((uint64_t)w[0] * (uint64_t)cnt) >> 32)];
}

// Instantiate a call for a run-time variant (KIND_ is the compile-time value).
#define GGNS_DISPATCH_KIND(var, CALL)                                    \
    switch (var) {                                                       \
        case VAR_GAUSS_DIAG: { constexpr int KIND_ = VAR_GAUSS_DIAG; CALL; break; } \
        case VAR_GAUSS_FULL: { constexpr int KIND_ = VAR_GAUSS_FULL; CALL; break; } \
        case VAR_SHELLS2: { constexpr int KIND_ = VAR_SHELLS2; CALL; break; }       \
        case VAR_SHELLS8: { constexpr int KIND_ = VAR_SHELLS8; CALL; break; }       \
        case VAR_GAUSS_FULL_BF16: { constexpr int KIND_ = VAR_GAUSS_FULL_BF16; CALL; break; } \
        case VAR_TORUS: { constexpr int KIND_ = VAR_TORUS; CALL; break; }           \
        default: { constexpr int KIND_ = VAR_GMM; CALL; break; }                    \
    }

}  // namespace ggns
