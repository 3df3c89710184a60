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

// Uniform in (0,1) from the top 24 bits (prior draws), in double.
__device__ __forceinline__ double u24_open(uint32_t a) {
    return ((double)(a >> 8) + 0.5) * 0x1p-24;
}

// ---------------------------------------------------------------------------
// Lane-group reductions (group of G lanes, G a power of two <= 64, aligned).
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ bool group_any(bool pred, int G) {
    const unsigned long long b = __ballot(pred);
    const int lane = threadIdx.x & 63;
    const unsigned long long m = (G >= 64) ? ~0ull : (((1ull << G) - 1ull) << (lane & ~(G - 1)));
    return (b & m) != 0ull;
}

template <typename T>
__device__ __forceinline__ T fast_exp(T v) { return exp(v); }
template <>
__device__ __forceinline__ float fast_exp<float>(float v) { return __expf(v); }
template <typename T>
__device__ __forceinline__ T fast_log(T v) { return log(v); }
template <>
__device__ __forceinline__ float fast_log<float>(float v) { return __logf(v); }

// ---------------------------------------------------------------------------
// Log-likelihood and score in the lane-group layout.
//
// Converted parameter blocks (run precision T):
//   GAUSS_DIAG: mu[d], iv[d] = 1/sigma^2, cst = sum(-log(2 pi)/2 - log sigma)
//   GAUSS_FULL: mu[d], cst = -d log(2 pi)/2 + log det P / 2, P[d*d]
//   SHELLS:     K blocks {c[d], r, iw2 = 1/w^2, lognorm = -log(2 pi w^2)/2}
//   GMM_DIAG:   K blocks {mu[d], iv[d], lognorm = -log K + sum(-log(2 pi)/2 - log sigma)}
// Every lane returns the same log L (xor-butterfly sums are bitwise identical
// across the group); g[] receives the score of the lane's own coordinates
// (zero on padding coordinates a >= d).
// ---------------------------------------------------------------------------

template <typename T, int C>
__device__ __forceinline__ T lik_gauss_diag(const T *prm, int d, int a0, int G, const T (&x)[C],
                                            T (&g)[C]) {
    const T *mu = prm, *iv = prm + d;
    T q = T(0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int a = a0 + c;
        if (a < d) {
            const T r = x[c] - mu[a];
            const T t = r * iv[a];
            q += r * t;
            g[c] = -t;
        } else {
            g[c] = T(0);
        }
    }
    q = group_sum(q, G);
    return prm[2 * d] - T(0.5) * q;
}

template <typename T, int C>
__device__ __forceinline__ T lik_shells(const T *prm, int d, int K, int a0, int G, const T (&x)[C],
                                        T (&g)[C]) {
    const int stride = d + 3;
    T s[kMaxComp];
#pragma unroll
    for (int k = 0; k < kMaxComp; ++k) {
        s[k] = T(0);
        if (k < K) {
            const T *ck = prm + k * stride;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int a = a0 + c;
                if (a < d) {
                    const T dd = x[c] - ck[a];
                    s[k] += dd * dd;
                }
            }
            s[k] = group_sum(s[k], G);
        }
    }
    T lp[kMaxComp], rho[kMaxComp];
    T lmax = T(-INFINITY);
#pragma unroll
    for (int k = 0; k < kMaxComp; ++k) {
        if (k < K) {
            const T *ck = prm + k * stride;
            rho[k] = sqrt(s[k]);
            const T e = rho[k] - ck[d];
            lp[k] = ck[d + 2] - T(0.5) * e * e * ck[d + 1];
            lmax = lp[k] > lmax ? lp[k] : lmax;
        }
    }
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < kMaxComp; ++k)
        if (k < K) acc += exp(lp[k] - lmax);
    const T l = lmax + log(acc);
#pragma unroll
    for (int c = 0; c < C; ++c) g[c] = T(0);
#pragma unroll
    for (int k = 0; k < kMaxComp; ++k) {
        if (k < K) {
            const T *ck = prm + k * stride;
            const T coef = (rho[k] > T(0))
                               ? -exp(lp[k] - l) * (rho[k] - ck[d]) * ck[d + 1] / rho[k]
                               : T(0);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int a = a0 + c;
                if (a < d) g[c] += coef * (x[c] - ck[a]);
            }
        }
    }
    return l;
}

template <typename T, int C>
__device__ __forceinline__ T lik_gmm(const T *prm, int d, int K, int a0, int G, const T (&x)[C],
                                     T (&g)[C]) {
    const int stride = 2 * d + 1;
    T q[kMaxComp];
#pragma unroll
    for (int k = 0; k < kMaxComp; ++k) {
        q[k] = T(0);
        if (k < K) {
            const T *mu = prm + k * stride, *iv = mu + d;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int a = a0 + c;
                if (a < d) {
                    const T r = x[c] - mu[a];
                    q[k] += r * r * iv[a];
                }
            }
            q[k] = group_sum(q[k], G);
        }
    }
    T lmax = T(-INFINITY);
#pragma unroll
    for (int k = 0; k < kMaxComp; ++k) {
        if (k < K) {
            q[k] = prm[k * stride + 2 * d] - T(0.5) * q[k];   // now lp_k
            lmax = q[k] > lmax ? q[k] : lmax;
        }
    }
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < kMaxComp; ++k)
        if (k < K) acc += exp(q[k] - lmax);
    const T l = lmax + log(acc);
#pragma unroll
    for (int c = 0; c < C; ++c) g[c] = T(0);
#pragma unroll
    for (int k = 0; k < kMaxComp; ++k) {
        if (k < K) {
            const T *mu = prm + k * stride, *iv = mu + d;
            const T resp = exp(q[k] - l);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int a = a0 + c;
                if (a < d) g[c] -= resp * (x[c] - mu[a]) * iv[a];
            }
        }
    }
    return l;
}

// Correlated Gaussian on the vector ALUs: r goes through the group's LDS slot
// xch[d] so that every lane can form its rows of P r.
template <typename T, int C>
__device__ __forceinline__ T lik_gauss_full(const T *prm, int d, int a0, int G, const T (&x)[C],
                                            T (&g)[C], T *xch) {
    const T *mu = prm;
    const T cst = prm[d];
    const T *P = prm + d + 1;
    T r[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int a = a0 + c;
        r[c] = (a < d) ? x[c] - mu[a] : T(0);
        if (a < d) xch[a] = r[c];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    T q = T(0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int a = a0 + c;
        T y = T(0);
        if (a < d) {
            const T *row = P + (int64_t)a * d;
            for (int j = 0; j < d; ++j) y += row[j] * xch[j];
        }
        q += r[c] * y;
        g[c] = -y;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    q = group_sum(q, G);
    return cst - T(0.5) * q;
}

// Family chosen at compile time so that each kernel instance only carries the
// registers of its own likelihood.
template <typename T, int C, int KIND>
__device__ __forceinline__ T lik_eval(int K, const T *prm, int d, int a0, int G, const T (&x)[C],
                                      T (&g)[C], T *xch) {
    if constexpr (KIND == GGNS_LIK_GAUSS_DIAG) return lik_gauss_diag<T, C>(prm, d, a0, G, x, g);
    else if constexpr (KIND == GGNS_LIK_SHELLS) return lik_shells<T, C>(prm, d, K, a0, G, x, g);
    else if constexpr (KIND == GGNS_LIK_GMM_DIAG) return lik_gmm<T, C>(prm, d, K, a0, G, x, g);
    else return lik_gauss_full<T, C>(prm, d, a0, G, x, g, xch);
}

// Instantiate F<KIND>() for a run-time family.
#define GGNS_DISPATCH_KIND(kind, CALL)                                   \
    switch (kind) {                                                      \
        case GGNS_LIK_GAUSS_DIAG: { constexpr int KIND_ = 0; CALL; break; } \
        case GGNS_LIK_GAUSS_FULL: { constexpr int KIND_ = 1; CALL; break; } \
        case GGNS_LIK_SHELLS: { constexpr int KIND_ = 2; CALL; break; }     \
        default: { constexpr int KIND_ = 3; CALL; break; }                  \
    }

}  // namespace ggns
