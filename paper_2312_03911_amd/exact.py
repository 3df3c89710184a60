"""Closed-form evidences of the synthetic workloads (the exact quantity nested
sampling estimates, Eq. (evidence): Z = integral of L(theta) pi(theta)).

The prior is uniform on the box [lo, hi]^d, so Z = (integral of L over the box)
/ (hi - lo)^d.  These are mathematics about the inputs, not a step of the
sampler; they pin end-to-end results of both the GPU engine and the oracle.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special

from .inputs import RunConfig


def _log_box_mass_1d(mu, sigma, lo, hi):
    """log of P(lo < N(mu, sigma^2) < hi), elementwise, accurate in the tails."""
    a = (lo - mu) / sigma
    b = (hi - mu) / sigma
    # Phi(b) - Phi(a) = Phi(-a) - Phi(-b); use the side with the smaller tail.
    la = special.log_ndtr(b)
    lb = special.log_ndtr(a)
    out = la + np.log1p(-np.exp(np.minimum(lb - la, 0.0)))
    return out


def log_z_gauss_diag(mu, sigma, lo, hi):
    d = len(mu)
    return float(np.sum(_log_box_mass_1d(np.asarray(mu), np.asarray(sigma), lo, hi))
                 - d * math.log(hi - lo))


def log_z_gmm_diag(params, d, n_comp, lo, hi):
    terms = []
    for k in range(n_comp):
        blk = params[k * 2 * d:(k + 1) * 2 * d]
        terms.append(np.sum(_log_box_mass_1d(blk[:d], blk[d:], lo, hi)))
    return float(special.logsumexp(terms) - math.log(n_comp) - d * math.log(hi - lo))


def log_radial_integral(d, radius, width):
    """log of integral_0^inf phi(rho) rho^(d-1) drho, with
    phi(rho) = (2 pi w^2)^(-1/2) exp(-(rho - r)^2 / (2 w^2))."""
    def logf(rho):
        return (-0.5 * math.log(2 * math.pi * width * width)
                - 0.5 * (rho - radius) ** 2 / (width * width) + (d - 1) * math.log(rho))
    # mode of the integrand
    peak = 0.5 * (radius + math.sqrt(radius * radius + 4 * (d - 1) * width * width))
    lmax = logf(peak)
    lo = max(peak - 40 * width, 1e-12)
    hi = peak + 40 * width
    val, _ = integrate.quad(lambda r: math.exp(logf(r) - lmax), lo, hi,
                            epsabs=0.0, epsrel=1e-13, limit=400, points=[peak])
    return lmax + math.log(val)


def log_z_shells(d, n_comp, radius, width, lo, hi):
    """Sum of n_comp identical shells; the box truncation is neglected (the shells
    reach at most |x_0| = 3.5 + peak radius, below 6 up to d=64 and 6.007 at
    d=128, where the truncated mass is far below double precision)."""
    log_sphere = math.log(2.0) + 0.5 * d * math.log(math.pi) - special.gammaln(0.5 * d)
    return (math.log(n_comp) + log_sphere + log_radial_integral(d, radius, width)
            - d * math.log(hi - lo))


def log_z_gauss_full(d, logdet_p, lo, hi):
    """Normalised correlated Gaussian; the mass outside the box is neglected (the
    workloads keep every marginal sigma <= 1 at >= 9 sigma from the faces)."""
    del logdet_p
    return -d * math.log(hi - lo)


def log_z_torus(d, alpha, beta, c, lo, hi):
    """The torus reward over the uniform prior on [0, 2 pi)^d: the recursion of
    Appendix F, Z_d = 2 pi Z_{d-1} + 3 pi c (2 pi)^(d-1), Z_1 = 2 pi c^3 + 3 pi c,
    divided by the prior volume (2 pi)^d, is c^3 + 3 d c / 2.  It holds for
    nonzero integer frequencies (then every sine and cosine and the odd
    moments integrate to zero over whole periods)."""
    if not (alpha == int(alpha) and beta == int(beta) and alpha != 0 and beta != 0):
        raise ValueError("the torus normalisation needs nonzero integer alpha and beta")
    if abs(lo) > 1e-12 or abs(hi - 2 * math.pi) > 1e-12:
        raise ValueError("the torus normalisation is over [0, 2 pi)^d")
    return math.log(c ** 3 + 1.5 * d * c)


def log_z(cfg: RunConfig) -> float:
    d, p = cfg.d, cfg.params
    if cfg.kind == "gauss_diag":
        return log_z_gauss_diag(p[:d], p[d:2 * d], cfg.lo, cfg.hi)
    if cfg.kind == "gmm_diag":
        return log_z_gmm_diag(p, d, cfg.n_comp, cfg.lo, cfg.hi)
    if cfg.kind == "shells":
        return log_z_shells(d, cfg.n_comp, float(p[d]), float(p[d + 1]), cfg.lo, cfg.hi)
    if cfg.kind == "gauss_full":
        return log_z_gauss_full(d, float(p[d + d * d]), cfg.lo, cfg.hi)
    if cfg.kind == "torus":
        return log_z_torus(d, float(p[0]), float(p[1]), float(p[2]), cfg.lo, cfg.hi)
    raise ValueError(cfg.kind)
