"""Posterior samples of a finished run, and the mode report of a mixture.

The dead points of a nested-sampling run, with their importance weights
p_i = L_i w_i / Z (Appendix A), are weighted posterior samples.  For the
equal-weight Gaussian mixture the report follows the reading used for its
mode-recovery check: every weighted sample is assigned to the component of
largest responsibility; a mode counts as recovered when at least one sample
assigned to it lies within the 0.999 quantile of the chi-square distribution
with d degrees of freedom in that component's Mahalanobis distance; each
mode's posterior weight is reported next to the exact 1/K.

Host-side analysis of the engine's outputs (numpy); it is not part of the
sampler's path.
"""
from __future__ import annotations

import numpy as np
from scipy import stats

from .inputs import RunConfig


def normalized_log_weights(dead_logl, dead_logw, log_z: float) -> np.ndarray:
    """log p_i = log L_i + log w_i - log Z."""
    return np.asarray(dead_logl, np.float64) + np.asarray(dead_logw, np.float64) - log_z


def effective_sample_size(log_p) -> float:
    """Kish's effective number of samples of normalised log weights."""
    lp = np.asarray(log_p, np.float64)
    w = np.exp(lp - lp.max())
    return float(w.sum() ** 2 / (w * w).sum())


def equal_weight_samples(x, log_p, n: int | None = None, seed: int = 0) -> np.ndarray:
    """n equally weighted posterior samples from the weighted dead points, by
    systematic resampling (one uniform offset, n evenly spaced draws through
    the weight CDF), e.g. to train a downstream amortised sampler; n defaults
    to the effective sample size."""
    x = np.asarray(x)
    lp = np.asarray(log_p, np.float64)
    w = np.exp(lp - lp.max())
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    if n is None:
        n = max(1, int(round(effective_sample_size(lp))))
    u = (np.random.default_rng(seed).uniform() + np.arange(n)) / n
    idx = np.minimum(np.searchsorted(cdf, u, side="right"), len(cdf) - 1)
    return x[idx]


def engine_posterior(engine, r: int):
    """Dead-point positions of run r (kept with engine.keep_dead_x(r) before the
    run) and their normalised log weights, after the run has finished."""
    st = engine.stats()[r]
    dl, dw = engine.dead(r)
    lp = normalized_log_weights(dl.cpu().numpy(), dw.cpu().numpy(), st["log_z"])
    return engine.dead_x(r).cpu().numpy(), lp


def gmm_mode_report(x, log_p, cfg: RunConfig, weight_floor: float = 1e-12) -> dict:
    """Mode recovery of an equal-weight diagonal Gaussian mixture run.

    x: [N, d] dead-point positions; log_p: [N] normalised log weights.  Samples
    whose weight is below weight_floor times the largest are left out (they
    change no weight by more than N times that fraction)."""
    if cfg.kind != "gmm_diag":
        raise ValueError("mode report is defined for the Gaussian mixture")
    d, K = cfg.d, cfg.n_comp
    blocks = np.asarray(cfg.params, np.float64).reshape(K, 2, d)
    mu, sg = blocks[:, 0, :], blocks[:, 1, :]
    x = np.asarray(x, np.float64)
    lp = np.asarray(log_p, np.float64)
    keep = lp >= lp.max() + np.log(weight_floor)
    x, lp = x[keep], lp[keep]
    z2 = (((x[:, None, :] - mu[None]) / sg[None]) ** 2).sum(-1)        # [N, K]
    logresp = -0.5 * z2 - np.log(sg).sum(-1)[None]
    a = logresp.argmax(1)
    m2 = z2[np.arange(len(a)), a]
    thr = stats.chi2.ppf(0.999, d)
    w = np.exp(lp - lp.max())
    w /= w.sum()
    weights = np.array([w[a == k].sum() for k in range(K)])
    recovered = np.array([bool(np.any((a == k) & (m2 <= thr))) for k in range(K)])
    return {"modes": K, "recovered": int(recovered.sum()), "recovered_mask": recovered.tolist(),
            "weights": weights.tolist(), "weight_exact": 1.0 / K,
            "weight_max_abs_err": float(np.abs(weights - 1.0 / K).max()),
            "samples_used": int(keep.sum())}
