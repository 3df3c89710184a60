"""Pins for the oracle's likelihoods and gradients: scipy densities (an
independent implementation of the same normalised densities), central finite
differences for the score, and the BF16 operand rounding."""
import math

import numpy as np
import pytest
from scipy import special, stats

from paper_2312_03911_amd import inputs


def _cfgs():
    rng = np.random.default_rng(11)
    d = 6
    yield inputs.RunConfig(kind="gauss_diag", d=d, n_live=10,
                           params=inputs.gauss_diag_params(rng.uniform(-1, 1, d), rng.uniform(0.3, 1.5, d)),
                           lo=-5, hi=5)
    prm, _ = inputs.correlated_gaussian_params(d, rng)
    yield inputs.RunConfig(kind="gauss_full", d=d, n_live=10, params=prm, lo=-5, hi=5)
    yield inputs.config_shells(d=d, n_live=10)
    yield inputs.config_gmm(d=d, n_live=10, n_comp=3, param_seed=5)


def _scipy_logl(cfg, x):
    d, p = cfg.d, cfg.params
    if cfg.kind == "gauss_diag":
        return stats.norm.logpdf(x, p[:d], p[d:2 * d]).sum(axis=-1)
    if cfg.kind == "gauss_full":
        prec = p[d:d + d * d].reshape(d, d)
        return stats.multivariate_normal(p[:d], np.linalg.inv(prec)).logpdf(x)
    if cfg.kind == "shells":
        terms = []
        for k in range(cfg.n_comp):
            blk = p[k * (d + 2):(k + 1) * (d + 2)]
            rho = np.linalg.norm(x - blk[:d], axis=-1)
            terms.append(stats.norm.logpdf(rho, blk[d], blk[d + 1]))
        return special.logsumexp(terms, axis=0)
    if cfg.kind == "gmm_diag":
        terms = []
        for k in range(cfg.n_comp):
            blk = p[k * 2 * d:(k + 1) * 2 * d]
            terms.append(stats.norm.logpdf(x, blk[:d], blk[d:]).sum(axis=-1) - math.log(cfg.n_comp))
        return special.logsumexp(terms, axis=0)
    raise ValueError


@pytest.mark.parametrize("cfg", list(_cfgs()), ids=lambda c: c.kind)
def test_loglike_matches_scipy(orc, cfg):
    x = inputs.uniform_points(50, cfg.d, -2.5, 2.5, seed=4)
    if cfg.kind == "shells":
        x[:, 0] += 3.0
    l, _ = orc.loglike(cfg, x)
    np.testing.assert_allclose(l, _scipy_logl(cfg, x), rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("cfg", list(_cfgs()), ids=lambda c: c.kind)
def test_gradient_matches_finite_differences(orc, cfg):
    x = inputs.uniform_points(20, cfg.d, -2.0, 2.0, seed=5)
    if cfg.kind == "shells":
        x[:, 0] += 3.0
    _, g = orc.loglike(cfg, x)
    h = 1e-6 * (cfg.hi - cfg.lo)
    fd = np.zeros_like(x)
    for a in range(cfg.d):
        e = np.zeros(cfg.d); e[a] = h
        lp, _ = orc.loglike(cfg, x + e)
        lm, _ = orc.loglike(cfg, x - e)
        fd[:, a] = (lp - lm) / (2 * h)
    err = np.abs(g - fd).max() / max(np.abs(fd).max(), 1e-12)
    assert err < 1e-6


def test_shell_gradient_is_radial(orc):
    cfg = inputs.config_shells(d=4, n_live=10)
    x = np.array([[3.5 + 1.0, 1.0, 0.0, 0.0]])   # only the +3.5 shell matters
    _, g = orc.loglike(cfg, x)
    r = x[0] - np.array([3.5, 0, 0, 0])
    cos = g[0] @ r / (np.linalg.norm(g[0]) * np.linalg.norm(r))
    assert abs(abs(cos) - 1.0) < 1e-9
    # inside the radius (rho < r) the score points outward
    assert g[0] @ r > 0


def test_bf16_rounding(orc):
    vals = np.random.default_rng(0).standard_normal(2000) * 10.0 ** np.random.default_rng(1).integers(-3, 4, 2000)
    for v in vals:
        r = orc.round_bf16(v)
        # at most 8 significant bits, error at most half an ulp (2^-8 relative)
        m, _ = math.frexp(r)
        assert (m * 2 ** 8) == int(m * 2 ** 8)
        assert abs(r - v) <= 2.0 ** -8 * abs(v) * (1 + 1e-6) + 1e-300
    # ties go to the even mantissa
    assert orc.round_bf16(1.0 + 2.0 ** -8) == 1.0
    assert orc.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_bf16_emulated_quadratic_form_close(orc):
    cfg = inputs.config_corr_gauss(d=64, n_live=10, param_seed=3, precision="bf16mma")
    x = inputs.uniform_points(20, 64, -1.5, 1.5, seed=9)
    l64, g64 = orc.loglike(cfg, x, bf16=False)
    l16, g16 = orc.loglike(cfg, x, bf16=True)
    q = -2 * (l64 - (-0.5 * 64 * math.log(2 * math.pi) + 0.5 * cfg.params[-1]))
    # operand rounding: relative error of the quadratic form ~ 2^-8 sqrt-averaged
    assert np.all(np.abs(l16 - l64) < 0.05 * np.abs(q))
    assert np.any(l16 != l64)
