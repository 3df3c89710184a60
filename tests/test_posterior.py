"""Posterior post-processing on samples with known answers (host logic): the
mixture mode report and equal-weight resampling."""
import numpy as np

from paper_2312_03911_amd import inputs
from paper_2312_03911_amd.posterior import gmm_mode_report, normalized_log_weights


def _gmm(d=16, K=8):
    return inputs.config_gmm(d=d, n_live=100, n_comp=K, seed=1, param_seed=77)


def _draw(cfg, counts, rng):
    blocks = cfg.params.reshape(cfg.n_comp, 2, cfg.d)
    xs = [blocks[k, 0] + blocks[k, 1] * rng.standard_normal((c, cfg.d)) for k, c in enumerate(counts)]
    return np.concatenate(xs)


def test_all_modes_recovered_with_equal_weights():
    cfg = _gmm()
    rng = np.random.default_rng(0)
    x = _draw(cfg, [400] * 8, rng)
    r = gmm_mode_report(x, np.zeros(len(x)), cfg)
    assert r["recovered"] == 8
    assert r["weight_max_abs_err"] < 1e-12            # 400 equal-weight samples each


def test_missing_mode_and_unequal_weights():
    cfg = _gmm()
    rng = np.random.default_rng(1)
    counts = [300, 300, 300, 300, 300, 300, 300, 0]
    x = _draw(cfg, counts, rng)
    logp = np.zeros(len(x))
    logp[:300] = np.log(2.0)                          # component 0 twice as heavy
    r = gmm_mode_report(x, logp, cfg)
    assert r["recovered"] == 7 and not r["recovered_mask"][7]
    np.testing.assert_allclose(r["weights"][0], 2.0 / 8.0, rtol=1e-12)
    np.testing.assert_allclose(r["weights"][1], 1.0 / 8.0, rtol=1e-12)


def test_far_sample_does_not_count_as_recovery():
    cfg = _gmm()
    blocks = cfg.params.reshape(8, 2, cfg.d)
    # a single sample 12 sigma from component 3 along every axis
    x = (blocks[3, 0] + 12.0 * blocks[3, 1])[None]
    r = gmm_mode_report(x, np.zeros(1), cfg)
    assert r["recovered"] == 0


def test_normalized_log_weights():
    lw = normalized_log_weights([1.0, 2.0], [-3.0, -4.0], 0.5)
    np.testing.assert_allclose(lw, [-2.5, -2.5])


def test_equal_weight_resampling_follows_the_weights():
    """Systematic resampling: each point appears floor or ceil of n times its
    weight, and the effective sample size of equal weights is their count."""
    from paper_2312_03911_amd.posterior import effective_sample_size, equal_weight_samples
    rng = np.random.default_rng(3)
    w = rng.uniform(0.0, 1.0, 50)
    w /= w.sum()
    x = np.arange(50)
    n = 10000
    s = equal_weight_samples(x, np.log(w), n=n, seed=5)
    counts = np.bincount(s, minlength=50)
    assert np.all(np.abs(counts - n * w) <= 1.0 + 1e-9)
    assert abs(effective_sample_size(np.zeros(40)) - 40.0) < 1e-12
    assert len(equal_weight_samples(x, np.zeros(50))) == 50
