"""Pins for the torus reward (Eq. torus, Appendix F): its normalisation, the
oracle's reward and score, and a whole oracle run against the closed form.

The closed form c^3 + 3 d c / 2 (the recursion of Appendix F over the uniform
prior on [0, 2 pi)^d) is pinned by quadrature of the one-dimensional base case
and by the trapezoid rule on a full periodic grid, which integrates a
trigonometric polynomial of degree below the grid size exactly; the grid
values come from the oracle's reward, so the same check pins the oracle."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2312_03911_amd import exact, inputs


@pytest.mark.parametrize("freq,c", [(1, 1.5), (2, 2.0), (3, 5.0)])
def test_base_case_by_quadrature(freq, c):
    """Z_1 = 2 pi c^3 + 3 pi c for sin and for cos (Appendix F, the base case)."""
    for f in (lambda x: (math.sin(freq * x) + c) ** 3, lambda x: (math.cos(freq * x) + c) ** 3):
        val, _ = integrate.quad(f, 0.0, 2 * math.pi, epsabs=0.0, epsrel=1e-13, limit=200)
        assert abs(val - (2 * math.pi * c ** 3 + 3 * math.pi * c)) < 1e-10 * val


@pytest.mark.parametrize("d,alpha,beta,m", [(1, 2, 3, 64), (2, 2, 3, 32), (3, 1, 2, 24), (4, 3, 1, 16)])
def test_grid_normalisation_matches_closed_form(orc, d, alpha, beta, m):
    """Mean of the oracle's reward over an m^d periodic grid (exact for the
    reward's trigonometric degree 3 max(alpha, beta) < m) equals the closed form."""
    cfg = inputs.config_torus(d=d, n_live=10, alpha=alpha, beta=beta)
    g = 2 * math.pi * np.arange(m) / m
    X = np.stack(np.meshgrid(*([g] * d), indexing="ij"), axis=-1).reshape(-1, d)
    logl, _ = orc.loglike(cfg, X)
    mean = float(np.mean(np.exp(logl)))
    assert abs(math.log(mean) - exact.log_z(cfg)) < 1e-12


def test_closed_form_needs_integer_frequencies():
    cfg = inputs.config_torus(d=3, n_live=10, alpha=2, beta=3)
    with pytest.raises(ValueError):
        exact.log_z(cfg.replace(params=inputs.torus_params(1.5, 3, 4.0)))
    # for a non-integer frequency the mean over the box differs from the formula
    c = 4.0
    val, _ = integrate.quad(lambda x: (math.sin(1.5 * x) + c) ** 3, 0.0, 2 * math.pi)
    assert abs(val / (2 * math.pi) - (c ** 3 + 1.5 * c)) > 1e-3


def test_index_convention_and_score(orc):
    """Odd 1-based coordinates carry cos(beta x), even ones sin(alpha x): at x = 0
    the sum is the number of odd indices; at x_j = pi/(2 alpha) on the even
    ones (sin = 1) and x = pi/(2 beta) on the odd ones (cos = 0) it is d/2.  The
    score matches central differences."""
    d, alpha, beta = 7, 2, 3
    cfg = inputs.config_torus(d=d, n_live=10, alpha=alpha, beta=beta)
    c = float(cfg.params[2])
    l0, _ = orc.loglike(cfg, np.zeros((1, d)))
    assert abs(l0[0] - 3 * math.log((d + 1) // 2 + c)) < 1e-12
    x = np.array([[math.pi / (2 * beta) if (i % 2) else math.pi / (2 * alpha) for i in range(1, d + 1)]])
    l1, _ = orc.loglike(cfg, x)
    assert abs(l1[0] - 3 * math.log(d // 2 + c)) < 1e-12
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 2 * math.pi, size=(5, d))
    _, g = orc.loglike(cfg, X)
    h = 1e-6
    for a in range(d):
        e = np.zeros(d)
        e[a] = h
        lp, _ = orc.loglike(cfg, X + e)
        lm, _ = orc.loglike(cfg, X - e)
        np.testing.assert_allclose(g[:, a], (lp - lm) / (2 * h), rtol=1e-6, atol=1e-8)


def test_invalid_offset_stops_the_run(orc):
    """c <= d would let the reward reach zero or below: the run does not start."""
    cfg = inputs.config_torus(d=4, n_live=20, c=4.0)
    o = orc.Oracle(cfg).init()
    assert o.st.state == 3


def test_oracle_run_matches_closed_form(orc):
    """The full method on the torus (d = 8, c = 9): the mean log Z of six runs
    lies within three standard errors (and 3 sigma_KL / sqrt(6)) of the closed form."""
    truth = exact.log_z(inputs.config_torus(d=8))
    zs, sk = [], []
    for r in range(6):
        o = orc.Oracle(inputs.config_torus(d=8, n_live=200, seed=2700 + r, precision="fp64")).run()
        assert o.st.state == 1
        zs.append(o.st.lz)
        sk.append(o.st.sigma_kl)
    zs = np.array(zs)
    tol = max(3 * zs.std(ddof=1) / math.sqrt(len(zs)), 3 * np.mean(sk) / math.sqrt(len(zs)))
    assert abs(zs.mean() - truth) < tol, (zs.mean() - truth, tol)
