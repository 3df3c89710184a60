"""The plain FP64 per-step walk (the speed baseline) computes the same method
on the same random streams as the fused walk and the oracle."""
import numpy as np
import pytest

from paper_2312_03911_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _engine(cfgs):
    from paper_2312_03911_amd.engine import Engine
    return Engine(cfgs)


def test_plain_full_run_matches_oracle(torch, orc):
    for seed in (2100, 2103):
        cfg = inputs.config_gauss2d(seed=seed)
        eng = _engine([cfg])
        st = eng.run(poll_every=4, plain=True)[0]
        o = orc.Oracle(cfg).run()
        assert st["state"] == o.st.state == 1
        assert st["iter"] == o.st.iter and st["evals"] == o.st.evals
        assert abs(st["log_z"] - o.st.lz) < 1e-9
        assert abs(st["sigma_mom"] - o.st.sigma_mom) < 1e-7
        eng.close()


CASES = [
    ("shells6", lambda: inputs.config_shells(d=6, n_live=400, seed=81, precision="fp64")),
    ("gmm9", lambda: inputs.config_gmm(d=9, n_live=300, n_comp=5, seed=82, param_seed=21,
                                       precision="fp64")),
    ("diag13", lambda: inputs.RunConfig(
        kind="gauss_diag", d=13, n_live=300, lo=-4.0, hi=4.0, seed=83, precision="fp64",
        params=inputs.gauss_diag_params(np.linspace(-1, 1, 13), np.linspace(0.4, 1.0, 13)))),
    ("corr10", lambda: inputs.config_corr_gauss(d=10, n_live=200, seed=84, param_seed=22,
                                                precision="fp64", n_steps_max=50)),
    ("shells6_wnoise", lambda: inputs.config_shells(d=6, n_live=400, seed=86, precision="fp64",
                                                    noise="walker")),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_plain_iterations_match_fused_fp64(torch, name, make):
    cfg = make()
    a, b = _engine([cfg]), _engine([cfg])
    for _ in range(4):
        a.iterate(1)
        b.iterate(1, plain=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(a.start(0).cpu().numpy(), b.start(0).cpu().numpy())
        xa, xb = a.walk_x(0).cpu().numpy(), b.walk_x(0).cpu().numpy()
        la, lb = a.walk_logl(0).cpu().numpy(), b.walk_logl(0).cpu().numpy()
        scale = max(abs(cfg.lo), abs(cfg.hi))
        # the two sum in different orders; reflections amplify the last-bit
        # differences a little, and a decision within rounding of L* or a box
        # face may differ for a rare walker
        bad = (np.abs(xa - xb).max(axis=1) > 1e-8 * scale) | \
              (np.abs(la - lb) > 1e-8 * np.maximum(1.0, np.abs(la)))
        assert bad.sum() <= max(2, 0.01 * cfg.n_kill), bad.sum()
    sa, sb = a.stats()[0], b.stats()[0]
    assert sa["iter"] == sb["iter"] == 4
    assert abs(sa["dt"] - sb["dt"]) < 1e-12 * sa["dt"]
    assert abs(sa["log_z"] - sb["log_z"]) < 1e-8 * max(1.0, abs(sa["log_z"]))


def test_plain_rejects_non_fp64_runs(torch):
    from paper_2312_03911_amd._lib import GGNSError
    eng = _engine([inputs.config_shells(d=8, n_live=100, seed=85)])
    with pytest.raises(GGNSError):
        eng.hss_walk_plain()
