"""The walk with a likelihood written in torch (score by autograd): the same
walk as the plain FP64 walk with the library's own likelihood, and whole runs
that recover a closed-form evidence."""
import math

import numpy as np
import pytest

from paper_2312_03911_amd import exact, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _gauss_diag_fn(torch, cfg):
    d = cfg.d
    mu = torch.tensor(cfg.params[:d], dtype=torch.float64, device="cuda")
    sg = torch.tensor(cfg.params[d:2 * d], dtype=torch.float64, device="cuda")
    cst = float(np.sum(-0.5 * math.log(2 * math.pi) - np.log(cfg.params[d:2 * d])))

    def fn(x):
        return cst - 0.5 * (((x - mu) / sg) ** 2).sum(dim=1)
    return fn


def _torus_fn(torch, cfg):
    alpha, beta, c = (float(v) for v in cfg.params)
    idx = torch.arange(1, cfg.d + 1, device="cuda")
    even = (idx % 2 == 0)

    def fn(x):
        s = torch.where(even, torch.sin(alpha * x), torch.cos(beta * x)).sum(dim=1) + c
        return 3.0 * torch.log(s)
    return fn


def test_external_walk_matches_plain_walk(torch):
    """One iteration: the torch likelihood's walk reproduces the plain FP64
    walk with the library's likelihood (same starts, streams and decisions;
    positions and log L equal up to the likelihood's rounding)."""
    from paper_2312_03911_amd.engine import Engine
    from paper_2312_03911_amd.external import ExternalRuns
    cfg = inputs.RunConfig(kind="gauss_diag", d=6, n_live=300, lo=-4.0, hi=4.0, precision="fp64",
                           seed=77, n_steps_max=40, min_ref=1, max_ref=3,
                           params=inputs.gauss_diag_params(np.linspace(-1, 1, 6), np.linspace(0.4, 1.0, 6)))
    plain = Engine([cfg], device="cuda:0")
    ext = ExternalRuns([cfg], [_gauss_diag_fn(torch, cfg)], device="cuda:0")
    np.testing.assert_allclose(ext.eng.live_logl(0).cpu().numpy(), plain.live_logl(0).cpu().numpy(),
                               rtol=1e-13, atol=1e-13)
    for it in range(3):
        plain.evidence_update()
        plain.hss_walk_plain()
        ext.eng.evidence_update()
        ext.walk(0)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ext.eng.start(0).cpu().numpy(), plain.start(0).cpu().numpy())
        np.testing.assert_allclose(ext.eng.walk_x(0).cpu().numpy(), plain.walk_x(0).cpu().numpy(),
                                   rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(ext.eng.walk_logl(0).cpu().numpy(), plain.walk_logl(0).cpu().numpy(),
                                   rtol=1e-9, atol=1e-9)
        plain.replace_dead()
        ext.eng.replace_dead()
        sp, se = plain.stats()[0], ext.eng.stats()[0]
        assert sp["evals"] == se["evals"] and sp["iter"] == se["iter"] == it + 1
        assert abs(sp["dt"] - se["dt"]) < 1e-15
    plain.close()
    ext.close()


def test_external_torus_runs_match_closed_form(torch):
    """Six runs of the torus reward written in torch (d = 8, c = 9): the mean
    log Z lies within three standard errors of the closed form."""
    from paper_2312_03911_amd.external import ExternalRuns
    cfgs = inputs.replicate(inputs.config_torus(d=8, n_live=200, precision="fp64"), 6, base_seed=3100)
    runs = ExternalRuns(cfgs, [_torus_fn(torch, c) for c in cfgs], device="cuda:0")
    st = runs.run()
    truth = exact.log_z(cfgs[0])
    dz = np.array([s["log_z"] - truth for s in st])
    assert all(s["state"] == 1 for s in st)
    se = max(dz.std(ddof=1), np.mean([s["sigma_kl"] for s in st])) / math.sqrt(len(dz))
    assert abs(dz.mean()) < 3 * se, (dz.mean(), se)
    runs.close()


def test_external_walk_refuses_fp32(torch):
    from paper_2312_03911_amd.external import ExternalRuns
    with pytest.raises(ValueError):
        ExternalRuns([inputs.config_torus(d=4, n_live=50)], [lambda x: x.sum(1)])
