"""The likelihoods' torch.autograd binding: the backward pass is the adjoint
kernel.  FP64 runs pass torch.autograd.gradcheck (central finite differences
of the GPU forward pass); every precision's backward matches gout times the
oracle's analytic score."""
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


FP64 = [
    ("gauss2d", lambda: inputs.config_gauss2d(seed=71)),
    ("shells6", lambda: inputs.config_shells(d=6, n_live=64, seed=72, precision="fp64")),
    ("gmm5", lambda: inputs.config_gmm(d=5, n_live=64, n_comp=3, seed=73, param_seed=11,
                                       precision="fp64")),
    ("corr7", lambda: inputs.config_corr_gauss(d=7, n_live=64, seed=74, param_seed=12,
                                               precision="fp64")),
]


@pytest.mark.parametrize("name,make", FP64, ids=[c[0] for c in FP64])
def test_gradcheck_fp64(torch, name, make):
    from paper_2312_03911_amd.autograd import loglike
    cfg = make()
    eng = _engine([cfg])
    # points in the bulk of each likelihood, where log L is smooth and O(1)
    X = inputs.uniform_points(6, cfg.d, 0.1 * cfg.lo, 0.1 * cfg.hi, seed=3)
    if cfg.kind == "gauss_diag":
        X = 0.5 + 0.05 * inputs.uniform_points(6, cfg.d, -1.0, 1.0, seed=3)
    if cfg.kind == "shells":
        X[:, 0] += 3.5
        X[:, 1] += 2.0
    x = torch.tensor(X, dtype=torch.float64, device=eng.device, requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: loglike(eng, 0, t), (x,), eps=1e-6, atol=1e-6,
                                    rtol=1e-5)
    eng.close()


MIXED = [
    ("shells32_fp32", lambda: inputs.config_shells(d=32, n_live=100, seed=75)),
    ("gmm16_fp32", lambda: inputs.config_gmm(d=16, n_live=100, n_comp=8, seed=76, param_seed=13)),
    ("corr64_bf16", lambda: inputs.config_corr_gauss(d=64, n_live=128, seed=77, param_seed=14,
                                                     precision="bf16mma")),
]


@pytest.mark.parametrize("name,make", MIXED, ids=[c[0] for c in MIXED])
def test_backward_is_gout_times_oracle_score(torch, orc, name, make):
    from paper_2312_03911_amd.autograd import loglike
    cfg = make()
    eng = _engine([cfg])
    X = inputs.uniform_points(129, cfg.d, 0.3 * cfg.lo, 0.3 * cfg.hi, seed=4)
    x = torch.tensor(X, dtype=eng._fdtype(0), device=eng.device, requires_grad=True)
    l = loglike(eng, 0, x)
    w = torch.linspace(-1.0, 2.0, X.shape[0], dtype=torch.float64, device=eng.device)
    (l * w).sum().backward()
    Xr = x.detach().cpu().numpy().astype(np.float64)
    lo_, go_ = orc.loglike(cfg, Xr, bf16=cfg.precision == "bf16mma")
    want = go_ * w.cpu().numpy()[:, None]
    scale = np.maximum(np.abs(want).max(axis=1, keepdims=True), 1.0)
    tol = 5e-3 if cfg.precision == "bf16mma" else 2e-4
    got = x.grad.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - want) <= tol * scale)
    rel = np.abs(l.detach().cpu().numpy() - lo_) / np.maximum(1.0, np.abs(lo_))
    assert rel.max() < (1e-4 if cfg.precision == "bf16mma" else 1e-5)
    eng.close()
