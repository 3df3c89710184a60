"""GPU engine vs the FP64 oracle on identical seeded inputs, through the C ABI.

Tolerances: FP64 runs 1e-10 relative (per-step positions), FP32 runs 1e-4
relative to max(|x|, prior width), as stated for short walks.  Where floating
point decides a branch (outside / inside, a box face), a walker is compared only
up to the first step the oracle finds within tau of that decision (log L: tau
relative to max(1, |L*|) with tau 1e-9 in FP64 and 1e-4 in FP32; faces: 0.1 tau
times the prior width); the masked share must stay small.  Per-step log L is
compared with the oracle's log L at the GPU's own positions, which separates
the likelihood arithmetic from the (bounded) drift of FP32 trajectories."""
import math

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


def _engine(cfgs, tile_c=None):
    from paper_2312_03911_amd.engine import Engine
    return Engine(cfgs, tile_c=tile_c)


def _np(t):
    return t.detach().cpu().numpy()


def _load_state(torch, eng, o, r, X):
    """Same live set on both sides: the positions the GPU holds (rounded to the
    run's precision) and the log L the GPU computed for them.  The kill order
    is an integer decision taken from these values, so both sides take it on
    the same ones (an FP32 log L and the oracle's FP64 value of the same point
    can order two points differently); the likelihood itself is compared on
    its own, per step of the walk and in test_loglike_and_adjoint_match_oracle."""
    cfg = eng.cfgs[r]
    xd = torch.from_numpy(X).to(eng.device, eng._fdtype(r))
    eng.live_x(r).copy_(xd)
    l, _ = eng.loglike(r, eng.live_x(r).clone(), grad=False)
    eng.live_logl(r).copy_(l)
    Xo = _np(xd).astype(np.float64)          # the rounded positions the GPU holds
    o.set_state(live_x=Xo, live_logl=_np(l).astype(np.float64), log_z=-math.inf, log_x=0.0,
                dt=cfg.dt_init * (cfg.hi - cfg.lo), iteration=0)
    torch.cuda.synchronize()
    return Xo


CASES = [
    ("gauss2d_fp64", lambda: inputs.config_gauss2d(seed=11), 1e-10, 1e-9),
    ("shells32_fp32", lambda: inputs.config_shells(d=32, n_live=1000, seed=12), 1e-4, 1e-4),
    ("shells32_fp64", lambda: inputs.config_shells(d=32, n_live=1000, seed=12, precision="fp64"),
     1e-10, 1e-9),
    ("gmm16_fp32", lambda: inputs.config_gmm(d=16, n_live=600, n_comp=8, seed=13, param_seed=5),
     1e-4, 1e-4),
    ("gauss_diag24_fp32", lambda: inputs.RunConfig(
        kind="gauss_diag", d=24, n_live=400, lo=-5.0, hi=5.0, seed=14, n_steps_max=60,
        params=inputs.gauss_diag_params(np.linspace(-1, 1, 24), np.linspace(0.3, 1.2, 24))),
     1e-4, 1e-4),
    ("corr12_fp32", lambda: inputs.config_corr_gauss(d=12, n_live=300, seed=15, param_seed=7,
                                                     precision="fp32", n_steps_max=60), 1e-4, 1e-4),
    ("shells5_fp64", lambda: inputs.config_shells(d=5, n_live=200, seed=16, precision="fp64"),
     1e-10, 1e-9),
    # BF16 matrix-core walk: compared with the oracle's BF16-operand emulation
    ("corr40_bf16", lambda: inputs.config_corr_gauss(d=40, n_live=300, seed=17, param_seed=8,
                                                     precision="bf16mma", n_steps_max=60), 1e-4, 1e-4),
    ("corr128_bf16", lambda: inputs.config_corr_gauss(d=128, n_live=256, seed=18, param_seed=9,
                                                      precision="bf16mma"), 1e-4, 1e-4),
    # the largest shapes of the vector-ALU walk: 256 coordinates over 64 lanes
    # (both cross-row butterfly levels) and 4096 live points
    ("gauss_diag256_fp64", lambda: inputs.RunConfig(
        kind="gauss_diag", d=256, n_live=300, lo=-6.0, hi=6.0, seed=25, n_steps_max=40,
        precision="fp64", params=inputs.gauss_diag_params(np.linspace(-1, 1, 256), np.linspace(0.5, 1.5, 256))),
     1e-10, 1e-9),
    # (log L ~ -1e6 here: the masking band is tau |L*|, so tau is set where the
    # FP32 error of such a sum, ~1e-6 relative, still sits well inside it)
    ("gmm256_fp32", lambda: inputs.config_gmm(d=256, n_live=200, n_comp=3, seed=26, param_seed=11,
                                              n_steps_max=40), 1e-4, 1e-5),
    ("gauss_diag8_n4096_fp32", lambda: inputs.RunConfig(
        kind="gauss_diag", d=8, n_live=4096, lo=-4.0, hi=4.0, seed=27, n_steps_max=30,
        params=inputs.gauss_diag_params(np.zeros(8), np.full(8, 0.7))), 1e-4, 1e-4),
    # torus reward (hardware sin/cos in FP32, the library's in FP64)
    ("torus16_fp32", lambda: inputs.config_torus(d=16, n_live=400, seed=23), 1e-4, 1e-4),
    ("torus9_fp64", lambda: inputs.config_torus(d=9, n_live=200, seed=24, precision="fp64"),
     1e-10, 1e-9),
    # one noise normal per walker and step (noise_mode 1)
    ("gauss2d_fp64_wnoise", lambda: inputs.config_gauss2d(seed=19, noise="walker"), 1e-10, 1e-9),
    ("shells32_fp32_wnoise", lambda: inputs.config_shells(d=32, n_live=1000, seed=20, noise="walker"),
     1e-4, 1e-4),
    ("gmm16_fp64_wnoise", lambda: inputs.config_gmm(d=16, n_live=300, n_comp=4, seed=21, param_seed=6,
                                                    precision="fp64", noise="walker"), 1e-10, 1e-9),
    ("corr72_bf16_wnoise", lambda: inputs.config_corr_gauss(d=72, n_live=200, seed=22, param_seed=10,
                                                            precision="bf16mma", n_steps_max=60,
                                                            noise="walker"), 1e-4, 1e-4),
    # one normal per coordinate (noise_mode 0) in the batch-minimum loop
    ("gmm16_fp32_cnoise", lambda: inputs.config_gmm(d=16, n_live=600, n_comp=8, seed=28, param_seed=5,
                                                    noise="component"), 1e-4, 1e-4),
    ("corr40_bf16_cnoise", lambda: inputs.config_corr_gauss(d=40, n_live=300, seed=29, param_seed=8,
                                                            precision="bf16mma", n_steps_max=60,
                                                            noise="component"), 1e-4, 1e-4),
    # each walker stopping and saving by its own reflection count (walk_mode 0)
    ("gmm16_fp32_perwalker", lambda: inputs.config_gmm(d=16, n_live=600, n_comp=8, seed=30,
                                                       param_seed=5, stop="walker", save="walker"),
     1e-4, 1e-4),
    ("corr40_bf16_perwalker", lambda: inputs.config_corr_gauss(d=40, n_live=300, seed=31, param_seed=8,
                                                               precision="bf16mma", n_steps_max=60,
                                                               stop="walker", save="walker"),
     1e-4, 1e-4),
]


@pytest.mark.parametrize("name,make,tol,tau", CASES, ids=[c[0] for c in CASES])
def test_init_matches_oracle(torch, orc, name, make, tol, tau):
    cfg = make()
    eng = _engine([cfg])
    torch.cuda.synchronize()
    o = orc.Oracle(cfg).init()
    x = _np(eng.live_x(0)).astype(np.float64)
    scale = max(abs(cfg.lo), abs(cfg.hi))
    err = np.abs(x - o.live_x).max() / scale
    assert err < (1e-15 if cfg.precision == "fp64" else 1e-7)
    l = _np(eng.live_logl(0))
    rel = np.abs(l - o.live_logl) / np.maximum(1.0, np.abs(o.live_logl))
    assert rel.max() < {"fp64": 1e-12, "fp32": 2e-5, "bf16mma": 1e-4}[cfg.precision]
    st = eng.stats()[0]
    assert st["state"] == 0 and st["evals"] == cfg.n_live
    assert abs(st["dt"] - cfg.dt_init * (cfg.hi - cfg.lo)) < 1e-15
    eng.close()


@pytest.mark.parametrize("name,make,tol,tau", CASES, ids=[c[0] for c in CASES])
def test_kill_and_walk_trace_match_oracle(torch, orc, name, make, tol, tau):
    _trace_check(torch, orc, make(), tol, tau)


# every coordinates-per-lane choice of the FP32 vector walk on d = 32 (groups of
# 32, 16, 8 and 4 lanes; 16, 8 and 4 run the kernels with the group size fixed
# at compile time), in both noise readings
VALU_SHAPES = [(c, noise) for c in (1, 2, 4, 8) for noise in ("component", "walker")]


@pytest.mark.parametrize("c,noise", VALU_SHAPES, ids=[f"c{c}_{n}" for c, n in VALU_SHAPES])
def test_valu_walk_shapes_match_oracle(torch, orc, c, noise):
    cfg = inputs.config_shells(d=32, n_live=300, seed=400 + c, noise=noise, n_steps_max=60)
    _trace_check(torch, orc, cfg, 1e-4, 1e-4, tile_c=[c], steps=20)


# every tile shape of the matrix-core walk: (d, wavefronts per 16 walkers)
MMA_SHAPES = [(20, 1), (20, 2), (64, 1), (64, 4), (72, 3), (128, 2), (128, 8), (150, 5),
              (180, 6), (200, 7), (256, 4), (256, 8)]


@pytest.mark.parametrize("d,waves", MMA_SHAPES, ids=[f"d{d}_w{w}" for d, w in MMA_SHAPES])
def test_mma_walk_shapes_match_oracle(torch, orc, d, waves):
    cfg = inputs.config_corr_gauss(d=d, n_live=96, seed=300 + d, param_seed=40 + d,
                                   precision="bf16mma", n_steps_max=40)
    _trace_check(torch, orc, cfg, 1e-4, 1e-4, tile_c=[waves], steps=12)


def _trace_state(cfg):
    """Start state of a trace check: uniform points at the first iteration's
    step; for the shells a mid-run state instead (points around both shells
    and the step the run has adapted to by then: at the first iteration's step,
    0.1 of the prior width times |p| ~ sqrt(d), the thin shell is a strongly
    chaotic billiard where each bounce multiplies the FP32-vs-FP64 difference
    several fold, which no short-walk tolerance can absorb)."""
    if cfg.kind == "shells":
        rng = np.random.default_rng(99)
        v = rng.standard_normal((cfg.n_live, cfg.d))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        X = v * rng.uniform(1.7, 2.3, size=(cfg.n_live, 1))
        X[:, 0] += np.where(np.arange(cfg.n_live) % 2 == 0, 3.5, -3.5)
        return X, 0.005 * (cfg.hi - cfg.lo)
    return inputs.uniform_points(cfg.n_live, cfg.d, cfg.lo, cfg.hi, seed=99), cfg.dt_init * (cfg.hi - cfg.lo)


def _prepare_trace(torch, eng, orc, r, T):
    """Load the trace start state of run r into the engine and a fresh oracle;
    record T steps of every walker of run r on the GPU."""
    cfg = eng.cfgs[r]
    o = orc.Oracle(cfg, trace_steps=T).init()
    X, dt = _trace_state(cfg)
    _load_state(torch, eng, o, r, X)
    eng.write_vars(r, -math.inf, 0.0, dt, 0)
    o.set_state(dt=dt)
    return o, eng.set_trace(r, T)


def _compare_trace(torch, orc, eng, r, o, trace, tol, tau):
    """After the kill and the walk: kill order, survivors, threshold, evidence,
    starts exactly; per-step positions within tol relative (walkers masked from
    the first step at which a floating-point decision is within tau of its
    boundary), outside flags exactly, log L at the GPU's positions against the
    oracle's likelihood."""
    cfg = eng.cfgs[r]
    tx, tl, to = trace
    np.testing.assert_array_equal(_np(eng.killed(r)), o.killed)
    np.testing.assert_array_equal(_np(eng.survivors(r)), o.surv[:cfg.n_live - cfg.n_kill])
    st = eng.stats()[r]
    assert abs(st["lstar"] - o.st.lstar) <= tau * max(1.0, abs(o.st.lstar))
    assert abs(st["log_z"] - o.st.lz) < (1e-12 if tol < 1e-6 else 2e-5) * max(1.0, abs(o.st.lz))
    assert abs(st["log_x"] - o.st.lx) < 1e-13
    np.testing.assert_array_equal(_np(eng.start(r)), o.start)
    gx, gl, go = _np(tx).astype(np.float64), _np(tl), _np(to)
    width = cfg.hi - cfg.lo
    lstar = o.st.lstar
    masked, compared, worst = 0, 0, 0.0
    for m in range(cfg.n_kill):
        steps = int((o.trace_x[:, m] != 0).any(axis=1).sum())
        cut = steps
        for t in range(steps):
            near_l = abs(o.trace_logl[t, m] - lstar) < tau * max(1.0, abs(lstar))
            xo = o.trace_x[t, m]
            near_f = np.any(np.minimum(np.abs(xo - cfg.lo), np.abs(xo - cfg.hi)) < 0.1 * tau * width)
            if near_l or near_f:
                cut = t
                break
        if cut < steps:
            masked += 1
        if cut == 0:
            continue
        ref = o.trace_x[:cut, m]
        err = np.abs(gx[:cut, m] - ref).max(axis=1) / np.maximum(np.abs(ref).max(axis=1), width)
        worst = max(worst, err.max())
        np.testing.assert_array_equal(go[:cut, m], o.trace_out[:cut, m])
        lref, _ = orc.loglike(cfg, gx[:cut, m], bf16=cfg.precision == "bf16mma")
        lrel = np.abs(gl[:cut, m] - lref) / np.maximum(1.0, np.abs(lref))
        assert lrel.max() < (1e-12 if tol < 1e-6 else (1e-4 if cfg.precision == "bf16mma" else 2e-5))
        compared += 1
    assert worst < tol, worst
    assert masked <= max(4, 0.03 * cfg.n_kill), masked
    assert compared >= 0.9 * cfg.n_kill


def _trace_check(torch, orc, cfg, tol, tau, tile_c=None, steps=20):
    eng = _engine([cfg], tile_c)
    if tile_c is not None:
        c, g = eng.tile_shape(0)
        assert g == (4 * tile_c[0] if cfg.precision == "bf16mma" else g)
    o, trace = _prepare_trace(torch, eng, orc, 0, steps)
    eng.evidence_update()
    o.evidence_update()
    torch.cuda.synchronize()
    eng.hss_walk()
    o.hss_walk()
    torch.cuda.synchronize()
    _compare_trace(torch, orc, eng, 0, o, trace, tol, tau)
    eng.close()


# the configurations bench.py times, at their full sizes
FULL = [
    ("shells32_n1000_fp32", lambda: inputs.config_shells(d=32, n_live=1000, seed=50), 1e-4, 1e-4),
    ("gmm64_n4000_fp32", lambda: inputs.config_gmm(seed=51), 1e-4, 1e-4),
    ("corr256_n2000_bf16", lambda: inputs.config_corr_gauss(seed=52), 1e-4, 1e-4),
]


@pytest.mark.parametrize("name,make,tol,tau", FULL, ids=[c[0] for c in FULL])
def test_full_size_walk_trace_matches_oracle(torch, orc, name, make, tol, tau):
    _trace_check(torch, orc, make(), tol, tau, steps=10)


def test_batch64_sampled_runs_match_oracle(torch, orc):
    """The 64-run batch in one launch per kernel (every walk class on its own
    stream, as bench.py times it): three of its runs, one of each family, follow
    the oracle step by step while the other 61 walk beside them."""
    cfgs = inputs.config_batch()
    eng = _engine(cfgs)
    picks = {}
    for r, c in enumerate(cfgs):
        picks.setdefault(c.kind, r)
    checks = {r: _prepare_trace(torch, eng, orc, r, 10) for r in picks.values()}
    eng.evidence_update()
    for o, _ in checks.values():
        o.evidence_update()
    torch.cuda.synchronize()
    eng.hss_walk()
    for o, _ in checks.values():
        o.hss_walk()
    torch.cuda.synchronize()
    for r, (o, trace) in checks.items():
        _compare_trace(torch, orc, eng, r, o, trace, 1e-4, 1e-4)
    eng.close()


def test_staged_mixture_walk_matches_oracle(torch, orc):
    """A mixture walk class with more wavefronts than the register kernel fills
    the device with (five d = 64 runs of 4000 live points: 5 x 2000 walkers x 16
    lanes = 2500 wavefronts against two per SIMD on 1024 SIMDs) runs the kernel
    that reads the parameter block from LDS at every step; two of its runs
    follow the oracle step by step."""
    cfgs = inputs.replicate(inputs.config_gmm(seed=53), 5, base_seed=53)
    eng = _engine(cfgs)
    checks = {r: _prepare_trace(torch, eng, orc, r, 10) for r in (0, 4)}
    eng.evidence_update()
    for o, _ in checks.values():
        o.evidence_update()
    torch.cuda.synchronize()
    eng.hss_walk()
    for o, _ in checks.values():
        o.hss_walk()
    torch.cuda.synchronize()
    for r, (o, trace) in checks.items():
        _compare_trace(torch, orc, eng, r, o, trace, 1e-4, 1e-4)
    eng.close()


@pytest.mark.parametrize("name,make,tol,tau", CASES, ids=[c[0] for c in CASES])
def test_loglike_and_adjoint_match_oracle(torch, orc, name, make, tol, tau):
    cfg = make()
    eng = _engine([cfg])
    X = inputs.uniform_points(257, cfg.d, 0.3 * cfg.lo, 0.3 * cfg.hi, seed=5)
    xd = torch.from_numpy(X).to(eng.device, eng._fdtype(0))
    Xr = _np(xd).astype(np.float64)
    l, g = eng.loglike(0, xd)
    bf = cfg.precision == "bf16mma"
    lo_, go_ = orc.loglike(cfg, Xr, bf16=bf)
    torch.cuda.synchronize()
    rel = {"fp64": 1e-12, "fp32": 1e-5, "bf16mma": 1e-4}[cfg.precision]
    assert np.all(np.abs(_np(l) - lo_) <= rel * np.maximum(1.0, np.abs(lo_)))
    gs = np.abs(go_).max(axis=1, keepdims=True)
    assert np.all(np.abs(_np(g) - go_) <= {"fp64": 1e-10, "fp32": 2e-4, "bf16mma": 5e-3}[cfg.precision]
                  * np.maximum(gs, 1.0))
    gout = torch.linspace(-2.0, 3.0, 257, dtype=torch.float64, device=eng.device)
    gx = eng.loglike_vjp(0, xd, gout)
    np.testing.assert_allclose(_np(gx), _np(g) * _np(gout)[:, None], rtol=1e-6, atol=1e-6 * gs.max())
    # empty input is a no-op
    l0, _ = eng.loglike(0, xd[:0])
    assert l0.numel() == 0


@pytest.mark.parametrize("term_kind", [0, 1, 2])
def test_gauss2d_fp64_full_run_matches_oracle(torch, orc, term_kind):
    """The whole FP64 run (init, iterations, final sweep) reproduces the oracle,
    under each termination test (remaining evidence at 1e-3, the two X*L peak
    forms at 0.01)."""
    tol = 1e-3 if term_kind == 0 else 0.01
    for seed in ((2100, 2101, 2102) if term_kind == 0 else (2103, 2104)):
        cfg = inputs.config_gauss2d(seed=seed, term_kind=term_kind, term_tol=tol)
        eng = _engine([cfg])
        st = eng.run(poll_every=4)[0]
        o = orc.Oracle(cfg).run()
        assert st["state"] == o.st.state == 1
        assert st["iter"] == o.st.iter
        assert st["evals"] == o.st.evals
        assert abs(st["log_z"] - o.st.lz) < 1e-9
        assert abs(st["sigma_kl"] - o.st.sigma_kl) < 1e-9
        assert abs(st["sigma_mom"] - o.st.sigma_mom) < 1e-7
        assert abs(st["log_z2"] - o.st.lz2) < 1e-9
        dl, dw = eng.dead(0)
        ol, ow = o.dead()
        np.testing.assert_allclose(_np(dl), ol, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(_np(dw), ow, rtol=1e-12, atol=1e-11)
        eng.close()


@pytest.mark.parametrize("n", [1000, 2000, 4096])
def test_gauss2d_fp64_large_run_matches_oracle(torch, orc, n):
    """Whole FP64 runs at 1000, 2000 and 4096 live points (above 1024 every kill
    after the first sorts only the new points and merges them with the previous
    survivors' order): the runs reproduce the oracle's (iterations,
    evaluations, log Z, dead records)."""
    cfg = inputs.config_gauss2d(seed=2105 + n, n_live=n)
    eng = _engine([cfg])
    st = eng.run(poll_every=4)[0]
    o = orc.Oracle(cfg).run()
    assert st["state"] == o.st.state == 1
    assert st["iter"] == o.st.iter and st["iter"] > 3
    assert st["evals"] == o.st.evals
    assert abs(st["log_z"] - o.st.lz) < 1e-9
    dl, dw = eng.dead(0)
    ol, ow = o.dead()
    np.testing.assert_allclose(_np(dl), ol, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(_np(dw), ow, rtol=1e-12, atol=1e-11)
    eng.close()


# (n, k, perturb a survivor): above 1024 live points the second kill merges
# the new points with the first kill's survivor order when both lists fit the
# sort of the new points (1024 entries up to 2048 live points, 2048 above) and
# the survivors are untouched; a changed survivor, the sizes or a live set of
# at most 1024 make it sort all
MERGE_SIZES = [(4096, 2048, False), (3000, 1500, False), (2500, 2000, False), (4095, 2048, False),
               (2049, 1, False), (4000, 1900, False), (4096, 2048, True), (3000, 1500, True),
               (2000, 1000, False), (2048, 1024, False), (1500, 500, False), (1100, 50, False),
               (2000, 1000, True), (1000, 500, False), (1024, 512, False), (700, 300, False),
               (600, 50, False), (64, 32, False), (1000, 500, True)]


@pytest.mark.parametrize("n,k,perturb", MERGE_SIZES,
                         ids=[f"n{n}_k{k}" + ("_perturbed" if p else "") for n, k, p in MERGE_SIZES])
def test_second_kill_order_matches_oracle(torch, orc, n, k, perturb):
    """Two kills on identical live sets with exact ties, the killed slots
    refilled with new log L (tied among themselves and with survivors) before
    the second: both kill orders, survivors, thresholds and evidences match the
    oracle exactly."""
    d = 3
    cfg = inputs.RunConfig(kind="gauss_diag", d=d, n_live=n, n_kill=k, lo=-3.0, hi=3.0,
                           precision="fp64", seed=90 + n + k,
                           params=inputs.gauss_diag_params(np.zeros(d), np.ones(d)))
    X = inputs.uniform_points(n, d, cfg.lo, cfg.hi, seed=n + 5 * k)
    rng = np.random.default_rng(n * 11 + k)
    L = np.round(rng.normal(-5.0, 2.0, size=n), 1)
    eng = _engine([cfg])
    o = orc.Oracle(cfg).init()
    for kill in range(2):
        eng.live_x(0).copy_(torch.from_numpy(X).to(eng.device))
        eng.live_logl(0).copy_(torch.from_numpy(L).to(eng.device))
        eng.write_vars(0, -math.inf, 0.0, 0.1, 0)
        o.set_state(live_x=X, live_logl=L, log_z=-math.inf, log_x=0.0, dt=0.1, iteration=0)
        eng.evidence_update()
        o.evidence_update()
        torch.cuda.synchronize()
        killed = _np(eng.killed(0))
        np.testing.assert_array_equal(killed, o.killed)
        np.testing.assert_array_equal(_np(eng.survivors(0)), o.surv[:n - k])
        st = eng.stats()[0]
        assert st["lstar"] == o.st.lstar
        assert abs(st["log_z"] - o.st.lz) < 1e-12 * max(1.0, abs(o.st.lz))
        # refill the killed slots above the threshold, with ties
        L = L.copy()
        L[killed] = np.round(o.st.lstar + np.abs(rng.normal(0.0, 1.5, size=k)), 1)
        if perturb:
            surv = np.setdiff1d(np.arange(n), killed)
            L[surv[rng.integers(len(surv))]] = np.round(L.max() + 1.0, 1)
    eng.close()


KILL_SIZES = [(4096, 2048, 8), (4096, 1, 3), (4095, 4094, 2), (2049, 1024, 5), (2048, 1000, 1),
              (1537, 1536, 3), (1025, 512, 2), (1024, 512, 4), (7, 3, 2), (2, 1, 1)]


@pytest.mark.parametrize("n,k,d", KILL_SIZES, ids=[f"n{n}_k{k}_d{d}" for n, k, d in KILL_SIZES])
def test_kill_order_at_edge_sizes(torch, orc, n, k, d):
    """The kill step on identical live sets (positions and FP64 log L loaded on
    both sides, with exact ties among them): killed slots in kill order,
    survivors, threshold, evidence and volume match the oracle exactly at the
    largest live set, at every register layout of the sort (1, 2 and 4 keys per
    thread) and at ragged, tiny and extreme kill counts."""
    cfg = inputs.RunConfig(kind="gauss_diag", d=d, n_live=n, n_kill=k, lo=-3.0, hi=3.0,
                           precision="fp64", seed=40 + n + k,
                           params=inputs.gauss_diag_params(np.zeros(d), np.ones(d)))
    X = inputs.uniform_points(n, d, cfg.lo, cfg.hi, seed=n + 3 * k)
    rng = np.random.default_rng(n * 7 + k)
    L = np.round(rng.normal(-5.0, 2.0, size=n), 1)          # many exact ties
    eng = _engine([cfg])
    eng.live_x(0).copy_(torch.from_numpy(X).to(eng.device))
    eng.live_logl(0).copy_(torch.from_numpy(L).to(eng.device))
    eng.write_vars(0, -math.inf, 0.0, 0.1, 0)
    o = orc.Oracle(cfg).init()
    o.set_state(live_x=X, live_logl=L, log_z=-math.inf, log_x=0.0, dt=0.1, iteration=0)
    eng.evidence_update()
    o.evidence_update()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(eng.killed(0)), o.killed)
    np.testing.assert_array_equal(_np(eng.survivors(0)), o.surv[:n - k])
    st = eng.stats()[0]
    assert st["lstar"] == o.st.lstar
    assert abs(st["log_z"] - o.st.lz) < 1e-12 * max(1.0, abs(o.st.lz))
    assert abs(st["log_x"] - o.st.lx) < 1e-13
    dl, dw = eng.dead(0)
    ol, ow = o.dead()
    np.testing.assert_array_equal(_np(dl), ol)
    np.testing.assert_allclose(_np(dw), ow, rtol=1e-13, atol=1e-13)
    eng.close()
