"""Engine behaviour on the GPU: batching, graph replay, determinism,
checkpoint/resume, per-run failure states, end-to-end agreement with the
oracle within the runs' own error."""
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


def _engine(cfgs, **kw):
    from paper_2312_03911_amd.engine import Engine
    return Engine(cfgs, **kw)


def _np(t):
    return t.detach().cpu().numpy()


def _small_mix():
    return [inputs.config_shells(d=8, n_live=300, seed=31),
            inputs.config_gmm(d=8, n_live=200, n_comp=4, seed=32, param_seed=3),
            inputs.RunConfig(kind="gauss_diag", d=4, n_live=120, lo=-4, hi=4, seed=33,
                             params=inputs.gauss_diag_params([0.1, -0.2, 0.3, 0.0], [0.5, 0.7, 0.9, 1.1])),
            inputs.config_gauss2d(seed=34)]


def test_run_inside_batch_equals_run_alone(torch):
    cfgs = _small_mix()
    both = _engine(cfgs)
    both.iterate(6)
    for r, c in enumerate(cfgs):
        one = _engine([c])
        one.iterate(6)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(_np(both.live_x(r)), _np(one.live_x(0)))
        np.testing.assert_array_equal(_np(both.live_logl(r)), _np(one.live_logl(0)))
        a, b = both.stats()[r], one.stats()[0]
        for key in ("log_z", "log_x", "dt", "lstar", "iter", "evals", "steps_out", "prunes"):
            assert a[key] == b[key], key
        one.close()
    both.close()


def _class_mix():
    """Runs spread over several kernel classes: vector FP32 and FP64, the
    matrix-core walk, batch-minimum walks and a cluster-mode run."""
    return _small_mix() + [
        inputs.config_corr_gauss(d=64, n_live=300, seed=35, n_steps_max=200),
        inputs.config_gmm(d=8, n_live=400, n_comp=4, seed=36, param_seed=4, cluster=1),
        inputs.config_torus(d=8, n_live=200, seed=37)]


def test_iterate_chains_equal_per_call_iterations(torch):
    """ggns_iterate (one chain of iterations per kernel class) gives bitwise the
    runs of one evidence / walk / replace call per iteration, eagerly and as a
    replayed graph, across blocks in which some runs stop."""
    cfgs = _class_mix()
    calls, chains, graph = _engine(cfgs), _engine(cfgs), _engine(cfgs)
    for block in range(6):
        calls.iterate(4, per_call=True)
        chains.iterate(4)
        graph.step_block(4, use_graph=True)
        torch.cuda.synchronize()
        s_c, s_i, s_g = calls.stats(), chains.stats(), graph.stats()
        for r in range(len(cfgs)):
            for e in (chains, graph):
                np.testing.assert_array_equal(_np(calls.live_x(r)), _np(e.live_x(r)))
                np.testing.assert_array_equal(_np(calls.live_logl(r)), _np(e.live_logl(r)))
            assert s_c[r] == s_i[r] == s_g[r], (block, r)
        for r, c in enumerate(cfgs):
            if c.cluster:
                np.testing.assert_array_equal(_np(calls.labels(r)), _np(chains.labels(r)))
    for e in (calls, chains, graph):
        e.close()


def test_iterate_rejects_negative_counts(torch):
    from paper_2312_03911_amd import _lib
    e = _engine(_small_mix())
    assert e.L.ggns_iterate(e.ctx, -1, e._stream()) == _lib.GGNS_EINVAL
    assert e.L.ggns_iterate(e.ctx, 0, e._stream()) == _lib.GGNS_OK
    e.close()


def test_same_seed_is_bitwise_reproducible(torch):
    cfgs = _small_mix()
    a, b = _engine(cfgs), _engine(cfgs)
    a.iterate(5)
    b.iterate(5)
    torch.cuda.synchronize()
    for r in range(len(cfgs)):
        np.testing.assert_array_equal(_np(a.live_x(r)), _np(b.live_x(r)))
        assert a.stats()[r] == b.stats()[r]


def test_graph_replays_match_eager_iterations(torch):
    cfgs = _small_mix()
    eager, graph = _engine(cfgs), _engine(cfgs)
    for block in range(4):
        eager.iterate(3)
        graph.step_block(3, use_graph=True)
        torch.cuda.synchronize()
        # eager work and synchronisation between replays
        s_e, s_g = eager.stats(), graph.stats()
        for r in range(len(cfgs)):
            np.testing.assert_array_equal(_np(eager.live_x(r)), _np(graph.live_x(r)))
            np.testing.assert_array_equal(_np(eager.live_logl(r)), _np(graph.live_logl(r)))
            assert s_e[r] == s_g[r], (block, r)


def test_pipelined_run_matches_synchronous_run(torch):
    """Reading the states one block behind (no drain between blocks) gives the
    same runs as reading them after every block; the asynchronous stats copy
    carries the same states as the synchronous read."""
    cfgs = _small_mix()
    a = _engine(cfgs)
    sa = a.run(poll_every=3, pipelined=False)
    b = _engine(cfgs)
    sb = b.run(poll_every=3, pipelined=True)
    for x, y in zip(sa, sb):
        assert x == y
    assert list(b.states_async(1)()) == [s["state"] for s in sb]
    a.close()
    b.close()


def test_reset_and_graph_replay_repeat_the_whole_run(torch):
    """Engine.reset re-initialises the runs on the same arena: a whole run
    replayed through the block graph captured before the reset gives the same
    stats, bitwise, as the first run and as a fresh engine (the benchmark's and
    the tuner's pass protocol)."""
    cfgs = _small_mix()
    a = _engine(cfgs)
    s1 = a.run(poll_every=4, use_graph=True)
    a.reset()
    s2 = a.run(poll_every=4, use_graph=True)
    b = _engine(cfgs)
    s3 = b.run(poll_every=4)
    for x, y, z in zip(s1, s2, s3):
        assert x == y == z
    a.close()
    b.close()


def test_checkpoint_and_resume_is_exact(torch):
    cfgs = _small_mix()
    a = _engine(cfgs)
    a.iterate(3)
    torch.cuda.synchronize()
    saved = a.arena.cpu().clone()
    a.iterate(4)
    torch.cuda.synchronize()
    restored = saved.to(a.device)
    b = _engine(cfgs, attach_arena=restored)
    b.iterate(4)
    torch.cuda.synchronize()
    for r in range(len(cfgs)):
        np.testing.assert_array_equal(_np(a.live_x(r)), _np(b.live_x(r)))
        assert a.stats()[r] == b.stats()[r]


def test_nonfinite_run_stops_alone(torch):
    good = inputs.config_shells(d=8, n_live=200, seed=41)
    bad = inputs.config_gauss2d(seed=42)
    bad.params = np.array([0.5, math.nan, 0.05, 0.05])
    eng = _engine([good, bad])
    alone = _engine([good])
    eng.iterate(3)
    alone.iterate(3)
    torch.cuda.synchronize()
    st = eng.stats()
    assert st[1]["state"] == 3 and st[0]["state"] == 0
    np.testing.assert_array_equal(_np(eng.live_x(0)), _np(alone.live_x(0)))


def test_max_iter_state_and_final_sweep(torch):
    cfg = inputs.config_gauss2d(seed=43, max_iter=4)
    eng = _engine([cfg])
    st = eng.run(poll_every=2)[0]
    assert st["state"] == 2 and st["iter"] == 4
    assert st["n_dead"] == 4 * cfg.n_kill + cfg.n_live
    assert math.isfinite(st["sigma_kl"]) and st["sigma_kl"] > 0


def test_forced_final_sweep(torch, orc):
    cfg = inputs.config_gauss2d(seed=44)
    eng = _engine([cfg])
    eng.iterate(5)
    eng.evidence_update(final_sweep=True)
    eng.finalize()
    o = orc.Oracle(cfg).init()
    for _ in range(5):
        o.iterate()
    o.evidence_update(final_sweep=True)
    st = eng.stats()[0]
    assert st["state"] == 1 and o.st.state == 1
    assert abs(st["log_z"] - o.st.lz) < 1e-9 and abs(st["h"] - o.st.h) < 1e-8


def test_shells_end_to_end_agree_with_oracle_within_error(torch, orc):
    """FP32 GPU and FP64 oracle runs of the shell problem: their log Z agree within
    the combined statistical error (trajectories differ after FP32 roundings)."""
    gz, oz, gs, os_ = [], [], [], []
    cfgs = inputs.replicate(inputs.config_shells(d=16, n_live=200), 6, base_seed=500)
    eng = _engine(cfgs)
    st = eng.run(poll_every=8)
    for c, s in zip(cfgs, st):
        o = orc.Oracle(c).run()
        gz.append(s["log_z"]); oz.append(o.st.lz)
        gs.append(s["sigma_mom"]); os_.append(o.st.sigma_mom)
        assert s["state"] == 1
    diff = np.mean(gz) - np.mean(oz)
    err = math.sqrt((np.mean(gs) ** 2 + np.mean(os_) ** 2) / len(cfgs))
    assert abs(diff) < 4 * err, (diff, err)


def test_torus_runs_match_closed_form_and_oracle(torch, orc):
    """Torus reward, FP32 on the GPU: ten d = 32 runs in one batch; their mean
    log Z lies within three standard errors of the closed form, like the FP64
    oracle's runs of the same problem; a run with c <= d stops before walking."""
    cfgs = inputs.replicate(inputs.config_torus(d=32, n_live=200), 10, base_seed=2800)
    bad = inputs.config_torus(d=8, n_live=100, c=8.0)
    eng = _engine(cfgs + [bad])
    st = eng.run(poll_every=8)
    truth = exact.log_z(cfgs[0])
    dz = np.array([s["log_z"] - truth for s in st[:-1]])
    assert all(s["state"] == 1 for s in st[:-1])
    assert st[-1]["state"] == 3 and st[-1]["iter"] == 0
    se = max(dz.std(ddof=1), np.mean([s["sigma_kl"] for s in st[:-1]])) / math.sqrt(len(dz))
    assert abs(dz.mean()) < 3 * se, (dz.mean(), se)
    oz = np.array([orc.Oracle(c.replace(precision="fp64")).run().st.lz - truth for c in cfgs[:4]])
    assert abs(oz.mean()) < 3 * max(oz.std(ddof=1), 0.02) / 2 + 3 * se


def test_tile_shapes_agree_and_autotune_picks_one(torch):
    """Every coordinates-per-lane choice computes the same walk (FP64: up to
    summation order), and the autotuner returns an admissible choice."""
    from paper_2312_03911_amd.autotune import candidates, tune
    cfg = inputs.config_shells(d=12, n_live=160, seed=61, precision="fp64")
    ref = None
    for c in candidates(cfg):
        eng = _engine([cfg], tile_c=[c])
        assert eng.tile_shape(0)[0] == c
        eng.iterate(3)
        torch.cuda.synchronize()
        x = _np(eng.live_x(0))
        if ref is None:
            ref = x
        else:
            assert np.abs(x - ref).max() < 1e-9, c
        eng.close()
    choice = tune([cfg, cfg.replace(seed=62)])
    assert choice[0] == choice[1] and choice[0] in candidates(cfg)


def test_dead_positions_follow_the_dead_records(torch):
    """With positions kept, row j of dead_x is the live point the j-th dead
    record came from: after one kill the killed rows in kill order, after the
    final sweep every remaining live point, and their log L are the records'."""
    cfg = inputs.config_gmm(d=12, n_live=200, n_comp=4, seed=45, param_seed=12)
    eng = _engine([cfg])
    eng.keep_dead_x(0)
    lx = _np(eng.live_x(0)).copy()
    ll = _np(eng.live_logl(0)).copy()
    eng.evidence_update()
    torch.cuda.synchronize()
    killed = _np(eng.killed(0))
    dl, _ = eng.dead(0)
    dx = _np(eng.dead_x(0))
    assert dx.shape == (cfg.n_kill, cfg.d)
    np.testing.assert_array_equal(dx, lx[killed])
    np.testing.assert_array_equal(_np(dl), ll[killed])
    eng.hss_walk()
    eng.replace_dead()
    st = eng.run(poll_every=4)[0]
    n_dead = st["n_dead"]
    dl, dw = eng.dead(0)
    dx = _np(eng.dead_x(0))
    assert dx.shape[0] == n_dead
    l_re, _ = eng.loglike(0, eng.dead_x(0)[-cfg.n_live:].clone(), grad=False)
    np.testing.assert_allclose(_np(l_re), _np(dl)[-cfg.n_live:], rtol=2e-6, atol=1e-6)
    # the mode report runs on the samples and finds the mixture's modes
    from paper_2312_03911_amd.posterior import gmm_mode_report, normalized_log_weights
    rep = gmm_mode_report(dx, normalized_log_weights(_np(dl), _np(dw), st["log_z"]), cfg)
    assert rep["recovered"] >= 1 and abs(sum(rep["weights"]) - 1.0) < 1e-9
