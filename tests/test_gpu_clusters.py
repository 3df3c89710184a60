"""Cluster mode on the GPU against the oracle on identical inputs: cluster
finding, per-cluster kill weights and volumes, grouped survivors, spawning,
and whole FP64 runs."""
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


def _engine(cfgs):
    from paper_2312_03911_amd.engine import Engine
    return Engine(cfgs)


def _np(t):
    return t.detach().cpu().numpy()


def _blob_cfg(d, n, precision, seed):
    return inputs.RunConfig(kind="gauss_diag", d=d, n_live=n, lo=-20.0, hi=20.0, precision=precision,
                            params=inputs.gauss_diag_params(np.zeros(d), np.full(d, 3.0)),
                            seed=seed, cluster=1, max_ref=0, n_steps_max=10)


def _blobs(centres, per, d, scale, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([c + scale * rng.standard_normal((per, d)) for c in centres])


def _moments_match(tab, o, nc, atol):
    """The cluster recursion's moments (logs of Zbar_p, (Z_p^2)bar, (Z X_p)bar,
    (Z_p X_p)bar, (X_p^2)bar and the cross (X_p X_q)bar) of the first nc
    clusters equal the oracle's: the same -inf pattern, finite values within
    atol."""
    cm = o.cm
    for name, off in (("log_zp", 0), ("log_z2p", 64), ("log_zx", 128), ("log_zpx", 192), ("log_x2", 256)):
        np.testing.assert_allclose(tab[name][:nc], cm[off:off + nc], rtol=0, atol=atol, err_msg=name)
    xx = cm[320:].reshape(64, 64)[:nc, :nc].copy()
    g = tab["log_xx"][:nc, :nc].copy()
    np.fill_diagonal(xx, 0.0)
    np.fill_diagonal(g, 0.0)
    np.testing.assert_allclose(g, xx, rtol=0, atol=atol, err_msg="log_xx")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cluster_step_matches_oracle(torch, orc, precision):
    d, per = 5, 100
    centres = [np.full(d, -8.0), np.zeros(d), np.full(d, 8.0), np.array([8.0, -8.0, 8.0, -8.0, 8.0])]
    X = _blobs(centres, per, d, 0.6, seed=3)
    cfg = _blob_cfg(d, 4 * per, precision, seed=31)
    eng = _engine([cfg])
    xd = torch.from_numpy(X).to(eng.device, eng._fdtype(0))
    eng.live_x(0).copy_(xd)
    l, _ = eng.loglike(0, eng.live_x(0).clone(), grad=False)
    eng.live_logl(0).copy_(l)
    o = orc.Oracle(cfg).init()
    o.set_state(live_x=_np(xd).astype(np.float64), live_logl=_np(l))
    eng.evidence_update()
    o.evidence_update()
    torch.cuda.synchronize()
    tab = eng.clusters(0)
    assert tab["n_clusters"] == o.st.n_clusters == 4 and tab["n_splits"] == o.st.n_splits == 1
    np.testing.assert_array_equal(_np(eng.labels(0)), o.label)
    nc = o.st.n_clusters
    np.testing.assert_array_equal(tab["n_live"][:nc], o.cn[:nc])
    np.testing.assert_allclose(tab["log_xbar"][:nc], o.clx[:nc], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(_np(eng.killed(0)), o.killed)
    np.testing.assert_array_equal(_np(eng.survivors(0)), o.surv[:cfg.n_live - cfg.n_kill])
    np.testing.assert_array_equal(tab["surv_off"][:nc + 1], o.surv_off[:nc + 1])
    dl, dw = eng.dead(0)
    np.testing.assert_array_equal(_np(dl), o.dead_logl[:o.n_dead])
    np.testing.assert_allclose(_np(dw), o.dead_logw[:o.n_dead], rtol=0, atol=1e-12)
    st = eng.stats()[0]
    assert abs(st["log_z"] - o.st.lz) < 1e-12 and abs(st["log_x"] - o.st.lx) < 1e-12
    assert st["n_clusters"] == 4
    # the split into four (Eqs. new0-new6) and the kill that follows
    # (Eqs. update1-update9): every moment, and the run's Z2bar
    _moments_match(tab, o, nc, 1e-12)
    assert abs(st["log_z2"] - o.st.lz2) < 1e-12
    # spawning: the same clusters and starts for every walker
    eng.hss_walk()
    o.hss_walk()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(eng.start(0)), o.start)
    eng.replace_dead()
    o.replace_dead()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(eng.labels(0)), o.label)
    np.testing.assert_array_equal(eng.clusters(0)["n_live"][:nc], o.cn[:nc])


def test_one_blob_stays_one_cluster(torch):
    d, n = 6, 300
    cfg = _blob_cfg(d, n, "fp64", seed=32)
    eng = _engine([cfg])
    X = inputs.ball_points(n, d, np.zeros(d), 3.0, seed=4)
    eng.live_x(0).copy_(torch.from_numpy(X).to(eng.device))
    l, _ = eng.loglike(0, eng.live_x(0).clone(), grad=False)
    eng.live_logl(0).copy_(l)
    eng.evidence_update()
    torch.cuda.synchronize()
    assert eng.clusters(0)["n_clusters"] == 1


@pytest.mark.parametrize("seed", [900, 901])
def test_cluster_mode_fp64_full_run_matches_oracle(torch, orc, seed):
    d = 4
    prm = inputs.gmm_params(np.array([np.full(d, -4.0), np.full(d, 4.0)]), np.full((2, d), 0.5))
    cfg = inputs.RunConfig(kind="gmm_diag", d=d, n_live=200, n_comp=2, params=prm, lo=-8.0, hi=8.0,
                           seed=seed, precision="fp64", cluster=1, noise="walker", max_ref=0,
                           n_steps_max=40)
    eng = _engine([cfg])
    st = eng.run(poll_every=4)[0]
    o = orc.Oracle(cfg).run()
    assert st["state"] == o.st.state == 1
    assert st["iter"] == o.st.iter and st["n_clusters"] == o.st.n_clusters >= 2
    assert abs(st["log_z"] - o.st.lz) < 1e-9
    assert abs(st["sigma_kl"] - o.st.sigma_kl) < 1e-9
    # the cluster recursion's second moment and the error it gives
    assert abs(st["log_z2"] - o.st.lz2) < 1e-9
    assert o.st.sigma_mom > 0 and abs(st["sigma_mom"] - o.st.sigma_mom) < 1e-9
    _moments_match(eng.clusters(0), o, o.st.n_clusters, 1e-9)


def test_cluster_mode_runs_batched_with_plain_runs(torch):
    """A cluster-mode run and ordinary runs in one batch: each equals itself
    run alone."""
    d = 4
    prm = inputs.gmm_params(np.array([np.full(d, -4.0), np.full(d, 4.0)]), np.full((2, d), 0.5))
    ccfg = inputs.RunConfig(kind="gmm_diag", d=d, n_live=200, n_comp=2, params=prm, lo=-8.0,
                            hi=8.0, seed=950, precision="fp32", cluster=1)
    cfgs = [inputs.config_shells(d=8, n_live=200, seed=951), ccfg]
    both = _engine(cfgs)
    both.iterate(12)
    alone = _engine([ccfg])
    alone.iterate(12)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(both.live_x(1)), _np(alone.live_x(0)))
    np.testing.assert_array_equal(_np(both.labels(1)), _np(alone.labels(0)))
    assert both.stats()[1] == alone.stats()[0]


def _exact_knn(X, K):
    """FP64 neighbour lists of one cluster holding every point, in (squared
    distance, slot) order (distances as sums of squared differences), and the
    relative gap between consecutive ranks."""
    n = len(X)
    order = np.empty((n, K + 1), np.int64)
    dd = np.empty((n, K + 1))
    for a in range(0, n, 256):
        D = ((X[a:a + 256, None, :] - X[None, :, :]) ** 2).sum(-1)
        D[np.arange(D.shape[0]), np.arange(a, a + D.shape[0])] = np.inf
        part = np.argpartition(D, K + 1, axis=1)[:, :K + 2]
        for i in range(D.shape[0]):
            c = part[i]
            o = c[np.lexsort((c, D[i, c]))][:K + 1]
            order[a + i], dd[a + i] = o, D[i, o]
    gap = np.abs(np.diff(dd, axis=1)) / np.maximum(dd[:, 1:], 1e-300)
    return order[:, :K], dd[:, :K], gap


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_knn_lists_match_fp64_distances(torch, orc, precision):
    """The first pass of neighbours at the d = 64, 4000-point size (one cluster
    holding the prior draws): the GPU's lists equal exact FP64 neighbour
    lists at every rank whose order is decided by a margin larger than the
    run precision's distance error (relative gap to the next rank 1e-10 in
    FP64, 1e-5 in FP32); the masked share stays small."""
    cfg = inputs.config_gmm(precision=precision, cluster=1, seed=9310)
    eng = _engine([cfg])
    eng.evidence_update()
    torch.cuda.synchronize()
    X = _np(eng.live_x(0)).astype(np.float64)
    slots, dist = eng.knn(0)
    g = _np(slots)[:, :8]
    ref, refd, gap = _exact_knn(X, 8)
    tau = 1e-10 if precision == "fp64" else 1e-5
    # a rank is decided when its distance is apart from both neighbours' ranks
    near = np.zeros_like(ref, bool)
    near[:, :8] |= gap[:, :8] < tau
    near[:, 1:] |= gap[:, :7] < tau
    ok = ~near
    assert ok.mean() > 0.98, ok.mean()
    np.testing.assert_array_equal(g[ok], ref[ok])
    np.testing.assert_allclose(_np(dist)[:, :8][ok], refd[ok], rtol=1e-12 if precision == "fp64" else 2e-5)
    eng.close()


def test_cluster_step_with_deep_neighbour_loop_matches_oracle(torch, orc):
    """The d = 64, 4000-point mixture (config 4) in cluster mode, FP64: two
    iterations on both sides from the same seed, then the third iteration's
    cluster finding, whose loop runs to k = 13 (the second pass of eight
    neighbours): clusters, labels, volumes and the kill that follows match
    the oracle exactly."""
    cfg = inputs.config_gmm(precision="fp64", cluster=1, seed=9300)
    eng = _engine([cfg])
    o = orc.Oracle(cfg).init()
    for _ in range(2):
        eng.iterate(1)
        o.iterate()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(eng.labels(0)), o.label)
    np.testing.assert_allclose(_np(eng.live_x(0)), o.live_x, rtol=0, atol=1e-9)
    before = o.st.kstop_max
    eng.evidence_update()
    o.evidence_update()
    torch.cuda.synchronize()
    assert o.st.kstop_max > 8 >= before
    tab = eng.clusters(0)
    nc = o.st.n_clusters
    assert tab["n_clusters"] == nc and tab["n_splits"] == o.st.n_splits and tab["n_cut"] == 0
    np.testing.assert_array_equal(_np(eng.labels(0)), o.label)
    np.testing.assert_array_equal(tab["n_live"][:nc], o.cn[:nc])
    np.testing.assert_allclose(tab["log_xbar"][:nc], o.clx[:nc], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(_np(eng.killed(0)), o.killed)
    st = eng.stats()[0]
    assert abs(st["log_z"] - o.st.lz) < 1e-12 * max(1.0, abs(o.st.lz))
    # moments after three kills of 2000 points and the splits between them
    assert abs(st["log_z2"] - o.st.lz2) < 1e-10 * max(1.0, abs(o.st.lz2))
    _moments_match(tab, o, nc, 1e-9)
    eng.close()
