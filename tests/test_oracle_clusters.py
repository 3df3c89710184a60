"""Cluster recognition and volume-proportional spawning in the oracle
(cluster_mode 1), pinned on cases whose answer is known."""
import math

import numpy as np

from paper_2312_03911_amd import exact, inputs

TAG_START = 2


def _cfg(d, n, **kw):
    base = dict(kind="gauss_diag", d=d, n_live=n, lo=-20.0, hi=20.0, precision="fp64",
                params=inputs.gauss_diag_params(np.zeros(d), np.full(d, 3.0)), seed=123, cluster=1,
                max_ref=0, n_steps_max=10)
    base.update(kw)
    return inputs.RunConfig(**base)


def _blobs(centres, per, d, scale, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([c + scale * rng.standard_normal((per, d)) for c in centres])


def test_separated_blobs_become_clusters_with_volume_by_count(orc):
    d, per = 4, 100
    centres = [np.full(d, -8.0), np.zeros(d), np.full(d, 8.0)]
    X = _blobs(centres, per, d, 0.5, seed=1)
    cfg = _cfg(d, 3 * per)
    o = orc.Oracle(cfg).init()
    o.set_state(live_x=X)
    o.evidence_update()
    assert o.st.n_clusters == 3 and o.st.n_splits == 1
    lab = o.label.copy()
    for b in range(3):
        assert len(set(lab[b * per:(b + 1) * per])) == 1      # one label per blob
    assert len(set(lab)) == 3
    # the first blob (smallest slots) keeps cluster 0
    assert lab[0] == 0
    # the first dead point of each cluster was weighted with Xbar_p / (n_p + 1)
    # where Xbar_p = n_p / n of the whole volume (split by count)
    dl, dw = o.dead_logl[:o.n_dead], o.dead_logw[:o.n_dead]
    killed = o.killed
    seen = set()
    for j, s in enumerate(killed):
        c = lab[s]
        if c in seen:
            continue
        seen.add(c)
        assert abs(dw[j] - (math.log(per / (3 * per)) - math.log(per + 1))) < 1e-12
    # the run's volume is the sum of the clusters' volumes
    assert abs(o.st.lx - np.log(np.sum(np.exp(o.clx[:3])))) < 1e-12


def test_one_blob_is_not_split(orc):
    d, n = 6, 300
    X = inputs.ball_points(n, d, np.zeros(d), 3.0, seed=4)
    cfg = _cfg(d, n)
    o = orc.Oracle(cfg).init()
    o.set_state(live_x=X)
    o.evidence_update()
    assert o.st.n_clusters == 1 and o.st.n_splits == 0


def test_spawning_draws_clusters_by_volume(orc):
    """Each walker's cluster is the inverse-CDF pick of its start stream's
    second word over the clusters' volumes, and its start is a survivor of
    that cluster picked by the first word."""
    d, per = 3, 200
    centres = [np.full(d, -6.0), np.full(d, 6.0)]
    X = _blobs(centres, per, d, 0.4, seed=2)
    cfg = _cfg(d, 2 * per, seed=9)
    o = orc.Oracle(cfg).init()
    o.set_state(live_x=X)
    o.evidence_update()
    assert o.st.n_clusters == 2
    o.hss_walk()
    off = o.surv_off[:3].copy()
    w = np.exp(o.clx[:2] - o.clx[:2].max())
    cum = np.cumsum(w)
    picks = []
    for m in range(cfg.n_kill):
        u = orc.stream_words(cfg.seed, 0, m, 0, TAG_START)
        target = (float(u[1]) + 0.5) * 2.0 ** -32 * cum[-1]
        p = int(np.searchsorted(cum, target, side="right"))
        assert o.start_cl[m] == p
        cnt = off[p + 1] - off[p]
        assert o.start[m] == o.surv[off[p] + ((int(u[0]) * int(cnt)) >> 32)]
        assert o.label[o.start[m]] == p
        picks.append(p)
    frac = np.mean(np.array(picks) == 0)
    expect = w[0] / w.sum()
    assert abs(frac - expect) < 4 * math.sqrt(expect * (1 - expect) / len(picks))


def test_cluster_mode_two_modes_match_closed_form(orc):
    """Two far-apart, equal-weight isotropic modes in d=4: with clusters the
    runs split them and their mean log Z is within three standard errors of
    the closed form (one noise normal per walker, fixed 10d-step walks)."""
    d = 4
    prm = inputs.gmm_params(np.array([np.full(d, -4.0), np.full(d, 4.0)]), np.full((2, d), 0.5))
    dz, sk, ncl = [], [], []
    for r in range(12):
        cfg = inputs.RunConfig(kind="gmm_diag", d=d, n_live=200, n_comp=2, params=prm, lo=-8.0,
                               hi=8.0, seed=900 + r, precision="fp64", cluster=1, noise="walker",
                               max_ref=0, n_steps_max=40)
        o = orc.Oracle(cfg).run()
        dz.append(o.st.lz - exact.log_z(cfg))
        sk.append(o.st.sigma_kl)
        ncl.append(o.st.n_clusters)
    assert min(ncl) >= 2
    assert abs(np.mean(dz)) < 3 * np.mean(sk) / math.sqrt(len(dz)), (np.mean(dz), dz)


def test_single_cluster_mode_matches_plain_run(orc):
    """With one cluster that never splits, cluster mode is the plain method:
    the same log Z to rounding (the same kills, weights and starts)."""
    cfg = inputs.config_gauss2d(seed=77)
    a = orc.Oracle(cfg).run()
    b = orc.Oracle(cfg.replace(cluster=1, cluster_kmax=2)).run()
    assert b.st.n_splits == 0
    assert abs(a.st.lz - b.st.lz) < 1e-9 and a.st.iter == b.st.iter
