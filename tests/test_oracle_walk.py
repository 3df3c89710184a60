"""Pins for the oracle's HSS walk (Algorithm GGNS HSS; Eq. reflection; the
outside-point scheme of Section 2.3; trajectory preservation, noise and pruning
of Section 3).  Each test sets up one iteration with a chosen live set and
checks the recorded trajectory against geometry that holds independently of
the code: straight lines, the mirror law, norm conservation, the stream
definitions and the uniform law inside a fixed ball."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2312_03911_amd import inputs

TAG_P0, TAG_EPS, TAG_RES = 3, 4, 5


def _gauss(d, sigma=1.0, lo=-100.0, hi=100.0, **kw):
    prm = inputs.gauss_diag_params(np.zeros(d), np.full(d, sigma))
    base = dict(kind="gauss_diag", d=d, n_live=2, params=prm, lo=lo, hi=hi, precision="fp64",
                n_steps_max=30, max_ref=0, min_ref=1, delta_p=0.0, prune_streak=0, seed=77)
    base.update(kw)
    return inputs.RunConfig(**base)


def one_walk(orc, cfg, killed_x, surv_x, dt, trace_steps=0, killed_logl=None, surv_logl=None):
    """Load killed (lowest) and surviving points, run one kill + walk."""
    k, n = len(killed_x), len(killed_x) + len(surv_x)
    cfg = cfg.replace(n_live=n, n_kill=k)
    o = orc.Oracle(cfg, trace_steps=trace_steps)
    o.init()
    X = np.concatenate([killed_x, surv_x])
    l, _ = orc.loglike(cfg, X)
    if killed_logl is not None:
        l[:k] = killed_logl
    if surv_logl is not None:
        l[k:] = surv_logl
    o.set_state(live_x=X, live_logl=l, log_z=-math.inf, log_x=0.0, dt=dt, iteration=0)
    o.evidence_update()
    assert sorted(o.killed.tolist()) == list(range(k))
    o.hss_walk()
    return o


def p0_of(orc, seed, walker, d, iteration=0, sub=0):
    z = []
    for b in range((d + 3) // 4):
        z.extend(orc.box_muller4(orc.stream_words(seed, b, walker, iteration, TAG_P0, sub)))
    return np.array(z[:d])


def momenta(o, x0):
    """Momenta implied by consecutive trace positions (valid when delta_p = 0
    between the recorded steps): q_t = (y_t - y_{t-1}) / dt."""
    y = o.trace_x                                   # [T, k, d]
    prev = np.concatenate([x0[None], y[:-1]], axis=0)
    return (y - prev) / o.st.dt


def test_straight_line_when_never_outside(orc):
    d = 3
    cfg = _gauss(d)
    x0 = np.array([[0.3, -0.2, 0.1]])
    o = one_walk(orc, cfg, killed_x=np.array([[50.0, 50.0, 50.0]]), surv_x=x0, dt=0.05,
                 trace_steps=30, killed_logl=[-1e300])
    p0 = p0_of(orc, cfg.seed, 0, d)
    t = np.arange(1, 31)[:, None]
    np.testing.assert_allclose(o.trace_x[:, 0, :], x0 + t * 0.05 * p0, rtol=0, atol=1e-12)
    assert o.trace_out.sum() == 0
    # no reflection: no point saved after min_ref=1, output is the last in-slice point
    np.testing.assert_allclose(o.out_x[0], o.trace_x[-1, 0])


def test_hand_reflection_head_on(orc):
    """Slice = unit disc of N(0, I_2).  Start at 0.9 along p0, step 0.2 along
    p0: lands at 1.1 (outside), normal -p0/|p0|, so p -> -p and the next
    position is back at 0.9."""
    d = 2
    cfg = _gauss(d, n_steps_max=4)
    p0 = p0_of(orc, cfg.seed, 0, d)
    u = p0 / np.linalg.norm(p0)
    x0 = 0.9 * u
    killed = np.array([[1.0, 0.0]])               # on the unit circle: L* = L(r = 1)
    o = one_walk(orc, cfg, killed_x=killed, surv_x=x0[None], dt=0.2 / np.linalg.norm(p0),
                 trace_steps=4)
    y = o.trace_x[:, 0, :]
    np.testing.assert_allclose(y[0], 1.1 * u, atol=1e-14)
    np.testing.assert_allclose(y[1], 0.9 * u, atol=1e-14)
    np.testing.assert_allclose(y[2], 0.7 * u, atol=1e-14)
    assert o.trace_out[:, 0].tolist()[:3] == [1, 0, 0]


def test_hand_reflection_oblique(orc):
    """x0 = (0.8, 0) moving with p = (1, 1)/sqrt(2) * |p0| is not available from
    the stream, so place x0 so that p0 hits the unit circle obliquely and check
    the mirror law at the landing point against its explicit normal."""
    d = 2
    cfg = _gauss(d, n_steps_max=3)
    p0 = p0_of(orc, cfg.seed, 0, d)
    u = p0 / np.linalg.norm(p0)
    perp = np.array([-u[1], u[0]])
    x0 = 0.6 * perp + 0.7 * u                      # |x0| = sqrt(0.85) < 1
    dt = 0.15 / np.linalg.norm(p0)
    o = one_walk(orc, cfg, killed_x=np.array([[1.0, 0.0]]), surv_x=x0[None], dt=dt, trace_steps=3)
    y0 = x0 + 0.15 * u                             # = 0.6 perp + 0.85 u, |y0| = 1.0404... > 1
    assert np.linalg.norm(y0) > 1.0
    np.testing.assert_allclose(o.trace_x[0, 0], y0, atol=1e-14)
    nvec = -y0 / np.linalg.norm(y0)                # unit score direction of N(0, I)
    p1 = p0 - 2 * (p0 @ nvec) * nvec
    np.testing.assert_allclose(o.trace_x[1, 0], y0 + dt * p1, atol=1e-13)
    # mirror law: tangential part kept, normal part reversed, norm kept
    q = (o.trace_x[1, 0] - y0) / dt
    assert abs(np.linalg.norm(q) - np.linalg.norm(p0)) < 1e-12
    assert abs(q @ nvec + p0 @ nvec) < 1e-12
    t = np.array([-nvec[1], nvec[0]])
    assert abs(q @ t - p0 @ t) < 1e-12


@pytest.mark.parametrize("d", [2, 5, 16])
def test_reflection_law_on_every_outside_step(orc, d):
    """delta_p = 0: every outside step reflects with the unit score at the
    landing point (or flips violated box axes); |p| never changes."""
    cfg = _gauss(d, lo=-0.8, hi=0.8, n_steps_max=40)
    n_w = 64
    rng = np.random.default_rng(d)
    sv = inputs.ball_points(n_w, d, np.zeros(d), 0.7, seed=d)
    sv = np.clip(sv, -0.79, 0.79)
    killed = np.tile(np.eye(d)[:1], (n_w, 1))      # L* = L(r = 1)
    o = one_walk(orc, cfg, killed_x=killed, surv_x=sv, dt=0.05, trace_steps=40)
    x0 = o.live_x[o.start]
    q = momenta(o, x0)                             # [T, k, d]
    norms = np.linalg.norm(q, axis=-1)
    np.testing.assert_allclose(norms, norms[:1].repeat(40, 0), rtol=1e-10)
    n_checked = 0
    for t in range(39):
        for m in range(n_w):
            y = o.trace_x[t, m]
            qa, qb = q[t, m], q[t + 1, m]
            if not o.trace_out[t, m]:
                np.testing.assert_allclose(qb, qa, rtol=1e-9, atol=1e-12)
                continue
            viol = (y < cfg.lo) | (y > cfg.hi)
            if viol.any():
                np.testing.assert_allclose(qb, np.where(viol, -qa, qa), rtol=1e-9, atol=1e-12)
            else:
                nv = -y / np.linalg.norm(y)
                np.testing.assert_allclose(qb, qa - 2 * (qa @ nv) * nv, rtol=1e-9, atol=1e-12)
            n_checked += 1
    assert n_checked > 50


def test_noise_is_componentwise_multiplicative_from_eps_stream(orc):
    d = 6
    cfg = _gauss(d, delta_p=0.05, n_steps_max=12, noise="component")
    x0 = np.zeros((1, d))
    o = one_walk(orc, cfg, killed_x=np.full((1, d), 50.0), surv_x=x0, dt=0.01, trace_steps=12,
                 killed_logl=[-1e300])
    q = momenta(o, x0)[:, 0, :]
    eps = np.zeros((12, 8))
    for b in range(2):
        w = orc.xoshiro_stream(orc.stream_words(cfg.seed, b, 0, 0, TAG_EPS), 4 * 12).reshape(12, 4)
        for t in range(12):
            eps[t, 4 * b:4 * b + 4] = orc.box_muller4(w[t])
    for t in range(11):
        np.testing.assert_allclose(q[t + 1], q[t] * (1 + 0.05 * eps[t, :d]), rtol=1e-9)


def test_walker_noise_scales_all_components_by_one_normal(orc):
    """noise_mode 1: p is multiplied by the same (1 + delta_p eps0) in every
    component, eps0 the first normal of the Box-Muller pair of two words of
    the walker's block-0 stream per step, so the direction of p is unchanged
    by the noise."""
    d = 6
    cfg = _gauss(d, delta_p=0.05, n_steps_max=12).replace(noise="walker")
    x0 = np.zeros((1, d))
    o = one_walk(orc, cfg, killed_x=np.full((1, d), 50.0), surv_x=x0, dt=0.01, trace_steps=12,
                 killed_logl=[-1e300])
    q = momenta(o, x0)[:, 0, :]
    w = orc.xoshiro_stream(orc.stream_words(cfg.seed, 0, 0, 0, TAG_EPS), 2 * 12).reshape(12, 2)
    for t in range(11):
        e0 = orc.box_muller4(np.concatenate([w[t], w[t]]))[0]
        np.testing.assert_allclose(q[t + 1], q[t] * (1 + 0.05 * e0), rtol=1e-9)
        cos = q[t + 1] @ q[t] / np.linalg.norm(q[t + 1]) / np.linalg.norm(q[t])
        assert abs(cos - 1.0) < 1e-12


def test_reservoir_follows_res_stream_and_is_uniform(orc):
    d = 4
    cfg = _gauss(d, delta_p=0.05, n_steps_max=40, min_ref=1)
    n_w = 400
    sv = inputs.ball_points(n_w, d, np.zeros(d), 0.8, seed=3)
    killed = np.tile(np.eye(d)[:1], (n_w, 1))
    o = one_walk(orc, cfg, killed_x=killed, surv_x=sv, dt=0.08, trace_steps=40)
    ranks = []
    for m in range(n_w):
        out = o.trace_out[:, m]
        nref = np.cumsum(out)
        res = orc.xoshiro_stream(orc.stream_words(cfg.seed, 0, m, 0, TAG_RES), 40)
        nsave, pick = 0, None
        for t in range(40):
            if not out[t] and nref[t] >= 1:
                nsave += 1
                if int(res[t]) * nsave < 2 ** 32:
                    pick = t
        if pick is None:
            continue
        np.testing.assert_array_equal(o.out_x[m], o.trace_x[pick, m])
        saved = [t for t in range(40) if not out[t] and nref[t] >= 1]
        j = saved.index(pick)
        ranks.append((j + 0.5) / len(saved))
    assert len(ranks) > 300
    assert stats.kstest(ranks, "uniform").pvalue > 1e-3


def test_prune_resets_to_start_with_fresh_momentum(orc):
    d = 3
    cfg = _gauss(d, n_steps_max=9, prune_streak=3)
    x0 = np.array([[0.1, 0.2, 0.3]])
    # survivors carry a fake, huge log L so that L* is above every real value:
    # every step is outside
    o = one_walk(orc, cfg, killed_x=np.full((1, d), 50.0), surv_x=x0, dt=0.01, trace_steps=9,
                 killed_logl=[1e299], surv_logl=[1e300])
    assert o.trace_out[:, 0].all()
    p1 = p0_of(orc, cfg.seed, 0, d, sub=1)
    p2 = p0_of(orc, cfg.seed, 0, d, sub=2)
    np.testing.assert_allclose(o.trace_x[3, 0], x0[0] + 0.01 * p1, atol=1e-14)
    np.testing.assert_allclose(o.trace_x[6, 0], x0[0] + 0.01 * p2, atol=1e-14)
    assert o.summary()["prunes"] == 3
    # nothing was ever inside: the output falls back to the start point
    np.testing.assert_array_equal(o.out_x[0], x0[0])


def test_max_ref_stops_each_walker(orc):
    """The per-walker reading of the loop: each walker stops at its own
    max_ref-th reflection."""
    d = 3
    cfg = _gauss(d, n_steps_max=500, max_ref=3, min_ref=1, stop="walker", save="walker")
    sv = inputs.ball_points(50, d, np.zeros(d), 0.8, seed=8)
    o = one_walk(orc, cfg, killed_x=np.tile(np.eye(d)[:1], (50, 1)), surv_x=sv, dt=0.1,
                 trace_steps=500)
    for m in range(50):
        out = o.trace_out[:, m]
        steps = int(np.flatnonzero(np.cumsum(out) >= 3)[0]) + 1
        assert np.all(o.trace_x[steps:, m] == 0.0)   # nothing recorded after the stop
    assert o.summary()["it_steps"] < 50 * 500


def _ball_walk(orc, d, n_w, dt, **kw):
    cfg = _gauss(d, **kw)
    sv = inputs.ball_points(n_w, d, np.zeros(d), 1.0, seed=100 + d)
    v = np.random.default_rng(d).standard_normal((n_w, d))
    killed = v / np.linalg.norm(v, axis=1, keepdims=True)
    lr, _ = orc.loglike(cfg.replace(n_live=2), killed[:1])
    return one_walk(orc, cfg, killed_x=killed, surv_x=sv, dt=dt,
                    killed_logl=np.full(n_w, lr[0]))


@pytest.mark.parametrize("d", [2, 32])
def test_uniform_in_fixed_ball(orc, d):
    """Walk outputs inside a fixed ball slice follow P(r <= s) = s^d and
    E r^2 = d/(d+2) (plain HSS: no noise, no pruning, long fixed walks)."""
    o = _ball_walk(orc, d, 6000, dt=0.1 / math.sqrt(d), n_steps_max=200, min_ref=0)
    r = np.linalg.norm(o.out_x, axis=1)
    assert r.max() < 1.0
    assert stats.kstest(r ** d, "uniform").pvalue > 1e-3
    assert abs(np.mean(r ** 2) - d / (d + 2)) < 0.01


def test_walk_deterministic_and_thread_independent(orc):
    cfg = inputs.config_shells(d=8, n_live=200)
    a = orc.Oracle(cfg).init()
    for _ in range(3):
        a.iterate()
    orc.set_threads(1)
    b = orc.Oracle(cfg).init()
    for _ in range(3):
        b.iterate()
    orc.set_threads(4)
    np.testing.assert_array_equal(a.live_x, b.live_x)
    np.testing.assert_array_equal(a.live_logl, b.live_logl)
    assert a.summary() == b.summary()


def _first_step(flags, t0=0):
    """1-based step at which a boolean step sequence first holds (inf if never)."""
    idx = np.flatnonzero(flags)
    return int(idx[0]) + 1 if len(idx) else math.inf


def test_batch_minimum_loop_and_save_window(orc):
    """Algorithm GGNS HSS as written: every walker moves until the batch
    minimum of num_reflections reaches max_ref, and a point is saved once the
    batch minimum has reached min_ref.  From the trace: every walker makes the
    same number of steps T = max over walkers of its max_ref-th reflection;
    the saved window starts at Ta = max over walkers of its min_ref-th
    reflection; each output is the reservoir pick (RES stream) over the
    walker's in-slice steps in [Ta, T]; a prune keeps the reflection count."""
    d = 3
    cfg = _gauss(d, n_steps_max=400, max_ref=3, min_ref=1, delta_p=0.05, prune_streak=4)
    assert cfg.stop_id == 1 and cfg.save_id == 1
    n_w = 40
    sv = inputs.ball_points(n_w, d, np.zeros(d), 0.8, seed=11)
    o = one_walk(orc, cfg, killed_x=np.tile(np.eye(d)[:1], (n_w, 1)), surv_x=sv, dt=0.12,
                 trace_steps=400)
    out = o.trace_out.astype(bool)                      # [T, k]
    nref = np.cumsum(out, axis=0)
    b = [_first_step(nref[:, m] >= 3) for m in range(n_w)]
    a = [_first_step(nref[:, m] >= 1) for m in range(n_w)]
    T, Ta = max(b), max(a)
    assert T < 400
    assert o.summary()["it_steps"] == n_w * T
    # nothing is recorded after step T, for any walker
    assert np.all(o.trace_x[T:] == 0.0)
    assert np.all(np.any(o.trace_x[T - 1] != 0.0, axis=1))
    assert o.summary()["prunes"] > 0                    # the count survives a prune
    n_pick = 0
    for m in range(n_w):
        res = orc.xoshiro_stream(orc.stream_words(cfg.seed, 0, m, 0, TAG_RES), T)
        nsave, pick = 0, None
        for s in range(1, T + 1):
            if not out[s - 1, m] and s >= Ta:
                nsave += 1
                if int(res[s - 1]) * nsave < 2 ** 32:
                    pick = s
        if pick is not None:
            np.testing.assert_array_equal(o.out_x[m], o.trace_x[pick - 1, m])
            n_pick += 1
    assert n_pick > 30


def test_pooled_draw_indexes_the_batch_archive(orc):
    """draw = pooled: the saved points of the whole batch form one archive in
    the order the loop appends them (step by step, walkers in index order);
    new point j is archive[floor(u_j N / 2^32)] with u_j word 0 of the RES
    stream, sub 1, walker index j."""
    d = 3
    cfg = _gauss(d, n_steps_max=300, max_ref=3, min_ref=1, delta_p=0.05, draw="pooled")
    n_w = 30
    sv = inputs.ball_points(n_w, d, np.zeros(d), 0.8, seed=12)
    o = one_walk(orc, cfg, killed_x=np.tile(np.eye(d)[:1], (n_w, 1)), surv_x=sv, dt=0.12,
                 trace_steps=300)
    out = o.trace_out.astype(bool)
    nref = np.cumsum(out, axis=0)
    T = o.summary()["it_steps"] // n_w
    Ta = max(_first_step(nref[:, m] >= 1) for m in range(n_w))
    arch = [o.trace_x[s - 1, m] for s in range(Ta, T + 1) for m in range(n_w) if not out[s - 1, m]]
    assert len(arch) > n_w
    for j in range(n_w):
        u = int(orc.stream_words(cfg.seed, 0, j, 0, TAG_RES, 1)[0])
        np.testing.assert_array_equal(o.out_x[j], arch[(u * len(arch)) >> 32])


def test_isotropic_noise_adds_a_scaled_normal_vector(orc):
    """noise = isotropic (an option): p += delta_p (|p| / sqrt d) eps with eps
    the walker's per-coordinate normals; its law has no preferred axis."""
    d = 6
    cfg = _gauss(d, delta_p=0.05, n_steps_max=12, noise="isotropic")
    x0 = np.zeros((1, d))
    o = one_walk(orc, cfg, killed_x=np.full((1, d), 50.0), surv_x=x0, dt=0.01, trace_steps=12,
                 killed_logl=[-1e300])
    q = momenta(o, x0)[:, 0, :]
    eps = np.zeros((12, 8))
    for b in range(2):
        w = orc.xoshiro_stream(orc.stream_words(cfg.seed, b, 0, 0, TAG_EPS), 4 * 12).reshape(12, 4)
        for t in range(12):
            eps[t, 4 * b:4 * b + 4] = orc.box_muller4(w[t])
    for t in range(11):
        sc = 0.05 * np.linalg.norm(q[t]) / math.sqrt(d)
        np.testing.assert_allclose(q[t + 1], q[t] + sc * eps[t, :d], rtol=1e-9)


def _ball_batches(orc, d, k, n_batches, **kw):
    """Walk outputs in a fixed unit-ball slice (isotropic Gaussian, L* at r = 1),
    k walkers per batch, dt adapted first as the sampler adapts it (x0.9 above
    an out_frac of 0.15, x1.1 below 0.05)."""
    def batch(dt, seed):
        cfg = _gauss(d, n_steps_max=max(64, 5 * d), max_ref=3, min_ref=1, delta_p=0.05,
                     prune_streak=10, seed=seed, **kw)
        sv = inputs.ball_points(k, d, np.zeros(d), 1.0, seed=seed + 1)
        v = np.random.default_rng(seed + 2).standard_normal((k, d))
        killed = v / np.linalg.norm(v, axis=1, keepdims=True)
        lr, _ = orc.loglike(cfg.replace(n_live=2), killed[:1])
        o = one_walk(orc, cfg, killed_x=killed, surv_x=sv, dt=dt, killed_logl=np.full(k, lr[0]))
        s = o.summary()
        return o.out_x, s["it_outs"] / s["it_steps"]
    dt = 0.1
    for it in range(60):
        _, of = batch(dt, 100 + it)
        dt = dt * 0.9 if of > 0.15 else (dt * 1.1 if of < 0.05 else dt)
    outs, ofs = [], []
    for b in range(n_batches):
        x, of = batch(dt, 10000 + 7 * b)
        outs.append(x)
        ofs.append(of)
    return np.concatenate(outs), float(np.mean(ofs))


@pytest.mark.parametrize("d", [8, 32])
def test_uniform_in_fixed_ball_at_adapted_step(orc, d):
    """The default walk (batch-minimum loop and save, one pick per walker,
    walker noise, pruning) at the step the run adapts to leaves a fixed ball
    slice uniform: with 2e5 outputs E[d log r] = -1 is resolved to +-0.0022
    (one standard error).  The per-walker stop, under the same conditions,
    is pushed outward far beyond that (d = 32)."""
    x, of = _ball_batches(orc, d, 100, 2000)
    assert 0.05 <= of <= 0.15
    v = d * np.log(np.linalg.norm(x, axis=1))
    se = v.std() / math.sqrt(len(v))
    assert se < 0.0025
    assert abs(v.mean() + 1.0) < 0.0075, (v.mean(), se)
    if d == 32:
        xw, _ = _ball_batches(orc, d, 100, 2000, stop="walker", save="walker")
        vw = d * np.log(np.linalg.norm(xw, axis=1))
        sew = vw.std() / math.sqrt(len(vw))
        assert vw.mean() + 1.0 > max(0.0075, 4 * sew), (vw.mean(), sew)
