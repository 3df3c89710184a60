"""Pins for the oracle's random streams (statistical properties; the paper
fixes no generator, the engine's choice is Philox4x32-10 + xoshiro128++ with
Box-Muller normals).  A wrong round count, a dropped key bump or a broken
transform shows up as failed diffusion or a wrong distribution here."""
import numpy as np
import pytest
from scipy import stats

TAG_INIT, TAG_START, TAG_P0, TAG_EPS, TAG_RES = 1, 2, 3, 4, 5


def _bits(words):
    w = np.asarray(words, dtype=np.uint32)
    return ((w[..., None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.int8)


def test_philox_uniform_words(orc):
    words = np.concatenate([orc.stream_words(12345, i, 7, 3, TAG_EPS) for i in range(8192)])
    top = words >> 26                                   # 64 bins
    counts = np.bincount(top, minlength=64)
    assert stats.chisquare(counts).pvalue > 1e-4
    bit_means = _bits(words).mean(axis=0)
    assert np.all(np.abs(bit_means - 0.5) < 0.02)


def test_philox_avalanche(orc):
    """Each input bit of counter and key flips each output bit with
    probability ~1/2 (strict avalanche); a cipher with too few rounds or a lost
    key schedule fails this."""
    rng = np.random.default_rng(7)
    n = 256
    flips = np.zeros((192, 128))
    for _ in range(n):
        ctr = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        base = _bits(orc.philox(ctr, key)).ravel()
        for b in range(192):
            c2, k2 = ctr.copy(), key.copy()
            if b < 128:
                c2[b // 32] ^= np.uint64(1 << (b % 32))
            else:
                k2[(b - 128) // 32] ^= np.uint64(1 << ((b - 128) % 32))
            flips[b] += base != _bits(orc.philox(c2, k2)).ravel()
    p = flips / n
    assert abs(p.mean() - 0.5) < 0.01
    assert p.min() > 0.33 and p.max() < 0.67


def test_philox_counter_and_key_separate_streams(orc):
    a = orc.stream_words(1, 0, 0, 0, TAG_P0)
    assert not np.array_equal(a, orc.stream_words(2, 0, 0, 0, TAG_P0))
    assert not np.array_equal(a, orc.stream_words(1, 0, 0, 0, TAG_EPS))
    assert not np.array_equal(a, orc.stream_words(1, 0, 1, 0, TAG_P0))
    assert not np.array_equal(a, orc.stream_words(1, 0, 0, 0, TAG_P0, sub=1))
    assert np.array_equal(a, orc.stream_words(1, 0, 0, 0, TAG_P0))


def test_xoshiro_stream_uniform_and_uncorrelated(orc):
    seed = orc.stream_words(99, 0, 0, 0, TAG_EPS)
    w = orc.xoshiro_stream(seed, 60000).astype(np.float64)
    u = (w + 0.5) / 2**32
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    lag1 = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(lag1) < 0.02
    bit_means = _bits(w.astype(np.uint32)).mean(axis=0)
    assert np.all(np.abs(bit_means - 0.5) < 0.02)


def test_xoshiro_zero_state_is_fixed_point(orc):
    # the generator is linear: the all-zero state maps to itself, which is why
    # seeding replaces an all-zero Philox output
    assert np.all(orc.xoshiro_stream([0, 0, 0, 0], 4) == 0)


def test_box_muller_normals(orc):
    rng = np.random.default_rng(3)
    z = np.concatenate([orc.box_muller4(rng.integers(0, 2**32, size=4, dtype=np.uint64))
                        for _ in range(20000)])
    assert stats.kstest(z, "norm").pvalue > 1e-4
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.02
    pairs = z.reshape(-1, 2)
    assert abs(np.corrcoef(pairs[:, 0], pairs[:, 1])[0, 1]) < 0.02
    ang = np.arctan2(pairs[:, 1], pairs[:, 0])
    assert stats.kstest((ang + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-4
    # radius^2 of a pair is chi-square with 2 degrees of freedom
    assert stats.kstest((pairs ** 2).sum(1), "chi2", args=(2,)).pvalue > 1e-4


def test_box_muller_extremes_finite(orc):
    z = orc.box_muller4([0, 0, 0xFFFFFFFF, 0xFFFFFFFF])
    assert np.all(np.isfinite(z))
    # smallest open uniform is 2^-25: radius sqrt(50 ln 2) ~ 5.89
    assert abs(np.hypot(z[0], z[1]) - np.sqrt(-2 * np.log(0.5 / 2**24))) < 1e-12
