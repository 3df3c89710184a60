"""Seeded synthetic workloads: likelihood parameters and run settings.

This module only draws inputs.  It holds no step of the sampler: no kill, no
walk, no evidence arithmetic.  Both the GPU engine and the FP64 test oracle read
the same `RunConfig` objects it builds.

The workloads stand in for the paper's experiments (none of its data ships):
  * Gaussian, d=2 (the Section 4.1 family of diagonal Gaussians at low d);
  * two Gaussian shells, d=32 (the classic nested-sampling shell benchmark);
  * a correlated Gaussian, d=256 (stand-in for the 256-dimensional Gaussian
    posterior of the lensing experiment, Section 4.3);
  * an 8-component diagonal Gaussian mixture, d=64 (multimodal, Section 4.2 and
    Appendix G style mode counting);
  * a table of 64 uneven runs mixing the three families.

Hyperparameter defaults follow the paper's Appendix C table (min_ref=1,
max_ref=3, delta_p=0.05), dt_ini=0.1 (Appendix G) and the out_frac band
(0.05, 0.15) with factors 1.1 / 0.9 (Appendix H, Algorithm GGNS).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

KINDS = {"gauss_diag": 0, "gauss_full": 1, "shells": 2, "gmm_diag": 3, "torus": 4}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16mma": 2}
NOISE = {"component": 0, "walker": 1, "isotropic": 2}
STOP = {"walker": 0, "batch": 1}
SAVE = {"walker": 0, "batch": 1}
DRAW = {"walker": 0, "pooled": 1}


@dataclasses.dataclass
class RunConfig:
    """One nested-sampling run: problem, prior box, walk and termination settings."""

    kind: str
    d: int
    n_live: int
    params: np.ndarray            # raw FP64 parameter block (layout per kind, below)
    lo: float
    hi: float
    n_comp: int = 1
    n_kill: int = 0               # 0 -> n_live // 2
    precision: str = "fp32"
    dt_init: float = 0.1          # in units of the prior width
    n_steps_max: int = 20         # fixed-step length when max_ref == 0, else a cap
    min_ref: int = 1
    max_ref: int = 3
    prune_streak: int = 10
    delta_p: float = 0.05
    out_hi: float = 0.15
    out_lo: float = 0.05
    dt_down: float = 0.9
    dt_up: float = 1.1
    term_kind: int = 0            # 0: remaining evidence fraction, 1: X*L_max peak, 2: X*L_dead peak
    term_tol: float = 1e-3
    max_iter: int = 0             # 0 -> a generous bound from d, width and n_live
    seed: int = 0
    name: str = ""
    noise: str = "walker"         # eps of p *= 1 + delta_p eps: one per walker ("walker"), per coordinate ("component"), isotropic (oracle only)
    cluster: int = 0              # 1: cluster recognition and volume-proportional spawning
    cluster_kmax: int = 32        # largest neighbour count the cluster finding tries (0: every k, oracle only)
    stop: str = ""                # walk ends at the batch minimum of reflections ("batch") or each walker's own ("walker"); "" = batch with max_ref > 0
    save: str = ""                # points saved once the batch minimum ("batch") or the walker's own count ("walker") reaches min_ref; "" = batch with max_ref > 0
    draw: str = "walker"          # new point: one pick per walker ("walker") or pooled draws from all saved points ("pooled", oracle only)

    def __post_init__(self):
        self.params = np.ascontiguousarray(self.params, dtype=np.float64)
        if self.n_kill <= 0:
            self.n_kill = self.n_live // 2
        if self.max_iter <= 0:
            n, k = self.n_live, self.n_kill
            width = self.hi - self.lo
            shrink = math.log((n + 1.0) / (n + 1.0 - k))
            self.max_iter = 3 * int(math.ceil((self.d * max(math.log(width), 0.0)
                                               + 2.0 * self.d + 50.0) / shrink))

    @property
    def kind_id(self) -> int:
        return KINDS[self.kind]

    @property
    def precision_id(self) -> int:
        return PRECISIONS[self.precision]

    @property
    def noise_id(self) -> int:
        return NOISE[self.noise]

    @property
    def stop_id(self) -> int:
        # a fixed-step walk (max_ref == 0) has no reflection loop: per walker
        return STOP[self.stop or ("batch" if self.max_ref > 0 else "walker")]

    @property
    def save_id(self) -> int:
        return SAVE[self.save or ("batch" if self.max_ref > 0 else "walker")]

    @property
    def draw_id(self) -> int:
        return DRAW[self.draw]

    def replace(self, **kw) -> "RunConfig":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# Parameter layouts (FP64):
#   gauss_diag: mu[d], sigma[d]
#   gauss_full: mu[d], P[d*d] (precision matrix, row-major), log det P
#   shells:     n_comp blocks of {centre[d], radius, width}
#   gmm_diag:   n_comp blocks of {mu[d], sigma[d]}, equal weights
#   torus:      {alpha, beta, c} of the torus reward (Eq. torus)
# ---------------------------------------------------------------------------

def gauss_diag_params(mu, sigma) -> np.ndarray:
    return np.concatenate([np.asarray(mu, np.float64), np.asarray(sigma, np.float64)])


def shells_params(centres, radius, width) -> np.ndarray:
    blocks = [np.concatenate([np.asarray(c, np.float64), [radius, width]]) for c in centres]
    return np.concatenate(blocks)


def gmm_params(mus, sigmas) -> np.ndarray:
    return np.concatenate([np.concatenate([m, s]) for m, s in zip(mus, sigmas)]).astype(np.float64)


def torus_params(alpha, beta, c) -> np.ndarray:
    return np.array([alpha, beta, c], np.float64)


def haar_orthogonal(d: int, rng: np.random.Generator) -> np.ndarray:
    """Random orthogonal matrix from the Haar measure: QR of a Gaussian matrix
    with the signs of R's diagonal moved into Q (Mezzadri 2007)."""
    a = rng.standard_normal((d, d))
    q, r = np.linalg.qr(a)
    return q * np.sign(np.diag(r))[None, :]


def correlated_gaussian_params(d: int, rng: np.random.Generator, mean_range=1.0,
                               log_eig_lo=math.log(1e-2), log_eig_hi=0.0):
    """Covariance Q diag(lambda) Q^T with log-uniform eigenvalues; returns the
    parameter block (mu, precision P = Q diag(1/lambda) Q^T, log det P) and the
    eigenvalues."""
    q = haar_orthogonal(d, rng)
    lam = np.exp(rng.uniform(log_eig_lo, log_eig_hi, size=d))
    mu = rng.uniform(-mean_range, mean_range, size=d)
    prec = (q / lam[None, :]) @ q.T
    prec = 0.5 * (prec + prec.T)
    logdet = float(-np.sum(np.log(lam)))
    return np.concatenate([mu, prec.ravel(), [logdet]]), lam


# ---------------------------------------------------------------------------
# The five workloads.
# ---------------------------------------------------------------------------

def config_gauss2d(seed: int = 2100, **kw) -> RunConfig:
    """Plain FP64 method: d=2 Gaussian N((.5,.5), .05^2 I) on [0,1]^2,
    n_live=100, 20-step walks, stop when the remaining evidence < 1e-3."""
    prm = gauss_diag_params([0.5, 0.5], [0.05, 0.05])
    base = dict(kind="gauss_diag", d=2, n_live=100, params=prm, lo=0.0, hi=1.0,
                precision="fp64", n_steps_max=20, max_ref=0, seed=seed,
                name="gauss_d2_nlive100_fp64")
    base.update(kw)
    return RunConfig(**base)


def config_shells(d: int = 32, n_live: int = 1000, seed: int = 2200, **kw) -> RunConfig:
    """Two Gaussian shells, radius 2, width 0.1, centres +-3.5 on axis 0, prior
    [-6,6]^d, FP32 walks of 5*d steps."""
    c0 = np.zeros(d); c0[0] = 3.5
    c1 = np.zeros(d); c1[0] = -3.5
    prm = shells_params([c0, c1], 2.0, 0.1)
    base = dict(kind="shells", d=d, n_live=n_live, params=prm, lo=-6.0, hi=6.0,
                n_comp=2, precision="fp32", n_steps_max=5 * d, max_ref=0, seed=seed,
                name=f"shells_d{d}_nlive{n_live}_fp32")
    base.update(kw)
    return RunConfig(**base)


def config_corr_gauss(d: int = 256, n_live: int = 2000, seed: int = 2300,
                      param_seed: int = 1003, precision: str = "bf16mma", **kw) -> RunConfig:
    """Correlated Gaussian: covariance Q diag(lambda) Q^T, lambda log-uniform in
    [1e-2, 1], mean U[-1,1]^d, prior [-10,10]^d; min_ref 1, max_ref 3, cap 5d."""
    rng = np.random.default_rng(param_seed)
    prm, _ = correlated_gaussian_params(d, rng)
    base = dict(kind="gauss_full", d=d, n_live=n_live, params=prm, lo=-10.0, hi=10.0,
                precision=precision, n_steps_max=5 * d, min_ref=1, max_ref=3, seed=seed,
                name=f"corr_gauss_d{d}_nlive{n_live}_{precision}")
    base.update(kw)
    return RunConfig(**base)


def config_gmm(d: int = 64, n_live: int = 4000, n_comp: int = 8, seed: int = 2400,
               param_seed: int = 1004, **kw) -> RunConfig:
    """Equal-weight diagonal mixture: means U[-5,5]^d, sigmas U[0.05, 0.2],
    prior [-8,8]^d; FP32 walks, min_ref 1, max_ref 3, cap 5d."""
    rng = np.random.default_rng(param_seed)
    mus = [rng.uniform(-5.0, 5.0, size=d) for _ in range(n_comp)]
    sgs = [rng.uniform(0.05, 0.2, size=d) for _ in range(n_comp)]
    prm = gmm_params(mus, sgs)
    base = dict(kind="gmm_diag", d=d, n_live=n_live, params=prm, lo=-8.0, hi=8.0,
                n_comp=n_comp, precision="fp32", n_steps_max=5 * d, min_ref=1,
                max_ref=3, seed=seed, name=f"gmm{n_comp}_d{d}_nlive{n_live}_fp32")
    base.update(kw)
    return RunConfig(**base)


def config_torus(d: int = 32, n_live: int = 500, alpha: int = 2, beta: int = 3, c=None,
                 seed: int = 2600, **kw) -> RunConfig:
    """Torus reward (Eq. torus) on the prior box [0, 2 pi)^d with integer
    frequencies alpha = 2, beta = 3 and c = d + 1 (the smallest integer with a
    positive reward everywhere; the paper states neither); FP32 walks with the
    paper's walk defaults (min_ref 1, max_ref 3), cap max(64, 5d)."""
    cc = float(d + 1) if c is None else float(c)
    base = dict(kind="torus", d=d, n_live=n_live, params=torus_params(alpha, beta, cc), lo=0.0,
                hi=2.0 * math.pi, precision="fp32", n_steps_max=max(64, 5 * d), min_ref=1,
                max_ref=3, seed=seed, name=f"torus_d{d}_nlive{n_live}_a{alpha}b{beta}")
    base.update(kw)
    return RunConfig(**base)


def config_batch(n_runs: int = 64, table_seed: int = 5005, dims=(8, 16, 32, 64, 128),
                 n_live_range=(200, 2000), corr_precision: str = "bf16mma") -> List[RunConfig]:
    """Table of uneven runs: d from `dims`, n_live uniform in n_live_range (even),
    kind drawn from correlated Gaussian, shells and mixture, each with its own
    walk rules (shells: fixed 5d steps; the others: min_ref 1, max_ref 3), with
    per-run parameter seeds 6000 + j and run seeds 7000 + j."""
    rng = np.random.default_rng(table_seed)
    runs = []
    kinds = ["gauss_full", "shells", "gmm_diag"]
    for j in range(n_runs):
        d = int(rng.choice(dims))
        n_live = 2 * int(rng.integers(n_live_range[0] // 2, n_live_range[1] // 2 + 1))
        kind = kinds[int(rng.integers(0, 3))]
        if kind == "gauss_full":
            cfg = config_corr_gauss(d=d, n_live=n_live, seed=7000 + j, param_seed=6000 + j,
                                    precision=corr_precision)
        elif kind == "shells":
            cfg = config_shells(d=d, n_live=n_live, seed=7000 + j)
        else:
            cfg = config_gmm(d=d, n_live=n_live, seed=7000 + j, param_seed=6000 + j)
        cfg.name = f"batch{j}_{cfg.name}"
        runs.append(cfg)
    return runs


def replicate(cfg: RunConfig, n: int, base_seed: int) -> List[RunConfig]:
    """The paper's protocol of repeated runs (10 in Sections 4.1 and 4.2):
    identical problems, seeds base_seed + r."""
    return [cfg.replace(seed=base_seed + r, name=f"{cfg.name}_r{r}") for r in range(n)]


def uniform_points(n: int, d: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Seeded uniform points in a box (test inputs, point-major [n, d])."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, d))


def ball_points(n: int, d: int, centre, radius: float, seed: int) -> np.ndarray:
    """Seeded points uniform in a d-ball (test inputs for a fixed slice)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, d))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = radius * rng.uniform(0.0, 1.0, size=(n, 1)) ** (1.0 / d)
    return np.asarray(centre, np.float64)[None, :] + r * v
