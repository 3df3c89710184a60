"""Tile-shape autotuner of the walk kernels.

The vector-ALU walk gives each walker a group of G lanes with C coordinates
per lane (G = next power of two of ceil(d / C)).  Fewer coordinates per lane
means more lanes per step and more wavefronts to hide latency with, but a
longer reduction butterfly and more redundant stream work; the best C depends
on the family, the dimension, the precision and on how many walkers the batch
holds.  The matrix-core walk shares a group of 16 walkers between W wavefronts
(dp / 4W dimensions per lane): more wavefronts spread the per-coordinate work
but read the residuals from LDS once each and meet at more barriers.
The tuner times the walk of each group of like runs (same family, precision,
dimension and component count) for every admissible C on the batch itself and
keeps the fastest.  Results are independent of C up to floating-point
summation order (the random streams are per coordinate block, not per lane).
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

from .inputs import RunConfig

_CACHE: Dict[Tuple, int] = {}


def candidates(cfg: RunConfig) -> List[int]:
    """Tile shapes the library accepts for this run.  Vector-ALU runs:
    coordinates per lane (1, 2, 4, 8), leaving out shapes whose lanes would
    hold padding only.  Matrix-core runs: wavefronts per group of 16 walkers
    giving 16, 8 or 4 dimensions per lane."""
    from . import _lib
    from .engine import make_descs
    L = _lib.load()

    def ok(t):
        descs, _ = make_descs([cfg], [t])
        return L.ggns_arena_bytes(descs, 1) > 0

    if cfg.precision == "bf16mma":
        dp = (cfg.d + 31) // 32 * 32
        return [w for w in (dp // 64, dp // 32, dp // 16) if w >= 1 and ok(w)]
    out = []
    for c in (1, 2, 4, 8):
        g = 1
        while g * c < cfg.d:
            g *= 2
        if c > 1 and g == 1 and c >= 2 * cfg.d:
            continue        # lanes of padding only
        if ok(c):
            out.append(c)
    return out


def _group_key(cfg: RunConfig) -> Tuple:
    return (cfg.kind, cfg.precision, cfg.d, cfg.n_comp, cfg.max_ref, cfg.n_steps_max)


def _time_walk(cfgs: Sequence[RunConfig], c, warm: int, reps: int, device: str):
    """Mean walk launch time (ms) after `warm` iterations with tile shape `c`
    (one for all runs, or a list), or None when a run ends before the timed
    walks are over (nothing comparable to time)."""
    import torch

    from . import _lib
    from .engine import Engine
    tiles = list(c) if isinstance(c, (list, tuple)) else [c] * len(cfgs)
    eng = Engine(cfgs, device=device, tile_c=tiles)
    eng.iterate(warm)
    stream = torch.cuda.current_stream(eng.device)
    t = 0.0
    for _ in range(reps):
        eng.evidence_update()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        eng.hss_walk()
        b.record(stream)
        eng.replace_dead()
        b.synchronize()
        t += a.elapsed_time(b)
    ended = any(s["state"] != _lib.RUN_ACTIVE for s in eng.stats())
    eng.close()
    return None if ended else t / reps


def _time_pass(cfgs: Sequence[RunConfig], tiles: Sequence[int], device: str) -> float:
    """Wall time (s) of one whole pass of the batch (every run to its stop) with
    the given tile shapes, run as the benchmark runs it: blocks of iterations
    replayed as one captured graph.  A first pass captures the graph and loads
    the kernels; the second, on the re-initialised arena, is timed."""
    import time

    import torch

    from .engine import Engine
    eng = Engine(cfgs, device=device, tile_c=list(tiles))
    eng.run(use_graph=True)
    eng.reset()
    torch.cuda.synchronize(eng.device)
    t0 = time.perf_counter()
    eng.run(use_graph=True)
    torch.cuda.synchronize(eng.device)
    t = time.perf_counter() - t0
    eng.close()
    return t


def tune(configs: Sequence[RunConfig], device: str = "cuda", warm: int = 2, reps: int = 3,
         verbose: bool = False, warm_reflect: int = 30) -> List[int]:
    """Coordinates per lane for every run of the batch (0 = library default).

    Fixed-step groups are timed after `warm` iterations.  Reflection-mode groups
    (max_ref > 0) are timed after `warm_reflect`: in their first iterations the
    step is still far too large, every walker meets its reflections within a
    few steps, and walks of that length favour other tile shapes than the
    adapted walks that make up the run."""
    groups: Dict[Tuple, List[int]] = {}
    for i, c in enumerate(configs):
        groups.setdefault(_group_key(c), []).append(i)
    choice = [0] * len(configs)
    for key, idx in groups.items():
        sub = [configs[i] for i in idx]
        cands = candidates(sub[0])
        ckey = key + (len(sub), sum(c.n_live for c in sub))
        if ckey not in _CACHE:
            if len(cands) <= 1:
                _CACHE[ckey] = cands[0] if cands else 0
            else:
                w = warm if sub[0].max_ref == 0 else max(warm, warm_reflect)
                times = {c: _time_walk(sub, c, w, reps, device) for c in cands}
                if any(t is None for t in times.values()):
                    _CACHE[ckey] = 0    # runs too short to time: the library default
                else:
                    _CACHE[ckey] = min(times, key=times.get)
                if verbose:
                    print("autotune", key, {c: (None if t is None else round(t, 4)) for c, t in times.items()},
                          "->", _CACHE[ckey], flush=True)
        for i in idx:
            choice[i] = _CACHE[ckey]
    if len(groups) > 1 and any(choice):
        # the groups were timed alone; in the batch their walks share the chip,
        # where fewer, fuller wavefronts can win, and the walks' lengths change
        # as the runs go on.  Keep the per-group choices only if whole passes
        # of the batch (the best of two each, interleaved) are faster with them
        # than with the library defaults
        default = [0] * len(configs)
        t_tuned = t_default = float("inf")
        for _ in range(2):
            t_tuned = min(t_tuned, _time_pass(configs, choice, device))
            t_default = min(t_default, _time_pass(configs, default, device))
        if verbose:
            print("autotune batch: tuned", t_tuned, "default", t_default, flush=True)
        if t_default <= 1.02 * t_tuned:
            return default
    return choice
