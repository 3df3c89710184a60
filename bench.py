"""Benchmark: likelihood+gradient evaluations per second of the batched HSS walk.

One step = one whole nested-sampling pass over the workload's batch of runs:
init (prior draws), iterations of evidence_update -> hss_walk -> replace_dead
until every run has stopped, final sweep and run summary.  Inputs are
synthetic and seeded; the closed-form log Z of every run is reported next to
the estimate.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2312_03911_amd import exact, inputs  # noqa: E402

PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "bf16mma": 2500.0}

# HBM bytes per walk launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# (KiB per dispatch, averaged over the launches that did work, as the launch
# duration is), each scaled by what the counter reads for a device copy of
# known size (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0), with the hash of the kernel
# sources they were taken on; reported only while the sources still hash the same
TRAFFIC = {"shells32x10": {"bytes": (645.69 * 2.0 + 702.86) * 1024,
                            "sources_sha1": "2a3497947888d4c7ec846b4c1314a9dc25e7cf48"}}


def traffic_for(workload: str):
    import hashlib
    t = TRAFFIC.get(workload)
    if t is None:
        return None
    csrc = os.path.join(ROOT, "paper_2312_03911_amd", "csrc")
    blob = b"".join(open(os.path.join(csrc, f), "rb").read()
                    for f in ("walk_valu.hip", "ggns_device.h"))
    return t["bytes"] if hashlib.sha1(blob).hexdigest() == t["sources_sha1"] else None


def workload(name: str):
    if name == "shells32x10":
        # Gaussian shells d=32, n_live=1000, FP32, 5d-step walks; the paper's
        # protocol of 10 runs per setting, batched into one launch
        return inputs.replicate(inputs.config_shells(d=32, n_live=1000), 10, base_seed=2200)
    if name == "shells32":
        return [inputs.config_shells(d=32, n_live=1000)]
    if name == "shells32x100":
        # the same problem, 100 seeded runs in one batch: 50,000 walkers, enough
        # wavefronts to fill every SIMD several times over (the batched form at
        # full occupancy; the default keeps the paper's 10-run protocol)
        return inputs.replicate(inputs.config_shells(d=32, n_live=1000), 100, base_seed=2200)
    if name == "gauss2d":
        return [inputs.config_gauss2d()]
    if name == "gauss2dx10":
        return inputs.replicate(inputs.config_gauss2d(), 10, base_seed=2100)
    if name == "gmm64":
        return [inputs.config_gmm()]
    if name == "gmm64_clusters":
        # the same mixture with cluster recognition and volume-proportional spawning
        return [inputs.config_gmm(cluster=1)]
    if name == "gmm64_clusters_x10":
        return inputs.replicate(inputs.config_gmm(cluster=1), 10, base_seed=2400)
    if name == "corr256":
        return [inputs.config_corr_gauss()]
    if name == "corr256x10":
        # the paper's 10-run protocol for the d=256 correlated Gaussian, one batch
        return inputs.replicate(inputs.config_corr_gauss(), 10, base_seed=2300)
    if name == "gmm64x10":
        return inputs.replicate(inputs.config_gmm(), 10, base_seed=2400)
    if name == "batch64":
        return inputs.config_batch()
    if name == "torus_sweep":
        # the torus reward (Eq. torus) at d = 2 ... 128, c = d + 1, alpha = 2,
        # beta = 3, n_live 500, 10 runs per d, all in one batch
        out = []
        for d in (2, 4, 8, 16, 32, 64, 128):
            out += inputs.replicate(inputs.config_torus(d=d, n_live=500), 10, base_seed=9000 + 100 * d)
        return out
    if name.startswith("gauss_sweep"):
        # the dimension sweep of the paper's comparison (diagonal Gaussian,
        # n_live = 200 at every d, 10 runs each): the d=2 Gaussian's family,
        # mean 0.5 and width 0.05 per axis in the unit box, FP32 walks with the
        # paper's default walk settings.  Termination at tol 0.01 by the X L
        # peak with L the largest live likelihood (gauss_sweep), with L the dead
        # point's (gauss_sweep_dead), or by the remaining evidence
        # (gauss_sweep_classic); ablations of the last: a fixed step of 0.1 or
        # 0.5 prior widths (_dt01, _dt05), no momentum noise (_dp0)
        parts = name.split("_")[2:]
        term = 1
        kw = {}
        for p_ in parts:
            if p_ == "dead":
                term = 2
            elif p_ == "classic":
                term = 0
            elif p_ in ("dt01", "dt05"):
                kw.update(dt_init=0.1 if p_ == "dt01" else 0.5, dt_up=1.0, dt_down=1.0)
            elif p_ == "dp0":
                kw.update(delta_p=0.0)
            else:
                raise SystemExit(f"unknown workload {name}")
        out = []
        for d in (2, 4, 8, 16, 32, 64, 128):
            base = inputs.RunConfig(kind="gauss_diag", d=d, n_live=200, lo=0.0, hi=1.0,
                                    params=inputs.gauss_diag_params(np.full(d, 0.5), np.full(d, 0.05)),
                                    precision="fp32", term_kind=term, term_tol=0.01,
                                    n_steps_max=max(64, 5 * d), name=f"gauss_d{d}", **kw)
            out += inputs.replicate(base, 10, base_seed=8000 + 100 * d)
        return out
    raise SystemExit(f"unknown workload {name}")


def valu_flops_per_eval(cfg, out_frac: float) -> float:
    """Algorithmic vector-ALU FP operations of one walker step, the normals
    excluded (they are costed at the generator's measured rate): drift, log L
    and score, reflection on outside steps, p *= 1 + delta_p eps.  For matrix-
    core runs the contraction P r is left out here (it is the MFMA term)."""
    d, K = cfg.d, cfg.n_comp
    drift = 2 * d
    if cfg.kind == "gauss_diag":
        lik = 4 * d + 2
    elif cfg.kind == "shells":
        lik = 5 * K * d + 10 * K
    elif cfg.kind == "gmm_diag":
        lik = 7 * K * d + 10 * K
    elif cfg.kind == "torus":
        # per coordinate: argument (FMA), sine and cosine (one each), f cos, the
        # sum, p.(f cos) and |f cos|^2 (FMAs), the score; log and quotient
        lik = 11 * d + 10
    elif cfg.precision == "bf16mma":
        lik = 3 * d + 2
    else:
        lik = 2 * d * d + 3 * d + 2
    reflect = 6 * d * out_frac
    noise = 2 * d
    return drift + lik + reflect + noise


def mfma_flops_per_eval(cfg) -> float:
    return 2.0 * cfg.d * cfg.d if cfg.precision == "bf16mma" else 0.0


def rng_rate(torch, L) -> float:
    """Normals per second of the walk's noise generator (xoshiro128++ words,
    FP32 Box-Muller) alone at full occupancy: 2^20 threads, 512 steps."""
    import ctypes as C
    W, B, T = 1 << 16, 16, 512
    cs = torch.empty(W * B, dtype=torch.float32, device="cuda:0")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    L.ggns_noise_normals(1, 0, W, B, 8, None, None, cs.data_ptr(), s)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    best = 0.0
    for _ in range(3):
        a.record()
        rc = L.ggns_noise_normals(1, 0, W, B, T, None, None, cs.data_ptr(), s)
        b.record()
        b.synchronize()
        if rc != 0:
            raise RuntimeError("ggns_noise_normals failed")
        best = max(best, W * B * T * 4 / (a.elapsed_time(b) / 1e3))
    return best


def probe_rates(torch, L) -> dict:
    """TFLOP/s this build reaches on the vector ALU (FP32 FMA chains, one FMA
    per lane and instruction, as the walks are compiled) and on the BF16 matrix
    cores (the walk's 16x16x32 MFMA), at eight wavefronts per SIMD: best of
    three launches of ggns_probe_valu / ggns_probe_mfma after a warm-up."""
    import ctypes as C
    blocks = 2048
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda:0")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {}
    for name, fn, iters, flop_per_round in (
            ("valu_fp32_fma", L.ggns_probe_valu, 4096, blocks * 256 * 16.0),
            ("mfma_bf16", L.ggns_probe_mfma, 2048, blocks * 4 * 4 * 16384.0)):
        if fn(blocks, 8, 0.5, 0.25, out.data_ptr(), s) != 0:
            raise RuntimeError(f"{name} probe failed")
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        best = 0.0
        for _ in range(3):
            a.record()
            fn(blocks, iters, 0.5, 0.25, out.data_ptr(), s)
            b.record()
            b.synchronize()
            best = max(best, flop_per_round * iters / (a.elapsed_time(b) / 1e3) / 1e12)
        res[name] = best
    return res


def _oracle_sample(O, cfgs, budget_s: float):
    """The workload's runs in order (cycling if they finish early) until the
    budget is used; a run cut by the budget counts the iterations it did.
    Returns evaluations, whole runs, iterations, the cut run's note, seconds
    and (index, log Z) of every whole run."""
    t0 = time.perf_counter()
    ev, whole, its, j = 0, 0, 0, 0
    last, done = "", []
    while time.perf_counter() - t0 < budget_s:
        cfg = cfgs[j % len(cfgs)]
        o = O.Oracle(cfg).init()
        it = 0
        while o.active and time.perf_counter() - t0 < budget_s:
            o.iterate()
            it += 1
        if not o.active:
            whole += 1
            if j < len(cfgs):
                done.append((j, float(o.st.lz)))
        else:
            last = f" + {it} iterations of {cfg.name}"
        ev += o.st.evals
        its += it
        j += 1
    return ev, whole, its, last, time.perf_counter() - t0, done


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfgs, budget_s: float = 12.0, budget_single_s: float = 6.0):
    """The oracle on the host cores (OpenMP over walkers, every thread), on a
    bounded sample of the workload, and single-threaded on a shorter one (its
    results are identical: the random streams are counter-based)."""
    import oracle.oracle as O
    cores = O.num_threads()
    ev, whole, its, last, dt, done = _oracle_sample(O, cfgs, budget_s)
    O.set_threads(1)
    ev1, _, its1, _, dt1, _ = _oracle_sample(O, cfgs, budget_single_s)
    O.set_threads(cores)
    return {"value": ev / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{whole} whole runs{last} of the workload ({its} iterations, "
                      f"{ev} evaluations) in {dt:.1f} s",
            "single_thread_value": ev1 / dt1,
            "single_thread_sample": f"{its1} iterations, {ev1} evaluations in {dt1:.1f} s",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "whole_runs_log_z": done}


def plain_baseline(cfgs, fused_value: float, fused_ms_per_run: float, fused_stats, truth,
                   budget_s: float = 20.0):
    """The plain FP64 GPU method (one thread per walker, one launch per step,
    state in HBM, runs one after another) on the workload's runs switched to
    FP64, as many whole runs as fit the budget; its log Z next to the fused
    FP32 estimate of the same runs."""
    import torch

    from paper_2312_03911_amd.engine import Engine
    evals, secs, dz, dfz = 0, 0.0, [], []
    n = 0
    for j, c in enumerate(cfgs):
        if secs > budget_s:
            break
        eng = Engine([c.replace(precision="fp64")], device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = eng.run(poll_every=8, plain=True)[0]
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        eng.close()
        evals += st["evals"]
        dz.append(st["log_z"] - truth[j])
        dfz.append(st["log_z"] - fused_stats[j]["log_z"])
        n += 1
    value = evals / secs
    return {"value": value, "unit": "evals/s", "kind": "plain FP64 per-step GPU walk",
            "runs": n, "ms_per_run": 1e3 * secs / n, "fused_ms_per_run": fused_ms_per_run,
            "speedup": fused_value / value,
            "logz_minus_closed_form_mean": float(np.mean(dz)),
            "logz_minus_fused_mean": float(np.mean(dfz)),
            "logz_minus_fused_sd": float(np.std(dfz))}


def sweep_report(cfgs, stats, truth) -> dict:
    """Mean evaluations, log Z error and sigma_KL of the runs of each dimension,
    and the log-log slope of evaluations against d."""
    by_d = {}
    for c, st_, t in zip(cfgs, stats, truth):
        by_d.setdefault(c.d, []).append((st_["evals"], st_["log_z"] - t, st_["sigma_kl"]))
    ds = sorted(by_d)
    col = lambda j, f: [float(f([v[j] for v in by_d[d]])) for d in ds]  # noqa: E731
    ev = col(0, np.mean)
    return {"d": ds, "evals_mean": ev,
            "logz_minus_closed_form_mean": col(1, np.mean),
            "logz_minus_closed_form_sd": col(1, np.std),
            "sigma_kl_mean": col(2, np.mean),
            "loglog_slope_evals_vs_d": float(np.polyfit(np.log(ds), np.log(ev), 1)[0])}


def run_environment(torch) -> dict:
    """Versions, the device and its current shader and memory clock levels,
    read from the driver's sysfs tables (the level marked '*'; no child
    process, so nothing runs under a profiler's preloaded library)."""
    import glob
    env = {"torch": torch.__version__, "hip": getattr(torch.version, "hip", None),
           "device": torch.cuda.get_device_name(0)}
    clocks = []
    for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
        for name in ("pp_dpm_sclk", "pp_dpm_mclk"):
            try:
                with open(os.path.join(dev, name)) as f:
                    cur = [ln.strip() for ln in f if ln.strip().endswith("*")]
            except OSError:
                continue
            if cur:
                clocks.append(f"{os.path.basename(os.path.dirname(dev))} {name[-4:]}: {cur[0]}")
    env["clocks"] = clocks or None
    return env


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="shells32x10")
    ap.add_argument("--poll", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-alt", action="store_true",
                    help="skip the untimed pass under the per-walker noise reading")
    ap.add_argument("--launch", default="graph", choices=["graph", "eager"],
                    help="throughput passes: each block of --poll iterations replayed as one captured "
                         "HIP graph, or launched kernel by kernel")
    ap.add_argument("--tile", default="auto", choices=["auto", "default"],
                    help="walk tile shape: autotuned per group of like runs, or the library default")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device a few times (the reference kernel "
                         "that scales HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": n, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        raise SystemExit(2)

    import torch

    from paper_2312_03911_amd.engine import Engine

    cfgs = workload(args.workload)
    truth = [exact.log_z(c) for c in cfgs]
    tile_c = None
    if args.tile == "auto":
        from paper_2312_03911_amd.autotune import tune
        tile_c = tune(cfgs, device="cuda:0", verbose=True)
    eng = Engine(cfgs, device="cuda:0", tile_c=tile_c)
    shapes = sorted({eng.tile_shape(r) for r in range(len(cfgs))})
    stream = torch.cuda.current_stream()

    walk_ms = []

    def full_run(record: bool):
        # re-initialise every run on the same arena, then iterate to the end:
        # blocks of `poll` iterations, the runs' states copied back after each
        # block and read one block later, so the stream never drains between
        # blocks (the block enqueued after the last run stopped is no-ops)
        from paper_2312_03911_amd import _lib
        eng.reset()
        evs = []
        pending, b = None, 0
        while True:
            if args.launch == "graph" and not record:
                # the block as one captured graph (captured once: every pass
                # re-initialises the same arena, so the launches' arguments,
                # all inside the arena, stay valid)
                eng.step_block(args.poll, use_graph=True)
                nxt = eng.states_async(b & 1)
                b += 1
                if pending is not None and (pending() != _lib.RUN_ACTIVE).all():
                    break
                pending = nxt
                continue
            for _ in range(args.poll):
                eng.evidence_update()
                if record:
                    a = torch.cuda.Event(enable_timing=True)
                    e = torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    eng.hss_walk()
                    e.record(stream)
                    evs.append((a, e))
                else:
                    eng.hss_walk()
                eng.replace_dead()
            nxt = eng.states_async(b & 1)
            b += 1
            if pending is not None and (pending() != _lib.RUN_ACTIVE).all():
                break
            pending = nxt
        eng.finalize()
        st = eng.stats()
        for a, e in evs:
            walk_ms.append(a.elapsed_time(e))
        return st

    for _ in range(args.warmup):
        full_run(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    pass_ms = []
    for _ in range(args.steps):
        t1 = time.perf_counter()
        stats = full_run(False)      # ends by reading the stats: the pass is complete
        pass_ms.append(1e3 * (time.perf_counter() - t1))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the same passes again with HIP events around every walk launch, for the
    # walk kernel's launch durations (kept out of the throughput figure: each
    # event adds a few microseconds between launches)
    for _ in range(args.steps):
        full_run(True)
    torch.cuda.synchronize()

    evals = sum(s["evals"] for s in stats)
    ms_per_step = 1e3 * elapsed / args.steps
    value = evals * args.steps / elapsed
    # roofline of the walk: the time its algorithmic work needs at the chip's
    # peaks (vector-ALU FP operations at the FP32 or FP64 vector peak, normals at
    # the generator's measured rate, the BF16 contraction at the matrix-core
    # peak; per run the larger of the vector and matrix terms, summed over runs)
    # over the measured walk time
    steps_total = sum(s["steps_out"] + s["steps_in"] for s in stats)
    out_frac = sum(s["steps_out"] for s in stats) / max(steps_total, 1)
    r_rng = rng_rate(torch, eng.L)
    reach = probe_rates(torch, eng.L)
    t_valu = t_mfma = t_bound = t_reach = 0.0
    flops_valu = flops_mfma = normals = 0.0
    for c, s in zip(cfgs, stats):
        e = s["steps_out"] + s["steps_in"]
        fo = s["steps_out"] / max(e, 1)
        fv, fm = valu_flops_per_eval(c, fo) * e, mfma_flops_per_eval(c) * e
        pv = PEAK_TFLOPS["fp64" if c.precision == "fp64" else "fp32"] * 1e12
        rr = r_rng / 2 if c.precision == "fp64" else r_rng
        tv = fv / pv + c.d * e / rr
        tm = fm / (PEAK_TFLOPS["bf16mma"] * 1e12)
        t_valu += tv
        t_mfma += tm
        t_bound += max(tv, tm)
        # the same bound at the rates the probes reach (FP32 vector and BF16
        # matrix cores; FP64 runs keep the published vector peak)
        pv_r = pv if c.precision == "fp64" else reach["valu_fp32_fma"] * 1e12
        t_reach += max(fv / pv_r + c.d * e / rr, fm / (reach["mfma_bf16"] * 1e12))
        flops_valu += fv
        flops_mfma += fm
        normals += c.d * e
    # only launches that did work (the trailing polled iterations of finished runs are no-ops)
    n_launch_work = max(1, max(s["iter"] for s in stats)) * args.steps
    wm = sorted(walk_ms, reverse=True)[:n_launch_work]
    walk_time_s = sum(wm) / 1e3 / args.steps
    prec = cfgs[0].precision
    frac = t_bound / walk_time_s
    bound = "mfma" if t_mfma > t_valu else "alu"
    peak = PEAK_TFLOPS["bf16mma"] if bound == "mfma" else \
        PEAK_TFLOPS["fp64" if all(c.precision == "fp64" for c in cfgs) else "fp32"]
    achieved = frac * peak
    dz = [s["log_z"] - t for s, t in zip(stats, truth)]
    zs = [d / max(s["sigma_kl"], 1e-12) for d, s in zip(dz, stats)]
    res = {
        "metric": "likelihood+grad evals/sec in HSS walks at stated logZ error; roofline fraction",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "runs": len(cfgs),
                   "d": sorted({c.d for c in cfgs}), "n_live": sorted({c.n_live for c in cfgs}),
                   "kinds": sorted({c.kind for c in cfgs}), "precision": sorted({c.precision for c in cfgs}),
                   "evals_per_step": evals, "iterations": [s["iter"] for s in stats][:16],
                   "tile": {"mode": args.tile, "coords_per_lane_x_lanes": shapes},
                   "launch": args.launch},
        "pass_ms": {"median": float(np.median(pass_ms)),
                    "iqr": float(np.percentile(pass_ms, 75) - np.percentile(pass_ms, 25)),
                    "min": float(np.min(pass_ms)), "max": float(np.max(pass_ms))},
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": frac, "traffic": traffic_for(args.workload),
                     "frac_resources_overlapped": max(t_valu, t_mfma) / walk_time_s,
                     "kernel": ("walk_mfma_kernel" if bound == "mfma" or
                                all(c.precision == "bf16mma" for c in cfgs) else "walk_valu_kernel"),
                     "walk_ms_per_step": 1e3 * walk_time_s,
                     "walk_launch_us": 1e6 * walk_time_s / max(1, n_launch_work // args.steps),
                     "walk_evals_per_s": steps_total / walk_time_s, "out_frac": out_frac,
                     "valu_flops_per_step": flops_valu, "mfma_flops_per_step": flops_mfma,
                     "normals_per_step": normals, "normals_per_s_peak": r_rng,
                     "t_bound_ms": 1e3 * t_bound, "t_valu_ms": 1e3 * t_valu,
                     "t_mfma_ms": 1e3 * t_mfma,
                     "probe_tflops": reach,
                     "frac_of_probed_rates": t_reach / walk_time_s},
        "accuracy": {"noise": "per component",
                     "logz_minus_closed_form_mean": float(np.mean(dz)),
                     "logz_minus_closed_form_sd": float(np.std(dz)),
                     "z_scores_max_abs": float(np.max(np.abs(zs))),
                     "sigma_kl_mean": float(np.mean([s["sigma_kl"] for s in stats])),
                     "sigma_mom_mean": float(np.mean([s["sigma_mom"] for s in stats]))},
    }
    # evaluations and log Z error against dimension (the sweep workloads)
    if args.workload.startswith("gauss_sweep") or args.workload == "torus_sweep":
        res["dimension_sweep"] = sweep_report(cfgs, stats, truth)
    # mode recovery of the mixture runs (one untimed pass with the dead points'
    # positions kept)
    if not args.no_alt and any(c.kind == "gmm_diag" for c in cfgs):
        from paper_2312_03911_amd.posterior import gmm_mode_report, normalized_log_weights
        eng.close()
        me = Engine(cfgs, device="cuda:0", tile_c=tile_c)
        idx = [i for i, c in enumerate(cfgs) if c.kind == "gmm_diag"]
        for i in idx:
            me.keep_dead_x(i)
        st_m = me.run(poll_every=args.poll)
        reps = []
        for i in idx:
            dl, dw = me.dead(i)
            reps.append(gmm_mode_report(me.dead_x(i).cpu().numpy(),
                                        normalized_log_weights(dl.cpu().numpy(), dw.cpu().numpy(),
                                                               st_m[i]["log_z"]), cfgs[i]))
        me.close()
        res["accuracy"]["modes"] = {
            "runs": len(reps), "recovered": sum(r["recovered"] for r in reps),
            "of": sum(r["modes"] for r in reps),
            "weight_max_abs_err": max(r["weight_max_abs_err"] for r in reps),
            "weights_run0": [round(w, 4) for w in reps[0]["weights"]]}
    # the same workload under the other reading of the momentum noise (one
    # normal per walker and step), one untimed pass: its log Z against the
    # closed form
    if not args.no_alt:
        eng.close()
        alt = Engine([c.replace(noise="walker") for c in cfgs], device="cuda:0", tile_c=tile_c)
        st_alt = alt.run(poll_every=args.poll)
        alt.close()
        dza = [s_["log_z"] - t for s_, t in zip(st_alt, truth)]
        if args.workload.startswith("gauss_sweep") or args.workload == "torus_sweep":
            res["dimension_sweep_walker_noise"] = sweep_report(cfgs, st_alt, truth)
        res["accuracy_walker_noise"] = {
            "noise": "one normal per walker and step",
            "logz_minus_closed_form_mean": float(np.mean(dza)),
            "logz_minus_closed_form_sd": float(np.std(dza)),
            "logz_minus_closed_form_sem": float(np.std(dza) / math.sqrt(max(1, len(dza) - 1))),
            "sigma_kl_mean": float(np.mean([s_["sigma_kl"] for s_ in st_alt])),
            "evals": int(sum(s_["evals"] for s_ in st_alt))}
    if not args.no_plain and all(c.kind != "gauss_full" for c in cfgs):
        res["plain_baseline"] = plain_baseline(cfgs, value, ms_per_step / len(cfgs), stats,
                                               truth)
    if not args.no_cpu:
        cb = cpu_baseline(cfgs)
        done = cb.pop("whole_runs_log_z")
        res["cpu_baseline"] = cb
        if done:
            # the same runs (same seeds) on the GPU against the FP64 oracle: FP32
            # trajectories part from FP64 ones, so this is a statistical comparison
            dzo = [stats[j]["log_z"] - lz for j, lz in done]
            res["accuracy"]["logz_minus_oracle"] = {"runs": len(dzo), "mean": float(np.mean(dzo)),
                                                    "max_abs": float(np.max(np.abs(dzo)))}
    res["env"] = run_environment(torch)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
