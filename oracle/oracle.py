"""Python handle on the FP64 C oracle (ns_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the CPU
baseline leg of bench.py, never by the GPU engine.  It imports nothing from the
engine package; run settings are read from any object carrying the RunConfig
attributes (kind_id, d, n_live, params, ...).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ns_oracle.c")
_LIB = os.path.join(_HERE, "libns_oracle.so")
_lock = threading.Lock()
_lib = None

ST_ACTIVE, ST_DONE, ST_MAXITER, ST_NONFINITE = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over walkers, no hand SIMD)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Desc(C.Structure):
    _fields_ = [("d", C.c_int32), ("n_live", C.c_int32), ("n_kill", C.c_int32),
                ("kind", C.c_int32), ("n_comp", C.c_int32), ("bf16", C.c_int32),
                ("lo", C.c_double), ("hi", C.c_double), ("dt_init", C.c_double),
                ("n_steps_max", C.c_int32), ("min_ref", C.c_int32), ("max_ref", C.c_int32),
                ("prune_streak", C.c_int32),
                ("delta_p", C.c_double), ("out_hi", C.c_double), ("out_lo", C.c_double),
                ("dt_down", C.c_double), ("dt_up", C.c_double),
                ("term_kind", C.c_int32), ("max_iter", C.c_int32),
                ("term_tol", C.c_double), ("seed", C.c_uint64),
                ("noise_mode", C.c_int32), ("cluster_mode", C.c_int32),
                ("cluster_kmax", C.c_int32), ("stop_mode", C.c_int32),
                ("save_mode", C.c_int32), ("draw_mode", C.c_int32), ("pad_desc", C.c_int32)]


_PD = C.POINTER(C.c_double)
_PI = C.POINTER(C.c_int32)


class _State(C.Structure):
    _fields_ = [("live_x", _PD), ("live_logl", _PD), ("dead_logl", _PD), ("dead_logw", _PD),
                ("dead_cap", C.c_int64), ("n_dead", C.c_int64),
                ("killed", _PI), ("surv", _PI), ("start", _PI),
                ("out_x", _PD), ("out_logl", _PD),
                ("lz", C.c_double), ("lx", C.c_double), ("lz2", C.c_double),
                ("lzx", C.c_double), ("lx2", C.c_double),
                ("lxl_max", C.c_double), ("dt", C.c_double), ("lstar", C.c_double),
                ("iter", C.c_int64), ("evals", C.c_int64), ("steps_out", C.c_int64),
                ("steps_in", C.c_int64), ("prunes", C.c_int64), ("nosave", C.c_int64),
                ("it_outs", C.c_int64), ("it_steps", C.c_int64),
                ("state", C.c_int32), ("pad", C.c_int32),
                ("h", C.c_double), ("sigma_kl", C.c_double), ("sigma_mom", C.c_double),
                ("trace_x", _PD), ("trace_logl", _PD), ("trace_out", _PI),
                ("trace_steps", C.c_int32), ("pad2", C.c_int32),
                ("label", _PI), ("clx", _PD), ("cn", _PI), ("surv_off", _PI), ("start_cl", _PI),
                ("n_clusters", C.c_int32), ("n_splits", C.c_int32),
                ("split_kmax", C.c_int32), ("kstop_max", C.c_int32),
                ("cm", _PD)]

CL_MAX = 64
CM_SIZE = 5 * CL_MAX + CL_MAX * CL_MAX


def stale() -> bool:
    """True when libns_oracle.so is missing or older than its source."""
    return not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)


def lib():
    """The compiled oracle.  It is never compiled here: a process that has
    started the GPU may not start a compiler, so a missing or stale library is
    an error (build it first with build(), or __graft_entry__.build())."""
    global _lib
    with _lock:
        if _lib is None:
            if stale():
                raise RuntimeError("oracle/libns_oracle.so is missing or older than ns_oracle.c: "
                                   "run __graft_entry__.build() (or oracle.oracle.build()) first")
            L = C.CDLL(_LIB)
            L.orc_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
            L.orc_xoshiro_next.argtypes = [C.POINTER(C.c_uint32)]
            L.orc_xoshiro_next.restype = C.c_uint32
            L.orc_box_muller4.argtypes = [C.POINTER(C.c_uint32), _PD]
            L.orc_loglike.argtypes = [C.c_int, C.c_int, _PD, C.c_int, _PD, _PD, _PD, C.c_int]
            L.orc_loglike.restype = C.c_int
            for fn in ("orc_init", "orc_hss_walk"):
                getattr(L, fn).argtypes = [C.POINTER(_Desc), _PD, C.POINTER(_State)]
            L.orc_run.argtypes = [C.POINTER(_Desc), _PD, C.POINTER(_State)]
            L.orc_evidence_update.argtypes = [C.POINTER(_Desc), C.POINTER(_State), C.c_int]
            L.orc_replace_dead.argtypes = [C.POINTER(_Desc), C.POINTER(_State)]
            L.orc_stream_words.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                           C.c_uint32, C.c_uint32, C.POINTER(C.c_uint32)]
            L.orc_round_bf16.argtypes = [C.c_double]
            L.orc_round_bf16.restype = C.c_double
            L.orc_moment_sequence.argtypes = [C.c_int, C.c_int, _PI, _PI, _PD, _PI, _PI, _PD]
            L.orc_moment_sequence.restype = C.c_int
            L.orc_num_threads.restype = C.c_int
            L.orc_set_threads.argtypes = [C.c_int]
            _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_PD)


def _ip(a):
    return a.ctypes.data_as(_PI)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ---------------------------------------------------------------- generators

def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def stream_words(seed, c0, c1, c2, tag, sub=0) -> np.ndarray:
    o = (C.c_uint32 * 4)()
    lib().orc_stream_words(C.c_uint64(seed), c0, c1, c2, tag, sub, o)
    return np.array(list(o), dtype=np.uint32)


def xoshiro_stream(state4, n: int) -> np.ndarray:
    s = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in state4])
    out = np.empty(n, dtype=np.uint32)
    for i in range(n):
        out[i] = lib().orc_xoshiro_next(s)
    return out


def box_muller4(words) -> np.ndarray:
    w = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in words])
    z = np.zeros(4)
    lib().orc_box_muller4(w, _dp(z))
    return z


def round_bf16(v: float) -> float:
    return float(lib().orc_round_bf16(float(v)))


# ---------------------------------------------------------------- likelihood

def loglike(cfg, x, bf16: bool = False):
    """log L and grad log L at points x [n, d] (FP64)."""
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    n, d = x.shape
    prm = np.ascontiguousarray(cfg.params, dtype=np.float64)
    logl = np.empty(n)
    grad = np.empty((n, d))
    L = lib()
    for i in range(n):
        rc = L.orc_loglike(cfg.kind_id, cfg.n_comp, _dp(prm), d, _dp(x[i]),
                           _dp(logl[i:i + 1]), _dp(grad[i]), int(bf16))
        if rc != 0:
            raise ValueError("oracle likelihood rejected its arguments")
    return logl, grad


def moment_sequence(n0: int, events) -> dict:
    """The cluster recursion (Eqs. update0-update9, new0-new6) over an event
    list: ("kill", p, logL), ("add", p), ("split", p, [counts...])."""
    typ, cl, lv, nco, cnts = [], [], [], [], []
    for ev in events:
        if ev[0] == "kill":
            typ.append(0); cl.append(ev[1]); lv.append(float(ev[2])); nco.append(0)
        elif ev[0] == "add":
            typ.append(1); cl.append(ev[1]); lv.append(0.0); nco.append(0)
        else:
            typ.append(2); cl.append(ev[1]); lv.append(0.0); nco.append(len(ev[2])); cnts.extend(ev[2])
    t = np.array(typ, np.int32); c = np.array(cl, np.int32); lv = np.array(lv, np.float64)
    nc = np.array(nco, np.int32); cn = np.array(cnts or [0], np.int32)
    out = np.zeros(2 + 3 * CL_MAX)
    rc = lib().orc_moment_sequence(int(n0), len(t), _ip(t), _ip(c), _dp(lv), _ip(nc), _ip(cn), _dp(out))
    if rc != 0:
        raise ValueError("inconsistent event sequence")
    return {"log_z": out[0], "log_z2": out[1], "log_zp": out[2:2 + CL_MAX],
            "log_z2p": out[2 + CL_MAX:2 + 2 * CL_MAX], "log_xp": out[2 + 2 * CL_MAX:]}


# ---------------------------------------------------------------- sampler

class Oracle:
    """One FP64 nested-sampling run, driven step by step like the GPU engine
    (init -> [evidence_update -> hss_walk -> replace_dead]* -> final sweep)."""

    def __init__(self, cfg, bf16: bool | None = None, trace_steps: int = 0):
        self.cfg = cfg
        d, n, k = cfg.d, cfg.n_live, cfg.n_kill
        if bf16 is None:
            bf16 = cfg.precision == "bf16mma"
        self.desc = _Desc(d=d, n_live=n, n_kill=k, kind=cfg.kind_id, n_comp=cfg.n_comp,
                          bf16=int(bf16), lo=cfg.lo, hi=cfg.hi, dt_init=cfg.dt_init,
                          n_steps_max=cfg.n_steps_max, min_ref=cfg.min_ref,
                          max_ref=cfg.max_ref, prune_streak=cfg.prune_streak,
                          delta_p=cfg.delta_p, out_hi=cfg.out_hi, out_lo=cfg.out_lo,
                          dt_down=cfg.dt_down, dt_up=cfg.dt_up, term_kind=cfg.term_kind,
                          max_iter=cfg.max_iter, term_tol=cfg.term_tol,
                          seed=C.c_uint64(int(cfg.seed) & (2**64 - 1)),
                          noise_mode=cfg.noise_id, cluster_mode=int(cfg.cluster),
                          cluster_kmax=int(cfg.cluster_kmax),
                          stop_mode=int(getattr(cfg, "stop_id", 0)),
                          save_mode=int(getattr(cfg, "save_id", 0)),
                          draw_mode=int(getattr(cfg, "draw_id", 0)))
        self.params = np.ascontiguousarray(cfg.params, dtype=np.float64)
        cap = k * cfg.max_iter + n
        self.live_x = np.zeros((n, d))
        self.live_logl = np.zeros(n)
        self.dead_logl = np.zeros(cap)
        self.dead_logw = np.zeros(cap)
        self.killed = np.zeros(k, np.int32)
        self.surv = np.zeros(max(n - k, 1), np.int32)
        self.start = np.zeros(k, np.int32)
        self.out_x = np.zeros((k, d))
        self.out_logl = np.zeros(k)
        self.trace_steps = int(trace_steps)
        ts = max(self.trace_steps, 1)
        self.trace_x = np.zeros((ts, k, d))
        self.trace_logl = np.zeros((ts, k))
        self.trace_out = np.zeros((ts, k), np.int32)
        self.st = _State(live_x=_dp(self.live_x), live_logl=_dp(self.live_logl),
                         dead_logl=_dp(self.dead_logl), dead_logw=_dp(self.dead_logw),
                         dead_cap=cap, n_dead=0, killed=_ip(self.killed), surv=_ip(self.surv),
                         start=_ip(self.start), out_x=_dp(self.out_x), out_logl=_dp(self.out_logl),
                         trace_x=_dp(self.trace_x) if trace_steps else None,
                         trace_logl=_dp(self.trace_logl), trace_out=_ip(self.trace_out),
                         trace_steps=self.trace_steps)
        self.label = np.zeros(n, np.int32)
        self.clx = np.full(CL_MAX, -np.inf)
        self.cn = np.zeros(CL_MAX, np.int32)
        self.surv_off = np.zeros(CL_MAX + 1, np.int32)
        self.start_cl = np.zeros(k, np.int32)
        self.st.label, self.st.clx, self.st.cn = _ip(self.label), _dp(self.clx), _ip(self.cn)
        self.st.surv_off, self.st.start_cl = _ip(self.surv_off), _ip(self.start_cl)
        self.cm = np.full(CM_SIZE, -np.inf)
        self.st.cm = _dp(self.cm)

    # -- steps
    def init(self):
        lib().orc_init(C.byref(self.desc), _dp(self.params), C.byref(self.st))
        return self

    def evidence_update(self, final_sweep: bool = False):
        lib().orc_evidence_update(C.byref(self.desc), C.byref(self.st), int(final_sweep))

    def hss_walk(self):
        lib().orc_hss_walk(C.byref(self.desc), _dp(self.params), C.byref(self.st))

    def replace_dead(self):
        lib().orc_replace_dead(C.byref(self.desc), C.byref(self.st))

    def iterate(self):
        self.evidence_update()
        if self.active:
            self.hss_walk()
            self.replace_dead()

    def run(self):
        lib().orc_run(C.byref(self.desc), _dp(self.params), C.byref(self.st))
        return self

    # -- state access
    def set_state(self, live_x=None, live_logl=None, log_z=None, log_x=None, dt=None,
                  iteration=None):
        """Load a live set / accumulators (test inputs)."""
        if live_x is not None:
            self.live_x[...] = live_x
            if live_logl is None:
                live_logl, _ = loglike(self.cfg, self.live_x, bool(self.desc.bf16))
        if live_logl is not None:
            self.live_logl[...] = live_logl
        if log_z is not None:
            self.st.lz = log_z
        if log_x is not None:
            self.st.lx = log_x
        if dt is not None:
            self.st.dt = dt
        if iteration is not None:
            self.st.iter = iteration

    @property
    def active(self) -> bool:
        return self.st.state == ST_ACTIVE

    @property
    def n_dead(self) -> int:
        return int(min(self.st.n_dead, self.st.dead_cap))

    def summary(self) -> dict:
        s = self.st
        return dict(log_z=s.lz, log_x=s.lx, log_z2=s.lz2, dt=s.dt, lstar=s.lstar,
                    iter=int(s.iter), evals=int(s.evals), n_dead=int(s.n_dead),
                    steps_out=int(s.steps_out), steps_in=int(s.steps_in),
                    prunes=int(s.prunes), nosave=int(s.nosave), state=int(s.state),
                    h=s.h, sigma_kl=s.sigma_kl, sigma_mom=s.sigma_mom,
                    it_outs=int(s.it_outs), it_steps=int(s.it_steps))

    def dead(self):
        n = self.n_dead
        return self.dead_logl[:n].copy(), self.dead_logw[:n].copy()
