"""Device-memory plumbing and the run loop on top of the C ABI.

PyTorch provides the device memory (one arena tensor per engine, one FP64
parameter tensor) and the stream; every step of the sampler runs in the HIP
kernels of libggns.so.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import numpy as np

from . import _lib
from .inputs import RunConfig

def _torch():
    import torch
    return torch


def walk_mode_of(c: RunConfig) -> int:
    """The library's walk_mode for a run's walk readings: 1 for the loop and
    the saving on the batch minimum of num_reflections, 0 for both per walker
    (and for fixed-step walks); other combinations, the pooled draw and the
    isotropic noise exist in the test oracle only."""
    if c.draw_id != 0:
        raise ValueError("the pooled x_saved draw is not implemented by the engine")
    if c.noise_id not in (0, 1):
        raise ValueError(f"noise reading {c.noise!r} is not implemented by the engine")
    if c.max_ref == 0:
        if c.save_id != 0:
            raise ValueError("fixed-step walks save per walker in the engine")
        return 0
    if (c.stop_id, c.save_id) == (1, 1):
        return 1
    if (c.stop_id, c.save_id) == (0, 0):
        return 0
    raise ValueError("the engine walks stop and save both per walker or both on the batch minimum")


def make_descs(configs: Sequence[RunConfig], tile_c=None):
    """The C run descriptors of a batch and its packed FP64 parameter blocks."""
    n = len(configs)
    descs = (_lib.ggns_run_desc * n)()
    off = 0
    blocks = []
    for i, c in enumerate(configs):
        D = descs[i]
        D.d, D.n_live, D.n_kill = c.d, c.n_live, c.n_kill
        D.lik_kind, D.precision, D.n_comp = c.kind_id, c.precision_id, c.n_comp
        D.param_offset = off
        D.prior_lo, D.prior_hi, D.dt_init = c.lo, c.hi, c.dt_init
        D.n_steps_max, D.min_ref, D.max_ref = c.n_steps_max, c.min_ref, c.max_ref
        D.prune_streak, D.delta_p = c.prune_streak, c.delta_p
        D.out_hi, D.out_lo, D.dt_down, D.dt_up = c.out_hi, c.out_lo, c.dt_down, c.dt_up
        D.term_kind, D.max_iter, D.term_tol = c.term_kind, c.max_iter, c.term_tol
        D.seed = int(c.seed) & (2 ** 64 - 1)
        D.tile_c = int(tile_c[i]) if tile_c is not None else 0
        D.noise_mode = c.noise_id
        D.cluster_mode, D.cluster_kmax = int(c.cluster), int(c.cluster_kmax)
        D.walk_mode = walk_mode_of(c)
        blocks.append(np.asarray(c.params, np.float64))
        off += len(c.params)
    return descs, blocks


class Engine:
    """Many independent nested-sampling runs advanced together.

    One iteration = ggns_evidence_update -> ggns_hss_walk -> ggns_replace_dead
    for every active run; a block of iterations goes through ggns_iterate,
    which gives each kernel class its own chain of them.  `run()` repeats
    blocks (optionally as a captured HIP graph) until every run has stopped.
    """

    def __init__(self, configs: Sequence[RunConfig], device: str = "cuda",
                 tile_c=None, attach_arena=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("the GGNS engine needs a ROCm GPU; no CPU path exists")
        self.torch = torch
        self.device = torch.device(device)
        self.cfgs: List[RunConfig] = list(configs)
        if isinstance(tile_c, str):
            if tile_c != "auto":
                raise ValueError("tile_c must be a list of ints or 'auto'")
            from .autotune import tune
            tile_c = tune(self.cfgs, device=str(self.device))
        L = _lib.load()
        self.L = L
        n = len(self.cfgs)
        self.descs, blocks = make_descs(self.cfgs, tile_c)
        self.params = torch.from_numpy(np.concatenate(blocks)).to(self.device)
        nbytes = int(L.ggns_arena_bytes(self.descs, n))
        if nbytes < 0:
            _lib.check(nbytes, "ggns_arena_bytes")
        self.arena_bytes = nbytes
        if attach_arena is not None:
            self.arena = attach_arena
        else:
            self.arena = torch.zeros(nbytes, dtype=torch.uint8, device=self.device)
        if self.arena.data_ptr() % 256:
            raise RuntimeError("arena is not 256-byte aligned")
        self.ctx = C.c_void_p()
        fn = L.ggns_attach if attach_arena is not None else L.ggns_init
        _lib.check(fn(C.byref(self.ctx), self.descs, n, self.params.data_ptr(),
                      self.params.numel(), self.arena.data_ptr(), nbytes, self._stream()),
                   "ggns_init")
        self.layouts = []
        for r in range(n):
            lay = _lib.ggns_layout()
            _lib.check(L.ggns_run_layout(self.ctx, r, C.byref(lay)), "ggns_run_layout")
            self.layouts.append(lay)
        self._graph = None
        self._graph_iters = 0
        self._trace = {}
        self._dead_x = {}
        self._stat_bufs = None

    # ------------------------------------------------------------------ plumbing
    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _view(self, off, nbytes, dtype, shape):
        return self.arena[off:off + nbytes].view(dtype).view(*shape)

    def walk_mode(self, r: int) -> int:
        return int(self.descs[r].walk_mode)

    def _fdtype(self, r):
        return self.torch.float64 if self.layouts[r].elem_bytes == 8 else self.torch.float32

    def close(self):
        if self.ctx:
            self.L.ggns_free(self.ctx)
            self.ctx = C.c_void_p()

    def reset(self):
        """Re-initialise every run on the same arena (same descriptors and
        parameters): prior draws and accumulators start afresh.  A captured
        block graph stays valid (its launches' arguments all point into the
        arena); traces and dead-position buffers set on the old context are not
        carried over."""
        self.close()
        _lib.check(self.L.ggns_init(C.byref(self.ctx), self.descs, len(self.cfgs),
                                    self.params.data_ptr(), self.params.numel(),
                                    self.arena.data_ptr(), self.arena_bytes, self._stream()),
                   "ggns_init")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ steps
    def evidence_update(self, final_sweep: bool = False):
        _lib.check(self.L.ggns_evidence_update(self.ctx, int(final_sweep), self._stream()),
                   "ggns_evidence_update")

    def finalize(self):
        _lib.check(self.L.ggns_finalize(self.ctx, self._stream()), "ggns_finalize")

    def hss_walk(self):
        _lib.check(self.L.ggns_hss_walk(self.ctx, self._stream()), "ggns_hss_walk")

    def hss_walk_plain(self):
        """The plain FP64 per-step walk (speed baseline; FP64 runs only)."""
        if getattr(self, "_plain_ws", None) is None:
            nb = int(self.L.ggns_plain_workspace_bytes(self.ctx))
            _lib.check(nb if nb < 0 else 0, "ggns_plain_workspace_bytes")
            self._plain_ws = self.torch.empty(max(nb, 256), dtype=self.torch.uint8, device=self.device)
        _lib.check(self.L.ggns_hss_walk_plain(self.ctx, self._plain_ws.data_ptr(),
                                              self._plain_ws.numel(), self._stream()),
                   "ggns_hss_walk_plain")

    def replace_dead(self):
        _lib.check(self.L.ggns_replace_dead(self.ctx, self._stream()), "ggns_replace_dead")

    def hss_walk_plain_static(self):
        """The same plain walk with its workspace in the library's fixed
        device buffer (no allocation; FP64 runs that fit the buffer only)."""
        _lib.check(self.L.ggns_hss_walk_plain_static(self.ctx, self._stream()),
                   "ggns_hss_walk_plain_static")

    def iterate(self, n: int = 1, plain: bool = False, per_call: bool = False):
        """n iterations.  The fused path goes through ggns_iterate (each kernel
        class on its own chain of iterations); `per_call` issues the same work
        as one evidence / walk / replace call per iteration instead."""
        if not plain and not per_call:
            _lib.check(self.L.ggns_iterate(self.ctx, int(n), self._stream()), "ggns_iterate")
            return
        for _ in range(n):
            self.evidence_update()
            if plain:
                self.hss_walk_plain()
            else:
                self.hss_walk()
            self.replace_dead()

    def capture(self, iters: int):
        """Capture `iters` iterations as one HIP graph (kernels only)."""
        torch = self.torch
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                self.iterate(iters)
        torch.cuda.current_stream(self.device).wait_stream(side)
        self._graph = g
        self._graph_iters = iters

    def step_block(self, iters: int, use_graph: bool, plain: bool = False):
        if plain:
            self.iterate(iters, plain=True)
        elif use_graph:
            if self._graph is None or self._graph_iters != iters:
                self.capture(iters)
            self._graph.replay()
        else:
            self.iterate(iters)

    def run(self, poll_every: int = 8, use_graph: bool = False, max_blocks: int = 10 ** 6,
            plain: bool = False, pipelined: bool = True):
        """Iterate until every run stopped; returns the per-run stats.

        Pipelined (the default): the runs' states are copied back after every
        block of `poll_every` iterations without draining the stream, and read
        one block later, while the next block runs; the block enqueued after
        the last run stopped is all no-op launches.  Results are the same
        either way."""
        if plain or not pipelined:
            for _ in range(max_blocks):
                self.step_block(poll_every, use_graph, plain)
                st = self.stats()
                if all(s["state"] != _lib.RUN_ACTIVE for s in st):
                    self.finalize()
                    return self.stats()
            raise RuntimeError("runs did not terminate")
        pending = None
        for b in range(max_blocks):
            self.step_block(poll_every, use_graph)
            nxt = self.states_async(b & 1)
            if pending is not None and not (pending() == _lib.RUN_ACTIVE).any():
                self.finalize()
                return self.stats()
            pending = nxt
        raise RuntimeError("runs did not terminate")

    def states_async(self, slot: int = 0):
        """Enqueue the copy of every run's stats into pinned host buffer `slot`
        (0 or 1) on the engine's stream; returns a function that waits for it
        and gives the runs' states (numpy int32)."""
        torch = self.torch
        n = len(self.cfgs)
        rec = C.sizeof(_lib.ggns_run_stats)
        if self._stat_bufs is None:
            self._stat_bufs = [torch.empty(n * rec, dtype=torch.uint8, pin_memory=True)
                               for _ in range(2)]
        buf = self._stat_bufs[slot]
        _lib.check(self.L.ggns_read_stats_async(self.ctx, buf.data_ptr(), self._stream()),
                   "ggns_read_stats_async")
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(self.device))
        off = _lib.ggns_run_stats.state.offset

        def wait():
            ev.synchronize()
            return buf.numpy().view(np.int32)[off // 4::rec // 4][:n].copy()
        return wait

    # ------------------------------------------------------------------ state
    def stats(self) -> List[dict]:
        n = len(self.cfgs)
        out = (_lib.ggns_run_stats * n)()
        _lib.check(self.L.ggns_read_stats(self.ctx, out, self._stream()), "ggns_read_stats")
        res = []
        for s in out:
            res.append({f: getattr(s, f) for f, _ in _lib.ggns_run_stats._fields_
                        if f != "reserved"})
        return res

    def write_vars(self, r: int, log_z: float, log_x: float, dt: float, iteration: int):
        v = _lib.ggns_run_vars(log_z=log_z, log_x=log_x, dt=dt, iter=iteration)
        _lib.check(self.L.ggns_write_vars(self.ctx, r, C.byref(v), self._stream()),
                   "ggns_write_vars")

    def tile_shape(self, r: int):
        c, g = C.c_int32(), C.c_int32()
        _lib.check(self.L.ggns_tile_shape(self.ctx, r, C.byref(c), C.byref(g)), "ggns_tile_shape")
        return c.value, g.value

    # views into the arena (device tensors)
    def live_x(self, r):
        c, lay = self.cfgs[r], self.layouts[r]
        return self._view(lay.live_x, c.n_live * c.d * lay.elem_bytes, self._fdtype(r),
                          (c.n_live, c.d))

    def live_logl(self, r):
        c, lay = self.cfgs[r], self.layouts[r]
        return self._view(lay.live_logl, c.n_live * 8, self.torch.float64, (c.n_live,))

    def killed(self, r):
        c, lay = self.cfgs[r], self.layouts[r]
        return self._view(lay.killed, c.n_kill * 4, self.torch.int32, (c.n_kill,))

    def survivors(self, r):
        c, lay = self.cfgs[r], self.layouts[r]
        m = c.n_live - c.n_kill
        return self._view(lay.survivors, m * 4, self.torch.int32, (m,))

    def start(self, r):
        c, lay = self.cfgs[r], self.layouts[r]
        return self._view(lay.start, c.n_kill * 4, self.torch.int32, (c.n_kill,))

    def walk_x(self, r):
        c, lay = self.cfgs[r], self.layouts[r]
        return self._view(lay.walk_x, c.n_kill * c.d * lay.elem_bytes, self._fdtype(r),
                          (c.n_kill, c.d))

    def walk_logl(self, r):
        c, lay = self.cfgs[r], self.layouts[r]
        return self._view(lay.walk_logl, c.n_kill * 8, self.torch.float64, (c.n_kill,))

    def dead(self, r, n_dead: Optional[int] = None):
        lay = self.layouts[r]
        if n_dead is None:
            n_dead = int(self.stats()[r]["n_dead"])
        n_dead = min(n_dead, lay.dead_cap)
        return (self._view(lay.dead_logl, n_dead * 8, self.torch.float64, (n_dead,)),
                self._view(lay.dead_logw, n_dead * 8, self.torch.float64, (n_dead,)))

    def labels(self, r):
        """Cluster of each live slot (cluster mode)."""
        c, lay = self.cfgs[r], self.layouts[r]
        if lay.label < 0:
            raise ValueError("run is not in cluster mode")
        return self._view(lay.label, c.n_live * 4, self.torch.int32, (c.n_live,))

    def clusters(self, r) -> dict:
        """The run's cluster table, copied to the host (cluster mode)."""
        lay = self.layouts[r]
        if lay.cluster_table < 0:
            raise ValueError("run is not in cluster mode")
        raw = self.arena[lay.cluster_table:lay.cluster_table + 1816].cpu().numpy()
        f64, i32 = raw[:1024].view(np.float64), raw[1024:1816].view(np.int32)
        nc = int(i32[194])
        ext = self.arena[lay.cluster_table + 1816:lay.cluster_table + 2088].cpu().numpy().view(np.int32)
        mom = self.arena[lay.cluster_table + 2088:lay.cluster_table + 37416].cpu().numpy().view(np.float64)
        return {"log_xbar": f64[:64].copy(), "cdf": f64[64:128].copy(), "n_live": i32[:64].copy(),
                "surv_off": i32[64:129].copy(), "member_off": i32[129:194].copy(),
                "n_clusters": nc, "n_splits": int(i32[195]), "stopping": int(i32[196]),
                "n_cut": int(ext[65]),
                # moments of the cluster recursion, as logarithms
                "log_zp": mom[0:64].copy(), "log_z2p": mom[64:128].copy(),
                "log_zx": mom[128:192].copy(), "log_zpx": mom[192:256].copy(),
                "log_x2": mom[256:320].copy(), "log_xx": mom[320:].reshape(64, 64).copy()}

    def knn(self, r):
        """The run's neighbour lists (cluster mode): slots [n_live, 32] and
        squared distances."""
        c, lay = self.cfgs[r], self.layouts[r]
        if lay.knn < 0:
            raise ValueError("run is not in cluster mode")
        return (self._view(lay.knn, c.n_live * 32 * 4, self.torch.int32, (c.n_live, 32)),
                self._view(lay.knn_dist, c.n_live * 32 * 8, self.torch.float64, (c.n_live, 32)))

    def set_trace(self, r: int, steps: int):
        """Record the first `steps` steps of every walker of run r."""
        torch = self.torch
        c = self.cfgs[r]
        if steps <= 0:
            _lib.check(self.L.ggns_set_trace(self.ctx, r, None, None, None, 0), "ggns_set_trace")
            self._trace.pop(r, None)
            return None
        tx = torch.zeros((steps, c.n_kill, c.d), dtype=self._fdtype(r), device=self.device)
        tl = torch.zeros((steps, c.n_kill), dtype=torch.float64, device=self.device)
        to = torch.zeros((steps, c.n_kill), dtype=torch.int32, device=self.device)
        _lib.check(self.L.ggns_set_trace(self.ctx, r, tx.data_ptr(), tl.data_ptr(), to.data_ptr(),
                                         steps), "ggns_set_trace")
        self._trace[r] = (tx, tl, to)
        return self._trace[r]

    def keep_dead_x(self, r: int):
        """Record the positions of run r's dead points from now on (a device
        tensor [dead_cap, d] in the run's precision)."""
        c, lay = self.cfgs[r], self.layouts[r]
        buf = self.torch.zeros((lay.dead_cap, c.d), dtype=self._fdtype(r), device=self.device)
        _lib.check(self.L.ggns_set_dead_x(self.ctx, r, buf.data_ptr(), lay.dead_cap), "ggns_set_dead_x")
        self._dead_x[r] = buf
        return buf

    def dead_x(self, r: int, n_dead: Optional[int] = None):
        if n_dead is None:
            n_dead = int(self.stats()[r]["n_dead"])
        return self._dead_x[r][:min(n_dead, self.layouts[r].dead_cap)]

    # ------------------------------------------------------------------ likelihood
    def loglike(self, r: int, x, grad: bool = True):
        torch = self.torch
        x = x.to(device=self.device, dtype=self._fdtype(r)).contiguous()
        n = x.shape[0]
        logl = torch.empty(n, dtype=torch.float64, device=self.device)
        g = torch.empty_like(x) if grad else None
        _lib.check(self.L.ggns_loglike_grad(self.ctx, r, x.data_ptr(), n, logl.data_ptr(),
                                            g.data_ptr() if g is not None else None,
                                            self._stream()), "ggns_loglike_grad")
        return logl, g

    def loglike_vjp(self, r: int, x, gout):
        torch = self.torch
        x = x.to(device=self.device, dtype=self._fdtype(r)).contiguous()
        gout = gout.to(device=self.device, dtype=torch.float64).contiguous()
        gx = torch.empty_like(x)
        _lib.check(self.L.ggns_loglike_vjp(self.ctx, r, x.data_ptr(), x.shape[0], gout.data_ptr(),
                                           gx.data_ptr(), self._stream()), "ggns_loglike_vjp")
        return gx


def run_configs(configs: Sequence[RunConfig], poll_every: int = 8, use_graph: bool = False,
                device: str = "cuda") -> List[dict]:
    eng = Engine(configs, device=device)
    st = eng.run(poll_every=poll_every, use_graph=use_graph)
    eng.close()
    return st
