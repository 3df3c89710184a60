"""Nested sampling with a likelihood written in torch.

The likelihood is any differentiable torch function of a [n, d] FP64 batch of
points returning [n] log-likelihoods; its score comes from torch.autograd
(the differentiable-programming route of Section 3).  The walk itself (starts,
momenta, reflections, noise, kept points, pruning, stop), the kill and the
evidence run in the library's kernels: per walk step the caller-side function
is evaluated once for every walker, then ggns_ext_step advances the walkers
(see ggns_ext_begin in the C header).  Runs must be FP64; the likelihood family
named in the run's configuration is only a placeholder for the library.
"""
from __future__ import annotations

import ctypes as C
from typing import Callable, List, Sequence

from . import _lib
from .engine import Engine
from .inputs import RunConfig


def value_and_score(fn: Callable, x):
    """log L and its gradient at the rows of x (torch autograd)."""
    import torch
    with torch.enable_grad():
        xr = x.detach().requires_grad_(True)
        logl = fn(xr)
        (g,) = torch.autograd.grad(logl.sum(), xr)
    return logl.detach(), g


class ExternalRuns:
    """Independent runs whose likelihoods are torch functions, one per run."""

    def __init__(self, configs: Sequence[RunConfig], fns: Sequence[Callable], device: str = "cuda"):
        if len(configs) != len(fns):
            raise ValueError("one likelihood function per run")
        if any(c.precision != "fp64" for c in configs):
            raise ValueError("the external-likelihood walk runs in FP64")
        self.eng = Engine(configs, device=device)
        self.fns: List[Callable] = list(fns)
        torch = self.eng.torch
        self._ws = []
        for r in range(len(configs)):
            nb = int(self.eng.L.ggns_ext_workspace_bytes(self.eng.ctx, r))
            _lib.check(nb if nb < 0 else 0, "ggns_ext_workspace_bytes")
            self._ws.append(torch.empty(nb, dtype=torch.uint8, device=self.eng.device))
            # the live set's log L from the caller's likelihood
            l, _ = value_and_score(self.fns[r], self.eng.live_x(r))
            self.eng.live_logl(r).copy_(l.to(torch.float64))

    def _buffers(self, r: int):
        torch = self.eng.torch
        c = self.eng.cfgs[r]
        ptrs = [C.c_void_p() for _ in range(4)]
        ws = self._ws[r]
        _lib.check(self.eng.L.ggns_ext_buffers(self.eng.ctx, r, ws.data_ptr(), ws.numel(),
                                               *[C.byref(p) for p in ptrs]), "ggns_ext_buffers")
        base = ws.data_ptr()

        def view(ptr, count, dtype, shape):
            off = ptr.value - base
            esz = torch.empty((), dtype=dtype).element_size()
            return ws[off:off + count * esz].view(dtype).view(*shape)
        k, d = c.n_kill, c.d
        x = view(ptrs[0], d * k, torch.float64, (d, k))
        logl = view(ptrs[1], k, torch.float64, (k,))
        grad = view(ptrs[2], d * k, torch.float64, (d, k))
        active = view(ptrs[3], c.n_steps_max + 1, torch.int32, (c.n_steps_max + 1,))
        return x, logl, grad, active

    def walk(self, r: int, poll_every: int = 8):
        """One walk of run r's killed points (after evidence_update)."""
        c = self.eng.cfgs[r]
        ws = self._ws[r]
        s = self.eng._stream()
        x, logl, grad, active = self._buffers(r)
        _lib.check(self.eng.L.ggns_ext_begin(self.eng.ctx, r, ws.data_ptr(), ws.numel(), s),
                   "ggns_ext_begin")
        # the batch-minimum loop takes one call more: the last step's save rule
        batch = self.eng.walk_mode(r) == 1
        n_calls = c.n_steps_max + (1 if batch else 0)
        for t in range(n_calls):
            if t < c.n_steps_max:
                l, g = value_and_score(self.fns[r], x.t())
                logl.copy_(l)
                grad.copy_(g.t())
            _lib.check(self.eng.L.ggns_ext_step(self.eng.ctx, r, ws.data_ptr(), ws.numel(), t, s),
                       "ggns_ext_step")
            if (t + 1) % poll_every == 0 and int(active[t].item()) == 0:
                break

    def iterate(self, n: int = 1):
        for _ in range(n):
            self.eng.evidence_update()
            for r in range(len(self.fns)):
                self.walk(r)
            self.eng.replace_dead()

    def run(self, poll_every: int = 8, max_iter_blocks: int = 10 ** 6) -> List[dict]:
        """Iterate until every run stopped; returns the per-run stats."""
        for _ in range(max_iter_blocks):
            self.iterate(poll_every)
            st = self.eng.stats()
            if all(x["state"] != _lib.RUN_ACTIVE for x in st):
                self.eng.finalize()
                return self.eng.stats()
        raise RuntimeError("runs did not terminate")

    def close(self):
        self.eng.close()
