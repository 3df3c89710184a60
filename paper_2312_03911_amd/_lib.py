"""ctypes binding of libggns.so: the structs and entry points of include/ggns.h,
with the same names.  Argument marshalling only; there is no fallback: loading
fails loudly when the library is missing."""
from __future__ import annotations

import ctypes as C
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libggns.so")

GGNS_OK, GGNS_EINVAL, GGNS_EHIP, GGNS_EUNSUPPORTED, GGNS_ESTATE, GGNS_ESCRATCH = 0, -1, -2, -3, -4, -5
STATIC_SCRATCH_BYTES = 16 << 20   # GGNS_STATIC_SCRATCH_BYTES
RUN_ACTIVE, RUN_DONE, RUN_MAXITER, RUN_NONFINITE = 0, 1, 2, 3

# every symbol the header declares
SYMBOLS = ("ggns_arena_bytes", "ggns_init", "ggns_attach", "ggns_evidence_update", "ggns_finalize",
           "ggns_hss_walk", "ggns_replace_dead", "ggns_iterate", "ggns_loglike_grad", "ggns_loglike_vjp",
           "ggns_run_layout", "ggns_read_stats", "ggns_read_stats_async", "ggns_write_vars",
           "ggns_set_trace", "ggns_tile_shape", "ggns_plain_workspace_bytes", "ggns_hss_walk_plain",
           "ggns_hss_walk_plain_static",
           "ggns_noise_normals", "ggns_set_dead_x", "ggns_ext_workspace_bytes", "ggns_ext_buffers",
           "ggns_ext_begin", "ggns_ext_step", "ggns_probe_valu", "ggns_probe_mfma", "ggns_free",
           "ggns_status_string")


class ggns_run_desc(C.Structure):
    _fields_ = [("d", C.c_int32), ("n_live", C.c_int32), ("n_kill", C.c_int32),
                ("lik_kind", C.c_int32), ("precision", C.c_int32), ("n_comp", C.c_int32),
                ("param_offset", C.c_int64),
                ("prior_lo", C.c_double), ("prior_hi", C.c_double), ("dt_init", C.c_double),
                ("n_steps_max", C.c_int32), ("min_ref", C.c_int32), ("max_ref", C.c_int32),
                ("prune_streak", C.c_int32),
                ("delta_p", C.c_double), ("out_hi", C.c_double), ("out_lo", C.c_double),
                ("dt_down", C.c_double), ("dt_up", C.c_double),
                ("term_kind", C.c_int32), ("max_iter", C.c_int32), ("term_tol", C.c_double),
                ("seed", C.c_uint64), ("tile_c", C.c_int32), ("noise_mode", C.c_int32),
                ("cluster_mode", C.c_int32), ("cluster_kmax", C.c_int32),
                ("walk_mode", C.c_int32), ("reserved0", C.c_int32)]


class ggns_layout(C.Structure):
    _fields_ = [("live_x", C.c_int64), ("live_logl", C.c_int64), ("killed", C.c_int64),
                ("survivors", C.c_int64), ("start", C.c_int64), ("walk_x", C.c_int64),
                ("walk_logl", C.c_int64), ("dead_logl", C.c_int64), ("dead_logw", C.c_int64),
                ("dead_cap", C.c_int64), ("elem_bytes", C.c_int32), ("reserved", C.c_int32),
                ("label", C.c_int64), ("cluster_table", C.c_int64),
                ("knn", C.c_int64), ("knn_dist", C.c_int64)]


class ggns_run_stats(C.Structure):
    _fields_ = [("log_z", C.c_double), ("log_x", C.c_double), ("log_z2", C.c_double),
                ("dt", C.c_double), ("lstar", C.c_double), ("log_xl_max", C.c_double),
                ("h", C.c_double), ("sigma_kl", C.c_double), ("sigma_mom", C.c_double),
                ("iter", C.c_int64), ("evals", C.c_int64), ("n_dead", C.c_int64),
                ("steps_out", C.c_int64), ("steps_in", C.c_int64), ("prunes", C.c_int64),
                ("nosave", C.c_int64), ("it_outs", C.c_int64), ("it_steps", C.c_int64),
                ("replayed", C.c_int64), ("state", C.c_int32), ("n_clusters", C.c_int32)]


class ggns_run_vars(C.Structure):
    _fields_ = [("log_z", C.c_double), ("log_x", C.c_double), ("dt", C.c_double),
                ("iter", C.c_int64)]


_lock = threading.Lock()
_lib = None


def load() -> C.CDLL:
    """Load libggns.so (built in-tree by paper_2312_03911_amd.build)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2312_03911_amd.build` (no CPU fallback exists)")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded, so both see the same devices, streams and allocations (a
        # second runtime loaded beside torch's finds no device)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        PD = C.POINTER(ggns_run_desc)
        L.ggns_arena_bytes.argtypes = [PD, i32]
        L.ggns_arena_bytes.restype = i64
        for fn in (L.ggns_init, L.ggns_attach):
            fn.argtypes = [C.POINTER(vp), PD, i32, vp, i64, vp, i64, vp]
            fn.restype = C.c_int
        L.ggns_evidence_update.argtypes = [vp, i32, vp]
        L.ggns_hss_walk.argtypes = [vp, vp]
        L.ggns_finalize.argtypes = [vp, vp]
        L.ggns_replace_dead.argtypes = [vp, vp]
        L.ggns_iterate.argtypes = [vp, i32, vp]
        L.ggns_loglike_grad.argtypes = [vp, i32, vp, i64, vp, vp, vp]
        L.ggns_loglike_vjp.argtypes = [vp, i32, vp, i64, vp, vp, vp]
        L.ggns_run_layout.argtypes = [vp, i32, C.POINTER(ggns_layout)]
        L.ggns_read_stats.argtypes = [vp, C.POINTER(ggns_run_stats), vp]
        L.ggns_read_stats_async.argtypes = [vp, vp, vp]
        L.ggns_write_vars.argtypes = [vp, i32, C.POINTER(ggns_run_vars), vp]
        L.ggns_set_trace.argtypes = [vp, i32, vp, vp, vp, i32]
        L.ggns_tile_shape.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32)]
        L.ggns_plain_workspace_bytes.argtypes = [vp]
        L.ggns_plain_workspace_bytes.restype = i64
        L.ggns_hss_walk_plain.argtypes = [vp, vp, i64, vp]
        L.ggns_hss_walk_plain_static.argtypes = [vp, vp]
        L.ggns_hss_walk_plain_static.restype = C.c_int
        L.ggns_noise_normals.argtypes = [C.c_uint64, i32, i32, i32, i32, vp, vp, vp, vp]
        L.ggns_noise_normals.restype = C.c_int
        for name in ("ggns_probe_valu", "ggns_probe_mfma"):
            getattr(L, name).argtypes = [i32, i32, C.c_float, C.c_float, vp, vp]
            getattr(L, name).restype = C.c_int
        L.ggns_set_dead_x.argtypes = [vp, i32, vp, i64]
        L.ggns_set_dead_x.restype = C.c_int
        L.ggns_ext_workspace_bytes.argtypes = [vp, i32]
        L.ggns_ext_workspace_bytes.restype = i64
        dpp = C.POINTER(C.c_void_p)
        L.ggns_ext_buffers.argtypes = [vp, i32, vp, i64, dpp, dpp, dpp, dpp]
        L.ggns_ext_buffers.restype = C.c_int
        L.ggns_ext_begin.argtypes = [vp, i32, vp, i64, vp]
        L.ggns_ext_begin.restype = C.c_int
        L.ggns_ext_step.argtypes = [vp, i32, vp, i64, i32, vp]
        L.ggns_ext_step.restype = C.c_int
        L.ggns_free.argtypes = [vp]
        L.ggns_free.restype = None
        L.ggns_status_string.argtypes = [C.c_int]
        L.ggns_status_string.restype = C.c_char_p
        for name in ("ggns_evidence_update", "ggns_finalize", "ggns_hss_walk", "ggns_replace_dead",
                     "ggns_iterate",
                     "ggns_loglike_grad", "ggns_loglike_vjp", "ggns_run_layout",
                     "ggns_read_stats", "ggns_read_stats_async", "ggns_write_vars",
                     "ggns_set_trace", "ggns_tile_shape", "ggns_hss_walk_plain"):
            getattr(L, name).restype = C.c_int
        _lib = L
        return L


class GGNSError(RuntimeError):
    pass


def check(rc: int, what: str) -> None:
    if rc != GGNS_OK:
        msg = load().ggns_status_string(rc).decode()
        raise GGNSError(f"{what} failed: {msg} ({rc})")
