"""ctypes binding of libpca.so: the C-ABI entry points of include/pca.h, same names.

Argument marshalling only.  Device memory and streams come from torch; every step of
the sampler runs in the library's HIP kernels.  Importing this module does not touch
the GPU; loading fails loudly if the built library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpca.so")

PCA_OK, PCA_EINVAL, PCA_ENOMEM, PCA_EDEVICE, PCA_ESTATE, PCA_EBUSY = 0, -1, -2, -3, -4, -5
PCA_PRIOR_POTTS, PCA_PRIOR_TRUNC_LINEAR = 0, 1

EXPORTED = ("pca_init", "pca_sweep", "pca_posterior_mean", "pca_marginal_map", "pca_get_state", "pca_set_state",
            "pca_stats", "pca_sweeps_per_launch", "pca_get_accumulators", "pca_set_accumulators", "pca_sync", "pca_destroy",
            "pca_batch_init", "pca_batch_autotune", "pca_batch_config", "pca_batch_set_config", "pca_batch_sweep", "pca_batch_posterior_mean", "pca_batch_marginal_map",
            "pca_batch_get_state", "pca_batch_stats", "pca_batch_sync", "pca_batch_destroy", "pca_server_create",
            "pca_server_submit", "pca_server_step", "pca_server_completed", "pca_server_status", "pca_server_result",
            "pca_server_release", "pca_server_stats", "pca_server_set_shedding", "pca_server_shed_count",
            "pca_server_destroy", "pca_run_static", "pca_last_error")


class PcaError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what} failed ({code}): {msg}")
        self.code = code


class pca_params(ctypes.Structure):
    _fields_ = [
        ("height", ctypes.c_int32), ("width", ctypes.c_int32), ("levels", ctypes.c_int32),
        ("chains", ctypes.c_int32), ("neighbourhood", ctypes.c_int32), ("prior", ctypes.c_int32),
        ("trunc", ctypes.c_int32),
        ("J", ctypes.c_float), ("q", ctypes.c_float), ("sigma", ctypes.c_float),
        ("vmin", ctypes.c_float), ("vmax", ctypes.c_float),
        ("beta", ctypes.POINTER(ctypes.c_float)), ("beta_len", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("init_mode", ctypes.c_int32), ("burn_in", ctypes.c_int32), ("tally_stride", ctypes.c_int32),
        ("inertia", ctypes.c_int32),
    ]


_lib = None


def load():
    """The loaded libpca.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback implementation)")
        lib = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        pp = ctypes.POINTER(pca_params)
        lib.pca_init.argtypes = [pp, vp, vp, ctypes.POINTER(vp)]
        lib.pca_sweep.argtypes = [vp, ctypes.c_int32, vp]
        lib.pca_posterior_mean.argtypes = [vp, vp, vp]
        lib.pca_marginal_map.argtypes = [vp, vp, vp]
        lib.pca_get_state.argtypes = [vp, vp, vp]
        lib.pca_set_state.argtypes = [vp, vp, ctypes.c_int64, vp]
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.pca_stats.argtypes = [vp, i64p, i64p, i64p]
        lib.pca_sweeps_per_launch.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        lib.pca_get_accumulators.argtypes = [vp, vp, vp, vp]
        lib.pca_set_accumulators.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int64, vp]
        lib.pca_sync.argtypes = [vp]
        lib.pca_destroy.argtypes = [vp]
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.pca_batch_init.argtypes = [pp, ctypes.POINTER(vp), ctypes.c_int32, vp, ctypes.POINTER(vp)]
        lib.pca_batch_autotune.argtypes = [vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_float)]
        lib.pca_batch_config.argtypes = [vp, i32p, i32p, i32p]
        lib.pca_batch_set_config.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp]
        lib.pca_batch_sweep.argtypes = [vp, ctypes.c_int32, vp]
        lib.pca_batch_posterior_mean.argtypes = [vp, ctypes.c_int32, vp, vp]
        lib.pca_batch_marginal_map.argtypes = [vp, ctypes.c_int32, vp, vp]
        lib.pca_batch_get_state.argtypes = [vp, ctypes.c_int32, vp, vp]
        lib.pca_batch_stats.argtypes = [vp, ctypes.c_int32, i64p, i64p, i64p]
        lib.pca_batch_sync.argtypes = [vp]
        lib.pca_batch_destroy.argtypes = [vp]
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.pca_server_create.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                          ctypes.POINTER(vp)]
        lib.pca_server_submit.argtypes = [vp, pp, vp, ctypes.c_int32, i64p]
        lib.pca_server_step.argtypes = [vp, vp, i32p]
        lib.pca_server_completed.argtypes = [vp, i64p, ctypes.c_int32, i32p]
        lib.pca_server_status.argtypes = [vp, ctypes.c_int64, i32p, i64p]
        lib.pca_server_result.argtypes = [vp, ctypes.c_int64, vp, vp, vp]
        lib.pca_server_release.argtypes = [vp, ctypes.c_int64]
        lib.pca_server_stats.argtypes = [vp, i32p, i32p, u64p, i64p, i64p]
        lib.pca_server_set_shedding.argtypes = [vp, ctypes.c_double]
        lib.pca_server_shed_count.argtypes = [vp, i64p]
        lib.pca_server_destroy.argtypes = [vp]
        lib.pca_run_static.argtypes = [pp, vp, ctypes.c_int32, vp, vp, vp, vp]
        lib.pca_last_error.argtypes = []
        lib.pca_last_error.restype = ctypes.c_char_p
        for name in EXPORTED[:-1]:
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def pca_last_error() -> str:
    return load().pca_last_error().decode()


def _check(rc: int, what: str):
    if rc != PCA_OK:
        raise PcaError(rc, what, pca_last_error())


def make_params(*, height: int, width: int, levels: int, chains: int = 1, neighbourhood: int = 4,
                prior: int = PCA_PRIOR_TRUNC_LINEAR, trunc: int = 1, J: float = 0.0, q: float = 0.0,
                sigma: float = 1.0, vmin: float = 0.0, vmax: Optional[float] = None,
                beta: Sequence[float] = (), seed: int = 0, init_mode: int = 0, burn_in: int = 0,
                tally_stride: int = 0, inertia: int = 0):
    """A pca_params struct plus the beta buffer it points to (keep both alive)."""
    if vmax is None:
        vmax = float(levels - 1)
    beta = list(beta)
    buf = (ctypes.c_float * max(1, len(beta)))(*beta) if beta else None
    p = pca_params(height, width, levels, chains, neighbourhood, prior, trunc, J, q, sigma, vmin, vmax,
                   ctypes.cast(buf, ctypes.POINTER(ctypes.c_float)) if buf is not None else None, len(beta),
                   seed & 0xFFFFFFFFFFFFFFFF, init_mode, burn_in, tally_stride, inertia)
    return p, buf


def pca_init(params: pca_params, obs_ptr: int, stream: int = 0) -> int:
    ctx = ctypes.c_void_p()
    _check(load().pca_init(ctypes.byref(params), ctypes.c_void_p(obs_ptr), ctypes.c_void_p(stream),
                           ctypes.byref(ctx)), "pca_init")
    return ctx.value


def pca_sweep(ctx: int, n: int, stream: int = 0):
    _check(load().pca_sweep(ctypes.c_void_p(ctx), int(n), ctypes.c_void_p(stream)), "pca_sweep")


def pca_posterior_mean(ctx: int, out_ptr: int, stream: int = 0):
    _check(load().pca_posterior_mean(ctypes.c_void_p(ctx), ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream)),
           "pca_posterior_mean")


def pca_marginal_map(ctx: int, out_ptr: int, stream: int = 0):
    _check(load().pca_marginal_map(ctypes.c_void_p(ctx), ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream)),
           "pca_marginal_map")


def pca_get_state(ctx: int, out_ptr: int, stream: int = 0):
    _check(load().pca_get_state(ctypes.c_void_p(ctx), ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream)),
           "pca_get_state")


def pca_set_state(ctx: int, in_ptr: int, t: int, stream: int = 0):
    _check(load().pca_set_state(ctypes.c_void_p(ctx), ctypes.c_void_p(in_ptr), int(t), ctypes.c_void_p(stream)),
           "pca_set_state")


def pca_stats(ctx: int):
    s, c, t = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().pca_stats(ctypes.c_void_p(ctx), ctypes.byref(s), ctypes.byref(c), ctypes.byref(t)), "pca_stats")
    return s.value, c.value, t.value


def pca_sweeps_per_launch(ctx: int) -> int:
    n = ctypes.c_int32()
    _check(load().pca_sweeps_per_launch(ctypes.c_void_p(ctx), ctypes.byref(n)), "pca_sweeps_per_launch")
    return n.value


def pca_get_accumulators(ctx: int, sum_ptr: int, hist_ptr: int = 0, stream: int = 0):
    _check(load().pca_get_accumulators(ctypes.c_void_p(ctx), ctypes.c_void_p(sum_ptr), ctypes.c_void_p(hist_ptr or None),
                                       ctypes.c_void_p(stream)), "pca_get_accumulators")


def pca_set_accumulators(ctx: int, sum_ptr: int, hist_ptr: int, count: int, tallies: int, stream: int = 0):
    _check(load().pca_set_accumulators(ctypes.c_void_p(ctx), ctypes.c_void_p(sum_ptr), ctypes.c_void_p(hist_ptr or None),
                                       int(count), int(tallies), ctypes.c_void_p(stream)), "pca_set_accumulators")


def pca_sync(ctx: int):
    _check(load().pca_sync(ctypes.c_void_p(ctx)), "pca_sync")


def pca_destroy(ctx: int):
    _check(load().pca_destroy(ctypes.c_void_p(ctx)), "pca_destroy")


# ------------------------------------------------------------------------------- batches

def pca_batch_init(params_list, obs_ptrs, stream: int = 0) -> int:
    """params_list: sequence of pca_params structs; obs_ptrs: device pointers, same length."""
    n = len(params_list)
    arr = (pca_params * n)(*params_list)
    ptrs = (ctypes.c_void_p * n)(*[ctypes.c_void_p(int(p)) for p in obs_ptrs])
    b = ctypes.c_void_p()
    _check(load().pca_batch_init(arr, ptrs, n, ctypes.c_void_p(stream), ctypes.byref(b)), "pca_batch_init")
    return b.value


def pca_batch_autotune(b: int, trial_sweeps: int, stream: int = 0) -> float:
    ms = ctypes.c_float()
    _check(load().pca_batch_autotune(ctypes.c_void_p(b), int(trial_sweeps), ctypes.c_void_p(stream),
                                     ctypes.byref(ms)), "pca_batch_autotune")
    return ms.value


def pca_batch_config(b: int):
    g, s, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().pca_batch_config(ctypes.c_void_p(b), ctypes.byref(g), ctypes.byref(s), ctypes.byref(t)),
           "pca_batch_config")
    return g.value, s.value, t.value


def pca_batch_set_config(b: int, chains_per_thread: int, share: int, tiled: int, stream: int = 0):
    _check(load().pca_batch_set_config(ctypes.c_void_p(b), int(chains_per_thread), int(share), int(tiled),
                                       ctypes.c_void_p(stream)), "pca_batch_set_config")


def pca_batch_sweep(b: int, n: int, stream: int = 0):
    _check(load().pca_batch_sweep(ctypes.c_void_p(b), int(n), ctypes.c_void_p(stream)), "pca_batch_sweep")


def pca_batch_posterior_mean(b: int, i: int, out_ptr: int, stream: int = 0):
    _check(load().pca_batch_posterior_mean(ctypes.c_void_p(b), int(i), ctypes.c_void_p(out_ptr),
                                           ctypes.c_void_p(stream)), "pca_batch_posterior_mean")


def pca_batch_marginal_map(b: int, i: int, out_ptr: int, stream: int = 0):
    _check(load().pca_batch_marginal_map(ctypes.c_void_p(b), int(i), ctypes.c_void_p(out_ptr),
                                         ctypes.c_void_p(stream)), "pca_batch_marginal_map")


def pca_batch_get_state(b: int, i: int, out_ptr: int, stream: int = 0):
    _check(load().pca_batch_get_state(ctypes.c_void_p(b), int(i), ctypes.c_void_p(out_ptr),
                                      ctypes.c_void_p(stream)), "pca_batch_get_state")


def pca_batch_stats(b: int, i: int):
    s, c, t = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().pca_batch_stats(ctypes.c_void_p(b), int(i), ctypes.byref(s), ctypes.byref(c), ctypes.byref(t)),
           "pca_batch_stats")
    return s.value, c.value, t.value


def pca_batch_sync(b: int):
    _check(load().pca_batch_sync(ctypes.c_void_p(b)), "pca_batch_sync")


def pca_batch_destroy(b: int):
    _check(load().pca_batch_destroy(ctypes.c_void_p(b)), "pca_batch_destroy")


# -------------------------------------------------------------------------------- server

def pca_server_create(hbm_budget_bytes: int, max_active: int, sweeps_per_step: int, step_ms: float = 20.0) -> int:
    sv = ctypes.c_void_p()
    _check(load().pca_server_create(int(hbm_budget_bytes), int(max_active), int(sweeps_per_step), float(step_ms),
                                    ctypes.byref(sv)), "pca_server_create")
    return sv.value


def pca_server_submit(sv: int, params: pca_params, obs_host_ptr: int, sweeps: int) -> int:
    rid = ctypes.c_int64()
    _check(load().pca_server_submit(ctypes.c_void_p(sv), ctypes.byref(params), ctypes.c_void_p(obs_host_ptr),
                                    int(sweeps), ctypes.byref(rid)), "pca_server_submit")
    return rid.value


def pca_server_set_shedding(sv: int, max_backlog_s: float):
    _check(load().pca_server_set_shedding(ctypes.c_void_p(sv), float(max_backlog_s)), "pca_server_set_shedding")


def pca_server_shed_count(sv: int) -> int:
    n = ctypes.c_int64()
    _check(load().pca_server_shed_count(ctypes.c_void_p(sv), ctypes.byref(n)), "pca_server_shed_count")
    return n.value


def pca_server_step(sv: int, stream: int = 0) -> int:
    n = ctypes.c_int32()
    _check(load().pca_server_step(ctypes.c_void_p(sv), ctypes.c_void_p(stream), ctypes.byref(n)), "pca_server_step")
    return n.value


def pca_server_completed(sv: int, capacity: int = 4096):
    ids = (ctypes.c_int64 * max(1, capacity))()
    n = ctypes.c_int32()
    _check(load().pca_server_completed(ctypes.c_void_p(sv), ids, int(capacity), ctypes.byref(n)),
           "pca_server_completed")
    return [ids[i] for i in range(n.value)]


def pca_server_status(sv: int, rid: int):
    st, sw = ctypes.c_int32(), ctypes.c_int64()
    _check(load().pca_server_status(ctypes.c_void_p(sv), int(rid), ctypes.byref(st), ctypes.byref(sw)),
           "pca_server_status")
    return st.value, sw.value


def pca_server_result(sv: int, rid: int, mean_ptr: int, mpm_ptr: int, state_ptr: int):
    _check(load().pca_server_result(ctypes.c_void_p(sv), int(rid), ctypes.c_void_p(mean_ptr), ctypes.c_void_p(mpm_ptr),
                                    ctypes.c_void_p(state_ptr)), "pca_server_result")


def pca_server_release(sv: int, rid: int):
    _check(load().pca_server_release(ctypes.c_void_p(sv), int(rid)), "pca_server_release")


def pca_server_stats(sv: int):
    q, a, u, st, sw = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_uint64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().pca_server_stats(ctypes.c_void_p(sv), ctypes.byref(q), ctypes.byref(a), ctypes.byref(u),
                                   ctypes.byref(st), ctypes.byref(sw)), "pca_server_stats")
    return q.value, a.value, u.value, st.value, sw.value


def pca_server_destroy(sv: int):
    _check(load().pca_server_destroy(ctypes.c_void_p(sv)), "pca_server_destroy")


def pca_run_static(params: pca_params, obs_ptr: int, sweeps: int, mean_ptr: int = 0, mpm_ptr: int = 0,
                   state_ptr: int = 0, stream: int = 0):
    _check(load().pca_run_static(ctypes.byref(params), ctypes.c_void_p(obs_ptr), int(sweeps),
                                 ctypes.c_void_p(mean_ptr or None), ctypes.c_void_p(mpm_ptr or None),
                                 ctypes.c_void_p(state_ptr or None), ctypes.c_void_p(stream)), "pca_run_static")
