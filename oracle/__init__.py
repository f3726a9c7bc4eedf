"""CPU oracle for the lazy PCA sampler and the sequential Gibbs sampler.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers.  The product path never
imports this package.  The arithmetic lives in ``orc.c`` (plain scalar C, the
paper's definitions and the arithmetic convention written in that file's header);
this module only compiles it and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

OK, EINVAL, ENOMEM, ESTATE = 0, -1, -2, -4
POTTS, TRUNC_LINEAR = 0, 1


def build(force: bool = True) -> str:
    """Compile ``orc.c`` into ``liborc.so`` (generic x86-64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out: str) -> str:
    """Compile ``orc.c`` with AddressSanitizer and UndefinedBehaviorSanitizer (any report
    aborts) into ``out``; load it by setting ORC_LIB to that path in a process started with
    the ASan runtime preloaded."""
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-o", out, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _Params(ctypes.Structure):
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


@dataclass
class Params:
    """Model and run parameters (same meaning as the C-ABI's ``pca_params``)."""
    height: int
    width: int
    levels: int
    chains: int = 1
    neighbourhood: int = 4
    prior: int = TRUNC_LINEAR
    trunc: int = 1
    J: float = 0.0
    q: float = 0.0
    sigma: float = 1.0
    vmin: float = 0.0
    vmax: Optional[float] = None
    beta: Sequence[float] = field(default_factory=list)
    seed: int = 0
    init_mode: int = 0
    burn_in: int = 0
    tally_stride: int = 0
    inertia: int = 0

    def __post_init__(self):
        if self.vmax is None:
            self.vmax = float(self.levels - 1)


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORC_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(path):
                build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        u8, u16, u32, f32 = P(ctypes.c_uint8), P(ctypes.c_uint16), P(ctypes.c_uint32), P(ctypes.c_float)
        i32, i64 = P(ctypes.c_int32), P(ctypes.c_int64)
        pp = P(_Params)
        L.orc_philox4x32_10.argtypes = [u32, u32, u32]
        L.orc_philox4x32_10.restype = None
        L.orc_exp2s.argtypes = [ctypes.c_float]
        L.orc_exp2s.restype = ctypes.c_float
        L.orc_uniform.argtypes = [ctypes.c_uint32]
        L.orc_uniform.restype = ctypes.c_float
        L.orc_level_obs.argtypes = [pp, ctypes.c_float]
        L.orc_level_obs.restype = ctypes.c_float
        L.orc_init_state.argtypes = [pp, f32, u8]
        L.orc_run.argtypes = [pp, f32, u8, ctypes.c_int64, ctypes.c_int32, u32, i64, u16, ctypes.c_int32]
        L.orc_update_sites.argtypes = [pp, f32, u8, ctypes.c_int64, ctypes.c_int64, i32, i64, u8]
        L.orc_site_acc.argtypes = [pp, f32, u8, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int64, ctypes.c_int32, f32]
        L.orc_posterior_mean.argtypes = [pp, u32, ctypes.c_int64, f32]
        L.orc_marginal_map.argtypes = [pp, u16, u8]
        L.orc_constants.argtypes = [pp, ctypes.c_int64, ctypes.c_int32, f32]
        L.orc_draw.argtypes = [f32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32]
        L.orc_draw.restype = ctypes.c_int32
        L.orc_pca_rows.argtypes = [pp, f32, u8, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, u8]
        L.orc_inertia_exponents.argtypes = [pp, f32, u8, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int64, f32, f32]
        for name in ("orc_init_state", "orc_run", "orc_update_sites", "orc_site_acc",
                     "orc_posterior_mean", "orc_marginal_map", "orc_constants", "orc_pca_rows",
                     "orc_inertia_exponents"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class _Bound:
    """Keeps the ctypes struct and the beta buffer alive together."""

    def __init__(self, p: Params):
        self.beta = np.ascontiguousarray(np.asarray(p.beta, dtype=np.float32))
        self.s = _Params(
            p.height, p.width, p.levels, p.chains, p.neighbourhood, p.prior, p.trunc,
            p.J, p.q, p.sigma, p.vmin, p.vmax,
            _ptr(self.beta, ctypes.c_float) if self.beta.size else None, int(self.beta.size),
            p.seed & 0xFFFFFFFFFFFFFFFF, p.init_mode, p.burn_in, p.tally_stride, p.inertia)

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _check(rc: int, what: str):
    if rc != OK:
        raise ValueError(f"{what} failed with code {rc}")


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def exp2s(y: float) -> float:
    return float(lib().orc_exp2s(float(np.float32(y))))


def uniform(r: int) -> float:
    return float(lib().orc_uniform(int(r)))


def constants(p: Params, t: int = 0, gibbs: bool = False):
    """(c2, R, a2) of sweep t as float32 values."""
    b = _Bound(p)
    out = np.zeros(3, dtype=np.float32)
    _check(lib().orc_constants(b.ref, t, int(gibbs), _ptr(out, ctypes.c_float)), "orc_constants")
    return out


def level_obs(p: Params, g: float) -> float:
    b = _Bound(p)
    return float(lib().orc_level_obs(b.ref, float(g)))


def init_state(p: Params, obs: np.ndarray) -> np.ndarray:
    b = _Bound(p)
    obs = np.ascontiguousarray(obs, dtype=np.float32)
    assert obs.shape == (p.height, p.width)
    st = np.zeros((p.chains, p.height, p.width), dtype=np.uint8)
    _check(lib().orc_init_state(b.ref, _ptr(obs, ctypes.c_float), _ptr(st, ctypes.c_uint8)), "orc_init_state")
    return st


class Run:
    """State and statistics of an oracle run, advanced with :meth:`sweep`."""

    def __init__(self, p: Params, obs: np.ndarray, gibbs: bool = False, state: Optional[np.ndarray] = None,
                 t: int = 0):
        self.p = p
        self.gibbs = bool(gibbs)
        self.obs = np.ascontiguousarray(obs, dtype=np.float32)
        assert self.obs.shape == (p.height, p.width)
        self.state = init_state(p, self.obs) if state is None else np.ascontiguousarray(state, dtype=np.uint8).copy()
        assert self.state.shape == (p.chains, p.height, p.width)
        self.t = int(t)
        self.sum = np.zeros((p.height, p.width), dtype=np.uint32)
        self.count = np.zeros(1, dtype=np.int64)
        self.hist = np.zeros((p.height, p.width, p.levels), dtype=np.uint16) if p.tally_stride > 0 else None
        self._b = _Bound(p)

    def sweep(self, n: int = 1) -> "Run":
        hist_ptr = _ptr(self.hist, ctypes.c_uint16) if self.hist is not None else None
        rc = lib().orc_run(self._b.ref, _ptr(self.obs, ctypes.c_float), _ptr(self.state, ctypes.c_uint8),
                           self.t, int(n), _ptr(self.sum, ctypes.c_uint32), _ptr(self.count, ctypes.c_int64),
                           hist_ptr, int(self.gibbs))
        _check(rc, "orc_run")
        self.t += int(n)
        return self

    def posterior_mean(self) -> np.ndarray:
        out = np.zeros((self.p.height, self.p.width), dtype=np.float32)
        rc = lib().orc_posterior_mean(self._b.ref, _ptr(self.sum, ctypes.c_uint32), int(self.count[0]),
                                      _ptr(out, ctypes.c_float))
        _check(rc, "orc_posterior_mean")
        return out

    def marginal_map(self) -> np.ndarray:
        if self.hist is None:
            raise ValueError("no histogram: tally_stride is 0")
        out = np.zeros((self.p.height, self.p.width), dtype=np.uint8)
        _check(lib().orc_marginal_map(self._b.ref, _ptr(self.hist, ctypes.c_uint16), _ptr(out, ctypes.c_uint8)),
               "orc_marginal_map")
        return out


def update_sites(p: Params, obs: np.ndarray, state: np.ndarray, t: int, chains: np.ndarray,
                 pixels: np.ndarray) -> np.ndarray:
    """PCA values after sweep t at the given (chain, pixel) sites of the full state."""
    b = _Bound(p)
    obs = np.ascontiguousarray(obs, dtype=np.float32)
    state = np.ascontiguousarray(state, dtype=np.uint8)
    chains = np.ascontiguousarray(chains, dtype=np.int32)
    pixels = np.ascontiguousarray(pixels, dtype=np.int64)
    out = np.zeros(chains.shape[0], dtype=np.uint8)
    rc = lib().orc_update_sites(b.ref, _ptr(obs, ctypes.c_float), _ptr(state, ctypes.c_uint8), int(t),
                                int(chains.shape[0]), _ptr(chains, ctypes.c_int32), _ptr(pixels, ctypes.c_int64),
                                _ptr(out, ctypes.c_uint8))
    _check(rc, "orc_update_sites")
    return out


def pca_rows(p: Params, obs: np.ndarray, state: np.ndarray, t: int, chain: int, r0: int, r1: int) -> np.ndarray:
    """New values of one chain after PCA sweep t for rows r0 .. r1-1, from the full
    previous state [C][H][W] (the oracle's C code runs outside the interpreter lock, so
    row bands may be computed in several threads)."""
    b = _Bound(p)
    obs = np.ascontiguousarray(obs, dtype=np.float32)
    state = np.ascontiguousarray(state, dtype=np.uint8)
    assert state.shape == (p.chains, p.height, p.width) and obs.shape == (p.height, p.width)
    out = np.zeros((r1 - r0, p.width), dtype=np.uint8)
    rc = lib().orc_pca_rows(b.ref, _ptr(obs, ctypes.c_float), _ptr(state, ctypes.c_uint8), int(t), int(chain),
                            int(r0), int(r1), _ptr(out, ctypes.c_uint8))
    _check(rc, "orc_pca_rows")
    return out


def pca_sweep_threaded(p: Params, obs: np.ndarray, state: np.ndarray, t: int, threads: int = 8,
                       band: int = 64) -> np.ndarray:
    """The whole next state [C][H][W] after PCA sweep t, computed in row bands of every
    chain by a pool of host threads."""
    from concurrent.futures import ThreadPoolExecutor
    obs = np.ascontiguousarray(obs, dtype=np.float32)
    state = np.ascontiguousarray(state, dtype=np.uint8)
    out = np.empty_like(state)
    jobs = [(ch, r0, min(r0 + band, p.height)) for ch in range(p.chains) for r0 in range(0, p.height, band)]

    def one(job):
        ch, r0, r1 = job
        out[ch, r0:r1] = pca_rows(p, obs, state, t, ch, r0, r1)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as pool:
        list(pool.map(one, jobs))
    return out


def inertia_exponents(p: Params, obs: np.ndarray, state: np.ndarray, chain: int, r: int, c: int, t: int = 0):
    """(F_0 .. F_{L-1}, Fmax): the unshifted L1/L2 exponents of one site and the O(1)
    shift the sampler subtracts from them."""
    b = _Bound(p)
    obs = np.ascontiguousarray(obs, dtype=np.float32)
    state = np.ascontiguousarray(state, dtype=np.uint8)
    F = np.zeros(p.levels, dtype=np.float32)
    fmax = np.zeros(1, dtype=np.float32)
    rc = lib().orc_inertia_exponents(b.ref, _ptr(obs, ctypes.c_float), _ptr(state, ctypes.c_uint8), chain, r, c,
                                     t, _ptr(F, ctypes.c_float), _ptr(fmax, ctypes.c_float))
    _check(rc, "orc_inertia_exponents")
    return F, float(fmax[0])


def site_acc(p: Params, obs: np.ndarray, state: np.ndarray, chain: int, r: int, c: int, t: int = 0,
             gibbs: bool = False) -> np.ndarray:
    """Running sums [acc_-1, acc_0, ..., acc_{L-1}] of one site."""
    b = _Bound(p)
    obs = np.ascontiguousarray(obs, dtype=np.float32)
    state = np.ascontiguousarray(state, dtype=np.uint8)
    out = np.zeros(p.levels + 1, dtype=np.float32)
    rc = lib().orc_site_acc(b.ref, _ptr(obs, ctypes.c_float), _ptr(state, ctypes.c_uint8), chain, r, c, t,
                            int(gibbs), _ptr(out, ctypes.c_float))
    _check(rc, "orc_site_acc")
    return out


def draw(acc: np.ndarray, x: int, rword: int) -> int:
    """The inverse-CDF draw from running sums [acc_-1, acc_0, ..., acc_{L-1}]."""
    acc = np.ascontiguousarray(acc, dtype=np.float32)
    return int(lib().orc_draw(_ptr(acc, ctypes.c_float), acc.size - 1, int(x), int(rword) & 0xFFFFFFFF))


def site_probs(p: Params, obs, state, chain, r, c, t=0, gibbs=False) -> np.ndarray:
    """Probability of each new level implied by the FP32 running sums (stay folded into x)."""
    acc = site_acc(p, obs, state, chain, r, c, t, gibbs).astype(np.float64)
    Z = acc[-1]
    w = np.diff(acc)  # weights of levels 0..L-1
    x = int(np.asarray(state)[chain, r, c])
    w[x] += acc[0]
    return w / Z
