"""Lazy Probabilistic Cellular Automaton sampler for lattice-MRF image denoising on
AMD Instinct MI355X (gfx950), after Costarelli, Piconi, Troiani (arXiv 2507.14869).

The sampler is the HIP library ``libpca.so`` behind the C ABI of ``include/pca.h``;
``_lib`` binds its entry points under the same names and :class:`Sampler` holds a
context together with the torch tensors that carry device memory and streams.
"""
from __future__ import annotations

from typing import Optional, Sequence

from . import _lib
from ._lib import (PCA_OK, PCA_EINVAL, PCA_ENOMEM, PCA_EDEVICE, PCA_ESTATE, PCA_EBUSY, PCA_PRIOR_POTTS, PCA_PRIOR_TRUNC_LINEAR, PcaError, make_params, pca_destroy,  # noqa
                   pca_get_state, pca_init, pca_last_error, pca_marginal_map, pca_posterior_mean, pca_set_state, pca_stats,
                   pca_sweeps_per_launch,
                   pca_sweep, pca_sync, pca_batch_init, pca_batch_autotune, pca_batch_config, pca_batch_set_config,
                   pca_batch_sweep, pca_batch_posterior_mean, pca_batch_marginal_map, pca_batch_get_state,
                   pca_batch_stats, pca_batch_sync, pca_batch_destroy, pca_server_create, pca_server_submit,
                   pca_server_step, pca_server_completed, pca_server_status, pca_server_result, pca_server_release,
                   pca_server_stats, pca_server_set_shedding, pca_server_shed_count, pca_server_destroy,
                   pca_get_accumulators, pca_set_accumulators, pca_run_static)


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


class Sampler:
    """One lazy-PCA run on the current GPU: ``obs`` is a float32 [H, W] tensor in value units.

    Keyword parameters are those of ``pca_params`` (include/pca.h).  All calls enqueue on
    ``stream`` (default: torch's current stream) and return torch tensors.
    """

    def __init__(self, obs, *, levels: int, chains: int = 1, neighbourhood: int = 4,
                 prior: int = PCA_PRIOR_TRUNC_LINEAR, trunc: int = 1, J: float = 0.0, q: float = 0.0,
                 sigma: float = 1.0, vmin: float = 0.0, vmax: Optional[float] = None,
                 beta: Sequence[float] = (), seed: int = 0, init_mode: int = 0, burn_in: int = 0,
                 tally_stride: int = 0, inertia: int = 0, stream=None):
        import torch
        _lib.load()
        if obs.dtype != torch.float32 or obs.dim() != 2 or not obs.is_cuda:
            raise ValueError("obs must be a float32 [H, W] CUDA tensor")
        self.obs = obs.contiguous()
        self.height, self.width = int(obs.shape[0]), int(obs.shape[1])
        self.levels, self.chains = levels, chains
        self.device = obs.device
        self.params, self._beta_buf = make_params(
            height=self.height, width=self.width, levels=levels, chains=chains, neighbourhood=neighbourhood,
            prior=prior, trunc=trunc, J=J, q=q, sigma=sigma, vmin=vmin, vmax=vmax, beta=beta, seed=seed,
            init_mode=init_mode, burn_in=burn_in, tally_stride=tally_stride, inertia=inertia)
        self.ctx = pca_init(self.params, self.obs.data_ptr(), _stream_handle(stream))

    def sweep(self, n: int = 1, stream=None) -> "Sampler":
        pca_sweep(self.ctx, n, _stream_handle(stream))
        return self

    def posterior_mean(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.height, self.width), dtype=torch.float32, device=self.device)
        pca_posterior_mean(self.ctx, out.data_ptr(), _stream_handle(stream))
        return out

    def marginal_map(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.height, self.width), dtype=torch.uint8, device=self.device)
        pca_marginal_map(self.ctx, out.data_ptr(), _stream_handle(stream))
        return out

    def state(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.chains, self.height, self.width), dtype=torch.uint8, device=self.device)
        pca_get_state(self.ctx, out.data_ptr(), _stream_handle(stream))
        return out

    def set_state(self, x, t: int, stream=None) -> "Sampler":
        import torch
        if x.dtype != torch.uint8 or tuple(x.shape) != (self.chains, self.height, self.width) or not x.is_cuda:
            raise ValueError("state must be a uint8 [chains, H, W] CUDA tensor")
        self._set_buf = x.contiguous()
        pca_set_state(self.ctx, self._set_buf.data_ptr(), t, _stream_handle(stream))
        return self

    def stats(self):
        """(sweep index, samples in the mean, tally sweeps)."""
        return pca_stats(self.ctx)

    def sweeps_per_launch(self) -> int:
        """Sweeps one kernel launch advances (1, or several from LDS tiles on small lattices)."""
        return pca_sweeps_per_launch(self.ctx)

    def accumulators(self, stream=None):
        """(sum, hist): the raw accumulators as int32 [H, W] and int16 [H, W, levels] CUDA
        tensors holding the bits of the uint32 level sums and uint16 level tallies (hist is
        None without a histogram).  With :meth:`state` and :meth:`stats` this checkpoints a
        run; :meth:`set_accumulators` restores it."""
        import torch
        s = torch.empty((self.height, self.width), dtype=torch.int32, device=self.device)
        h = (torch.empty((self.height, self.width, self.levels), dtype=torch.int16, device=self.device)
             if self.params.tally_stride > 0 else None)
        pca_get_accumulators(self.ctx, s.data_ptr(), h.data_ptr() if h is not None else 0, _stream_handle(stream))
        return s, h

    def set_accumulators(self, sum_, hist, count: int, tallies: int, stream=None) -> "Sampler":
        import torch
        if sum_.dtype != torch.int32 or tuple(sum_.shape) != (self.height, self.width) or not sum_.is_cuda:
            raise ValueError("sum must be an int32 [H, W] CUDA tensor")
        if hist is not None and (hist.dtype != torch.int16 or not hist.is_cuda
                                 or tuple(hist.shape) != (self.height, self.width, self.levels)):
            raise ValueError("hist must be an int16 [H, W, levels] CUDA tensor")
        self._acc_bufs = (sum_.contiguous(), hist.contiguous() if hist is not None else None)
        pca_set_accumulators(self.ctx, self._acc_bufs[0].data_ptr(),
                             self._acc_bufs[1].data_ptr() if hist is not None else 0, count, tallies,
                             _stream_handle(stream))
        return self

    def sync(self):
        pca_sync(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            pca_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent lattices advanced together, one kernel launch per sweep.

    ``problems`` is a sequence of (obs, params) pairs: obs a float32 [H, W] CUDA tensor and
    params a dict of ``pca_params`` fields (``levels`` required).  All lattices share the
    neighbourhood and the sweep index.
    """

    def __init__(self, problems, stream=None):
        import torch
        _lib.load()
        self._obs = []
        self._params = []
        self._bufs = []
        self.shapes = []
        for obs, kw in problems:
            if obs.dtype != torch.float32 or obs.dim() != 2 or not obs.is_cuda:
                raise ValueError("obs must be float32 [H, W] CUDA tensors")
            obs = obs.contiguous()
            H, W = int(obs.shape[0]), int(obs.shape[1])
            p, buf = make_params(height=H, width=W, **kw)
            self._obs.append(obs)
            self._params.append(p)
            self._bufs.append(buf)
            self.shapes.append((H, W, int(kw.get("chains", 1)), int(kw["levels"])))
        self.device = self._obs[0].device
        self.b = pca_batch_init(self._params, [o.data_ptr() for o in self._obs], _stream_handle(stream))

    def autotune(self, trial_sweeps: int = 3, stream=None) -> float:
        """Picks the fastest launch configuration (ms per sweep); resets the run to sweep 0."""
        return pca_batch_autotune(self.b, trial_sweeps, _stream_handle(stream))

    @property
    def config(self):
        return pca_batch_config(self.b)

    def set_config(self, chains_per_thread: int, share: int, tiled: int, stream=None):
        pca_batch_set_config(self.b, chains_per_thread, share, tiled, _stream_handle(stream))

    def sweep(self, n: int = 1, stream=None) -> "Batch":
        pca_batch_sweep(self.b, n, _stream_handle(stream))
        return self

    def posterior_mean(self, i: int, stream=None):
        import torch
        H, W, _, _ = self.shapes[i]
        out = torch.empty((H, W), dtype=torch.float32, device=self.device)
        pca_batch_posterior_mean(self.b, i, out.data_ptr(), _stream_handle(stream))
        return out

    def marginal_map(self, i: int, stream=None):
        import torch
        H, W, _, _ = self.shapes[i]
        out = torch.empty((H, W), dtype=torch.uint8, device=self.device)
        pca_batch_marginal_map(self.b, i, out.data_ptr(), _stream_handle(stream))
        return out

    def state(self, i: int, stream=None):
        import torch
        H, W, C, _ = self.shapes[i]
        out = torch.empty((C, H, W), dtype=torch.uint8, device=self.device)
        pca_batch_get_state(self.b, i, out.data_ptr(), _stream_handle(stream))
        return out

    def stats(self, i: int):
        return pca_batch_stats(self.b, i)

    def sync(self):
        pca_batch_sync(self.b)

    def close(self):
        if getattr(self, "b", None):
            pca_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server (see ``pca_server_*`` in include/pca.h).

    ``submit(obs, sweeps, **params)`` takes a host float32 [H, W] numpy array; ``step()``
    admits what fits the device-memory budget and advances every admitted request (at least
    one sweep each, the rest of a ``step_ms`` GPU-time budget half to the requests with the
    least remaining work, half to the oldest); ``result(id)`` returns (mean, mode, states)
    as numpy arrays.  ``set_shedding(s)`` makes ``submit`` raise :class:`PcaError` with
    code ``PCA_EBUSY`` while the predicted wait of the accepted work exceeds ``s`` seconds.
    """

    def __init__(self, hbm_budget_bytes: int, max_active: int = 256, sweeps_per_step: int = 300,
                 step_ms: float = 20.0):
        _lib.load()
        self.sv = pca_server_create(hbm_budget_bytes, max_active, sweeps_per_step, step_ms)
        self._shapes = {}

    def submit(self, obs, sweeps: int, **kw) -> int:
        import numpy as np
        obs = np.ascontiguousarray(obs, dtype=np.float32)
        H, W = obs.shape
        p, buf = make_params(height=H, width=W, **kw)
        rid = pca_server_submit(self.sv, p, obs.ctypes.data, sweeps)
        self._shapes[rid] = (H, W, int(kw.get("chains", 1)), int(kw.get("tally_stride", 0)) > 0)
        return rid

    def step(self, stream=None) -> int:
        return pca_server_step(self.sv, _stream_handle(stream))

    def set_shedding(self, max_backlog_s: float):
        pca_server_set_shedding(self.sv, max_backlog_s)

    @property
    def shed(self) -> int:
        """Submissions refused by the shedding limit so far."""
        return pca_server_shed_count(self.sv)

    def completed(self):
        return pca_server_completed(self.sv)

    def status(self, rid: int):
        return pca_server_status(self.sv, rid)

    def result(self, rid: int):
        import numpy as np
        H, W, C, has_mpm = self._shapes[rid]
        mean = np.empty((H, W), np.float32)
        state = np.empty((C, H, W), np.uint8)
        mpm = np.empty((H, W), np.uint8) if has_mpm else None
        pca_server_result(self.sv, rid, mean.ctypes.data, mpm.ctypes.data if mpm is not None else 0,
                          state.ctypes.data)
        return mean, mpm, state

    def release(self, rid: int):
        pca_server_release(self.sv, rid)
        self._shapes.pop(rid, None)

    def stats(self):
        """(queued, active, device bytes held, steps, sweeps launched)."""
        return pca_server_stats(self.sv)

    def close(self):
        if getattr(self, "sv", None):
            pca_server_destroy(self.sv)
            self.sv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
