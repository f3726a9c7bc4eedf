"""Helpers for the GPU parity tests: run the HIP path through the C ABI and the CPU oracle
on the same seeded inputs.  Inputs flow only oracle -> GPU (initial and resynchronised
states); expected values come only from the oracle."""
from __future__ import annotations

import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def params_dict(**kw):
    keys = ("height", "width", "levels", "chains", "neighbourhood", "prior", "trunc", "J", "q", "sigma", "vmin",
            "vmax", "beta", "seed", "init_mode", "burn_in", "tally_stride", "inertia")
    return {k: v for k, v in kw.items() if k in keys}


def gpu_sampler(obs: np.ndarray, **kw):
    torch = torch_cuda()
    from paper_2507_14869_amd import Sampler
    pd = params_dict(**kw)
    levels = pd.pop("levels")
    pd.pop("height", None)
    pd.pop("width", None)
    return Sampler(torch.from_numpy(np.ascontiguousarray(obs, dtype=np.float32)).cuda(), levels=levels, **pd)


def oracle_run(orc, obs: np.ndarray, gibbs=False, **kw):
    return orc.Run(orc.Params(**params_dict(**kw)), obs, gibbs=gibbs)


def stepwise(orc, obs, sweeps: int, *, resync: bool = True, **kw):
    """Advance both implementations one sweep at a time from the oracle's state.
    Returns (mismatching site updates, total site updates, oracle run, gpu sampler)."""
    torch = torch_cuda()
    ref = oracle_run(orc, obs, **kw)
    gpu = gpu_sampler(obs, **kw)
    st0 = gpu.state().cpu().numpy()
    assert np.array_equal(st0, ref.state), "initial states differ"
    bad = 0
    total = 0
    for _ in range(sweeps):
        if resync:
            gpu.set_state(torch.from_numpy(ref.state.copy()).cuda(), ref.t)
        ref.sweep(1)
        gpu.sweep(1)
        got = gpu.state().cpu().numpy()
        bad += int((got != ref.state).sum())
        total += ref.state.size
    return bad, total, ref, gpu
