"""pca_run_static (the entry point that allocates nothing) against the context entry
points it stands for: pca_init, pca_sweep(n), pca_posterior_mean, pca_marginal_map and
pca_get_state on the same inputs must give the same bytes.  Two calls in a row share the
library's device array, the second on a smaller lattice, then a third with no histogram:
whatever the earlier call left there must not reach the later results."""
import numpy as np
import pytest

from tests.gpu_util import gpu_sampler, torch_cuda

pytestmark = pytest.mark.gpu


def _case(height, width, levels, chains, sweeps, seed, **extra):
    from paper_2507_14869_amd import PCA_PRIOR_POTTS, PCA_PRIOR_TRUNC_LINEAR
    rng = np.random.default_rng(seed)
    obs = (rng.random((height, width), dtype=np.float32) * (levels - 1)
           + rng.normal(0.0, 0.15 * levels, (height, width)).astype(np.float32))
    kw = dict(height=height, width=width, levels=levels, chains=chains, neighbourhood=4,
              prior=PCA_PRIOR_TRUNC_LINEAR if levels > 2 else PCA_PRIOR_POTTS,
              trunc=min(4, levels - 1), J=0.3, q=1.2, sigma=0.2 * levels, vmin=0.0, vmax=float(levels - 1),
              seed=seed, init_mode=0, burn_in=sweeps // 4, tally_stride=1)
    kw.update(extra)
    return obs.astype(np.float32), kw, sweeps


def _context_run(obs, kw, sweeps):
    s = gpu_sampler(obs, **kw)
    s.sweep(sweeps)
    mean = s.posterior_mean().cpu().numpy()
    mpm = s.marginal_map().cpu().numpy() if kw["tally_stride"] > 0 else None
    state = s.state().cpu().numpy()
    s.close()
    return mean, mpm, state


def _static_run(obs, kw, sweeps):
    torch = torch_cuda()
    from paper_2507_14869_amd import _lib
    H, W, C = kw["height"], kw["width"], kw["chains"]
    dev_obs = torch.from_numpy(obs).cuda()
    mean = torch.full((H, W), float("nan"), dtype=torch.float32, device="cuda")
    mpm = torch.full((H, W), 255, dtype=torch.uint8, device="cuda") if kw["tally_stride"] > 0 else None
    state = torch.full((C, H, W), 255, dtype=torch.uint8, device="cuda")
    p, _buf = _lib.make_params(**kw)
    stream = torch.cuda.current_stream().cuda_stream
    _lib.pca_run_static(p, dev_obs.data_ptr(), sweeps, mean.data_ptr(), mpm.data_ptr() if mpm is not None else 0,
                        state.data_ptr(), stream)
    torch.cuda.synchronize()
    return mean.cpu().numpy(), (mpm.cpu().numpy() if mpm is not None else None), state.cpu().numpy()


def test_static_run_matches_the_context_entry_points_on_consecutive_calls():
    torch_cuda()
    cases = [
        # 96 x 80 (several workgroups and a ragged last one), 16 levels, 8 chains, a beta schedule
        _case(96, 80, 16, 8, 24, 11, beta=[0.6 + 0.05 * i for i in range(10)]),
        # smaller and with more levels: 33 x 21, 256 levels, 4 chains (16-level blocks)
        _case(33, 21, 256, 4, 9, 12, trunc=32, J=0.05, q=1.0),
        # no histogram, binary Potts, one chain
        _case(17, 29, 2, 1, 13, 13, tally_stride=0, J=0.8, q=2.0, sigma=0.6, vmin=-1.0, vmax=1.0),
    ]
    for obs, kw, sweeps in cases:
        print(f"pca_run_static vs context: {kw['height']}x{kw['width']} L={kw['levels']} C={kw['chains']} "
              f"sweeps={sweeps}", flush=True)
        want = _context_run(obs, kw, sweeps)
        got = _static_run(obs, kw, sweeps)
        assert np.array_equal(got[0].view(np.uint32), want[0].view(np.uint32)), "posterior mean differs"
        if want[1] is not None:
            assert np.array_equal(got[1], want[1]), "marginal mode differs"
        assert np.array_equal(got[2], want[2]), "last states differ"


def test_static_run_refuses_a_run_above_its_working_memory():
    torch = torch_cuda()
    from paper_2507_14869_amd import _lib
    obs = torch.zeros((2048, 2048), dtype=torch.float32, device="cuda")
    mean = torch.empty_like(obs)
    p, _buf = _lib.make_params(height=2048, width=2048, levels=256, chains=16, trunc=32, J=0.05, q=1.0, sigma=20.0,
                               tally_stride=1)
    with pytest.raises(_lib.PcaError) as e:
        _lib.pca_run_static(p, obs.data_ptr(), 2, mean.data_ptr(), 0, 0)
    assert e.value.code == _lib.PCA_EINVAL


def test_static_run_replays_from_a_captured_graph():
    """The use it is for: pca_run_static captured into a HIP graph (it launches kernels only,
    no allocation and no memset node) and replayed three times, with eager work on the
    same outputs in between; every replay gives the eager call's bytes."""
    torch = torch_cuda()
    from paper_2507_14869_amd import _lib
    obs, kw, sweeps = _case(64, 48, 16, 8, 12, 21, beta=[0.9, 1.0, 1.1])
    H, W, C = kw["height"], kw["width"], kw["chains"]
    want = _static_run(obs, kw, sweeps)  # eager, also looks the device array up before capture
    dev_obs = torch.from_numpy(obs).cuda()
    mean = torch.empty((H, W), dtype=torch.float32, device="cuda")
    mpm = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    state = torch.empty((C, H, W), dtype=torch.uint8, device="cuda")
    p, _buf = _lib.make_params(**kw)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        _lib.pca_run_static(p, dev_obs.data_ptr(), sweeps, mean.data_ptr(), mpm.data_ptr(), state.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        mean.fill_(float("nan"))
        mpm.fill_(255)
        state.fill_(255)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(mean.cpu().numpy().view(np.uint32), want[0].view(np.uint32)), rep
        assert np.array_equal(mpm.cpu().numpy(), want[1]), rep
        assert np.array_equal(state.cpu().numpy(), want[2]), rep
