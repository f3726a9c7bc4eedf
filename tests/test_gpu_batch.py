"""Batched sweeps (one launch per sweep over many lattices, graph-replayed) against the
single-lattice path and the CPU oracle: every lattice must come out bit-identical to
running it alone, for every launch configuration, across repeated graph replays with
eager work and synchronisation in between."""
import numpy as np
import pytest

try:  # import at collection so the first GPU test's time limit does not include it
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

from tests.gpu_util import gpu_sampler, oracle_run, torch_cuda
from workloads import synth

pytestmark = pytest.mark.gpu


def _problem(H, W, L, C, seed, **over):
    rng = np.random.default_rng(seed)
    truth = synth.random_image(H, W, L, max(2, H * W // 300), L > 2, rng)
    sigma = float(rng.uniform(0.1, 0.3) * L)
    obs = synth.noisy_observation(truth, L, 0.0, float(L - 1), sigma, rng)
    fam = {2: (0, 1, 0.8)}.get(L, (1, 4 if L <= 16 else 32, 0.4 if L <= 16 else 0.05))
    kw = dict(levels=L, chains=C, prior=fam[0], trunc=fam[1], J=float(fam[2] * rng.uniform(0.5, 1.5)),
              q=float(rng.uniform(1.0, 2.0)), sigma=sigma, vmin=0.0, vmax=float(L - 1), seed=int(seed) * 7919 + 1,
              burn_in=2, tally_stride=1, beta=[1.0, 1.25, 1.5])
    kw.update(over)
    return obs, kw


def _batch(problems):
    torch = torch_cuda()
    from paper_2507_14869_amd import Batch
    return Batch([(torch.from_numpy(o).cuda(), kw) for o, kw in problems])


def _alone(obs, kw, sweeps):
    return gpu_sampler(obs, height=obs.shape[0], width=obs.shape[1], **kw).sweep(sweeps)


MIXED = [(37, 53, 256, 4, 1), (64, 64, 2, 4, 2), (17, 200, 16, 4, 3), (1, 1, 16, 4, 4), (90, 33, 256, 4, 5),
         (128, 96, 2, 4, 6), (5, 7, 33, 4, 7)]
MIXED_CHAINS = [(30, 31, 16, 1, 11), (22, 40, 256, 2, 12), (19, 19, 2, 3, 13), (40, 12, 33, 5, 14),
                (16, 16, 7, 8, 15)]


@pytest.mark.parametrize("config", [(4, 1, 0), (4, 1, 1), (2, 2, 0), (2, 1, 1), (1, 4, 0), (1, 4, 1), (1, 2, 0),
                                    (1, 1, 1), (4, 1, 2), (2, 2, 2), (1, 4, 2), (1, 1, 2)])
def test_batch_matches_lattices_run_alone(config):
    problems = [_problem(*spec[:4], seed=spec[4]) for spec in MIXED]
    b = _batch(problems)
    b.set_config(*config)
    assert b.config == config
    done = 0
    for rep in range(3):  # three replays of the same captured graph, eager work in between
        b.sweep(4)
        done += 4
        for i, (obs, kw) in enumerate(problems):
            ref = _alone(obs, kw, done)
            assert np.array_equal(b.state(i).cpu().numpy(), ref.state().cpu().numpy()), (config, rep, i)
            assert np.array_equal(b.posterior_mean(i).cpu().numpy(), ref.posterior_mean().cpu().numpy())
            assert np.array_equal(b.marginal_map(i).cpu().numpy(), ref.marginal_map().cpu().numpy())
            assert b.stats(i) == ref.stats()
            ref.close()
        b.sync()
    b.close()


def test_long_calls_replay_bounded_graphs():
    """150 sweeps in one call replay the 64-sweep graph twice and a 22-sweep graph once;
    70 + 80 sweeps replay 64 + 6 and 64 + 16.  Both equal every lattice run alone."""
    problems = [_problem(*spec[:4], seed=spec[4]) for spec in MIXED[:4]]
    one = _batch(problems)
    one.sweep(150)
    two = _batch(problems)
    two.sweep(70)
    two.sweep(80)
    for i, (obs, kw) in enumerate(problems):
        ref = _alone(obs, kw, 150)
        want = ref.state().cpu().numpy()
        assert np.array_equal(one.state(i).cpu().numpy(), want), i
        assert np.array_equal(two.state(i).cpu().numpy(), want), i
        assert np.array_equal(one.posterior_mean(i).cpu().numpy(), ref.posterior_mean().cpu().numpy())
        assert np.array_equal(two.marginal_map(i).cpu().numpy(), ref.marginal_map().cpu().numpy())
        assert one.stats(i) == ref.stats() == two.stats(i)
        ref.close()
    one.close()
    two.close()


def test_batch_with_mixed_chain_counts():
    problems = [_problem(*spec[:4], seed=spec[4]) for spec in MIXED_CHAINS]
    b = _batch(problems)
    assert b.config[0] == 1  # only one chain per thread divides every chain count here
    b.sweep(5).sweep(5)
    for i, (obs, kw) in enumerate(problems):
        ref = _alone(obs, kw, 10)
        assert np.array_equal(b.state(i).cpu().numpy(), ref.state().cpu().numpy()), i
        assert np.array_equal(b.posterior_mean(i).cpu().numpy(), ref.posterior_mean().cpu().numpy())
    with pytest.raises(Exception):
        b.set_config(4, 1, 0)


def test_batch_autotune_restores_initial_state_and_keeps_results(orc):
    problems = [_problem(*spec[:4], seed=spec[4]) for spec in MIXED[:4]]
    b = _batch(problems)
    ms = b.autotune(2)
    assert ms > 0
    assert b.stats(0) == (0, 0, 0)
    b.sweep(6)
    for i, (obs, kw) in enumerate(problems):
        ref = oracle_run(orc, obs, height=obs.shape[0], width=obs.shape[1], **kw).sweep(6)
        assert np.array_equal(b.state(i).cpu().numpy(), ref.state), i
        assert np.array_equal(b.posterior_mean(i).cpu().numpy(), ref.posterior_mean())
        assert np.array_equal(b.marginal_map(i).cpu().numpy(), ref.marginal_map())


def test_batch_rejects_mixed_neighbourhoods_and_bad_configs():
    from paper_2507_14869_amd import PcaError
    p1 = _problem(16, 16, 16, 4, 1)
    p2 = _problem(16, 16, 16, 4, 2, neighbourhood=8)
    with pytest.raises(PcaError):
        _batch([p1, p2])
    b = _batch([p1])
    with pytest.raises(PcaError):
        b.set_config(3, 1, 0)
    with pytest.raises(PcaError):
        b.sweep(-1)
    with pytest.raises(PcaError):
        b.posterior_mean(0)  # nothing accumulated yet (burn-in 2)
    b.close()


def test_batch_eight_neighbour():
    problems = [_problem(24, 29, L, 4, s, neighbourhood=8, prior=0, trunc=1) for s, L in ((21, 5), (22, 9), (23, 33))]
    b = _batch(problems)
    b.sweep(7)
    for i, (obs, kw) in enumerate(problems):
        ref = _alone(obs, kw, 7)
        assert np.array_equal(b.state(i).cpu().numpy(), ref.state().cpu().numpy()), i


def test_batch_with_inertia_norms(orc):
    """Lattices with L1 and L2 inertia in one batch (their kernel differs from the
    indicator's, so a batch holds one form or the other)."""
    problems = [_problem(33, 20, 256, 4, 31, inertia=1, q=0.02), _problem(40, 17, 16, 4, 32, inertia=2, q=0.3),
                _problem(19, 25, 2, 2, 33, inertia=1), _problem(12, 70, 33, 8, 34, inertia=2, q=0.05)]
    b = _batch(problems)
    assert b.config[1] == 1
    b.sweep(3).sweep(3)
    for i, (obs, kw) in enumerate(problems):
        ref = oracle_run(orc, obs, height=obs.shape[0], width=obs.shape[1], **kw).sweep(6)
        assert np.array_equal(b.state(i).cpu().numpy(), ref.state), i
        assert np.array_equal(b.posterior_mean(i).cpu().numpy(), ref.posterior_mean())
        assert np.array_equal(b.marginal_map(i).cpu().numpy(), ref.marginal_map())
    from paper_2507_14869_amd import PcaError
    with pytest.raises(PcaError):
        b.set_config(4, 2, 0)
    with pytest.raises(PcaError):
        _batch([problems[0], _problem(16, 16, 16, 4, 35)])
    b.close()


@pytest.mark.parametrize("chains,configs", [(12, [(4, 1, 1), (2, 2, 1), (1, 4, 1), (1, 2, 1)]),
                                            (20, [(4, 1, 1), (2, 2, 1), (2, 1, 1)])])
def test_tiled_batch_with_pixels_that_do_not_fill_a_tile(orc, chains, configs):
    """Tiled traversal with 3, 5, 6, 10 or 12 threads per pixel: 256 threads then hold
    fewer than a whole number of 16-pixel tile rows, and the threads left over must not
    sweep pixels of the next tile (which would count them twice in the mean and the
    histogram).  Each lattice equals itself run alone, and one equals the CPU reference."""
    problems = [_problem(*spec, seed=60 + i) for i, spec in enumerate([(29, 37, 16, chains), (40, 21, 256, chains),
                                                                       (17, 33, 2, chains)])]
    for config in configs:
        b = _batch(problems)
        b.set_config(*config)
        assert b.config == config
        b.sweep(3).sweep(4)
        for i, (obs, kw) in enumerate(problems):
            ref = _alone(obs, kw, 7)
            assert np.array_equal(b.state(i).cpu().numpy(), ref.state().cpu().numpy()), (config, i)
            assert np.array_equal(b.posterior_mean(i).cpu().numpy(), ref.posterior_mean().cpu().numpy()), (config, i)
            assert np.array_equal(b.marginal_map(i).cpu().numpy(), ref.marginal_map().cpu().numpy()), (config, i)
            assert b.stats(i) == ref.stats()
            ref.close()
        obs, kw = problems[0]
        want = oracle_run(orc, obs, height=obs.shape[0], width=obs.shape[1], **kw).sweep(7)
        assert np.array_equal(b.posterior_mean(0).cpu().numpy(), want.posterior_mean())
        assert np.array_equal(b.marginal_map(0).cpu().numpy(), want.marginal_map())
        b.close()


def test_batch_patches_with_many_threads_per_pixel(orc):
    """Untiled batched launches lay out L > 16 lattices in 2-D pixel patches; with 32 and 64
    chains a pixel takes 8 and 16 threads (2x4 and 2x2-pixel patches per wave), mixed with a
    row-major L = 2 lattice in the same launches: every lattice equals the oracle's run."""
    problems = [_problem(23, 31, 40, 32, 41), _problem(9, 45, 256, 64, 42), _problem(30, 17, 2, 4, 43)]
    b = _batch(problems)
    b.set_config(4, 1, 0)
    b.sweep(5)
    for i, (obs, kw) in enumerate(problems):
        ref = oracle_run(orc, obs, height=obs.shape[0], width=obs.shape[1], **kw).sweep(5)
        assert np.array_equal(b.state(i).cpu().numpy(), ref.state), i
        assert np.array_equal(b.posterior_mean(i).cpu().numpy(), ref.posterior_mean()), i
        assert np.array_equal(b.marginal_map(i).cpu().numpy(), ref.marginal_map()), i



@pytest.mark.parametrize("calls", [(4, 4, 9), (150,), (1, 2, 64)])
def test_batch_of_small_lattices_several_sweeps_per_launch(orc, calls):
    """Traversal 2 with only lattices of at most 16 levels: every launch advances all of them
    by an odd number of sweeps (7, or the rest split into odd parts) from LDS tiles, and no
    one-sweep launch remains.  Sweep counts per call give chunks 3+1, 7s+1, 1, 1+1, 7s+1;
    every lattice equals the oracle's run (state, mean, mode)."""
    problems = [_problem(40, 33, 16, 4, 51), _problem(64, 64, 2, 4, 52), _problem(1, 30, 5, 4, 53),
                _problem(17, 9, 16, 8, 54, beta=[0.7 + 0.1 * i for i in range(10)])]
    b = _batch(problems)
    b.set_config(4, 1, 2)
    assert b.config == (4, 1, 2)
    for n in calls:
        b.sweep(n)
    total = sum(calls)
    for i, (obs, kw) in enumerate(problems):
        ref = oracle_run(orc, obs, height=obs.shape[0], width=obs.shape[1], **kw).sweep(total)
        assert np.array_equal(b.state(i).cpu().numpy(), ref.state), (calls, i)
        assert np.array_equal(b.posterior_mean(i).cpu().numpy(), ref.posterior_mean()), (calls, i)
        assert np.array_equal(b.marginal_map(i).cpu().numpy(), ref.marginal_map()), (calls, i)
    b.close()


def test_full_size_mixed_batch_against_the_oracle(orc):
    """The 64-lattice mixed batch of the benchmark (sides 128-1024, L in {2, 16, 256}, 4
    chains) at full size: two sweeps in the untiled and the tiled traversal, every site update
    and every lattice's posterior mean against the oracle (sweeps computed in row bands on the
    host's cores)."""
    import os
    torch = torch_cuda()
    from paper_2507_14869_amd import Batch
    wls = synth.batch_mix(64, sweeps=2)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    problems, want_state, want_mean = [], [], []
    for w in wls:
        kw = w.params(burn_in=0, tally_stride=1)
        p = orc.Params(**kw)
        x0 = orc.init_state(p, w.obs)
        x1 = orc.pca_sweep_threaded(p, w.obs, x0, 0, threads=threads)
        x2 = orc.pca_sweep_threaded(p, w.obs, x1, 1, threads=threads)
        want_state.append(x2)
        ref = orc.Run(p, w.obs)  # the oracle's mean of the accumulated level sums
        ref.sum[...] = x1.sum(axis=0, dtype=np.uint32) + x2.sum(axis=0, dtype=np.uint32)
        ref.count[0] = 2 * w.chains
        want_mean.append(ref.posterior_mean())
        kw.pop("height")
        kw.pop("width")
        problems.append((torch.from_numpy(w.obs).cuda(), kw))
    for cfg in ((4, 1, 0), (4, 1, 1)):
        b = Batch(problems)
        b.set_config(*cfg)
        b.sweep(2)
        for i in range(len(problems)):
            bad = int((b.state(i).cpu().numpy() != want_state[i]).sum())
            assert bad == 0, (cfg, i, bad)
            assert np.array_equal(b.posterior_mean(i).cpu().numpy(), want_mean[i]), (cfg, i)
        b.close()
