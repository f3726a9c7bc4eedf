"""Several sweeps per launch (lattices with L <= 16 too small to fill the GPU: each
workgroup advances an LDS tile with a halo as deep as the sweeps it runs) against the CPU
oracle.  The runs cross every boundary inside a launch: the beta schedule changes at
every sweep for the first twelve (the prior table is rebuilt inside a launch), burn-in ends
and tally sweeps fall in the middle of one, and 21 sweeps split into launches of 8 or fewer.
Lattice shapes give ragged edge tiles, 1x1 and one-row lattices, tiles of 4x4, 8x8 and
16x16 sites, level counts that are and are not powers of two, and chain counts whose
pixels take 1, 2, 3, 4, 8, 16 or 25 threads (3 and more than 4: global atomics for the
statistics).
States, posterior means and marginal modes must be identical."""
import numpy as np
import pytest

from tests.gpu_util import gpu_sampler, oracle_run, torch_cuda
from workloads import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", [
    # (H, W, L, chains, nbr, prior, T)
    (1, 1, 4, 1, 4, 1, 2),
    (1, 45, 16, 4, 8, 1, 4),
    (5, 3, 16, 12, 8, 1, 3),     # 3 threads per pixel
    (33, 29, 5, 6, 4, 1, 2),     # ragged 4x4 tiles, padded chain slots
    (64, 64, 2, 1, 4, 0, 1),     # the binary workload's shape
    (17, 70, 16, 8, 8, 1, 4),
    (40, 40, 9, 2, 4, 0, 1),
    (128, 128, 16, 4, 4, 1, 4),  # 8x8 tiles
    (20, 24, 3, 16, 4, 1, 2),    # 4 threads per pixel: 4 sweeps per launch fit, not 8
    (12, 10, 6, 29, 8, 1, 3),    # 8 threads per pixel: global atomics for the statistics
    (240, 256, 3, 1, 4, 1, 2),   # 16x16 tiles, 4 items per thread in the first sweep
    (9, 11, 8, 64, 4, 1, 2),     # 16 threads per pixel, 2 sweeps per launch
    (6, 7, 16, 100, 8, 1, 4),    # 25 threads per pixel: a pixel's threads span two waves
])
def test_several_sweeps_per_launch_match_the_oracle(orc, case):
    torch_cuda()
    H, W, L, C, nbr, prior, T = case
    rng = np.random.default_rng(H * 131 + W * 7 + C)
    truth = synth.random_image(H, W, L, max(2, H * W // 300), L > 2, rng)
    obs = synth.noisy_observation(truth, L, 0.0, float(L - 1), 0.25 * L, rng)
    kw = dict(height=H, width=W, levels=L, chains=C, neighbourhood=nbr, prior=prior, trunc=T, J=0.35, q=1.1,
              sigma=0.25 * L, vmin=0.0, vmax=float(L - 1), beta=[0.8 + 0.1 * i for i in range(12)],
              seed=900 + H + W, burn_in=3, tally_stride=2)
    ref = oracle_run(orc, obs, **kw).sweep(21)
    gpu = gpu_sampler(obs, **kw)
    assert gpu.sweeps_per_launch() > 1
    gpu.sweep(21)
    assert np.array_equal(gpu.state().cpu().numpy(), ref.state)
    assert np.array_equal(gpu.posterior_mean().cpu().numpy(), ref.posterior_mean())
    assert np.array_equal(gpu.marginal_map().cpu().numpy(), ref.marginal_map())
    # and split differently: 5 + 1 + 15 sweeps
    gpu2 = gpu_sampler(obs, **kw).sweep(5).sweep(1).sweep(15)
    assert np.array_equal(gpu2.state().cpu().numpy(), ref.state)
    assert np.array_equal(gpu2.posterior_mean().cpu().numpy(), ref.posterior_mean())
    gpu.close()
    gpu2.close()


@pytest.mark.parametrize("shape,expected", [
    # (H, W, L, chains, inertia), sweeps per launch
    ((64, 64, 2, 1, 0), 12),      # the binary workload: 4x4 tiles, 12 sweeps
    ((20, 24, 3, 16, 0), 4),      # 4 threads per pixel: the items of 8 or 10 sweeps do not fit
    ((64, 64, 2, 1, 1), 1),       # L1 inertia: one sweep per launch
    ((64, 64, 17, 1, 0), 1),      # more than 16 levels
    ((512, 512, 16, 8, 0), 1),    # fills the GPU with one sweep
])
def test_sweeps_per_launch_reports_the_plan(shape, expected):
    torch = torch_cuda()
    from paper_2507_14869_amd import Sampler
    H, W, L, C, inertia = shape
    obs = torch.zeros((H, W), dtype=torch.float32, device="cuda")
    s = Sampler(obs, levels=L, chains=C, prior=1, trunc=2, J=0.3, q=1.0, sigma=1.0, vmin=0.0, vmax=float(L - 1),
                seed=5, inertia=inertia)
    assert s.sweeps_per_launch() == expected
    s.close()


@pytest.mark.parametrize("seed", range(64))
def test_random_small_lattices_match_the_oracle(orc, seed):
    """Seeded random small lattices (sides 1-48, 2-16 levels, 1-24 chains, 4 or 8 neighbours,
    either prior, a beta schedule or none, burn-in and tally stride) run in random call
    splits: states, posterior means and marginal modes identical to the oracle's."""
    torch_cuda()
    rng = np.random.default_rng(7100 + seed)
    H, W = int(rng.integers(1, 49)), int(rng.integers(1, 49))
    L = int(rng.integers(2, 17))
    C = int(rng.choice([1, 2, 3, 4, 5, 8, 12, 16, 24]))
    nbr = int(rng.choice([4, 8]))
    prior = 0 if L == 2 else int(rng.integers(0, 2))
    T = int(rng.integers(1, 8))
    beta = [float(b) for b in rng.uniform(0.5, 2.0, size=int(rng.integers(0, 20)))]
    sweeps = int(rng.integers(1, 26))
    truth = synth.random_image(H, W, L, max(2, H * W // 200), L > 2, rng)
    obs = synth.noisy_observation(truth, L, 0.0, float(L - 1), float(rng.uniform(0.1, 0.3)) * L, rng)
    kw = dict(height=H, width=W, levels=L, chains=C, neighbourhood=nbr, prior=prior, trunc=T,
              J=float(rng.uniform(0.05, 0.8)), q=float(rng.uniform(0.0, 2.0)), sigma=float(rng.uniform(0.1, 0.3)) * L,
              vmin=0.0, vmax=float(L - 1), beta=beta, seed=int(rng.integers(0, 2**62)),
              burn_in=int(rng.integers(0, sweeps)), tally_stride=int(rng.integers(0, 4)))
    ref = oracle_run(orc, obs, **kw).sweep(sweeps)
    gpu = gpu_sampler(obs, **kw)
    done = 0
    while done < sweeps:
        n = int(rng.integers(1, sweeps - done + 1))
        gpu.sweep(n)
        done += n
    assert np.array_equal(gpu.state().cpu().numpy(), ref.state)
    if ref.count[0] > 0:
        assert np.array_equal(gpu.posterior_mean().cpu().numpy(), ref.posterior_mean())
    stride, b0 = kw["tally_stride"], kw["burn_in"]
    if stride > 0 and any(t >= b0 and (t - b0) % stride == 0 for t in range(sweeps)):
        assert np.array_equal(gpu.marginal_map().cpu().numpy(), ref.marginal_map())
    gpu.close()
