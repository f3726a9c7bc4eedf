"""HIP path vs the CPU oracle, through the C ABI, on seeded synthetic inputs.

Integer state trajectories must agree bit for bit (the arithmetic is the same FP32
convention on both sides; a threshold tie would show up as a mismatch and is allowed
at most once per 1e6 site updates).  Posterior means and marginal modes are integer
sums turned into values by one rounding, so they must agree exactly.
"""
import numpy as np
import pytest

try:  # import at collection so the first GPU test's time limit does not include it
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

from tests.gpu_util import gpu_sampler, oracle_run, stepwise, torch_cuda
from workloads import synth

pytestmark = pytest.mark.gpu

FLIP_BUDGET = 1e-6


def _obs(H, W, L, seed, vmin=0.0, vmax=None, sigma=None):
    vmax = float(L - 1) if vmax is None else vmax
    rng = np.random.default_rng(seed)
    truth = synth.random_image(H, W, L, max(2, H * W // 400), L > 2, rng)
    sigma = 0.2 * (vmax - vmin) if sigma is None else sigma
    return synth.noisy_observation(truth, L, vmin, vmax, sigma, rng)


def test_c1_free_running_200_sweeps(orc):
    """64x64 binary Ising/Potts image, 1 chain, 200 sweeps: full trajectory, mean and mode."""
    wl = synth.make_workload("c1")
    kw = wl.params()
    ref = oracle_run(orc, wl.obs, **kw).sweep(wl.sweeps)
    gpu = gpu_sampler(wl.obs, **kw).sweep(wl.sweeps)
    assert np.array_equal(gpu.state().cpu().numpy(), ref.state)
    assert np.array_equal(gpu.posterior_mean().cpu().numpy(), ref.posterior_mean())
    assert np.array_equal(gpu.marginal_map().cpu().numpy(), ref.marginal_map())
    assert gpu.stats() == (200, 150, 150)


@pytest.mark.parametrize("case", [
    # (H, W, L, chains, nbr, prior, T, J, q, sigma)
    (96, 80, 16, 8, 4, 1, 4, 0.4, 1.5, 2.0),      # c2-shaped, 2 threads per pixel
    (37, 41, 256, 16, 4, 1, 32, 0.05, 1.0, 20.0),  # c3-shaped, 4 threads per pixel
    (30, 29, 5, 3, 8, 0, 1, 1 / 3, 0.51, 1.0),     # paper-like 8-neighbour Potts, padded chain
    (23, 19, 33, 1, 8, 1, 3, 0.3, 0.7, 3.0),       # one chain per thread, partial last block
    (17, 26, 33, 2, 4, 1, 40, 0.2, 0.3, 4.0),      # two chains, truncation above L-1
    (12, 12, 2, 5, 4, 0, 1, 0.8, 2.0, 0.3),        # binary, 5 chains
    (9, 14, 200, 4, 8, 1, 9, 0.1, 0.0, 15.0),      # q = 0: naive synchronous update
    (16, 16, 16, 4, 4, 1, 4, 0.0, 1.0, 2.0),       # J = 0: independent sites
])
def test_stepwise_parity(orc, case):
    H, W, L, C, nbr, prior, T, J, q, sigma = case
    obs = _obs(H, W, L, seed=H * 1000 + W, sigma=sigma)
    kw = dict(height=H, width=W, levels=L, chains=C, neighbourhood=nbr, prior=prior, trunc=T, J=J, q=q,
              sigma=sigma, vmin=0.0, vmax=float(L - 1), beta=[1.25] * 2 + [1.5] * 2 + [2.0], seed=4242 + H,
              burn_in=1, tally_stride=2)
    bad, total, ref, gpu = stepwise(orc, obs, 6, **kw)
    assert bad <= FLIP_BUDGET * total, f"{bad} of {total} site updates differ"
    assert np.array_equal(gpu.posterior_mean().cpu().numpy(), ref.posterior_mean())
    assert np.array_equal(gpu.marginal_map().cpu().numpy(), ref.marginal_map())


@pytest.mark.parametrize("L,C,nbr", [(7, 6, 8), (40, 16, 8), (40, 16, 4), (40, 8, 4), (40, 4, 8)])
@pytest.mark.parametrize("shape", [(1, 1), (1, 37), (29, 1), (2, 2), (3, 300), (257, 3)])
def test_degenerate_lattices_free_running(orc, shape, L, C, nbr):
    """Thin and tiny lattices, in row-major order (L = 7) and in pixel patches that the
    lattice fills only in part (L = 40): 4x4-pixel wave patches in 8x8 tiles (16 chains),
    4x8 in 8x16 (8 chains) and 8x8 in 16x16 (4 chains)."""
    H, W = shape
    obs = _obs(H, W, L, seed=7 + H + W, sigma=0.2 * (L - 1))
    kw = dict(height=H, width=W, levels=L, chains=C, neighbourhood=nbr, prior=1, trunc=2 if L == 7 else 6, J=0.5,
              q=0.8, sigma=1.4 if L == 7 else 8.0, vmin=0.0, vmax=float(L - 1), seed=99, init_mode=1, tally_stride=1)
    ref = oracle_run(orc, obs, **kw).sweep(12)
    gpu = gpu_sampler(obs, **kw).sweep(12)
    assert np.array_equal(gpu.state().cpu().numpy(), ref.state)
    assert np.array_equal(gpu.posterior_mean().cpu().numpy(), ref.posterior_mean())
    assert np.array_equal(gpu.marginal_map().cpu().numpy(), ref.marginal_map())


def test_value_units_and_random_init(orc):
    """Observation in value units [-3, 5] with L = 9; random initial states."""
    H, W, L = 40, 33, 9
    obs = _obs(H, W, L, seed=5, vmin=-3.0, vmax=5.0, sigma=1.1)
    kw = dict(height=H, width=W, levels=L, chains=4, prior=1, trunc=3, J=0.35, q=0.9, sigma=1.1, vmin=-3.0,
              vmax=5.0, seed=(1 << 63) + 12345, init_mode=1, burn_in=3, tally_stride=1)
    ref = oracle_run(orc, obs, **kw)
    gpu = gpu_sampler(obs, **kw)
    assert np.array_equal(gpu.state().cpu().numpy(), ref.state)
    ref.sweep(20)
    gpu.sweep(20)
    assert np.array_equal(gpu.state().cpu().numpy(), ref.state)
    assert np.array_equal(gpu.posterior_mean().cpu().numpy(), ref.posterior_mean())


@pytest.mark.parametrize("case", [
    # (L, chains, tally stride, sweeps per call, reset the state after call i)
    (33, 5, 1, (3, 9, 1, 20), 1),
    (33, 5, 2, (5, 17, 4), None),
    (256, 16, 3, (8, 8, 8), 0),
    (16, 8, 5, (30,), None),
    (2, 2, 9, (7, 13, 11, 40), 2),
])
def test_deferred_tallies_match_oracle(orc, case):
    """Tally strides of 1 to 5 and sweep counts split over several calls: the mode read
    between calls, after a state reset or at any sweep count counts every tally sweep
    once, as the CPU reference does."""
    torch = torch_cuda()
    L, C, stride, calls, reset_after = case
    H, W = 21, 34
    obs = _obs(H, W, L, seed=L + C + stride, sigma=0.25 * L)
    kw = dict(height=H, width=W, levels=L, chains=C, prior=1 if L > 2 else 0, trunc=max(1, L // 8), J=0.3,
              q=1.2, sigma=0.25 * L, vmin=0.0, vmax=float(L - 1), seed=77 + stride, burn_in=2, tally_stride=stride)
    ref = oracle_run(orc, obs, **kw)
    gpu = gpu_sampler(obs, **kw)
    for i, n in enumerate(calls):
        ref.sweep(n)
        gpu.sweep(n)
        tallies = len(range(2, ref.t, stride))
        assert gpu.stats() == (ref.t, int(ref.count[0]), tallies)
        assert np.array_equal(gpu.state().cpu().numpy(), ref.state), i
        if tallies > 0 and i % 2 == 0:
            assert np.array_equal(gpu.marginal_map().cpu().numpy(), ref.marginal_map()), i
        if i == reset_after:  # a state write must not lose the pending tallies
            gpu.set_state(torch.from_numpy(ref.state.copy()).cuda(), ref.t)
    assert np.array_equal(gpu.posterior_mean().cpu().numpy(), ref.posterior_mean())
    assert np.array_equal(gpu.marginal_map().cpu().numpy(), ref.marginal_map())


@pytest.mark.parametrize("case", [
    # (H, W, L, chains, nbr, prior, T, J, q, sigma, inertia exponent)
    (37, 41, 256, 16, 4, 1, 32, 0.05, 0.02, 20.0, 1),  # c3-shaped, L1 inertia
    (37, 41, 256, 16, 4, 1, 32, 0.05, 0.002, 20.0, 2),  # c3-shaped, L2 inertia
    (40, 33, 16, 8, 4, 1, 4, 0.4, 0.4, 2.0, 1),       # c2-shaped, one block per level
    (29, 31, 33, 3, 8, 1, 3, 0.3, 0.2, 3.0, 2),       # padded chains, 8 neighbours
    (21, 18, 5, 1, 8, 0, 1, 1 / 3, 0.5, 0.6, 2),      # paper-like Potts, one chain
    (16, 19, 200, 2, 4, 1, 9, 0.1, 3.0, 1.0, 2),      # inertia far stronger than the data
])
def test_inertia_norm_stepwise_parity(orc, case):
    """The L1 and L2 inertia forms: same per-site arithmetic as the CPU reference."""
    H, W, L, C, nbr, prior, T, J, q, sigma, p = case
    obs = _obs(H, W, L, seed=H * 1000 + W + p, sigma=sigma)
    kw = dict(height=H, width=W, levels=L, chains=C, neighbourhood=nbr, prior=prior, trunc=T, J=J, q=q,
              sigma=sigma, vmin=0.0, vmax=float(L - 1), beta=[1.25, 1.5, 2.0], seed=5151 + H, burn_in=1,
              tally_stride=1, inertia=p, init_mode=1)
    bad, total, ref, gpu = stepwise(orc, obs, 5, **kw)
    assert bad <= FLIP_BUDGET * total, f"{bad} of {total} site updates differ"
    ref2 = oracle_run(orc, obs, **kw).sweep(12)
    gpu2 = gpu_sampler(obs, **kw).sweep(12)
    assert np.array_equal(gpu2.state().cpu().numpy(), ref2.state)
    assert np.array_equal(gpu2.posterior_mean().cpu().numpy(), ref2.posterior_mean())
    assert np.array_equal(gpu2.marginal_map().cpu().numpy(), ref2.marginal_map())


@pytest.mark.parametrize("case", [
    # (H, W, L, chains, nbr, prior, T, J, q, sigma, observation, inertia exponent)
    (24, 20, 256, 4, 8, 1, 255, 0.02, 1.0, 20.0, "image", 0),    # largest prior table: 8*255 + 1 entries
    (19, 23, 256, 16, 4, 1, 32, 0.05, 1.0, 5.0, "outside", 0),   # observations far outside [vmin, vmax]
    (21, 17, 33, 3, 4, 1, 4, 0.3, 1.0, 0.01, "image", 0),        # sigma 0.01 levels: the data decides
    (18, 22, 16, 8, 8, 1, 4, 0.4, 1.5, 1e5, "image", 0),         # flat data term
    (20, 20, 16, 2, 4, 1, 4, 20.0, 0.5, 2.0, "image", 0),        # prior factors underflow to zero
    (17, 19, 2, 5, 4, 0, 1, 0.8, 69.0, 0.3, "image", 0),         # q at its bound, beta q log2(e) < 100
    (22, 18, 200, 4, 8, 0, 1, 3.0, 0.5, 10.0, "outside", 0),     # strong Potts coupling, many levels
    (21, 19, 256, 4, 8, 1, 255, 0.02, 0.05, 20.0, "outside", 1),  # L1 inertia, largest table, far data
    (17, 16, 64, 2, 4, 1, 8, 0.3, 0.5, 0.01, "image", 2),        # L2 inertia with a sharp data term
])
def test_extreme_parameters(orc, case):
    """Parameters at the edges of the accepted range, where weights underflow, the stay
    weight is near its largest value or the observation lies far outside the level range:
    the same trajectories, means and modes as the CPU reference."""
    H, W, L, C, nbr, prior, T, J, q, sigma, observation, p = case
    if observation == "outside":
        obs = np.random.default_rng(H * W).uniform(-300.0, 600.0, size=(H, W)).astype(np.float32)
    else:
        obs = _obs(H, W, L, seed=H * 100 + W, sigma=min(sigma, 0.2 * L))
    beta = [1.0] if q * 1.4427 * 1.5 > 100.0 else [1.0, 1.25, 1.5]
    kw = dict(height=H, width=W, levels=L, chains=C, neighbourhood=nbr, prior=prior, trunc=T, J=J, q=q,
              sigma=sigma, vmin=0.0, vmax=float(L - 1), beta=beta, seed=6161 + H, burn_in=1, tally_stride=1,
              inertia=p, init_mode=1)
    bad, total, ref, gpu = stepwise(orc, obs, 4, **kw)
    assert bad <= FLIP_BUDGET * total, f"{bad} of {total} site updates differ"
    ref2 = oracle_run(orc, obs, **kw).sweep(10)
    gpu2 = gpu_sampler(obs, **kw).sweep(10)
    assert np.array_equal(gpu2.state().cpu().numpy(), ref2.state)
    assert np.array_equal(gpu2.posterior_mean().cpu().numpy(), ref2.posterior_mean())
    assert np.array_equal(gpu2.marginal_map().cpu().numpy(), ref2.marginal_map())


@pytest.mark.parametrize("C", [12, 32, 100, 1024])
def test_many_chains_per_pixel(orc, C):
    """Chain counts whose lanes per pixel (chains / 4) are 3, 8, 25 and 256: pixels whose
    lanes do not fill a quad, span several quads, or several waves.  The mean accumulator
    then takes the per-lane atomic path instead of the quad reduction."""
    H, W, L = 9, 7, 33 if C < 1024 else 5
    obs = _obs(H, W, L, seed=C)
    kw = dict(height=H, width=W, levels=L, chains=C, prior=1, trunc=4, J=0.3, q=0.9, sigma=0.2 * L, vmin=0.0,
              vmax=float(L - 1), beta=[1.2, 1.6], seed=31 + C, burn_in=1, tally_stride=1,
              init_mode=1)
    n = 6 if C < 1024 else 3
    ref = oracle_run(orc, obs, **kw).sweep(n)
    gpu = gpu_sampler(obs, **kw).sweep(n)
    assert np.array_equal(gpu.state().cpu().numpy(), ref.state)
    assert np.array_equal(gpu.posterior_mean().cpu().numpy(), ref.posterior_mean())
    assert np.array_equal(gpu.marginal_map().cpu().numpy(), ref.marginal_map())


@pytest.mark.parametrize("L,C", [(2, 64), (32, 32)])
def test_sweeps_larger_than_one_launch(orc, L, C):
    """16384 x 16400 pixels whose sweep needs more workgroups than one launch may hold
    (2^23 of 256 threads), so each sweep is issued as several launches with the last one
    ragged: L = 2 with 64 chains (row-major order, 16.8e6 workgroups, three launches) and
    L = 32 with 32 chains (2 x 4 pixel patches, 8.4e6 workgroups, two launches).  The
    first four chains must equal an unsplit run with 4 chains everywhere, that run must
    equal the CPU reference at sampled sites around the launch boundaries, and the mean
    accumulator must hold the per-pixel sum of the new state over all chains."""
    torch = torch_cuda()
    H, W = 16384, 16400
    rng = np.random.default_rng(8 + L)
    yy = np.arange(H, dtype=np.int32)[:, None]
    xx = np.arange(W, dtype=np.int32)[None, :]
    lo, hi = (-1.0, 1.0) if L == 2 else (0.0, float(L - 1))
    mid, amp = (lo + hi) / 2, (hi - lo) / 2
    obs = np.where(((yy // 512) + (xx // 640)) % 2 == 0, np.float32(mid + amp), np.float32(mid - amp))
    obs += np.float32(0.3 * amp) * rng.standard_normal((H, W), dtype=np.float32)
    if L == 2:
        model = dict(prior=0, trunc=1, J=0.8, q=2.0, sigma=0.6)
    else:
        model = dict(prior=1, trunc=4, J=0.3, q=1.0, sigma=0.3 * amp)
    kw = dict(height=H, width=W, levels=L, neighbourhood=4, vmin=lo, vmax=hi, seed=1616 + L, burn_in=0,
              tally_stride=0, **model)
    big = gpu_sampler(obs, chains=C, **kw).sweep(1)
    small = gpu_sampler(obs, chains=4, **kw).sweep(1)
    assert big.stats() == (1, C, 0)
    sb = big.state()
    ss = small.state()
    assert torch.equal(sb[:4], ss)
    acc, _ = big.accumulators()
    assert torch.equal(sb.sum(dim=0, dtype=torch.int32), acc)
    del sb, acc
    big.close()
    N = H * W
    if L == 2:  # row-major: first pixels of the second and third launch
        split = [(1 << 31) // 16, (1 << 32) // 16]
    else:  # 4 x 8 pixel tiles, 2050 per tile row: first tile of the second launch
        t = 1 << 23
        split = [(t // 2050) * 4 * W + (t % 2050) * 8]
    pix = np.concatenate([[0, W - 1, N - W, N - 1], [p + d for p in split for d in (-W - 1, -1, 0, 1, W, W + 1)],
                          rng.integers(0, N, size=3000)]).astype(np.int64)
    chains = rng.integers(0, 4, size=pix.shape[0]).astype(np.int32)
    p4 = orc.Params(chains=4, **kw)
    want = orc.update_sites(p4, obs, orc.init_state(p4, obs), 0, chains, pix)
    got = ss.view(4, -1)[torch.from_numpy(chains).long().cuda(), torch.from_numpy(pix).cuda()].cpu().numpy()
    assert np.array_equal(got, want)
    del ss
    small.close()
    torch.cuda.empty_cache()


def test_sweep_splitting_is_invisible(orc):
    wl = synth.make_workload("c2", height=64, width=48, chains=8)
    kw = wl.params(beta=[1.0, 1.5, 2.0], burn_in=2)
    a = gpu_sampler(wl.obs, **kw).sweep(3).sweep(4).sweep(0)
    b = gpu_sampler(wl.obs, **kw).sweep(7)
    assert np.array_equal(a.state().cpu().numpy(), b.state().cpu().numpy())
    assert np.array_equal(a.posterior_mean().cpu().numpy(), b.posterior_mean().cpu().numpy())
    assert np.array_equal(a.marginal_map().cpu().numpy(), b.marginal_map().cpu().numpy())


def test_chain_results_do_not_depend_on_chain_count():
    wl = synth.make_workload("c2", height=40, width=40)
    s16 = gpu_sampler(wl.obs, **wl.params(chains=16)).sweep(5).state().cpu().numpy()
    s3 = gpu_sampler(wl.obs, **wl.params(chains=3)).sweep(5).state().cpu().numpy()
    s1 = gpu_sampler(wl.obs, **wl.params(chains=1)).sweep(5).state().cpu().numpy()
    assert np.array_equal(s16[:3], s3) and np.array_equal(s16[:1], s1)


def test_streams_and_errors():
    torch = torch_cuda()
    from paper_2507_14869_amd import PcaError
    wl = synth.make_workload("c2", height=32, width=32)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = gpu_sampler(wl.obs, **wl.params(burn_in=5))
        g.sweep(3)
        with pytest.raises(PcaError):
            g.posterior_mean()  # nothing accumulated before burn-in
        with pytest.raises(PcaError):
            g.marginal_map()
        with pytest.raises(PcaError):
            g.sweep(-1)
        g.sweep(3)
        m = g.posterior_mean()
    s.synchronize()
    assert torch.isfinite(m).all()
    g.sync()
    g.close()


def test_sweep_index_stops_at_32_bits():
    """The sweep index is a 32-bit counter word of the random stream: sweeps may run up to
    it, and a call that would pass 2^32 - 1 is refused without side effects."""
    from paper_2507_14869_amd import PcaError
    wl = synth.make_workload("c2", height=16, width=16)
    g = gpu_sampler(wl.obs, **wl.params(burn_in=0))
    g.set_state(g.state(), (1 << 32) - 3)
    g.sweep(2)
    assert g.stats()[0] == (1 << 32) - 1
    before = g.state().cpu().numpy()
    with pytest.raises(PcaError):
        g.sweep(1)
    assert g.stats()[0] == (1 << 32) - 1
    assert np.array_equal(g.state().cpu().numpy(), before)
    g.close()


def _host_threads():
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def test_full_size_c3_whole_lattice(orc):
    """2048x2048, L = 256, 16 chains in the benchmark's launch configuration.  Sweep 0 from
    the oracle's initial state, checked at 3000 sampled (chain, pixel) sites and the
    lattice corners; then sweep 777 from an oracle-made random state, checked at every one
    of the 2048 x 2048 x 16 site updates against the oracle (computed in row bands on the
    host's cores).  The accumulators hold exactly the two new states: the uint32 level sum
    at every pixel, and the uint16 tallies on the first and last 64 rows."""
    torch = torch_cuda()
    wl = synth.make_workload("c3")
    kw = wl.params(burn_in=0)
    p = orc.Params(**kw)
    gpu = gpu_sampler(wl.obs, **kw)
    x0 = orc.init_state(p, wl.obs)
    assert np.array_equal(gpu.state().cpu().numpy(), x0)
    rng = np.random.default_rng(31)
    N = wl.height * wl.width
    gpu.sweep(1)
    new0 = gpu.state().cpu().numpy()
    chains = rng.integers(0, 16, size=3000).astype(np.int32)
    pix = rng.integers(0, N, size=3000).astype(np.int64)
    pix[:4] = [0, wl.width - 1, N - wl.width, N - 1]
    want = orc.update_sites(p, wl.obs, x0, 0, chains, pix)
    assert np.array_equal(new0.reshape(16, -1)[chains, pix], want)

    start = rng.integers(0, 256, size=x0.shape, dtype=np.uint8)
    gpu.set_state(torch.from_numpy(start).cuda(), 777)
    gpu.sweep(1)
    new1 = gpu.state().cpu().numpy()
    want1 = orc.pca_sweep_threaded(p, wl.obs, start, 777, threads=_host_threads())
    bad = int((new1 != want1).sum())
    assert bad == 0, f"{bad} of {new1.size} site updates differ"

    assert gpu.stats() == (778, 32, 2)
    s, h = gpu.accumulators()
    want_sum = new0.sum(axis=0, dtype=np.uint32) + new1.sum(axis=0, dtype=np.uint32)
    assert np.array_equal(s.cpu().numpy().view(np.uint32), want_sum)
    for rows in (slice(0, 64), slice(wl.height - 64, wl.height)):
        got_h = h[rows].cpu().numpy().view(np.uint16)
        both = np.concatenate([new0[:, rows], new1[:, rows]], axis=0).reshape(32, -1)
        cell = np.arange(both.shape[1], dtype=np.int64)[None, :] * 256 + both
        want_h = np.bincount(cell.reshape(-1), minlength=both.shape[1] * 256).reshape(got_h.shape)
        assert np.array_equal(got_h, want_h.astype(np.uint16))
    gpu.close()


def test_full_size_c2_whole_lattice(orc):
    """512x512, L = 16, 8 chains (the few-level kernel in the benchmark's configuration):
    12 sweeps from the oracle's initial state, every site update of every sweep against the
    oracle's (computed in row bands on the host's cores), and the accumulators of the 8
    sweeps after burn-in (level sums, tallies, mean and mode) against those states; then one
    sweep from an oracle-made random state at sweep 4321, checked at every site."""
    torch = torch_cuda()
    wl = synth.make_workload("c2")
    kw = wl.params(burn_in=4)
    p = orc.Params(**kw)
    gpu = gpu_sampler(wl.obs, **kw)
    x = orc.init_state(p, wl.obs)
    assert np.array_equal(gpu.state().cpu().numpy(), x)
    C, H, W, L = wl.chains, wl.height, wl.width, wl.levels
    want_sum = np.zeros((H, W), dtype=np.uint32)
    want_hist = np.zeros(H * W * L, dtype=np.int64)
    cell0 = np.arange(H * W, dtype=np.int64)[None, :] * L
    for t in range(12):
        x = orc.pca_sweep_threaded(p, wl.obs, x, t, threads=_host_threads())
        gpu.sweep(1)
        bad = int((gpu.state().cpu().numpy() != x).sum())
        assert bad == 0, f"{bad} of {x.size} site updates differ at sweep {t}"
        if t >= 4:
            want_sum += x.sum(axis=0, dtype=np.uint32)
            want_hist += np.bincount((cell0 + x.reshape(C, -1)).reshape(-1), minlength=H * W * L)
    assert gpu.stats() == (12, 8 * C, 8)
    s, h = gpu.accumulators()
    assert np.array_equal(s.cpu().numpy().view(np.uint32), want_sum)
    assert np.array_equal(h.cpu().numpy().view(np.uint16), want_hist.reshape(H, W, L).astype(np.uint16))
    ref = orc.Run(p, wl.obs)  # the oracle's read-outs of the same accumulators
    ref.sum[...] = want_sum
    ref.count[0] = 8 * C
    ref.hist[...] = want_hist.reshape(H, W, L)
    assert np.array_equal(gpu.posterior_mean().cpu().numpy(), ref.posterior_mean())
    assert np.array_equal(gpu.marginal_map().cpu().numpy(), ref.marginal_map())

    rng = np.random.default_rng(47)
    start = rng.integers(0, L, size=x.shape, dtype=np.uint8)
    gpu.set_state(torch.from_numpy(start).cuda(), 4321)
    gpu.sweep(1)
    want = orc.pca_sweep_threaded(p, wl.obs, start, 4321, threads=_host_threads())
    bad = int((gpu.state().cpu().numpy() != want).sum())
    assert bad == 0, f"{bad} of {want.size} site updates differ"
    gpu.close()


@pytest.mark.parametrize("H,W,L,C,nbr", [
    (264, 256, 16, 16, 4),  # 4 lanes per pixel, more than 15 chains: the row built as uint16 pairs
    (264, 256, 16, 14, 4),  # 4 lanes per pixel, 4-bit counters, a padded chain group
    (520, 512, 16, 3, 4),   # one lane per pixel owning the whole row
    (264, 512, 15, 8, 4),   # 2 lanes per pixel, 15 levels (a full row of 8 words)
    (264, 512, 7, 8, 4),    # rows of 4 words
    (264, 256, 2, 16, 4),   # rows of one word
    (520, 512, 12, 2, 4),   # two chains, rows of 6 words
    (264, 512, 16, 8, 8),   # the 8-neighbourhood (statistic table of plain terms)
    (264, 256, 16, 16, 8),  # 8 neighbours, the largest statistic (8 * 15)
])
def test_few_level_histogram_rows(orc, H, W, L, C, nbr):
    """The one-sweep few-level kernel (lattices large enough not to take the several-sweeps
    kernel) for each lanes-per-pixel layout of the histogram row and full and partial rows,
    and both neighbourhoods: four sweeps free-running from the oracle's initial state, then
    state, level sums, every tally, mean and mode against the oracle."""
    obs = _obs(H, W, L, seed=H + 7 * L + C, sigma=0.15 * L)
    kw = dict(height=H, width=W, levels=L, chains=C, neighbourhood=nbr, prior=1, trunc=15 if nbr == 8 else 3,
              J=0.4 if nbr == 4 else 0.1, q=1.2, sigma=0.15 * L, vmin=0.0, vmax=float(L - 1), seed=900 + C,
              burn_in=1, tally_stride=1)
    ref = oracle_run(orc, obs, **kw).sweep(4)
    gpu = gpu_sampler(obs, **kw)
    assert gpu.sweeps_per_launch() == 1
    gpu.sweep(4)
    assert np.array_equal(gpu.state().cpu().numpy(), ref.state)
    s, h = gpu.accumulators()
    assert np.array_equal(s.cpu().numpy().view(np.uint32), ref.sum)
    assert np.array_equal(h.cpu().numpy().view(np.uint16), ref.hist.astype(np.uint16))
    assert np.array_equal(gpu.posterior_mean().cpu().numpy(), ref.posterior_mean())
    assert np.array_equal(gpu.marginal_map().cpu().numpy(), ref.marginal_map())
    gpu.close()


def test_set_state_rejects_values_outside_the_levels():
    """A state value >= levels is refused (PCA_EINVAL) and leaves the context as it was;
    levels - 1 is accepted."""
    torch = torch_cuda()
    from paper_2507_14869_amd import PCA_EINVAL, PcaError
    wl = synth.make_workload("c2", height=24, width=20, chains=5)
    g = gpu_sampler(wl.obs, **wl.params(burn_in=0))
    g.sweep(2)
    before = g.state().cpu().numpy()
    bad = before.copy()
    bad[4, 23, 19] = 16  # one value past the last level, in the last chain's last pixel
    with pytest.raises(PcaError) as e:
        g.set_state(torch.from_numpy(bad).cuda(), 9)
    assert e.value.code == PCA_EINVAL
    assert g.stats()[0] == 2
    assert np.array_equal(g.state().cpu().numpy(), before)
    top = np.full_like(before, 15)
    g.set_state(torch.from_numpy(top).cuda(), 9)
    assert g.stats()[0] == 9
    assert np.array_equal(g.state().cpu().numpy(), top)
    g.close()


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_full_size_workload_restores_the_image(orc, name):
    """The whole workload as the benchmark runs it (c2: 512x512, L = 16, 8 chains, 1000
    sweeps; c3 with 200 sweeps): the posterior mean and the marginal mode are closer to
    the clean image than the observation is (by more than 6 dB), and the last sweep agrees
    with the CPU reference at sampled sites."""
    torch = torch_cuda()
    from workloads import metrics
    wl = synth.make_workload(name, sweeps=None if name == "c2" else 200)
    kw = wl.params()
    gpu = gpu_sampler(wl.obs, **kw).sweep(wl.sweeps - 1)
    before = gpu.state().cpu().numpy()
    gpu.sweep(1)
    truth = metrics.luminance_levels(wl.truth, wl.levels)
    noisy = metrics.luminance_values(np.clip(wl.obs, wl.vmin, wl.vmax), wl.vmin, wl.vmax)
    mean = metrics.luminance_values(gpu.posterior_mean().cpu().numpy(), wl.vmin, wl.vmax)
    mpm = metrics.luminance_levels(gpu.marginal_map().cpu().numpy(), wl.levels)
    base = metrics.psnr(truth, noisy)
    print(f"\n{name}: PSNR noisy {base:.2f} dB, mean {metrics.psnr(truth, mean):.2f}, mode {metrics.psnr(truth, mpm):.2f}")
    assert metrics.psnr(truth, mean) > base + 6.0
    assert metrics.psnr(truth, mpm) > base + 6.0
    rng = np.random.default_rng(5)
    N = wl.height * wl.width
    chains = rng.integers(0, wl.chains, size=2000).astype(np.int32)
    pix = rng.integers(0, N, size=2000).astype(np.int64)
    want = orc.update_sites(orc.Params(**kw), wl.obs, before, wl.sweeps - 1, chains, pix)
    got = gpu.state().cpu().numpy().reshape(wl.chains, -1)[chains, pix]
    assert np.array_equal(got, want)


def test_checkpoint_and_resume_is_bit_exact(orc):
    """State, sweep index and accumulators saved after 5 sweeps and loaded into a fresh
    context continue exactly as the uninterrupted run; the raw accumulators equal the
    CPU reference's level sums and tallies."""
    torch = torch_cuda()
    H, W, L = 23, 31, 33
    obs = _obs(H, W, L, seed=404)
    kw = dict(height=H, width=W, levels=L, chains=6, prior=1, trunc=5, J=0.3, q=0.8, sigma=6.0, vmin=0.0,
              vmax=float(L - 1), beta=[1.0, 1.2, 1.4], seed=4040, burn_in=2, tally_stride=1, init_mode=1)
    whole = gpu_sampler(obs, **kw).sweep(12)
    first = gpu_sampler(obs, **kw).sweep(5)
    ref = oracle_run(orc, obs, **kw).sweep(5)
    state = first.state()
    s, h = first.accumulators()
    t, count, tallies = first.stats()
    assert np.array_equal(s.cpu().numpy().view(np.uint32), ref.sum)
    assert np.array_equal(h.cpu().numpy().view(np.uint16), ref.hist)
    first.close()
    resumed = gpu_sampler(obs, **kw).set_state(state, t).set_accumulators(s, h, count, tallies).sweep(7)
    assert resumed.stats() == whole.stats()
    assert np.array_equal(resumed.state().cpu().numpy(), whole.state().cpu().numpy())
    assert np.array_equal(resumed.posterior_mean().cpu().numpy(), whole.posterior_mean().cpu().numpy())
    assert np.array_equal(resumed.marginal_map().cpu().numpy(), whole.marginal_map().cpu().numpy())
    from paper_2507_14869_amd import PcaError
    with pytest.raises(PcaError):
        resumed.set_accumulators(s, h, -1, 0)
    with pytest.raises(PcaError):
        resumed.set_accumulators(s, None, count, tallies)  # this run keeps a histogram
