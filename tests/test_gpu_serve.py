"""Continuous-batching server: requests admitted by device-memory footprint while others
run, their sweeps interleaved in shared launches; every result must equal the request
run alone (and the CPU oracle for a small one)."""
import numpy as np
import pytest

try:  # import at collection so the first GPU test's time limit does not include it
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

from tests.gpu_util import gpu_sampler, oracle_run, torch_cuda
from tests.test_gpu_batch import _problem
from workloads import synth

pytestmark = pytest.mark.gpu


def _server(budget, max_active=64, k=4, step_ms=0.05):
    torch_cuda()
    from paper_2507_14869_amd import Server
    return Server(budget, max_active=max_active, sweeps_per_step=k, step_ms=step_ms)


def _alone(obs, kw, sweeps):
    s = gpu_sampler(obs, height=obs.shape[0], width=obs.shape[1], **kw).sweep(sweeps)
    out = (s.posterior_mean().cpu().numpy(), s.marginal_map().cpu().numpy(), s.state().cpu().numpy())
    s.close()
    return out


SPECS = [(37, 53, 256, 2, 1, 9), (64, 64, 2, 2, 2, 14), (17, 200, 16, 2, 3, 6), (90, 33, 256, 2, 5, 11),
         (128, 96, 16, 2, 6, 7), (5, 7, 33, 2, 7, 13), (40, 40, 2, 4, 8, 10), (33, 65, 256, 1, 9, 8)]


@pytest.mark.parametrize("step_ms,k", [(0.05, 3), (2.0, 16)])
def test_requests_in_the_mix_equal_requests_alone(step_ms, k):
    sv = _server(budget=1 << 34, k=k, step_ms=step_ms)
    reqs = {}
    pending = list(SPECS)
    # submit half, run a step, submit the rest while the first ones are on the GPU
    for spec in pending[:4]:
        obs, kw = _problem(*spec[:4], seed=spec[4])
        reqs[sv.submit(obs, spec[5], **kw)] = (obs, kw, spec[5])
    sv.step()
    done = set(sv.completed())
    assert sv.stats()[1] + len(done) == 4  # admitted at once: running or already finished
    for spec in pending[4:]:
        obs, kw = _problem(*spec[:4], seed=spec[4])
        reqs[sv.submit(obs, spec[5], **kw)] = (obs, kw, spec[5])
    for _ in range(100):
        sv.step()
        done.update(sv.completed())
        if len(done) == len(reqs):
            break
    assert done == set(reqs)
    q, a, used, steps, _ = sv.stats()
    assert (q, a, used) == (0, 0, 0)
    for rid, (obs, kw, sweeps) in reqs.items():
        mean, mpm, state = sv.result(rid)
        ref = _alone(obs, kw, sweeps)
        assert np.array_equal(mean, ref[0]), rid
        assert np.array_equal(mpm, ref[1]), rid
        assert np.array_equal(state, ref[2]), rid
        assert sv.status(rid) == (2, sweeps)
    sv.close()


def test_memory_budget_queues_requests_and_keeps_results(orc):
    specs = SPECS[:5]
    probs = [_problem(*s[:4], seed=s[4]) for s in specs]
    from paper_2507_14869_amd import Server  # noqa: F401
    # a budget that holds the largest request but never all of them together
    sizes = []
    for (obs, kw), s in zip(probs, specs):
        H, W = obs.shape
        L = kw["levels"]
        Cp = kw["chains"] if kw["chains"] <= 2 else (kw["chains"] + 3) // 4 * 4
        sizes.append(H * W * (4 + 2 * Cp + 4 + 4 + ((L + 1) // 2) * 4) + 4096 + 8 * 3)
    budget = max(sizes) + min(sizes)
    sv = _server(budget=budget, max_active=8, k=5)
    ids = [sv.submit(obs, s[5], **kw) for (obs, kw), s in zip(probs, specs)]
    queued_while_running = False
    done = []
    for _ in range(200):
        sv.step()
        q, a, used, _, _ = sv.stats()
        assert used <= budget
        queued_while_running |= q > 0 and a > 0
        done += sv.completed()
        if len(done) == len(ids):
            break
    assert sorted(done) == sorted(ids)
    assert queued_while_running  # the budget held requests back until others finished
    for rid, (obs, kw), s in zip(ids, probs, specs):
        mean, mpm, state = sv.result(rid)
        ref = _alone(obs, kw, s[5])
        assert np.array_equal(mean, ref[0]) and np.array_equal(mpm, ref[1]) and np.array_equal(state, ref[2])
    # and one against the CPU oracle directly
    obs, kw = probs[2]
    ref = oracle_run(orc, obs, height=obs.shape[0], width=obs.shape[1], **kw).sweep(specs[2][5])
    mean, mpm, state = sv.result(ids[2])
    assert np.array_equal(mean, ref.posterior_mean()) and np.array_equal(state, ref.state)
    assert np.array_equal(mpm, ref.marginal_map())
    sv.release(ids[0])
    with pytest.raises(Exception):
        sv.status(ids[0])
    sv.close()


def test_server_rejects_bad_requests():
    from paper_2507_14869_amd import PcaError
    sv = _server(budget=1 << 20)
    obs, kw = _problem(64, 64, 256, 2, 3)
    with pytest.raises(PcaError):  # 64x64 with L=256 histogram needs more than 1 MiB
        sv.submit(obs, 5, **kw)
    small, kw2 = _problem(8, 8, 16, 2, 4)
    with pytest.raises(PcaError):
        sv.submit(small, 0, **kw2)
    rid = sv.submit(small, 3, **kw2)
    with pytest.raises(PcaError):
        sv.result(rid)  # not finished
    while sv.status(rid)[0] != 2:
        sv.step()
    sv.close()


def test_shedding_refuses_requests_while_the_backlog_is_long():
    """With a shedding limit, a submission is refused (PCA_EBUSY) while accepted work is
    pending and accepted again once the server has drained; the accepted request's result
    equals the request run alone.  A limit of 0 accepts everything."""
    from paper_2507_14869_amd import PCA_EBUSY, PcaError
    sv = _server(budget=1 << 32, k=8, step_ms=0.5)
    obs, kw = _problem(48, 40, 16, 2, 21)
    sv.set_shedding(1e-9)  # any pending work is too much
    first = sv.submit(obs, 24, **kw)  # an idle server accepts
    with pytest.raises(PcaError) as err:
        sv.submit(obs, 24, **kw)
    assert err.value.code == PCA_EBUSY
    assert sv.shed == 1
    while sv.status(first)[0] != 2:
        sv.step()
    again = sv.submit(obs, 24, **kw)  # drained: accepted again
    mean, mpm, state = sv.result(first)
    want = _alone(obs, kw, 24)
    assert np.array_equal(mean, want[0]) and np.array_equal(mpm, want[1]) and np.array_equal(state, want[2])
    sv.set_shedding(0.0)
    extra = [sv.submit(obs, 24, **kw) for _ in range(3)]
    assert sv.shed == 1
    with pytest.raises(PcaError):
        sv.set_shedding(-1.0)
    while any(sv.status(r)[0] != 2 for r in [again] + extra):
        sv.step()
    sv.close()


def test_requests_with_different_kernels_share_the_server():
    """Requests needing different kernels (4 or 8 neighbours, indicator or L2 inertia)
    are served in the same steps' rotation and each equals its run alone."""
    sv = _server(budget=1 << 34, k=4, step_ms=0.5)
    specs = [((30, 31, 16, 2, 41), {}), ((22, 40, 33, 2, 42), dict(inertia=2, q=0.1)),
             ((25, 25, 5, 2, 43), dict(neighbourhood=8, prior=0, trunc=1)),
             ((18, 33, 256, 2, 44), dict(inertia=1, q=0.02))]
    reqs = {}
    for spec, over in specs:
        obs, kw = _problem(*spec, **over)
        reqs[sv.submit(obs, 9, **kw)] = (obs, kw)
    done = set()
    for _ in range(200):
        sv.step()
        done.update(sv.completed())
        if len(done) == len(reqs):
            break
    assert done == set(reqs)
    for rid, (obs, kw) in reqs.items():
        mean, mpm, state = sv.result(rid)
        ref = _alone(obs, kw, 9)
        assert np.array_equal(state, ref[2]), rid
        assert np.array_equal(mean, ref[0]) and np.array_equal(mpm, ref[1]), rid
    sv.close()


def _drain(sv, ids, limit=400):
    done = []
    for _ in range(limit):
        sv.step()
        done += sv.completed()
        if set(done) >= set(ids):
            break
    return done


def test_failed_admission_waits_then_fails_without_stalling_the_queue(monkeypatch):
    """A request whose device allocation fails at admission (forced from the host with
    PCA_FAULT_INJECT) waits while another request holds device memory, then fails with
    PCA_ENOMEM once nothing else is admitted; the requests around it finish with results
    equal to each run alone."""
    from paper_2507_14869_amd import PCA_ENOMEM, PcaError
    sv = _server(budget=1 << 34, k=4, step_ms=0.05)
    probs = [_problem(40, 30, 16, 2, 51), _problem(30, 30, 256, 2, 52), _problem(25, 44, 2, 2, 53)]
    ids = [sv.submit(obs, 9, **kw) for obs, kw in probs]
    monkeypatch.setenv("PCA_FAULT_INJECT", f"admit:{ids[1]}")
    sv.step()
    assert sv.status(ids[1])[0] == 0  # the first request holds memory: the failed one waits
    assert sv.status(ids[0])[0] in (1, 2)
    done = _drain(sv, ids)
    assert sorted(done) == sorted(ids)
    assert sv.status(ids[1]) == (3, 0)
    with pytest.raises(PcaError) as err:
        sv.result(ids[1])
    assert err.value.code == PCA_ENOMEM
    for rid, (obs, kw) in ((ids[0], probs[0]), (ids[2], probs[2])):
        mean, mpm, state = sv.result(rid)
        ref = _alone(obs, kw, 9)
        assert np.array_equal(mean, ref[0]) and np.array_equal(mpm, ref[1]) and np.array_equal(state, ref[2])
    assert sv.stats()[:3] == (0, 0, 0)
    sv.release(ids[1])
    sv.close()


def test_request_larger_than_device_memory_fails_and_the_next_one_runs():
    """The budget is the caller's estimate: a request whose chain states exceed the
    device's whole memory passes the budget but its allocation fails; with nothing else
    admitted it fails with PCA_ENOMEM, and the small request queued behind it completes
    with the result it has alone."""
    torch = torch_cuda()
    from paper_2507_14869_amd import PCA_ENOMEM, PcaError
    total = torch.cuda.get_device_properties(0).total_memory
    chains = 1024
    side = int(np.ceil(np.sqrt(1.1 * total / (2 * chains))))  # two state buffers of side^2 x 1024 bytes
    sv = _server(budget=1 << 50, k=4, step_ms=0.05)
    big = np.zeros((side, side), dtype=np.float32)
    big_id = sv.submit(big, 1, levels=2, chains=chains, prior=0, J=0.8, q=1.0, sigma=0.5, vmin=0.0, vmax=1.0,
                       seed=1, burn_in=0, tally_stride=0)
    del big
    obs, kw = _problem(33, 27, 16, 2, 54)
    small_id = sv.submit(obs, 6, **kw)
    done = _drain(sv, [big_id, small_id])
    assert sorted(done) == sorted([big_id, small_id])
    assert sv.status(big_id)[0] == 3
    with pytest.raises(PcaError) as err:
        sv.result(big_id)
    assert err.value.code == PCA_ENOMEM
    mean, mpm, state = sv.result(small_id)
    ref = _alone(obs, kw, 6)
    assert np.array_equal(mean, ref[0]) and np.array_equal(mpm, ref[1]) and np.array_equal(state, ref[2])
    assert sv.stats()[:3] == (0, 0, 0)
    sv.close()


def test_failed_read_out_ends_the_request_without_an_extra_sweep(monkeypatch):
    """A request whose results cannot be copied out (host allocation forced to fail) ends
    as failed after exactly its sweeps, releases its device memory, and the other
    requests' results are unchanged."""
    from paper_2507_14869_amd import PCA_ENOMEM, PcaError
    sv = _server(budget=1 << 34, k=3, step_ms=0.05)
    probs = [_problem(36, 28, 33, 2, 55), _problem(20, 50, 16, 2, 56)]
    ids = [sv.submit(obs, 7, **kw) for obs, kw in probs]
    monkeypatch.setenv("PCA_FAULT_INJECT", f"readout:{ids[0]}")
    done = _drain(sv, ids)
    assert sorted(done) == sorted(ids)
    assert sv.status(ids[0]) == (3, 7)
    with pytest.raises(PcaError) as err:
        sv.result(ids[0])
    assert err.value.code == PCA_ENOMEM
    mean, mpm, state = sv.result(ids[1])
    ref = _alone(*probs[1], 7)
    assert np.array_equal(mean, ref[0]) and np.array_equal(mpm, ref[1]) and np.array_equal(state, ref[2])
    assert sv.stats()[:3] == (0, 0, 0)
    sv.close()


def _random_requests(rng):
    reqs = []
    for _ in range(int(rng.integers(3, 9))):
        H, W = int(rng.integers(4, 81)), int(rng.integers(4, 81))
        L = int(rng.choice([2, 5, 16, 33, 256]))
        sweeps = int(rng.integers(1, 26))
        truth = synth.random_image(H, W, L, max(2, H * W // 300), L > 2, rng)
        sigma = float(rng.uniform(0.1, 0.3) * L)
        obs = synth.noisy_observation(truth, L, 0.0, float(L - 1), sigma, rng)
        kw = dict(levels=L, chains=int(rng.integers(1, 5)), neighbourhood=int(rng.choice([4, 8])),
                  prior=0 if L == 2 else int(rng.integers(0, 2)), trunc=int(rng.integers(1, 40)),
                  J=float(rng.uniform(0.02, 0.8)), q=float(rng.uniform(0.0, 2.0)), sigma=sigma, vmin=0.0,
                  vmax=float(L - 1), beta=[float(b) for b in rng.uniform(0.5, 2.0, size=int(rng.integers(0, 6)))],
                  seed=int(rng.integers(0, 2**62)), burn_in=int(rng.integers(0, sweeps)),
                  tally_stride=int(rng.integers(1, 3)))
        reqs.append((obs, kw, sweeps))
    return reqs


@pytest.mark.parametrize("seed", range(10))
def test_random_serving_matches_the_oracle(orc, seed):
    """Seeded random request streams: 3-8 requests (sides 4-80, 2-256 levels, 1-4 chains,
    either neighbourhood and prior, beta schedules, burn-in and tally stride) submitted at
    random steps to a server with a random budget, slot count and sweeps per step; every
    request's mean, mode and final states equal the oracle's run of it alone."""
    rng = np.random.default_rng(6600 + seed)
    reqs = _random_requests(rng)
    fps = []
    for obs, kw, _ in reqs:
        N = obs.shape[0] * obs.shape[1]
        C = kw["chains"]
        Cp = C if C <= 2 else (C + 3) // 4 * 4
        fps.append(N * (4 + 2 * Cp + 4 + 4 + ((kw["levels"] + 1) // 2) * 4) + 4096 + 24)
    budget = max(fps) + int(rng.uniform(0.0, 1.0) * sum(fps))
    sv = _server(budget=budget, max_active=int(rng.integers(1, 9)), k=int(rng.integers(1, 10)))
    ids, done, nxt = {}, set(), 0
    for _ in range(3000):
        while nxt < len(reqs) and rng.integers(0, 3) == 0:
            obs, kw, sweeps = reqs[nxt]
            ids[sv.submit(obs, sweeps, **kw)] = nxt
            nxt += 1
        sv.step()
        done.update(sv.completed())
        if nxt == len(reqs) and len(done) == len(reqs):
            break
    assert done == set(ids)
    for rid, i in ids.items():
        obs, kw, sweeps = reqs[i]
        mean, mpm, state = sv.result(rid)
        ref = oracle_run(orc, obs, height=obs.shape[0], width=obs.shape[1], **kw).sweep(sweeps)
        assert np.array_equal(state, ref.state), (seed, i)
        assert np.array_equal(mean, ref.posterior_mean()), (seed, i)
        assert np.array_equal(mpm, ref.marginal_map()), (seed, i)
    sv.close()
