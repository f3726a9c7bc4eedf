"""Pins of the oracle's samplers against closed forms and exact enumerated laws.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a sign, a
wrong neighbour offset, swapped height/width, beta applied to the data term, a wrong
inertia reference) changes a checked quantity:

* empirical law of 2e5 independent oracle chains after t sweeps vs the exact float64
  law P^t(x0, .) of the enumerated transition matrix (PCA and systematic Gibbs);
* closed forms of special cases: discrete-Gaussian mean and variance (J = 0, q = 0;
  Poisson summation makes the mean equal g' to ~1e-15 in the interior), the L = 2
  logistic, the Potts and truncated-linear profiles with a flat data term, the
  inertia odds at a symmetric observation, corner/edge neighbour counts;
* inverse-CDF draw: frequencies over many chains vs the implied probabilities.
"""
import math

import numpy as np
import pytest
from scipy import stats

from tests import exact

M_CHAINS = 200_000


def chisq_pvalue(counts: np.ndarray, probs: np.ndarray) -> float:
    n = counts.sum()
    exp_ = probs * n
    order = np.argsort(exp_)
    # merge the smallest expected cells until every cell expects at least 5
    obs_m, exp_m = [], []
    acc_o = acc_e = 0.0
    for k in order:
        acc_o += counts[k]
        acc_e += exp_[k]
        if acc_e >= 5.0:
            obs_m.append(acc_o)
            exp_m.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0:
        obs_m[-1] += acc_o
        exp_m[-1] += acc_e
    obs_m, exp_m = np.array(obs_m), np.array(exp_m)
    exp_m *= obs_m.sum() / exp_m.sum()
    return float(stats.chisquare(obs_m, exp_m).pvalue)


CASES = [
    dict(H=3, W=3, L=2, nbr=4, potts=True, T=1, J=0.6, q=1.0, sigma=0.7, beta=1.0, seed=1, t=6),
    dict(H=2, W=3, L=3, nbr=8, potts=False, T=1, J=0.5, q=0.7, sigma=0.9, beta=1.3, seed=2, t=5),
    dict(H=2, W=2, L=4, nbr=4, potts=False, T=2, J=0.8, q=0.4, sigma=1.1, beta=0.8, seed=3, t=4),
    dict(H=3, W=2, L=2, nbr=8, potts=True, T=1, J=0.3, q=2.5, sigma=0.6, beta=1.0, seed=4, t=7),
    # L1 and L2 inertia norms (Sec. 3)
    dict(H=2, W=3, L=3, nbr=8, potts=False, T=1, J=0.5, q=0.7, sigma=0.9, beta=1.3, seed=2, t=5, p=1),
    dict(H=2, W=2, L=4, nbr=4, potts=False, T=2, J=0.8, q=0.4, sigma=1.1, beta=0.8, seed=3, t=4, p=2),
]


def make(case, orc, chains):
    rng = np.random.default_rng(case["seed"])
    H, W, L = case["H"], case["W"], case["L"]
    g = rng.uniform(-0.3, L - 0.7, size=(H, W)).astype(np.float32)
    m = exact.Model(H=H, W=W, L=L, nbr=case["nbr"], potts=case["potts"], T=case["T"], J=case["J"],
                    q=case["q"], sigma=case["sigma"], beta=case["beta"], g=g.astype(np.float64),
                    p=case.get("p", 0))
    p = orc.Params(height=H, width=W, levels=L, chains=chains, neighbourhood=case["nbr"],
                   prior=orc.POTTS if case["potts"] else orc.TRUNC_LINEAR, trunc=case["T"], J=case["J"],
                   q=case["q"], sigma=case["sigma"], vmin=0.0, vmax=float(L - 1), beta=[case["beta"]],
                   seed=1000 + case["seed"], inertia=case.get("p", 0))
    return m, p, g


@pytest.mark.parametrize("case", CASES)
def test_pca_empirical_law_matches_exact(orc, case):
    m, p, g = make(case, orc, M_CHAINS)
    run = orc.Run(p, g).sweep(case["t"])
    idx = exact.state_index(m, run.state.reshape(M_CHAINS, -1))
    counts = np.bincount(idx, minlength=m.L ** (m.H * m.W)).astype(np.float64)
    x0 = exact.state_index(m, run.state[:1].reshape(1, -1) * 0 + orc.init_state(
        orc.Params(**{**p.__dict__, "chains": 1}), g).reshape(1, -1))[0]
    law = exact.law_at(exact.pca_matrix(m), int(x0), case["t"])
    assert chisq_pvalue(counts, law) > 1e-4


@pytest.mark.parametrize("case", CASES[:3])
def test_gibbs_empirical_law_matches_exact(orc, case):
    m, p, g = make(case, orc, M_CHAINS)
    run = orc.Run(p, g, gibbs=True).sweep(case["t"])
    idx = exact.state_index(m, run.state.reshape(M_CHAINS, -1))
    counts = np.bincount(idx, minlength=m.L ** (m.H * m.W)).astype(np.float64)
    x0 = exact.state_index(m, orc.init_state(orc.Params(**{**p.__dict__, "chains": 1}), g).reshape(1, -1))[0]
    law = exact.law_at(exact.gibbs_sweep_matrix(m), int(x0), case["t"])
    assert chisq_pvalue(counts, law) > 1e-4
    # and the same sweep matrix converges to the joint posterior
    assert exact.tv(exact.law_at(exact.gibbs_sweep_matrix(m), int(x0), 300), exact.gibbs_posterior(m)) < 1e-6


def test_pca_long_run_matches_closed_form_stationary_law(orc):
    case = dict(CASES[0], J=0.2, q=0.5)  # second eigenvalue 0.63: mixed to 1e-8 by t = 40
    m, p, g = make(case, orc, M_CHAINS)
    run = orc.Run(p, g).sweep(40)
    idx = exact.state_index(m, run.state.reshape(M_CHAINS, -1))
    counts = np.bincount(idx, minlength=2 ** 9).astype(np.float64)
    pi = exact.pca_closed_form(m)
    x0 = exact.state_index(m, orc.init_state(orc.Params(**{**p.__dict__, "chains": 1}), g).reshape(1, -1))[0]
    assert exact.tv(exact.law_at(exact.pca_matrix(m), int(x0), 40), pi) < 1e-6
    assert chisq_pvalue(counts, pi) > 1e-4


# ------------------------------------------------------------- closed-form special cases

def one_site_probs(orc, L, g_c, nb_vals, *, J=0.0, q=0.0, sigma=1.0, beta=1.0, potts=False, T=1,
                   x_self=None, nbr=4, pos="centre", inertia=0):
    """Conditional of one site of a 3x3 lattice with the given neighbour values."""
    H = W = 3
    st = np.zeros((1, H, W), dtype=np.uint8)
    r, c = {"centre": (1, 1), "corner": (0, 0), "edge": (0, 1)}[pos]
    obs = np.full((H, W), 0.0, dtype=np.float32)
    obs[r, c] = g_c
    offs = [(-1, 0), (1, 0), (0, -1), (0, 1)] + ([(-1, -1), (-1, 1), (1, -1), (1, 1)] if nbr == 8 else [])
    vals = iter(nb_vals)
    for dr, dc in offs:
        rr, cc = r + dr, c + dc
        if 0 <= rr < H and 0 <= cc < W:
            st[0, rr, cc] = next(vals)
    if x_self is not None:
        st[0, r, c] = x_self
    p = orc.Params(height=H, width=W, levels=L, chains=1, neighbourhood=nbr,
                   prior=orc.POTTS if potts else orc.TRUNC_LINEAR, trunc=T, J=J, q=q, sigma=sigma,
                   vmin=0.0, vmax=float(L - 1), beta=[beta], seed=9, inertia=inertia)
    return orc.site_probs(p, obs, st, 0, r, c)


@pytest.mark.parametrize("g_c,sigma", [(20.0, 1.0), (31.37, 1.7), (40.5, 2.5), (25.25, 3.0)])
def test_discrete_gaussian_mean_and_variance(orc, g_c, sigma):
    """J = 0, q = 0: p(k) ~ exp(-(g-k)^2 / 2 sigma^2) on the integers; far from the ends its
    mean is g and its variance sigma^2 up to exp(-2 pi^2 sigma^2) (Poisson summation)."""
    p = one_site_probs(orc, 64, g_c, [0, 0, 0, 0], sigma=sigma)
    k = np.arange(64)
    mean = float((p * k).sum())
    var = float((p * (k - mean) ** 2).sum())
    tail = math.exp(-2 * math.pi ** 2 * sigma ** 2)
    assert abs(mean - np.float32(g_c)) < 2e-6 + tail
    assert abs(var - sigma ** 2) < 2e-5 * sigma ** 2 + 8 * tail


@pytest.mark.parametrize("g_c,sigma", [(0.5, 0.7), (0.2, 0.4), (0.9, 1.3), (-0.4, 0.6)])
def test_binary_logistic(orc, g_c, sigma):
    """L = 2, J = 0, q = 0: logit p(1) = ((g-0)^2 - (g-1)^2) / (2 sigma^2) = (2g-1)/(2 sigma^2)."""
    p = one_site_probs(orc, 2, g_c, [0, 0, 0, 0], sigma=sigma)
    want = 1.0 / (1.0 + math.exp(-(2 * float(np.float32(g_c)) - 1) / (2 * sigma ** 2)))
    assert abs(p[1] - want) < 1e-6


@pytest.mark.parametrize("beta,J", [(1.0, 0.3), (1.5, 0.5), (2.0, 1 / 3)])
def test_potts_profile_with_flat_data(orc, beta, J):
    """Potts, q = 0, data term flat (huge sigma), four neighbours all at level m: the level
    m is favoured by exp(2 beta J * 4) over every other level, which are all equal."""
    L, m = 5, 3
    p = one_site_probs(orc, L, 2.0, [m] * 4, J=J, beta=beta, potts=True, sigma=1e6)
    want = np.ones(L)
    want[m] = math.exp(2 * beta * J * 4)
    # level probabilities are differences of FP32 running sums: good to ~1 ulp of Z
    assert np.allclose(p, want / want.sum(), rtol=1e-6, atol=3e-7)


def test_potts_mixed_neighbours(orc):
    """Two neighbours at level 1, one at 3, one at 4: odds relative to an absent level 0 are
    exp(2 beta J * count)."""
    beta, J = 1.25, 0.4
    p = one_site_probs(orc, 5, 2.0, [1, 3, 1, 4], J=J, beta=beta, potts=True, sigma=1e6)
    want = np.exp(2 * beta * J * np.array([0, 2, 0, 1, 1]))
    assert np.allclose(p, want / want.sum(), rtol=1e-6, atol=3e-7)


@pytest.mark.parametrize("T", [1, 3, 6])
def test_truncated_linear_profile(orc, T):
    """Truncated linear, flat data: p(k) ~ exp(-beta J * 4 * min(|k - m|, T))."""
    L, m, beta, J = 16, 7, 1.0, 0.35
    p = one_site_probs(orc, L, 7.0, [m] * 4, J=J, beta=beta, T=T, sigma=1e6)
    k = np.arange(L)
    want = np.exp(-beta * J * 4 * np.minimum(np.abs(k - m), T))
    want /= want.sum()
    assert np.allclose(p, want, rtol=1e-6, atol=3e-7)


@pytest.mark.parametrize("pos,nbr,n_nb", [("corner", 4, 2), ("edge", 4, 3), ("corner", 8, 3),
                                           ("edge", 8, 5), ("centre", 8, 8)])
def test_free_boundary_neighbour_count(orc, pos, nbr, n_nb):
    """Only in-lattice neighbours count: with all of them at m and flat data, the odds of m
    against a level far beyond the truncation are exp(beta J T n)."""
    L, m, T, beta, J = 12, 2, 3, 1.0, 0.3
    p = one_site_probs(orc, L, 2.0, [m] * 8, J=J, beta=beta, T=T, sigma=1e6, nbr=nbr, pos=pos)
    k = np.arange(L)
    want = np.exp(-beta * J * T * n_nb) * np.exp(beta * J * (T - np.minimum(np.abs(k - m), T)) * n_nb)
    assert np.allclose(p, want / want.sum(), rtol=1e-6, atol=3e-7)
    assert abs(p[m] / p[11] - math.exp(beta * J * T * n_nb)) < 1e-4 * math.exp(beta * J * T * n_nb)


@pytest.mark.parametrize("beta,q", [(1.0, 0.5), (1.0, 2.0), (1.75, 0.71), (2.0, 3.0)])
def test_inertia_odds_at_symmetric_observation(orc, beta, q):
    """L = 2, J = 0, g = 1/2 so both levels have equal data weight: staying at the current
    value has probability 1/(1 + exp(-beta q)), whichever value that is."""
    for x in (0, 1):
        p = one_site_probs(orc, 2, 0.5, [0, 0, 0, 0], q=q, beta=beta, sigma=0.8, x_self=x)
        assert abs(p[x] - 1.0 / (1.0 + math.exp(-beta * q))) < 1e-6


@pytest.mark.parametrize("p,beta,q", [(1, 1.0, 0.5), (1, 1.5, 1.1), (2, 1.0, 0.3), (2, 2.0, 0.45)])
def test_inertia_norm_profile_with_flat_data(orc, p, beta, q):
    """J = 0 and a data term that is flat over the levels (huge sigma): the conditional is
    exp(-beta q |k - x|^p) normalised, a two-sided geometric law for p = 1 and a discrete
    Gaussian centred on the current value for p = 2 (Sec. 3 inertia q|x_i - w_i|^p)."""
    L, x = 13, 5
    got = one_site_probs(orc, L, 6.0, [0, 0, 0, 0], q=q, beta=beta, sigma=1e4, x_self=x, inertia=p)
    d = np.abs(np.arange(L) - x).astype(np.float64)
    want = np.exp(-beta * q * d ** p)
    assert np.allclose(got, want / want.sum(), rtol=1e-5, atol=3e-7)
    assert abs(got[x + 1] / got[x] - math.exp(-beta * q)) < 1e-5
    assert abs(got[x + 2] / got[x] - math.exp(-beta * q * 2 ** p)) < 1e-5


def test_inertia_norm_single_site_matches_exact_conditional(orc):
    rng = np.random.default_rng(15)
    for _ in range(30):
        p_ = int(rng.integers(1, 3))
        L = int(rng.integers(2, 40))
        nb = rng.integers(0, L, size=4).tolist()
        x = int(rng.integers(0, L))
        g_c = float(rng.uniform(-1, L))
        J, q, sigma, beta, T = rng.uniform(0, 1), rng.uniform(0, 2), rng.uniform(0.3, 4), rng.uniform(0.5, 2), int(
            rng.integers(1, L + 1))
        p = one_site_probs(orc, L, g_c, nb, J=J, q=q, sigma=sigma, beta=beta, T=T, x_self=x, inertia=p_)
        st = np.zeros(9, dtype=np.int64)
        st[[1, 7, 3, 5]] = nb
        st[4] = x
        m = exact.Model(H=3, W=3, L=L, nbr=4, potts=False, T=T, J=J, q=q, sigma=sigma, beta=beta,
                        g=np.array([[0, 0, 0], [0, np.float32(g_c), 0], [0, 0, 0]], dtype=np.float64), p=p_)
        want = exact.site_conditional(m, st, 4, inertia=True)
        # The data and inertia exponents are evaluated in FP32 in log2 units; where they
        # oppose each other they reach hundreds, and their rounding (2^-24 relative to the
        # magnitude) becomes a relative error of the weights.
        k = np.arange(L)
        F = (m.a * (np.float32(g_c) - k) ** 2 + beta * q * np.abs(k - x) ** p_) / math.log(2)
        rtol = 1e-6 + 2 * math.log(2) * 2.0 ** -24 * (F[want > 1e-9].max() + F.min())
        assert np.allclose(p, want, rtol=rtol, atol=3e-7), (p_, L, nb, x)


def test_beta_does_not_scale_the_data_term(orc):
    """J = q = 0: the conditional is the likelihood alone for every beta."""
    a = one_site_probs(orc, 16, 6.3, [2, 9, 4, 11], sigma=1.3, beta=1.0)
    b = one_site_probs(orc, 16, 6.3, [2, 9, 4, 11], sigma=1.3, beta=2.75)
    assert np.array_equal(a, b)


def test_beta_scales_prior_and_inertia_together(orc):
    """beta J and beta q enter only as products: (beta, J, q) and (2 beta, J/2, q/2) agree."""
    a = one_site_probs(orc, 16, 6.3, [2, 9, 4, 11], J=0.8, q=1.2, sigma=1.3, beta=1.0, x_self=5, T=4)
    b = one_site_probs(orc, 16, 6.3, [2, 9, 4, 11], J=0.4, q=0.6, sigma=1.3, beta=2.0, x_self=5, T=4)
    assert np.allclose(a, b, rtol=1e-6, atol=1e-12)


def test_single_site_matches_exact_conditional(orc):
    """Random neighbourhoods: the FP32 probabilities agree with the float64 conditional."""
    rng = np.random.default_rng(5)
    for _ in range(30):
        L = int(rng.integers(2, 40))
        nb = rng.integers(0, L, size=4).tolist()
        x = int(rng.integers(0, L))
        g_c = float(rng.uniform(-1, L))
        J, q, sigma, beta, T = rng.uniform(0, 1), rng.uniform(0, 2), rng.uniform(0.3, 4), rng.uniform(0.5, 2), int(
            rng.integers(1, L + 1))
        p = one_site_probs(orc, L, g_c, nb, J=J, q=q, sigma=sigma, beta=beta, T=T, x_self=x)
        st = np.zeros(9, dtype=np.int64)
        st[[1, 7, 3, 5]] = nb
        st[4] = x
        m = exact.Model(H=3, W=3, L=L, nbr=4, potts=False, T=T, J=J, q=q, sigma=sigma, beta=beta,
                        g=np.array([[0, 0, 0], [0, np.float32(g_c), 0], [0, 0, 0]], dtype=np.float64))
        want = exact.site_conditional(m, st, 4, inertia=True)
        assert np.allclose(p, want, rtol=1e-6, atol=3e-7), (L, nb, x)


# ---------------------------------------------------------------------- draw and chains

def test_draw_frequencies_match_conditional(orc):
    """All chains start in the same state, so after one sweep each site's value over the
    chains is a sample of its conditional: inverse-CDF frequencies match."""
    H, W, L, C = 4, 5, 9, M_CHAINS // 4
    rng = np.random.default_rng(11)
    obs = rng.uniform(0, L - 1, size=(H, W)).astype(np.float32)
    p = orc.Params(height=H, width=W, levels=L, chains=C, neighbourhood=8, prior=orc.TRUNC_LINEAR, trunc=3,
                   J=0.45, q=0.9, sigma=1.4, beta=[1.25], seed=77)
    run = orc.Run(p, obs)
    start = run.state.copy()
    run.sweep(1)
    for (r, c) in [(0, 0), (1, 2), (3, 4), (2, 0)]:
        probs = orc.site_probs(p, obs, start, 0, r, c)
        counts = np.bincount(run.state[:, r, c], minlength=L).astype(np.float64)
        assert chisq_pvalue(counts, probs) > 1e-4


def _acc(weights, stay):
    """FP32 running sums as the sampler forms them: the stay weight, then fma-free adds
    of exactly representable weights (so the sums are exact)."""
    acc = [np.float32(stay)]
    for w in weights:
        acc.append(np.float32(acc[-1] + np.float32(w)))
    return np.array(acc, dtype=np.float32)


def test_draw_rule_at_the_ends_of_the_uniform(orc):
    """u = 0 takes the first positive weight in the order (stay, 0, 1, ..., L-1); the
    largest u, 1 - 2^-24, takes the last positive one; zero weights are never drawn."""
    w = [0.0, 0.0, 0.25, 0.5, 0.0, 0.125, 0.0]
    acc = _acc(w, 0.0)
    assert orc.draw(acc, 3, 0) == 2 and orc.draw(acc, 3, 255) == 2  # both give u = 0
    assert orc.draw(acc, 3, 0xFFFFFFFF) == 5
    acc = _acc(w, 0.0625)
    assert orc.draw(acc, 6, 0) == 6             # positive stay weight: u = 0 stays, at a zero-weight level
    assert orc.draw(acc, 6, 0xFFFFFFFF) == 5


def test_draw_rule_is_monotone_and_exact_at_boundaries(orc):
    """The drawn position in (stay, 0, ..., L-1) never decreases with u, and u exactly at
    a cumulative boundary belongs to the next cell (strict inequality)."""
    rng = np.random.default_rng(21)
    for _ in range(20):
        L = int(rng.integers(2, 12))
        w = (rng.integers(0, 5, size=L) / 8.0).tolist()
        stay = float(rng.integers(0, 3) / 8.0)
        if sum(w) + stay == 0:
            w[0] = 0.125
        acc = _acc(w, stay)
        x = int(rng.integers(0, L))
        pos_of = lambda k, u_word: (-1 if k == x and float(acc[0]) > float(orc.uniform(u_word)) * float(acc[-1])  # noqa: E731
                                    else k)
        last = -2
        for r in range(0, 1 << 24, 1 << 14):
            word = r << 8
            k = orc.draw(acc, x, word)
            pos = pos_of(k, word)
            assert pos >= last
            last = pos
        Z = float(acc[-1])
        for j in range(1, L + 1):  # u with u*Z equal to the cumulative sum acc_{j-2}
            c = float(acc[j - 1])
            r = c / Z * (1 << 24)
            if r == int(r) and 0 <= r < (1 << 24) and c > 0:
                k = orc.draw(acc, x, int(r) << 8)
                cum = acc[1:]
                assert k == x or cum[k] > c


def test_draw_keeps_the_state_when_every_weight_is_zero(orc):
    acc = np.zeros(6, dtype=np.float32)
    for x in range(5):
        for word in (0, 0x12345678, 0xFFFFFFFF):
            assert orc.draw(acc, x, word) == x


def test_sweeps_compose_and_chains_are_independent_of_chain_count(orc):
    H, W, L = 6, 5, 16
    rng = np.random.default_rng(3)
    obs = rng.uniform(0, 15, size=(H, W)).astype(np.float32)
    base = dict(height=H, width=W, levels=L, neighbourhood=4, prior=orc.TRUNC_LINEAR, trunc=4, J=0.4, q=1.5,
                sigma=2.0, beta=[1.0, 1.25, 1.5], seed=2024, tally_stride=1)
    a = orc.Run(orc.Params(chains=7, **base), obs).sweep(3).sweep(4)
    b = orc.Run(orc.Params(chains=7, **base), obs).sweep(7)
    assert np.array_equal(a.state, b.state)
    assert np.array_equal(a.sum, b.sum) and a.count[0] == b.count[0] == 49
    assert np.array_equal(a.hist, b.hist)
    c = orc.Run(orc.Params(chains=3, **base), obs).sweep(7)
    assert np.array_equal(c.state, b.state[:3])
    g = orc.Run(orc.Params(chains=7, **base), obs, gibbs=True).sweep(7)
    assert not np.array_equal(g.state, b.state)


def test_random_init_is_uniform(orc):
    H, W, L, C = 16, 16, 7, 64
    p = orc.Params(height=H, width=W, levels=L, chains=C, J=0.1, sigma=1.0, init_mode=1, seed=5)
    st = orc.init_state(p, np.zeros((H, W), np.float32))
    counts = np.bincount(st.reshape(-1), minlength=L).astype(np.float64)
    assert chisq_pvalue(counts, np.full(L, 1.0 / L)) > 1e-4
    assert st.max() < L


def test_nearest_level_init_and_value_units(orc):
    """Values map to levels as vmin + k (vmax - vmin)/(L-1); init picks the nearest level."""
    p = orc.Params(height=1, width=5, levels=2, chains=2, J=0.8, q=2.0, sigma=0.6, vmin=-1.0, vmax=1.0)
    obs = np.array([[-3.0, -0.2, 0.0, 0.2, 2.5]], dtype=np.float32)
    st = orc.init_state(p, obs)
    assert st[0].tolist() == [[0, 0, 0, 1, 1]]  # 0.0 -> level 0.5 -> rint half-even -> 0
    assert orc.level_obs(p, 1.0) == 1.0 and orc.level_obs(p, -1.0) == 0.0


def test_posterior_mean_and_marginal_map_definitions(orc):
    p = orc.Params(height=1, width=4, levels=3, chains=2, sigma=1.0, vmin=-1.0, vmax=1.0, tally_stride=1)
    run = orc.Run(p, np.zeros((1, 4), np.float32))
    run.sum[:] = [0, 3, 5, 8]
    run.count[0] = 4
    mean = run.posterior_mean()
    # level mean sum/count in [0, 2] mapped to [-1, 1]
    assert mean[0].tolist() == [-1.0, -0.25, 0.25, 1.0]
    run.hist[0] = [[0, 0, 0], [2, 2, 1], [1, 3, 3], [0, 0, 5]]
    assert run.marginal_map().tolist() == [[0, 0, 1, 2]]


def test_statistics_respect_burn_in_and_tally_stride(orc):
    H, W, L, C = 3, 4, 5, 2
    obs = np.random.default_rng(1).uniform(0, 4, size=(H, W)).astype(np.float32)
    p = orc.Params(height=H, width=W, levels=L, chains=C, J=0.3, q=1.0, sigma=1.0, burn_in=3, tally_stride=2,
                   seed=8)
    run = orc.Run(p, obs)
    sums, hist = np.zeros((H, W), np.int64), np.zeros((H, W, L), np.int64)
    for t in range(8):
        run.sweep(1)
        if t >= 3:
            sums += run.state.astype(np.int64).sum(axis=0)
            if (t - 3) % 2 == 0:
                for ch in range(C):
                    np.add.at(hist, (np.arange(H)[:, None], np.arange(W)[None, :], run.state[ch]), 1)
    assert np.array_equal(run.sum, sums) and run.count[0] == 5 * C
    assert np.array_equal(run.hist, hist)


@pytest.mark.parametrize("bad", [dict(levels=1), dict(levels=257), dict(chains=0), dict(neighbourhood=6),
                                 dict(prior=2), dict(trunc=0), dict(J=-0.1), dict(q=-1.0), dict(sigma=0.0),
                                 dict(vmax=0.0), dict(init_mode=2), dict(burn_in=-1), dict(tally_stride=-1),
                                 dict(beta=[0.0]), dict(height=0), dict(q=80.0), dict(inertia=3),
                                 dict(inertia=-1)])
def test_invalid_parameters_rejected(orc, bad):
    kw = dict(height=2, width=2, levels=4, chains=1, prior=orc.TRUNC_LINEAR, trunc=1, J=0.1, q=0.5, sigma=1.0,
              vmin=0.0, vmax=3.0)
    kw.update(bad)
    with pytest.raises(ValueError):
        orc.init_state(orc.Params(**kw), np.zeros((kw["height"], 2), np.float32))
