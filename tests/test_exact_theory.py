"""The float64 exact laws used to pin the oracle, checked against the paper's theory.

These tests touch no sampler code; they establish that the enumerated transition
matrices behave as Sec. 3 says (reversibility, closed-form stationary law) so that the
oracle's empirical laws can be compared with them.
"""
import numpy as np
import pytest

from tests import exact


def _model(H, W, L, nbr, potts, T, J, q, sigma, beta, seed, p=0):
    rng = np.random.default_rng(seed)
    g = rng.uniform(-0.3, L - 0.7, size=(H, W)).astype(np.float32).astype(np.float64)
    return exact.Model(H=H, W=W, L=L, nbr=nbr, potts=potts, T=T, J=J, q=q, sigma=sigma, beta=beta, g=g, p=p)


CASES = [
    # 3x3 binary Potts, 4 neighbours (512 states)
    dict(H=3, W=3, L=2, nbr=4, potts=True, T=1, J=0.6, q=1.0, sigma=0.7, beta=1.0, seed=1),
    # 2x3 with 3 levels, truncated linear, 8 neighbours (729 states)
    dict(H=2, W=3, L=3, nbr=8, potts=False, T=1, J=0.5, q=0.7, sigma=0.9, beta=1.3, seed=2),
    # 2x2 with 4 levels, truncated linear T=2, 4 neighbours (256 states)
    dict(H=2, W=2, L=4, nbr=4, potts=False, T=2, J=0.8, q=0.4, sigma=1.1, beta=0.8, seed=3),
    # the L1 and L2 inertia norms of Sec. 3 on the 2x3 and 2x2 lattices
    dict(H=2, W=3, L=3, nbr=8, potts=False, T=1, J=0.5, q=0.7, sigma=0.9, beta=1.3, seed=2, p=1),
    dict(H=2, W=2, L=4, nbr=4, potts=False, T=2, J=0.8, q=0.4, sigma=1.1, beta=0.8, seed=3, p=2),
]


@pytest.mark.parametrize("case", CASES)
def test_pca_matrix_is_stochastic_and_reversible(case):
    m = _model(**case)
    P = exact.pca_matrix(m)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
    pi = exact.pca_closed_form(m)
    # detailed balance pi(x) P(x,w) = pi(w) P(w,x): Sec. 3 eq. (pca_detailed_balance)
    F = pi[:, None] * P
    assert np.max(np.abs(F - F.T)) < 1e-14


@pytest.mark.parametrize("case", CASES)
def test_pca_stationary_vector_equals_closed_form(case):
    m = _model(**case)
    P = exact.pca_matrix(m)
    assert exact.tv(exact.stationary(P), exact.pca_closed_form(m)) < 1e-11


@pytest.mark.parametrize("case", CASES)
def test_systematic_gibbs_preserves_joint_posterior(case):
    m = _model(**case)
    M = exact.gibbs_sweep_matrix(m)
    pi = exact.gibbs_posterior(m)
    assert exact.tv(pi @ M, pi) < 1e-12
    assert exact.tv(exact.stationary(M), pi) < 1e-10


def test_pca_differs_from_gibbs_at_finite_q():
    """The lazy PCA only approximates the posterior (Sec. 3, 'The lazy PCA')."""
    m = _model(**CASES[0])
    assert exact.tv(exact.pca_closed_form(m), exact.gibbs_posterior(m)) > 1e-2


def test_large_q_limit_is_squared_gibbs_law():
    """As q grows the PCA law tends to pi_GS^2 (doubled coupling and data precision),
    a sharpened form of the paper's q -> infinity remark (Sec. 3, 'Distinctive features')."""
    base = dict(CASES[0])
    d = []
    for q in (2.0, 4.0, 8.0):
        base["q"] = q
        m = _model(**base)
        d.append(exact.tv(exact.pca_closed_form(m), exact.gibbs_posterior(m, power=2.0)))
    assert d[0] > d[1] > d[2]
    assert d[2] < 2e-3


def test_q_zero_is_synchronous_product_of_gibbs_conditionals():
    """q = 0 gives the naive parallel update of Sec. 3 (product of full conditionals)."""
    case = dict(CASES[0])
    case["q"] = 0.0
    m = _model(**case)
    P = exact.pca_matrix(m)
    X = exact.states(m)
    for a in (0, 77, 300, 511):
        row = np.ones(X.shape[0])
        for i in range(m.H * m.W):
            row *= exact.site_conditional(m, X[a], i, inertia=False)[X[:, i]]
        assert np.allclose(P[a], row, atol=1e-15)


def test_halved_coupling_and_doubled_variance_target_the_posterior_as_q_grows():
    """Since the q -> infinity limit squares the Gibbs law, running the PCA with J/2 and
    sigma*sqrt(2) makes that limit the posterior itself (the correction offered by
    paper_2507_14869_amd.variants.posterior_matched)."""
    from paper_2507_14869_amd.variants import posterior_matched
    base = dict(CASES[0])
    target = exact.gibbs_posterior(_model(**base))
    d_plain, d_matched = [], []
    for q in (2.0, 4.0, 8.0):
        m = _model(**{**base, "q": q})
        d_plain.append(exact.tv(exact.pca_closed_form(m), target))
        adj = posterior_matched({"J": base["J"], "sigma": base["sigma"]})
        mm = _model(**{**base, "q": q, "J": adj["J"], "sigma": adj["sigma"]})
        d_matched.append(exact.tv(exact.pca_closed_form(mm), target))
    assert d_matched[0] > d_matched[1] > d_matched[2]
    assert d_matched[2] < 2e-3 < d_plain[2]


@pytest.mark.parametrize("p", [1, 2])
def test_large_q_limit_is_squared_gibbs_law_for_every_norm(p):
    """Any inertia that vanishes only at k = x_i has the same q -> infinity limit."""
    base = dict(CASES[2], p=p)
    d = []
    for q in (2.0, 4.0, 8.0):
        m = _model(**{**base, "q": q})
        d.append(exact.tv(exact.pca_closed_form(m), exact.gibbs_posterior(m, power=2.0)))
    assert d[0] > d[1] > d[2]
    assert d[2] < 2e-3


def test_norms_coincide_on_binary_lattices_and_differ_beyond():
    """With two levels |k - x| is 0 or 1, so the indicator, L1 and L2 inertias agree; with
    four levels a change by 2 costs q, 2q and 4q respectively."""
    for p in (1, 2):
        a = _model(**CASES[0])
        b = _model(**{**CASES[0], "p": p})
        assert np.array_equal(exact.pca_matrix(a), exact.pca_matrix(b))
    laws = [exact.pca_closed_form(_model(**{**CASES[2], "p": p})) for p in (0, 1, 2)]
    assert exact.tv(laws[0], laws[1]) > 1e-3 and exact.tv(laws[1], laws[2]) > 1e-3
