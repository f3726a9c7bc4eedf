"""The GPU sampler's empirical law against the exact float64 law of the enumerated
transition matrix, with no reference to the CPU oracle's code: 2e5 independent GPU chains
(200 seeds x 1024 chains) on lattices of 512 and 256 states, after t sweeps, against
P^t(x0, .) by chi-square (Sec. 3, product transition of the lazy PCA), and after a long
run against the closed-form stationary law."""
import numpy as np
import pytest

try:  # import at collection so the first GPU test's time limit does not include it
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

from tests import exact
from tests.gpu_util import gpu_sampler
from tests.test_oracle_sampler import chisq_pvalue

pytestmark = pytest.mark.gpu

SEEDS = 200
CHAINS = 1024


def _laws(case, sweeps):
    rng = np.random.default_rng(case["seed"])
    H, W, L = case["H"], case["W"], case["L"]
    g = rng.uniform(-0.3, L - 0.7, size=(H, W)).astype(np.float32)
    m = exact.Model(H=H, W=W, L=L, nbr=case["nbr"], potts=case["potts"], T=case["T"], J=case["J"], q=case["q"],
                    sigma=case["sigma"], beta=case["beta"], g=g.astype(np.float64), p=case.get("p", 0))
    kw = dict(height=H, width=W, levels=L, chains=CHAINS, neighbourhood=case["nbr"], prior=0 if case["potts"] else 1,
              trunc=case["T"], J=case["J"], q=case["q"], sigma=case["sigma"], vmin=0.0, vmax=float(L - 1),
              beta=[case["beta"]], inertia=case.get("p", 0))
    counts = np.zeros(L ** (H * W))
    x0 = None
    for s in range(SEEDS):
        smp = gpu_sampler(g, seed=90000 + 7919 * s, **kw)
        if x0 is None:
            x0 = exact.state_index(m, smp.state().cpu().numpy()[:1].reshape(1, -1))[0]
        st = smp.sweep(sweeps).state().cpu().numpy().reshape(CHAINS, -1)
        smp.close()
        counts += np.bincount(exact.state_index(m, st), minlength=counts.size)
    return m, int(x0), counts


@pytest.mark.parametrize("case", [
    dict(H=3, W=3, L=2, nbr=4, potts=True, T=1, J=0.6, q=1.0, sigma=0.7, beta=1.0, seed=1, t=6),
    dict(H=2, W=2, L=4, nbr=4, potts=False, T=2, J=0.8, q=0.4, sigma=1.1, beta=0.8, seed=3, t=4),
    dict(H=2, W=2, L=4, nbr=4, potts=False, T=2, J=0.8, q=0.4, sigma=1.1, beta=0.8, seed=3, t=4, p=2),
])
def test_gpu_law_after_t_sweeps(case):
    m, x0, counts = _laws(case, case["t"])
    law = exact.law_at(exact.pca_matrix(m), x0, case["t"])
    assert chisq_pvalue(counts, law) > 1e-4


def test_gpu_long_run_matches_closed_form_stationary_law():
    case = dict(H=3, W=3, L=2, nbr=4, potts=True, T=1, J=0.2, q=0.5, sigma=0.7, beta=1.0, seed=1)
    m, x0, counts = _laws(case, 40)  # second eigenvalue 0.63: mixed to 1e-8
    assert chisq_pvalue(counts, exact.pca_closed_form(m)) > 1e-4
