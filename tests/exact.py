"""Exact float64 laws of the samplers on lattices small enough to enumerate.

Independent of the oracle: these functions are written from the paper's formulas in
natural-log units and float64, and are what the oracle's empirical behaviour is pinned to.

* PCA transition (product of single-site conditionals): Sec. 3 eq. (general_pca_definition)
  with the lazy posterior conditional of Sec. 5.2 (inertia compares with the site's own
  previous value; indicator by default, or q|k - x_i|^p for p = 1, 2 as in Sec. 3).
* Closed-form stationary law of a PCA with a symmetric pair Hamiltonian, Sec. 3
  eq. (symm_ham_pca_stationary_measure): pi(x) ~ sum_w exp(-H(x,w)); with the data term
  added symmetrically this is exp(-D(x)) * prod_i Z_i(x).
* Gibbs posterior from the JOINT Hamiltonian over unordered neighbour pairs (the law whose
  single-site conditionals are Sec. 5.1 eq. (gibbs_sampler_elementary_step)).
* Systematic-scan Gibbs sweep matrix (Sec. 2, single-spin-flip sampler, fixed order).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np


@dataclass
class Model:
    H: int
    W: int
    L: int
    nbr: int          # 4 or 8
    potts: bool       # Potts (c = 2 beta J, T = 1) or truncated linear (c = beta J)
    T: int
    J: float
    q: float
    sigma: float      # level units
    beta: float
    g: np.ndarray     # [H, W] observation in level units
    p: int = 0        # inertia exponent: q |k - x_i|^p with 0^0 = 0 (p = 0: indicator)

    @property
    def c(self) -> float:
        return (2.0 if self.potts else 1.0) * self.beta * self.J

    @property
    def Teff(self) -> int:
        return 1 if self.potts else min(self.T, self.L - 1)

    @property
    def a(self) -> float:
        return 1.0 / (2.0 * self.sigma ** 2)


def neighbours(m: Model, i: int):
    r, c = divmod(i, m.W)
    offs = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    if m.nbr == 8:
        offs += [(-1, -1), (-1, 1), (1, -1), (1, 1)]
    out = []
    for dr, dc in offs:
        rr, cc = r + dr, c + dc
        if 0 <= rr < m.H and 0 <= cc < m.W:
            out.append(rr * m.W + cc)
    return out


def states(m: Model) -> np.ndarray:
    """All configurations, [L^N, N], site 0 varying slowest."""
    N = m.H * m.W
    return np.array(list(itertools.product(range(m.L), repeat=N)), dtype=np.int64)


def state_index(m: Model, x: np.ndarray) -> np.ndarray:
    """Index of configurations x [..., N] in the order of :func:`states`."""
    N = m.H * m.W
    w = m.L ** np.arange(N - 1, -1, -1)
    return (np.asarray(x, dtype=np.int64) * w).sum(axis=-1)


def log_site_weights(m: Model, x: np.ndarray, i: int, inertia: bool) -> np.ndarray:
    """log of the unnormalised conditional of site i given configuration x (natural log)."""
    g = m.g.reshape(-1)[i]
    k = np.arange(m.L)
    S = np.zeros(m.L)
    for j in neighbours(m, i):
        S += np.minimum(np.abs(k - x[j]), m.Teff)
    lw = -m.c * S - m.a * (g - k) ** 2
    if inertia:
        d = np.abs(k - x[i]).astype(np.float64)
        lw = lw - m.beta * m.q * ((d != 0) if m.p == 0 else d ** m.p)
    return lw


def site_conditional(m: Model, x, i, inertia: bool) -> np.ndarray:
    lw = log_site_weights(m, np.asarray(x), i, inertia)
    w = np.exp(lw - lw.max())
    return w / w.sum()


def pca_matrix(m: Model) -> np.ndarray:
    """P(x, w) = prod_i p_i(w_i | x)."""
    X = states(m)
    N = m.H * m.W
    P = np.ones((X.shape[0], X.shape[0]))
    for a, x in enumerate(X):
        for i in range(N):
            p = site_conditional(m, x, i, inertia=True)
            P[a] *= p[X[:, i]]
    return P


def data_energy(m: Model, X: np.ndarray) -> np.ndarray:
    g = m.g.reshape(-1)
    return (m.a * (g[None, :] - X) ** 2).sum(axis=1)


def pca_closed_form(m: Model) -> np.ndarray:
    """exp(-D(x)) prod_i Z_i(x), normalised (log-domain for stability)."""
    X = states(m)
    N = m.H * m.W
    logpi = -data_energy(m, X)
    for a, x in enumerate(X):
        for i in range(N):
            lw = log_site_weights(m, x, i, inertia=True)
            mx = lw.max()
            logpi[a] += mx + np.log(np.exp(lw - mx).sum())
    logpi -= logpi.max()
    pi = np.exp(logpi)
    return pi / pi.sum()


def edges(m: Model):
    N = m.H * m.W
    return [(i, j) for i in range(N) for j in neighbours(m, i) if j > i]


def gibbs_posterior(m: Model, power: float = 1.0) -> np.ndarray:
    """pi_GS(x) ~ exp(-c sum_{edges} min(|x_i - x_j|, T) - D(x)), raised to `power`."""
    X = states(m)
    logpi = -data_energy(m, X)
    for i, j in edges(m):
        logpi -= m.c * np.minimum(np.abs(X[:, i] - X[:, j]), m.Teff)
    logpi *= power
    logpi -= logpi.max()
    pi = np.exp(logpi)
    return pi / pi.sum()


def gibbs_sweep_matrix(m: Model) -> np.ndarray:
    """Systematic scan in row-major order: product of single-site update matrices."""
    X = states(m)
    nS = X.shape[0]
    N = m.H * m.W
    idx_of = {tuple(x): a for a, x in enumerate(X)}
    M = np.eye(nS)
    for i in range(N):
        K = np.zeros((nS, nS))
        for a, x in enumerate(X):
            p = site_conditional(m, x, i, inertia=False)
            for k in range(m.L):
                y = x.copy()
                y[i] = k
                K[a, idx_of[tuple(y)]] += p[k]
        M = M @ K
    return M


def stationary(P: np.ndarray) -> np.ndarray:
    """Left Perron vector of a row-stochastic matrix."""
    vals, vecs = np.linalg.eig(P.T)
    k = int(np.argmin(np.abs(vals - 1.0)))
    v = np.real(vecs[:, k])
    v = np.abs(v)
    return v / v.sum()


def tv(p: np.ndarray, q: np.ndarray) -> float:
    return 0.5 * float(np.abs(p - q).sum())


def law_at(P: np.ndarray, start: int, t: int) -> np.ndarray:
    v = np.zeros(P.shape[0])
    v[start] = 1.0
    for _ in range(t):
        v = v @ P
    return v
