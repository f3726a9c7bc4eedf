"""Pins of the oracle's per-site conditional at the parameter points the workloads run at.

The random-site pin in test_oracle_sampler.py draws its parameters from small ranges
(L < 40, four neighbours, truncated-linear prior).  Here the oracle's FP32 probabilities
are compared with the float64 conditional of the lazy PCA (Sec. 5.2, the transition after
eq. (denoising_pair_posterior_Hamiltonian); the 8-site neighbourhood of eq. (neighborhood))
at exactly the binary Potts point (L = 2, J = 0.8, q = 2, sigma = 0.6 in value units on
[-1, 1]), the 16-level point (T = 4, J = 0.4, q = 1.5, sigma = 2), the 256-level point
(T = 32, J = 0.05, q = 1, sigma = 20), with four and eight neighbours, at interior, edge
and corner sites, and at the paper's own experiment (8-neighbour Potts, J = 1/3, the beta
schedule and q grid of Sec. 6).

The tolerance is derived from the FP32 arithmetic of the convention, per level k:
exp2s has relative error below 4e-7; rounding the data exponent (about |a2 e_k^2| in log2
units) and the prior exponent (|c2 S_k|) costs ln2 * 2^-24 per unit of magnitude and
operation; the running sum rounds once per level, which moves Z by at most L * 2^-24
relative and each implied probability by at most 2 * 2^-24 absolute.  A dropped term, a
wrong sign, a truncation off by one or a wrong neighbour count moves some probability by
far more (the smallest such change here is a factor exp(-0.05) on a level's weight).
"""
import math

import numpy as np
import pytest

from tests import exact

ULP = 2.0 ** -24
OFFS4 = [(-1, 0), (1, 0), (0, -1), (0, 1)]
OFFS8 = OFFS4 + [(-1, -1), (-1, 1), (1, -1), (1, 1)]

# name: (L, potts, T, J, q, sigma in value units, vmin, vmax)
POINTS = {
    "binary_potts": (2, True, 1, 0.8, 2.0, 0.6, -1.0, 1.0),
    "L16_trunc4": (16, False, 4, 0.4, 1.5, 2.0, 0.0, 15.0),
    "L256_trunc32": (256, False, 32, 0.05, 1.0, 20.0, 0.0, 255.0),
}


def site_case(orc, rng, L, potts, T, J, q, sigma, vmin, vmax, nbr, beta, pos, near):
    """A 3x3 lattice with random neighbour levels (near the observation or uniform), the
    oracle's FP32 probabilities for one site and the float64 conditional."""
    H = W = 3
    r, c = {"centre": (1, 1), "edge": (0, 1), "corner": (2, 2)}[pos]
    delta = (vmax - vmin) / (L - 1)
    g_level = rng.uniform(-0.1 * L, 1.1 * L) if rng.random() < 0.2 else rng.uniform(0, L - 1)
    obs = np.zeros((H, W), dtype=np.float32)
    obs[r, c] = np.float32(vmin + g_level * delta)
    st = np.zeros((1, H, W), dtype=np.uint8)
    centre = int(np.clip(round(g_level), 0, L - 1))
    spread = max(1, L // 8)
    for rr in range(H):
        for cc in range(W):
            if near:
                st[0, rr, cc] = int(np.clip(centre + rng.integers(-spread, spread + 1), 0, L - 1))
            else:
                st[0, rr, cc] = int(rng.integers(0, L))
    p = orc.Params(height=H, width=W, levels=L, chains=1, neighbourhood=nbr,
                   prior=orc.POTTS if potts else orc.TRUNC_LINEAR, trunc=T, J=J, q=q, sigma=sigma, vmin=vmin,
                   vmax=vmax, beta=[beta], seed=17)
    got = orc.site_probs(p, obs, st, 0, r, c)
    gp = orc.level_obs(p, float(obs[r, c]))  # the FP32 observation in level units (C1)
    g = np.zeros((H, W))
    g[r, c] = gp
    m = exact.Model(H=H, W=W, L=L, nbr=nbr, potts=potts, T=T, J=J, q=q, sigma=sigma / delta, beta=beta, g=g)
    want = exact.site_conditional(m, st[0].reshape(-1), r * W + c, inertia=True)
    # per-level magnitudes of the two exponents (log2 units) for the tolerance
    k = np.arange(L)
    S = np.zeros(L)
    for dr, dc in (OFFS8 if nbr == 8 else OFFS4):
        if 0 <= r + dr < H and 0 <= c + dc < W:
            S += np.minimum(np.abs(k - int(st[0, r + dr, c + dc])), m.Teff)
    y_data = m.a * (gp - k) ** 2 / math.log(2)
    y_prior = m.c * S / math.log(2)
    rtol = 5e-7 + math.log(2) * ULP * (3 * y_data + 2 * y_prior + 3) + L * ULP
    return got, want, rtol


def check(got, want, rtol):
    err = np.abs(got - want)
    ok = err <= rtol * want + 2 * ULP + 1e-9
    return bool(ok.all()), float((err / np.maximum(want, 1e-300)).max())


@pytest.mark.parametrize("name", list(POINTS))
@pytest.mark.parametrize("nbr", [4, 8])
def test_conditional_at_workload_points(orc, name, nbr):
    L, potts, T, J, q, sigma, vmin, vmax = POINTS[name]
    rng = np.random.default_rng(hash((name, nbr)) % (1 << 32))
    for i in range(60):
        pos = ("centre", "edge", "corner")[i % 3]
        got, want, rtol = site_case(orc, rng, L, potts, T, J, q, sigma, vmin, vmax, nbr, 1.0, pos, near=i % 2 == 0)
        ok, worst = check(got, want, rtol)
        assert ok, (name, nbr, pos, i, worst)


@pytest.mark.parametrize("L,sigma01", [(5, 0.25), (9, 0.2), (33, 0.1)])
def test_conditional_at_the_paper_experiment(orc, L, sigma01):
    """8-neighbour Potts, J = 1/3, values in [0, 1] with the noise of the paper's test
    images, every beta of the schedule and the ends and middle of the q grid (Sec. 6)."""
    rng = np.random.default_rng(L)
    for beta in (1.25, 1.5, 1.75, 2.0):
        for q in (0.06, 0.31, 0.71):
            for pos in ("centre", "edge", "corner"):
                got, want, rtol = site_case(orc, rng, L, True, 1, 1 / 3, q, sigma01, 0.0, 1.0, 8, beta, pos,
                                            near=True)
                ok, worst = check(got, want, rtol)
                assert ok, (L, beta, q, pos, worst)


def test_tolerance_detects_plausible_mistakes(orc):
    """The bound above is tight enough to see the smallest model changes that matter:
    the truncation off by one, the coupling of one neighbour dropped, q off by 1%."""
    L, potts, T, J, q, sigma, vmin, vmax = POINTS["L256_trunc32"]
    rng = np.random.default_rng(99)
    seen = {"T-1": False, "J*0.99": False, "q*1.01": False}
    for i in range(20):
        got, want, rtol = site_case(orc, rng, L, potts, T, J, q, sigma, vmin, vmax, 4, 1.0, "centre", near=True)
        for tag, (T2, J2, q2) in {"T-1": (T - 1, J, q), "J*0.99": (T, J * 0.99, q), "q*1.01": (T, J, q * 1.01)}.items():
            rng2 = np.random.default_rng(99 + 1000 * i)  # same site again, perturbed model on the oracle side
            g2, _, _ = site_case(orc, rng2, L, potts, T2, J2, q2, sigma, vmin, vmax, 4, 1.0, "centre", near=True)
            rng3 = np.random.default_rng(99 + 1000 * i)
            _, w2, r2 = site_case(orc, rng3, L, potts, T, J, q, sigma, vmin, vmax, 4, 1.0, "centre", near=True)
            ok, _ = check(g2, w2, r2)
            seen[tag] = seen[tag] or not ok
    assert all(seen.values()), seen


@pytest.mark.parametrize("p", [1, 2])
def test_inertia_shift_is_the_plain_maximum(orc, p):
    """C8 shifts the L1/L2 exponents by their maximum over the levels, found in O(1) from
    the concavity of F_k in k; it equals the plain O(L) maximum of the same FP32 exponents,
    over random sites at every level count of the workloads, observations far outside the
    level range, sigma from 0.01 to 200 levels and q from 1e-4 to 30."""
    rng = np.random.default_rng(40 + p)
    for _ in range(3000):
        L = int(rng.choice([2, 5, 16, 33, 200, 256]))
        sigma = float(np.exp(rng.uniform(math.log(0.01), math.log(200.0))))
        q = float(np.exp(rng.uniform(math.log(1e-4), math.log(30.0))))
        beta = float(rng.uniform(0.5, 2.0))
        if beta * q * math.log2(math.e) > 100.0:
            continue
        g = rng.uniform(-50, L + 50) if rng.random() < 0.3 else rng.uniform(0, L - 1)
        x = int(rng.integers(0, L))
        prm = orc.Params(height=1, width=1, levels=L, chains=1, J=0.1, q=q, sigma=sigma, beta=[beta], inertia=p)
        F, fmax = orc.inertia_exponents(prm, np.array([[g]], dtype=np.float32), np.array([[[x]]], dtype=np.uint8),
                                        0, 0, 0)
        assert fmax == float(F.max()), (L, sigma, q, beta, g, x)
