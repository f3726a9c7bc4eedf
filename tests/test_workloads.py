"""Synthetic inputs, quality metrics, and the oracle's restoration quality on c1."""
import math

import numpy as np
import pytest

from workloads import synth, metrics


def test_named_workloads_are_seeded_and_shaped():
    a = synth.make_workload("c1")
    b = synth.make_workload("c1")
    assert np.array_equal(a.truth, b.truth) and np.array_equal(a.obs, b.obs)
    assert a.truth.shape == (64, 64) and a.truth.dtype == np.uint8 and a.obs.dtype == np.float32
    assert set(np.unique(a.truth)) <= {0, 1} and a.truth.mean() > 0.05
    # noise has the stated standard deviation in value units
    resid = a.obs - (-1.0 + 2.0 * a.truth)
    assert abs(resid.std() - 0.6) < 0.03
    c = synth.make_workload("c2", height=96, width=80)
    assert c.truth.shape == (96, 80) and c.truth.max() <= 15
    assert len(np.unique(c.truth)) > 5


def test_batch_and_trace_are_mixed():
    batch = synth.batch_mix(12, side_lo=16, side_hi=64)
    assert {w.levels for w in batch} <= {2, 16, 256}
    assert all(16 <= w.height <= 64 and 16 <= w.width <= 64 for w in batch)
    for w in batch:
        assert 0.1 * w.levels - 1e-9 <= w.sigma <= 0.3 * w.levels + 1e-9
    t, reqs = synth.serving_trace(30, side_lo=16, side_hi=48)
    assert np.all(np.diff(t) > 0) and len(reqs) == 30
    assert 0.2 < t[-1] / 30 * 50 < 5  # mean gap ~ 1/50 s


def test_psnr_closed_form():
    x = np.zeros((8, 8))
    x[2:5, 2:5] = 1.0
    y = x + 0.1
    assert abs(metrics.psnr(x, y) - 20 * math.log10(1.0 / 0.1)) < 1e-9
    assert metrics.psnr(x, x) == math.inf


def test_ssim_properties():
    rng = np.random.default_rng(0)
    x = rng.random((32, 32))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    assert abs(metrics.ssim_global(x, x) - 1.0) < 1e-12
    assert abs(metrics.ssim_windowed(x, x) - 1.0) < 1e-12
    assert abs(metrics.ssim_global(x, y) - metrics.ssim_global(y, x)) < 1e-12
    assert abs(metrics.ssim_windowed(x, y) - metrics.ssim_windowed(y, x)) < 1e-12
    assert metrics.ssim_windowed(x, y) < 0.99
    # global SSIM with zero constants is the product of the three correlation terms
    mx, my = x.mean(), y.mean()
    cxy = np.cov(x.ravel(), y.ravel())[0, 1]
    want = (2 * mx * my + 1e-4) * (2 * cxy + 9e-4) / ((mx ** 2 + my ** 2 + 1e-4) * (x.var(ddof=1) + y.var(ddof=1) + 9e-4))
    assert abs(metrics.ssim_global(x, y) - want) < 1e-12


def test_oracle_restores_c1(orc):
    """PCA and Gibbs posterior means both beat the raw observation on the binary image."""
    wl = synth.make_workload("c1", sweeps=60)
    p = orc.Params(**{**wl.params(), "burn_in": 20})
    truth = metrics.luminance_levels(wl.truth, 2)
    noisy = metrics.luminance_values(np.clip(wl.obs, -1, 1), -1, 1)
    base = metrics.psnr(truth, noisy)
    for gibbs in (False, True):
        run = orc.Run(p, wl.obs, gibbs=gibbs).sweep(wl.sweeps)
        mean = metrics.luminance_values(run.posterior_mean(), -1, 1)
        assert metrics.psnr(truth, mean) > base + 3.0
        mpm = run.marginal_map()
        assert metrics.psnr(truth, mpm.astype(np.float64)) > base + 3.0
