"""Synthetic denoising workloads standing in for the paper's private MRF test images.

The paper restores piecewise-regular grey images corrupted by additive Gaussian noise
(Sec. 6).  Its images are not available, so every workload here is painted from a seed:
axis-aligned rectangles and ellipses over a background (flat or a linear gradient),
quantised to L equally spaced levels (round half to even, clamped), plus N(0, sigma^2)
FP32 noise in value units.  Levels map to values as vmin + k (vmax - vmin)/(L-1).

Named workloads (sizes, level counts, noise, priors, chains and sweeps):
  c1  64x64 binary (values -1/+1), 3 rectangles and 2 ellipses, sigma 0.6, Potts 4-nbr
      J 0.8, q 2.0, 1 chain, 200 sweeps.
  c2  512x512, L 16, gradient + 20 shapes, sigma 2 levels, truncated linear T 4, J 0.4,
      q 1.5, 8 chains, 1000 sweeps.
  c3  2048x2048, L 256, gradient + 200 shapes, sigma 20 levels, truncated linear T 32,
      J 0.05, q 1.0, 16 chains, 1000 sweeps, posterior mean and marginal MAP.
  c4  batch of 64 images with log-uniform sides in [128, 1024] and mixed L (batch_mix).
  c5  Poisson request trace at 50 req/s with sides in [64, 4096] (serving_trace).
Data seed 1000 + index, sampler seed 2000 + index; burn-in is a quarter of the sweeps.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import List, Optional

import numpy as np

POTTS, TRUNC_LINEAR = 0, 1


@dataclass
class Workload:
    name: str
    height: int
    width: int
    levels: int
    chains: int
    sweeps: int
    prior: int
    trunc: int
    J: float
    q: float
    sigma: float          # value units
    vmin: float
    vmax: float
    neighbourhood: int = 4
    beta: List[float] = field(default_factory=list)
    seed: int = 0         # sampler (Philox) seed
    data_seed: int = 0
    burn_in: int = 0
    tally_stride: int = 0
    shapes: int = 0
    gradient: bool = False
    truth: Optional[np.ndarray] = None   # uint8 levels [H, W]
    obs: Optional[np.ndarray] = None     # float32 values [H, W]

    def params(self, **over) -> dict:
        d = {k: v for k, v in asdict(self).items() if k in PARAM_KEYS}
        d.update(over)
        return d

    @property
    def site_updates(self) -> int:
        return self.height * self.width * self.chains * self.sweeps


PARAM_KEYS = ("height", "width", "levels", "chains", "neighbourhood", "prior", "trunc", "J", "q", "sigma",
              "vmin", "vmax", "beta", "seed", "burn_in", "tally_stride")

WORKLOAD_RECIPES = {
    "c1": dict(height=64, width=64, levels=2, chains=1, sweeps=200, prior=POTTS, trunc=1, J=0.8, q=2.0,
               sigma=0.6, vmin=-1.0, vmax=1.0, shapes=5, gradient=False, burn_in=50, tally_stride=1),
    "c2": dict(height=512, width=512, levels=16, chains=8, sweeps=1000, prior=TRUNC_LINEAR, trunc=4, J=0.4,
               q=1.5, sigma=2.0, vmin=0.0, vmax=15.0, shapes=20, gradient=True, burn_in=250, tally_stride=1),
    "c3": dict(height=2048, width=2048, levels=256, chains=16, sweeps=1000, prior=TRUNC_LINEAR, trunc=32,
               J=0.05, q=1.0, sigma=20.0, vmin=0.0, vmax=255.0, shapes=200, gradient=True, burn_in=250,
               tally_stride=1),
}
CONFIG_INDEX = {"c1": 0, "c2": 1, "c3": 2, "c4": 3, "c5": 4}


def _paint(levels: np.ndarray, rng: np.random.Generator, n_shapes: int, L: int, binary: bool) -> None:
    H, W = levels.shape
    for s in range(n_shapes):
        if binary:
            kind = "rect" if s < 3 else "ellipse"
            value = L - 1
            if kind == "rect":
                h, w = rng.integers(8, 33, size=2) if min(H, W) >= 64 else rng.integers(1, max(2, min(H, W) // 2), 2)
            else:
                ah, aw = rng.integers(4, 17, size=2) if min(H, W) >= 64 else rng.integers(1, max(2, min(H, W) // 4), 2)
        else:
            kind = "rect" if rng.random() < 0.5 else "ellipse"
            value = int(rng.integers(0, L))
            h = int(rng.integers(max(1, H // 32), max(2, H // 4) + 1))
            w = int(rng.integers(max(1, W // 32), max(2, W // 4) + 1))
            ah, aw = max(1, h // 2), max(1, w // 2)
        if kind == "rect":
            r0 = int(rng.integers(0, max(1, H - h + 1)))
            c0 = int(rng.integers(0, max(1, W - w + 1)))
            levels[r0:r0 + h, c0:c0 + w] = value
        else:
            rc = int(rng.integers(0, H))
            cc = int(rng.integers(0, W))
            r0, r1 = max(0, rc - ah), min(H, rc + ah + 1)
            c0, c1 = max(0, cc - aw), min(W, cc + aw + 1)
            rr = (np.arange(r0, r1)[:, None] - rc) / float(ah)
            cr = (np.arange(c0, c1)[None, :] - cc) / float(aw)
            mask = rr * rr + cr * cr <= 1.0
            levels[r0:r1, c0:c1][mask] = value


def random_image(height: int, width: int, levels: int, shapes: int, gradient: bool, rng: np.random.Generator,
                 binary: Optional[bool] = None) -> np.ndarray:
    """Ground truth as uint8 level indices [H, W]."""
    if binary is None:
        binary = levels == 2
    if gradient:
        theta = rng.uniform(0, 2 * math.pi)
        rr, cc = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
        proj = rr * math.sin(theta) + cc * math.cos(theta)
        span = proj.max() - proj.min()
        base = (proj - proj.min()) / (span if span > 0 else 1.0) * (levels - 1)
        lv = np.clip(np.rint(base), 0, levels - 1).astype(np.int32)
    else:
        lv = np.zeros((height, width), dtype=np.int32)
    _paint(lv, rng, shapes, levels, binary)
    return np.clip(lv, 0, levels - 1).astype(np.uint8)


def noisy_observation(truth: np.ndarray, levels: int, vmin: float, vmax: float, sigma: float,
                      rng: np.random.Generator) -> np.ndarray:
    delta = (vmax - vmin) / (levels - 1)
    values = vmin + truth.astype(np.float64) * delta
    return (values + rng.normal(0.0, sigma, size=truth.shape)).astype(np.float32)


def make_workload(name: str, *, height: Optional[int] = None, width: Optional[int] = None,
                  chains: Optional[int] = None, sweeps: Optional[int] = None) -> Workload:
    """Named workload c1/c2/c3 with its truth and observation (optionally resized)."""
    cfg = dict(WORKLOAD_RECIPES[name])
    idx = CONFIG_INDEX[name]
    if height is not None:
        cfg["height"] = height
    if width is not None:
        cfg["width"] = width
    if chains is not None:
        cfg["chains"] = chains
    if sweeps is not None:
        cfg["sweeps"] = sweeps
        cfg["burn_in"] = sweeps // 4
    wl = Workload(name=name, seed=2000 + idx, data_seed=1000 + idx, **cfg)
    rng = np.random.default_rng(wl.data_seed)
    wl.truth = random_image(wl.height, wl.width, wl.levels, wl.shapes, wl.gradient, rng)
    wl.obs = noisy_observation(wl.truth, wl.levels, wl.vmin, wl.vmax, wl.sigma, rng)
    return wl


# Per-level-count prior families for the mixed batch and the serving trace.
_FAMILY = {2: (POTTS, 1, 0.8), 16: (TRUNC_LINEAR, 4, 0.4), 256: (TRUNC_LINEAR, 32, 0.05)}


def _mixed_request(rng: np.random.Generator, side_lo: int, side_hi: int, chains: int, sweeps: int,
                   idx: int, name: str, levels=(2, 16, 256)) -> Workload:
    H = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
    W = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
    L = int(rng.choice(list(levels)))
    prior, T, J0 = _FAMILY[L]
    sigma = float(rng.uniform(0.1, 0.3) * L)
    J = float(J0 * rng.uniform(0.5, 1.5))
    q = float(rng.uniform(1.0, 2.0))
    wl = Workload(name=f"{name}[{idx}]", height=H, width=W, levels=L, chains=chains, sweeps=sweeps, prior=prior,
                  trunc=T, J=J, q=q, sigma=sigma, vmin=0.0, vmax=float(L - 1), seed=int(rng.integers(0, 2**63)),
                  shapes=max(3, (H * W) // 20000), gradient=L > 2)
    wl.truth = random_image(H, W, L, wl.shapes, wl.gradient, rng)
    wl.obs = noisy_observation(wl.truth, L, wl.vmin, wl.vmax, sigma, rng)
    return wl


def batch_mix(n_images: int = 64, *, side_lo: int = 128, side_hi: int = 1024, chains: int = 4, sweeps: int = 500,
              seed: int = 1003, levels=(2, 16, 256)) -> List[Workload]:
    """Mixed-size batch: sides log-uniform, L drawn from `levels` (default {2, 16, 256}),
    sigma ~ U[0.1, 0.3] L."""
    rng = np.random.default_rng(seed)
    return [_mixed_request(rng, side_lo, side_hi, chains, sweeps, i, "c4", levels) for i in range(n_images)]


def serving_trace(n_requests: int, *, rate: float = 50.0, side_lo: int = 64, side_hi: int = 4096, chains: int = 2,
                  sweeps: int = 300, seed: int = 1004):
    """Poisson arrivals (seconds from 0) with mixed-size requests."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    reqs = [_mixed_request(rng, side_lo, side_hi, chains, sweeps, i, "c5") for i in range(n_requests)]
    return t, reqs
