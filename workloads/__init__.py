"""Seeded synthetic workloads and image-quality metrics.

Shared by the tests, the benchmark and the oracle's checks.  Holds none of the
sampler's arithmetic: it paints ground-truth images, adds Gaussian noise and scores
restorations.
"""
from .synth import WORKLOAD_RECIPES, Workload, make_workload, random_image, batch_mix, serving_trace  # noqa: F401
from .metrics import psnr, ssim_global, ssim_windowed  # noqa: F401
