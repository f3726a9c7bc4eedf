"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer reproduces its
frozen fixture (every golden run: binary Potts, L = 16 with a beta schedule, L = 33
8-neighbour random init, L = 256, L1 and L2 inertia, sequential Gibbs) and runs the
degenerate lattices (1 x 1, one row, one column, 8 neighbours) and the site and row entry
points with no sanitizer report: an out-of-bounds access or undefined operation anywhere in
those paths aborts the child process."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np
import oracle
from tests.golden import make_oracle_fixtures as fx
with open(fx.OUT) as f:
    stored = [l.rstrip("\n") for l in f if not l.startswith("#")]
assert fx.lines() == stored, "sanitized oracle differs from its fixture"
rng = np.random.default_rng(5)
for (H, W, L, C, nbr, inertia) in [(1, 1, 4, 1, 4, 0), (1, 37, 16, 5, 8, 0), (29, 1, 256, 2, 4, 1),
                                   (3, 4, 9, 3, 8, 2), (2, 2, 2, 6, 4, 0)]:
    p = oracle.Params(height=H, width=W, levels=L, chains=C, neighbourhood=nbr, prior=1 if L > 2 else 0,
                      trunc=min(4, L - 1), J=0.3, q=0.7, sigma=0.4 * L, vmin=0.0, vmax=float(L - 1), seed=9,
                      burn_in=1, tally_stride=1, inertia=inertia)
    obs = rng.uniform(-2.0, L + 1.0, size=(H, W)).astype(np.float32)
    for gibbs in (False, True):
        if gibbs and inertia:
            continue
        run = oracle.Run(p, obs, gibbs=gibbs).sweep(4)
        run.posterior_mean()
        run.marginal_map()
    x = run.state
    ch = rng.integers(0, C, size=50).astype(np.int32)
    px = rng.integers(0, H * W, size=50).astype(np.int64)
    oracle.update_sites(p, obs, x, 3, ch, px)
    oracle.pca_rows(p, obs, x, 3, C - 1, 0, H)
print("sanitized oracle: clean")
"""


def _asan_runtime():
    try:
        out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_is_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    import oracle
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = oracle.build_sanitized(str(tmp_path / "liborc_san.so"))
    env = dict(os.environ, ORC_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle: clean" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
