"""Writes oracle_convention.txt: the CPU reference's arithmetic convention frozen as text.

The paper prints no worked numerical example of the sampler (its tables are PSNR/SSIM on
images that are not available), so the values stored here are not the paper's: they are
the reference's own outputs on small seeded inputs, written by this script, which calls
only `oracle/`.  `tests/test_golden_oracle.py` recomputes them; a difference means the
reference's arithmetic changed, and the fixture may only be rewritten together with that
change and its justification.

Contents: exp2s at selected arguments (hex floats), Philox4x32-10 words at selected
counters and keys, uniform conversions, and for short runs of the lazy PCA (Sec. 5.2) and
of the sequential Gibbs sampler (Sec. 5.1) the SHA-256 of the final states, the level sum
and the marginal mode.

Run from the repository root:  python -m tests.golden.make_oracle_fixtures
"""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_convention.txt")

EXP2_ARGS = [0.0, 1.0, -1.0, 0.5, -0.5, 0.25, -124.75, -125.0, -125.5, 99.9, 3.3, -17.123, 1e-7]
PHILOX = [((0, 0, 0, 0), (0, 0)), ((1, 2, 3, 4), (5, 6)), ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF)),
          ((123456, 7, 2, 0), (2001, 0)), ((0, 999, 1, 1), (0xDEADBEEF, 0x12345678))]
UNIFORM = [0, 255, 256, 0x7FFFFFFF, 0xFFFFFFFF]

# name, params, sweeps, gibbs; observations come from the seeded generator below
RUNS = [
    ("binary potts 4-nbr", dict(height=9, width=11, levels=2, chains=3, neighbourhood=4, prior=0, trunc=1, J=0.8,
                                q=2.0, sigma=0.6, vmin=-1.0, vmax=1.0, seed=11, burn_in=2, tally_stride=1), 12, False),
    ("L16 truncated linear 8 chains", dict(height=12, width=10, levels=16, chains=8, neighbourhood=4, prior=1,
                                           trunc=4, J=0.4, q=1.5, sigma=2.0, vmin=0.0, vmax=15.0, seed=22,
                                           burn_in=3, tally_stride=2, beta=[1.0, 1.25, 1.5]), 10, False),
    ("L33 potts 8-nbr random init", dict(height=8, width=13, levels=33, chains=5, neighbourhood=8, prior=0,
                                         trunc=1, J=1 / 3, q=0.51, sigma=3.0, vmin=0.0, vmax=1.0, seed=33,
                                         init_mode=1, burn_in=1, tally_stride=1), 8, False),
    ("L256 truncated linear T32", dict(height=7, width=9, levels=256, chains=4, neighbourhood=4, prior=1, trunc=32,
                                       J=0.05, q=1.0, sigma=20.0, vmin=0.0, vmax=255.0, seed=44, burn_in=0,
                                       tally_stride=1), 5, False),
    ("L5 L1 inertia", dict(height=10, width=10, levels=5, chains=2, neighbourhood=4, prior=1, trunc=2, J=0.3,
                           q=0.6, sigma=0.8, vmin=0.0, vmax=4.0, seed=55, burn_in=1, tally_stride=1, inertia=1), 9,
     False),
    ("L9 L2 inertia 8-nbr", dict(height=6, width=14, levels=9, chains=3, neighbourhood=8, prior=1, trunc=3, J=0.3,
                                 q=0.2, sigma=1.2, vmin=0.0, vmax=8.0, seed=66, burn_in=2, tally_stride=1,
                                 inertia=2), 9, False),
    ("L9 sequential Gibbs", dict(height=9, width=9, levels=9, chains=2, neighbourhood=8, prior=0, trunc=1, J=1 / 3,
                                 q=0.0, sigma=0.2, vmin=0.0, vmax=1.0, seed=77, burn_in=1, tally_stride=1), 6, True),
]


def observation(name: str, p: dict) -> np.ndarray:
    """Seeded observation: uniform over the value range widened by a quarter each side."""
    seed = int.from_bytes(hashlib.sha256(name.encode()).digest()[:4], "little")
    rng = np.random.default_rng(seed)
    span = p["vmax"] - p["vmin"]
    return rng.uniform(p["vmin"] - 0.25 * span, p["vmax"] + 0.25 * span, size=(p["height"], p["width"])).astype(
        np.float32)


def lines() -> list[str]:
    out = []
    for y in EXP2_ARGS:
        out.append(f"exp2s {float(np.float32(y)).hex()} {float(np.float32(oracle.exp2s(float(np.float32(y))))).hex()}")
    for ctr, key in PHILOX:
        words = " ".join(f"{int(w):08x}" for w in oracle.philox4x32_10(ctr, key))
        out.append(f"philox {' '.join(f'{c:08x}' for c in ctr)} {key[0]:08x} {key[1]:08x} -> {words}")
    for r in UNIFORM:
        out.append(f"uniform {r:08x} {float(np.float32(oracle.uniform(r))).hex()}")
    for name, p, sweeps, gibbs in RUNS:
        obs = observation(name, p)
        run = oracle.Run(oracle.Params(**p), obs, gibbs=gibbs).sweep(sweeps)
        state = hashlib.sha256(run.state.tobytes()).hexdigest()
        total = int(run.sum.astype(np.uint64).sum())
        mpm = hashlib.sha256(run.marginal_map().tobytes()).hexdigest() if run.hist is not None else "-"
        out.append(f"run {name} | sweeps {sweeps} | state {state} | sum {total} | count {int(run.count[0])} | "
                   f"mode {mpm}")
    return out


def main():
    with open(OUT, "w") as f:
        f.write("# CPU reference convention fixtures, written by tests/golden/make_oracle_fixtures.py\n")
        f.write("# (exp2s and uniforms as hex floats; Philox words hex; runs as SHA-256 of the uint8 states)\n")
        for line in lines():
            f.write(line + "\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
