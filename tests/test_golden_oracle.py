"""The CPU reference's arithmetic convention against its frozen fixture
(tests/golden/oracle_convention.txt, written by tests/golden/make_oracle_fixtures.py from
the reference alone): exp2s, Philox words, uniforms and short seeded PCA and Gibbs runs
must reproduce it exactly.  The paper fixes no arithmetic, so this guards the convention
itself against unintended change; the laws it must obey are pinned by the other tests."""
import os

from tests.golden import make_oracle_fixtures as fx


def _stored():
    with open(fx.OUT) as f:
        return [line.rstrip("\n") for line in f if not line.startswith("#")]


def test_fixture_covers_every_case():
    stored = _stored()
    assert len(stored) == len(fx.EXP2_ARGS) + len(fx.PHILOX) + len(fx.UNIFORM) + len(fx.RUNS)
    assert os.path.basename(fx.OUT) == "oracle_convention.txt"


def test_reference_reproduces_its_frozen_convention():
    stored = _stored()
    now = fx.lines()
    diff = [(a, b) for a, b in zip(stored, now) if a != b]
    assert not diff, "\n".join(f"stored: {a}\n   now: {b}" for a, b in diff)
