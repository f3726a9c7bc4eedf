"""Host-side logic of the benchmark (no GPU): the one-GPU-share option's validation and the
roofline note, which must name the instruction mix of the kernel that runs."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_share_option_rejects_splits_that_do_not_divide_the_workload():
    for bad, msg in (("rows:3", "must divide the workload's height"), ("chains:5", "must divide the workload's chains"),
                     ("cols:2", "takes rows:N or chains:N"), ("rows:x", "takes rows:N or chains:N")):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--share", bad], capture_output=True,
                           text=True, timeout=180, cwd=ROOT)
        assert r.returncode == 2, (bad, r.stderr[-300:])
        assert msg in r.stderr, (bad, r.stderr[-300:])
        assert r.stdout == ""


def test_roofline_note_names_the_kernel_mix():
    sys.path.insert(0, ROOT)
    import bench
    from workloads import synth
    c1, c2, c3 = (synth.make_workload(n, sweeps=4) for n in ("c1", "c2", "c3"))
    assert "byte table" in bench.peak_note(c2, 0, 1)           # few levels, one sweep per launch
    assert "byte SADs, 24-bit mads" in bench.peak_note(c3, 0, 1)  # 256 levels
    assert "byte SADs, 24-bit mads" in bench.peak_note(c1, 0, 12)  # several sweeps per launch, 2 levels
    assert "byte table" in bench.peak_note(c2, 0, 8)            # several sweeps per launch, 16 levels
    assert "byte SADs, 24-bit mads" in bench.peak_note(c2, 1, 1)   # L1 inertia
