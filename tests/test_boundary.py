"""The C-ABI library loads and exports every entry point declared in include/pca.h, and
rejects invalid arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pca.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(pca_\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2507_14869_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import paper_2507_14869_amd.build as b
        b.build()
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("pca_init", "pca_sweep", "pca_posterior_mean", "pca_marginal_map", "pca_get_state",
              "pca_set_state", "pca_sync", "pca_destroy", "pca_last_error", "pca_stats"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(os.path.join(ROOT, "paper_2507_14869_amd", "libpca.so"))
    for name in declared_functions():
        assert hasattr(raw, name), name


def test_binding_names_match_the_boundary():
    from paper_2507_14869_amd import _lib
    for name in declared_functions():
        assert callable(getattr(_lib, name)), name


def test_null_context_is_rejected(lib):
    from paper_2507_14869_amd import _lib
    for call in (lambda: _lib.pca_sweep(None, 1), lambda: _lib.pca_posterior_mean(None, 0),
                 lambda: _lib.pca_marginal_map(None, 0), lambda: _lib.pca_get_state(None, 0),
                 lambda: _lib.pca_set_state(None, 0, 0), lambda: _lib.pca_stats(None), lambda: _lib.pca_sync(None),
                 lambda: _lib.pca_sweeps_per_launch(None)):
        with pytest.raises(_lib.PcaError) as e:
            call()
        assert e.value.code == _lib.PCA_EINVAL
    _lib.pca_destroy(None)  # no-op


@pytest.mark.parametrize("bad", [dict(levels=1), dict(levels=257), dict(chains=0), dict(chains=1025),
                                 dict(neighbourhood=6), dict(prior=2), dict(trunc=0), dict(J=-0.1), dict(q=-1.0),
                                 dict(sigma=0.0), dict(vmax=0.0), dict(init_mode=2), dict(burn_in=-1),
                                 dict(tally_stride=-1), dict(beta=[1.0, -2.0]), dict(height=0),
                                 dict(J=float("nan")), dict(q=80.0), dict(width=70000, height=70000),
                                 dict(inertia=3), dict(inertia=-1)])
def test_invalid_parameters_are_rejected_without_a_device(lib, bad):
    from paper_2507_14869_amd import _lib
    kw = dict(height=4, width=4, levels=4, chains=1, J=0.1, q=0.5, sigma=1.0)
    kw.update(bad)
    p, _buf = _lib.make_params(**kw)
    with pytest.raises(_lib.PcaError) as e:
        _lib.pca_init(p, 0x1000)
    assert e.value.code == _lib.PCA_EINVAL
    assert _lib.pca_last_error() != ""


def test_null_observation_is_rejected(lib):
    from paper_2507_14869_amd import _lib
    p, _buf = _lib.make_params(height=4, width=4, levels=4)
    with pytest.raises(_lib.PcaError) as e:
        _lib.pca_init(p, 0)
    assert e.value.code == _lib.PCA_EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with status 2 and says why,
    before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_injected_allocation_failure_in_init(lib, monkeypatch):
    """The failure-handling hook: with PCA_FAULT_INJECT naming the "init" site, pca_init
    fails as if device memory were exhausted (PCA_ENOMEM, no context), before any device
    work; other sites and an unset variable change nothing."""
    from paper_2507_14869_amd import _lib
    p, _buf = _lib.make_params(height=4, width=4, levels=4, J=0.1, q=0.5, sigma=1.0)
    for spec in ("init", "admit:3,init", "readout,init"):
        monkeypatch.setenv("PCA_FAULT_INJECT", spec)
        with pytest.raises(_lib.PcaError) as e:
            _lib.pca_init(p, 0x1000)
        assert e.value.code == _lib.PCA_ENOMEM
        assert "allocation" in _lib.pca_last_error()
    monkeypatch.setenv("PCA_FAULT_INJECT", "initx")  # not the init site: validation still comes first
    bad, _b2 = _lib.make_params(height=4, width=4, levels=1)
    with pytest.raises(_lib.PcaError) as e:
        _lib.pca_init(bad, 0x1000)
    assert e.value.code == _lib.PCA_EINVAL


@pytest.mark.parametrize("case", ["bad_params", "null_obs", "negative_sweeps", "no_output", "mode_without_histogram",
                                  "mean_without_accumulation", "too_large"])
def test_run_static_rejects_bad_calls_without_a_device(lib, case):
    """pca_run_static checks its arguments and the size of its working memory on the host,
    before it looks up the device array: every refusal here happens without a GPU."""
    from paper_2507_14869_amd import _lib
    kw = dict(height=8, width=8, levels=16, chains=4, J=0.1, q=0.5, sigma=1.0, tally_stride=1)
    obs, sweeps, mean, mpm, want = 0x1000, 3, 0x2000, 0x3000, _lib.PCA_EINVAL
    if case == "bad_params":
        kw["levels"] = 1
    elif case == "null_obs":
        obs = 0
    elif case == "negative_sweeps":
        sweeps = -1
    elif case == "no_output":
        mean = mpm = 0
    elif case == "mode_without_histogram":
        kw["tally_stride"] = 0
        want = _lib.PCA_ESTATE
    elif case == "mean_without_accumulation":
        kw["burn_in"] = 5
        want = _lib.PCA_ESTATE
    elif case == "too_large":
        # 2048 x 2048, 16 chains, 256 levels with a histogram: about 2.3 GB of working memory
        kw.update(height=2048, width=2048, chains=16, levels=256)
    p, _buf = _lib.make_params(**kw)
    with pytest.raises(_lib.PcaError) as e:
        _lib.pca_run_static(p, obs, sweeps, mean, mpm)
    assert e.value.code == want
    if case == "too_large":
        assert "working memory" in _lib.pca_last_error()
