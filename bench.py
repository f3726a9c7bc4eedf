#!/usr/bin/env python3
"""Throughput of the lazy-PCA denoising job on one MI355X.

A step is one whole job on a synthetic 2048x2048 image with L = 256 grey levels, 16
independent chains and 1000 sweeps (truncated-linear prior T = 32, J = 0.05, q = 1.0,
sigma = 20 levels): initialisation from the observation, every sweep with its running
mean and histogram, and the posterior-mean and marginal-mode readouts.  The observation
is resident in HBM before the timed region.  Prints one JSON line.

Roofline: the sweep kernel is bound by vector ALU work; `roofline` reports its
algorithmic VALU lane-operations per launch divided by its average launch time (HIP
events on the launch stream) against the MI355X VALU issue rate; `traffic` is the HBM
bytes per launch from the committed rocprofv3 counter summary when it was taken on the
current kernel source for this job.  `cpu_baseline` is the CPU reference timed on a
bounded sample of the same workload on this host.

Other workloads: --workload c1/c2 (smaller single images), c4 (a batch of 64 mixed
lattices in one launch per sweep, against one launch per lattice), c5 (a Poisson stream
of 250 mixed requests through the continuous-batching server, against one request at a
time; latency percentiles); --inertia, --q and --neighbourhood vary the model on c1-c3.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# 32-bit VALU issue rate: the FP32 vector peak of 157.3 TFLOP/s counts an FMA as two flops,
# i.e. 256 CUs x 128 lanes x 2.4 GHz = 78.6 T lane-operations/s.
PEAK_VALU_TOPS = 256 * 128 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2507_14869_amd", "csrc", f) for f in ("pca_sweep.h", "pca_kernels.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_c3_traffic.txt")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "sweep_kernel_c3_counters.txt")


def valu_ops_per_site_update(levels: int, chains: int, inertia: int = 0, nbr: int = 4) -> float:
    """Algorithmic VALU lane-ops per site update.  Indicator inertia: per (chain, level)
    three byte-SADs per four neighbours, the two-op table index and one fma; per (pixel,
    level) the 15-op data factor shared by the chains of the pixel.  L1/L2 inertia: per
    (chain, level) those plus |k - x|^p and its conversion (3), the exponent (2 fma/mul, 1
    subtraction) and exp2s (9); per (pixel, level) e and e*e (2)."""
    sads = 3.0 * nbr / 4.0
    if inertia:
        return levels * (sads + 18.0 + 2.0 / chains)
    return levels * (sads + 3.0 + 15.0 / chains)


def peak_note(wl, inertia: int, sweeps_per_launch: int) -> str:
    """What the VALU peak is and how the kernel's instruction mix relates to the ops model
    (the several-sweeps kernel keeps the byte SADs for at most 4 levels)."""
    base = ("32-bit VALU issue rate, 256 CUs x 128 lanes x 2.4 GHz (the FP32 vector peak counts an fma as "
            "two flops); ")
    if wl.levels <= 16 and inertia == 0 and (sweeps_per_launch == 1 or wl.levels > 4):
        return base + ("with at most 16 levels the kernel takes each (chain, level)'s neighbour statistic "
                       "from an LDS byte table (one byte extract and one fma per (chain, level) instead of "
                       "three byte SADs per four neighbours, a shift-add and a 24-bit mad), so the dense-"
                       "equivalent count is that of the SAD formulation")
    return base + ("the kernel's integer VOP3 instructions (byte SADs, 24-bit mads, shift-adds) are 5 of its 7 "
                   "per (chain, level)")


def model_bytes_per_site_update(chains: int) -> float:
    """HBM bytes the method must move per site update on an accumulating sweep: state read
    and write (2 per chain), observation read (4 per pixel) and the uint32 sum
    read-modify-write (8 per pixel), i.e. 2 + 12/C."""
    return 2.0 + 12.0 / chains


def hbm_bytes_per_sweep(N: int, chains: int, acc: bool, tally: bool) -> float:
    """State read and write and observation read; on accumulating sweeps the uint32 sum
    read-modify-write; on tally sweeps one uint16 counter read-modify-write per chain."""
    b = 2.0 * chains * N + 4.0 * N
    if acc:
        b += 8.0 * N
    if tally:
        b += 4.0 * chains * N
    return b


def hbm_bytes_per_launch(wl) -> float:
    """Algorithmic bytes per sweep launch averaged over the job's sweeps (burn-in sweeps
    accumulate nothing)."""
    N = wl.height * wl.width
    total = 0.0
    for t in range(wl.sweeps):
        acc = t >= wl.burn_in
        tally = acc and wl.tally_stride > 0 and (t - wl.burn_in) % wl.tally_stride == 0
        total += hbm_bytes_per_sweep(N, wl.chains, acc, tally)
    return total / wl.sweeps


def kernel_hash() -> str:
    """Hash of the sources the single-lattice sweep kernel is built from."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(per_launch_units: float):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source; otherwise None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sha256_16") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_valu_per_site_update():
    """VALU instructions per site update of the sweep kernel from the committed rocprofv3
    counter summary (SQ_INSTS_VALU per wave / site updates per wave) when it was taken on
    the current kernel source; otherwise None."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    txt = open(COUNTERS_FILE).read()
    if f"sha256[:16] = {kernel_hash()}" not in txt:
        return None
    for line in txt.splitlines():
        if line.startswith("# VALU instructions per wave") and "per site update:" in line:
            try:
                return float(line.rsplit(":", 1)[1])
            except ValueError:
                return None
    return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, seconds: float, inertia: int = 0, threads: int = 1):
    """The oracle timed on this host's cores on a bounded sample of the same job.  When a
    whole sweep fits in a third of `seconds`, whole sweeps of the job from its initial
    state (the oracle's own run, with its accumulators); otherwise row bands of every chain
    of sweep 0.  With threads > 1 the row bands are spread over a pool of host threads (the
    oracle's C code runs outside the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    p = oracle.Params(**wl.params(inertia=inertia))
    x0 = oracle.init_state(p, wl.obs)
    band = 8
    t0 = time.perf_counter()
    oracle.pca_rows(p, wl.obs, x0, 0, 0, 0, min(band, wl.height))
    per_sweep = (time.perf_counter() - t0) * wl.height / min(band, wl.height) * wl.chains / threads
    how = "single-threaded" if threads == 1 else f"in {threads} threads"
    if per_sweep <= seconds / 3:
        run = oracle.Run(p, wl.obs)
        k = 0
        t0 = time.perf_counter()
        while k < wl.sweeps and time.perf_counter() - t0 < seconds:
            if threads == 1:
                run.sweep(1)
            else:
                run.state = oracle.pca_sweep_threaded(p, wl.obs, run.state, run.t, threads=threads)
                run.t += 1
            k += 1
        dt = time.perf_counter() - t0
        done = k * wl.height * wl.width * wl.chains
        sample = f"{k} whole sweeps of the {wl.height}x{wl.width} L={wl.levels} job from its initial state"
    else:
        jobs = [(ch, r0) for r0 in range(0, wl.height, band) for ch in range(wl.chains)]
        done_rows = []
        t0 = time.perf_counter()

        def one(job):
            if time.perf_counter() - t0 >= seconds:
                return 0
            ch, r0 = job
            r1 = min(r0 + band, wl.height)
            oracle.pca_rows(p, wl.obs, x0, 0, ch, r0, r1)
            return r1 - r0

        with ThreadPoolExecutor(max_workers=threads) as pool:
            done_rows = list(pool.map(one, jobs))
        dt = time.perf_counter() - t0
        done = sum(done_rows) * wl.width
        sample = (f"{sum(done_rows)} rows ({band}-row bands, every chain) of sweep 0 of the {wl.height}x{wl.width} "
                  f"L={wl.levels} job")
    return {"value": done / dt, "unit": "site-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample}: {done} site updates in {dt:.1f} s {how}",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def quality(wl, mean, mpm):
    """PSNR and SSIM (windowed and the paper's single-window form) of the posterior mean and
    of the marginal mode against the ground truth, and of the noisy observation, all on
    luminance in [0, 1] (Sec. 6)."""
    import numpy as np
    from workloads import metrics
    truth = metrics.luminance_levels(wl.truth, wl.levels)
    noisy = metrics.luminance_values(np.clip(wl.obs, wl.vmin, wl.vmax), wl.vmin, wl.vmax)
    out = {}
    for name, img in (("observation", noisy), ("posterior_mean", metrics.luminance_values(mean, wl.vmin, wl.vmax)),
                      ("marginal_mode", None if mpm is None else metrics.luminance_levels(mpm, wl.levels))):
        if img is None:
            continue
        out[name] = {"psnr_db": metrics.psnr(truth, img), "ssim": metrics.ssim_windowed(truth, img),
                     "ssim_global": metrics.ssim_global(truth, img)}
    return out


def gibbs_comparison(wl):
    """The sequential single-site Gibbs sampler of Sec. 5.1 on the CPU (the oracle's), run
    for the same sweeps on the same data with the same seed: the paper's comparison
    (Table 1).  Returns its time and the quality of its posterior mean and mode."""
    import oracle
    p = oracle.Params(**wl.params())
    t0 = time.perf_counter()
    run = oracle.Run(p, wl.obs, gibbs=True).sweep(wl.sweeps)
    dt = time.perf_counter() - t0
    q = quality(wl, run.posterior_mean(), run.marginal_map() if wl.tally_stride > 0 else None)
    q.pop("observation", None)
    return {"sweeps": wl.sweeps, "seconds": dt, "cores": 1,
            "site_updates_per_s": wl.height * wl.width * wl.chains * wl.sweeps / dt, **q}


def gibbs_rate(wl, seconds: float):
    """The oracle's sequential Gibbs sampler (Sec. 5.1, one thread, raster order) timed on
    the same per-site work: whole sweeps of the workload's lattice, or of its top-left
    128x128 crop when the lattice is larger, until `seconds` have passed (at least one
    sweep)."""
    import numpy as np
    import oracle
    H, W = wl.height, wl.width
    if H * W > 128 * 128:
        H, W = min(H, 128), min(W, 128)
    p = oracle.Params(**{**wl.params(), "height": H, "width": W})
    run = oracle.Run(p, np.ascontiguousarray(wl.obs[:H, :W]), gibbs=True)
    k = 0
    t0 = time.perf_counter()
    while k == 0 or time.perf_counter() - t0 < seconds:
        run.sweep(1)
        k += 1
    dt = time.perf_counter() - t0
    su = k * H * W * wl.chains
    where = "the whole lattice" if (H, W) == (wl.height, wl.width) else f"its top-left {H}x{W} crop"
    return {"value": su / dt, "unit": "site-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} sequential Gibbs sweeps of {where} ({wl.chains} chains, L={wl.levels}): "
                      f"{su} site updates in {dt:.1f} s single-threaded"}


def workload_label(wl, inertia: int) -> str:
    if wl.prior == 0:
        prior = f"Potts prior J={wl.J} (2J per disagreeing neighbour)"
    else:
        prior = f"truncated-linear prior T={wl.trunc} J={wl.J}"
    scale = (wl.levels - 1) / (wl.vmax - wl.vmin)
    sig = f"sigma={wl.sigma:g} levels" if scale == 1.0 else f"sigma={wl.sigma:g} in value units ({wl.sigma * scale:g} levels)"
    return (f"{wl.name}: {wl.height}x{wl.width} image, L={wl.levels}, {wl.chains} chains, {wl.sweeps} sweeps, "
            f"{prior}, q={wl.q}, {sig}, {wl.neighbourhood}-neighbour, mean + marginal mode"
            + ("" if inertia == 0 else f", L{inertia} inertia"))


def copy_probe(mib: int, reps: int = 4):
    """A plain copy of known size: its HBM byte counters calibrate those of the sweep."""
    import torch
    n = mib * (1 << 20)
    a = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "reps": reps}), flush=True)


def bench_batch(args):
    """Mixed batch of 64 lattices (sides log-uniform in [128, 1024], L in {2, 16, 256},
    4 chains, 500 sweeps): one launch per sweep for the whole batch (graph-replayed,
    autotuned launch configuration) against one launch per lattice per sweep."""
    import torch
    from paper_2507_14869_amd import Batch, Sampler
    from workloads import synth

    sweeps = args.sweeps or 500
    wls = synth.batch_mix(64, sweeps=sweeps)
    stream = torch.cuda.current_stream()
    problems = []
    for w in wls:
        kw = w.params(burn_in=sweeps // 4, tally_stride=1)
        kw.pop("height")
        kw.pop("width")
        problems.append((torch.from_numpy(w.obs).cuda(), kw))
    su = sum(w.height * w.width * w.chains for w in wls) * sweeps

    def batched(cfg=None):
        b = Batch(problems)
        if cfg is not None:
            b.set_config(*cfg)
        b.sweep(sweeps)
        outs = [b.posterior_mean(i) for i in range(len(problems))]
        return b, outs

    def per_lattice():
        objs = []
        for obs, kw in problems:
            s = Sampler(obs, **kw).sweep(sweeps)
            objs.append((s, s.posterior_mean()))
        return objs

    tuner = Batch(problems)
    tune_ms = tuner.autotune(3)
    cfg = tuner.config
    tuner.close()
    for _ in range(args.warmup):
        b, _ = batched(cfg)
        b.sync()
        b.close()
        for s, _ in per_lattice():
            s.sync()
            s.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    keep = [batched(cfg) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    for b, _ in keep:
        b.close()
    t0 = time.perf_counter()
    keep = [per_lattice() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_single = (time.perf_counter() - t0) / args.steps
    for objs in keep:
        for s, _ in objs:
            s.close()
    out = {
        "metric": "site-updates/s",
        "value": su / t_batch,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_batch * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"c4: batch of {len(wls)} lattices, sides log-uniform in [128, 1024], L in {{2, 16, 256}}, "
                        f"4 chains, {sweeps} sweeps, one launch per sweep for the batch (graph-replayed)",
            "lattices": len(wls), "sweeps": sweeps, "site_updates_per_step": su,
            "levels_mix": {str(L): sum(1 for w in wls if w.levels == L) for L in (2, 16, 256)},
            "autotuned": {"chains_per_thread": cfg[0], "share": cfg[1], "tiled": cfg[2], "ms_per_sweep": tune_ms},
        },
        "one_launch_per_lattice": {"value": su / t_single, "ms_per_step": t_single * 1e3},
        "speedup_vs_one_launch_per_lattice": t_single / t_batch,
    }
    out["small_lattices"] = bench_small_batch(sweeps)
    print(json.dumps(out), flush=True)


def bench_small_batch(sweeps: int):
    """A batch of 64 small lattices (sides log-uniform in [32, 128], L in {2, 16}, 4 chains),
    whose sweeps are too short to fill the GPU: one launch per sweep (traversal 0) against
    7 sweeps per launch from LDS tiles (traversal 2), and the autotuner's choice."""
    import torch
    from paper_2507_14869_amd import Batch
    from workloads import synth
    wls = synth.batch_mix(64, side_lo=32, side_hi=128, sweeps=sweeps, seed=1013, levels=(2, 16))
    problems = []
    for w in wls:
        kw = w.params(burn_in=sweeps // 4, tally_stride=1)
        kw.pop("height")
        kw.pop("width")
        problems.append((torch.from_numpy(w.obs).cuda(), kw))
    su = sum(w.height * w.width * w.chains for w in wls) * sweeps

    def job(cfg):
        b = Batch(problems)
        b.set_config(*cfg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.sweep(sweeps)
        for i in range(len(problems)):
            b.posterior_mean(i)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b.close()
        return dt

    tuner = Batch(problems)
    tuner.autotune(3)
    tuned = tuner.config
    tuner.close()
    res = {}
    for name, cfg in (("one_sweep_per_launch", (4, 1, 0)), ("seven_sweeps_per_launch", (4, 1, 2)),
                      ("autotuned", tuned)):
        job(cfg)  # warm-up: graph capture
        dt = min(job(cfg) for _ in range(3))
        res[name] = {"config": list(cfg), "ms_per_job": dt * 1e3, "site_updates_per_s": su / dt}
    res["workload"] = (f"64 lattices, sides log-uniform in [32, 128], L in {{2, 16}}, 4 chains, {sweeps} sweeps, "
                       f"{su} site updates per job")
    return res


def bench_serve(args):
    """Poisson arrivals at 50 requests/s (sides log-uniform in [64, 4096], L in {2, 16, 256},
    sigma ~ U[0.1, 0.3] L, 2 chains, 300 sweeps) through the continuous-batching server, and
    through a one-request-at-a-time baseline on the same trace.  Latency is measured from
    each request's scheduled arrival to the end of the step that finished it.  The offered
    load rho is the arrival rate times the mean time a request takes on the GPU alone
    (measured in the one-at-a-time run).  The same requests are then served saturated (all
    arriving at once), both ways.  With --shed-backlog-s the server refuses submissions while
    its predicted wait exceeds the limit; latency, throughput and quality are then over the
    requests it served."""
    import numpy as np
    import torch
    from paper_2507_14869_amd import PCA_EBUSY, PcaError, Sampler, Server
    from workloads import metrics, synth

    sweeps = args.sweeps or 300
    arrivals, reqs = synth.serving_trace(args.requests, sweeps=sweeps)
    kws = []
    for w in reqs:
        kw = w.params(burn_in=sweeps // 4, tally_stride=1)
        kw.pop("height")
        kw.pop("width")
        kws.append(kw)
    su_of = [w.height * w.width * w.chains * sweeps for w in reqs]
    su_total = sum(su_of)

    def run_server(arrive, shed_s):
        sv = Server(160 << 30, max_active=512, sweeps_per_step=sweeps, step_ms=args.step_ms)
        sv.set_shedding(shed_s)
        done_at, rid_of = {}, {}
        i = 0
        t0 = time.perf_counter()
        busy = 0.0
        while len(done_at) < len(rid_of) or i < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and arrive[i] <= now:
                try:
                    rid_of[sv.submit(reqs[i].obs, sweeps, **kws[i])] = i
                except PcaError as err:  # refused by the shedding limit
                    if err.code != PCA_EBUSY:
                        raise
                i += 1
            q, a, _, _, _ = sv.stats()
            if q == 0 and a == 0:
                if i < len(reqs):
                    time.sleep(max(0.0, min(arrive[i] - now, 0.05)))
                continue
            ts = time.perf_counter()
            sv.step()
            busy += time.perf_counter() - ts
            t = time.perf_counter() - t0
            for rid in sv.completed():
                done_at[rid_of[rid]] = t
        makespan = time.perf_counter() - t0
        results = {}
        for rid, k in rid_of.items():
            results[k] = sv.result(rid)[0]
        steps = sv.stats()[3]
        sv.close()
        served = sorted(results)
        lat = np.array([done_at[k] - arrive[k] for k in served])
        return {"lat": lat, "makespan": makespan, "busy": busy, "steps": steps, "results": results, "served": served}

    def run_sequential(arrive):
        done_at, service, means = {}, {}, {}
        t0 = time.perf_counter()
        for k, w in enumerate(reqs):
            now = time.perf_counter() - t0
            if arrive[k] > now:
                time.sleep(arrive[k] - now)
            ts = time.perf_counter()
            s = Sampler(torch.from_numpy(w.obs).cuda(), **kws[k]).sweep(sweeps)
            means[k] = s.posterior_mean().cpu().numpy()
            s.close()
            te = time.perf_counter()
            service[k] = te - ts
            done_at[k] = te - t0
        makespan = time.perf_counter() - t0
        lat = np.array([done_at[k] - arrive[k] for k in range(len(reqs))])
        return {"lat": lat, "makespan": makespan, "service": service, "results": means}

    def pct(lat):
        return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                "mean": float(lat.mean()), "max": float(lat.max())}

    def psnr_of(k, img):
        w = reqs[k]
        return metrics.psnr(metrics.luminance_levels(w.truth, w.levels), metrics.luminance_values(img, w.vmin, w.vmax))

    # warm up the library and the kernels
    warm = Server(1 << 33, 8, 30)
    warm.submit(reqs[0].obs[:64, :64].copy(), 30, **{**kws[0], "burn_in": 5})
    while warm.stats()[1] or warm.stats()[0]:
        warm.step()
    warm.close()
    torch.cuda.synchronize()

    srv = run_server(arrivals, args.shed_backlog_s)
    served = srv["served"]
    su_served = sum(su_of[k] for k in served)
    seq = run_sequential(arrivals)
    mean_service = float(np.mean(list(seq["service"].values())))
    rate = len(reqs) / float(arrivals[-1])
    psnr_gain, psnr_delta = [], []
    for k in served:
        w = reqs[k]
        noisy = metrics.luminance_values(np.clip(w.obs, w.vmin, w.vmax), w.vmin, w.vmax)
        truth = metrics.luminance_levels(w.truth, w.levels)
        p_served = psnr_of(k, srv["results"][k])
        psnr_gain.append(p_served - metrics.psnr(truth, noisy))
        psnr_delta.append(abs(p_served - psnr_of(k, seq["results"][k])))
    out = {
        "metric": "site-updates/s",
        "value": su_served / srv["makespan"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": srv["makespan"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"c5: {len(reqs)} requests, Poisson arrivals at 50/s, sides log-uniform in [64, 4096], "
                        f"L in {{2, 16, 256}}, 2 chains, {sweeps} sweeps, continuous batching, {args.step_ms} ms steps",
            "requests": len(reqs), "site_updates": su_total,
        },
        "offered_load": {"rho": rate * mean_service, "arrival_rate_per_s": rate,
                         "mean_service_s": mean_service,
                         "service": "time of one request alone on the GPU (one-at-a-time run, upload to mean "
                                    "download)"},
        "shedding": {"max_backlog_s": args.shed_backlog_s, "served": len(served), "shed": len(reqs) - len(served),
                     "shed_fraction": 1.0 - len(served) / len(reqs)},
        "latency_s": pct(srv["lat"]),
        "requests_per_s": len(served) / srv["makespan"],
        "gpu_busy_fraction": srv["busy"] / srv["makespan"],
        "server_steps": srv["steps"],
        "mean_psnr_gain_db": float(np.mean(psnr_gain)),
        "max_psnr_delta_vs_alone_db": float(np.max(psnr_delta)),
        "one_request_at_a_time": {"value": su_total / seq["makespan"], "latency_s": pct(seq["lat"])},
    }
    if args.shed_backlog_s == 0.0:
        # saturated: every request waiting at time 0
        zero = np.zeros(len(reqs))
        srv0 = run_server(zero, 0.0)
        seq0 = run_sequential(zero)
        out["saturated"] = {
            "served": {"value": su_total / srv0["makespan"], "makespan_s": srv0["makespan"],
                       "latency_s": pct(srv0["lat"]), "server_steps": srv0["steps"]},
            "one_request_at_a_time": {"value": su_total / seq0["makespan"], "makespan_s": seq0["makespan"],
                                      "latency_s": pct(seq0["lat"])},
        }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--requests", type=int, default=250, help="c5: number of requests in the trace")
    ap.add_argument("--step-ms", type=float, default=50.0, help="c5: GPU time per server step")
    ap.add_argument("--shed-backlog-s", type=float, default=0.0,
                    help="c5: refuse submissions while the predicted wait exceeds this (0: never)")
    ap.add_argument("--sweeps", type=int, default=None, help="override the workload's sweep count")
    ap.add_argument("--inertia", type=int, default=0, choices=[0, 1, 2],
                    help="c1-c3: inertia norm exponent (0 indicator, 1 L1, 2 L2)")
    ap.add_argument("--q", type=float, default=None, help="c1-c3: override the inertia weight q")
    ap.add_argument("--neighbourhood", type=int, default=None, choices=[4, 8],
                    help="c1-c3: override the neighbourhood (the paper's experiments use 8)")
    ap.add_argument("--share", default=None, metavar="rows:N|chains:N",
                    help="c1-c3: run one GPU's share of an N-GPU split of the workload (a strip of H/N rows, "
                         "or C/N of the chains) on this GPU; the exchange between GPUs is not part of it")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the sampler has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2507_14869_amd import Sampler
    from workloads import synth

    if args.workload == "c4":
        bench_batch(args)
        return
    if args.workload == "c5":
        bench_serve(args)
        return

    share = None
    if args.share:
        split, _, n = args.share.partition(":")
        base = synth.make_workload(args.workload)
        if split not in ("rows", "chains") or not n.isdigit() or int(n) < 1:
            ap.error("--share takes rows:N or chains:N")
        n = int(n)
        if split == "rows" and base.height % n == 0:
            wl = synth.make_workload(args.workload, sweeps=args.sweeps, height=base.height // n)
        elif split == "chains" and base.chains % n == 0:
            wl = synth.make_workload(args.workload, sweeps=args.sweeps, chains=base.chains // n)
        else:
            ap.error(f"--share {args.share}: N must divide the workload's {'height' if split == 'rows' else 'chains'}")
        share = {"split": split, "of_gpus": n,
                 "note": "one GPU's share of the workload split over that many GPUs, run alone on one GPU (a "
                         "row strip is a separately drawn image of the strip's shape); the halo exchange of a "
                         "row split and the final reduce of the level sums and histograms are not measured"}
    else:
        wl = synth.make_workload(args.workload, sweeps=args.sweeps)
    if args.q is not None:
        wl.q = args.q
    if args.neighbourhood is not None:
        wl.neighbourhood = args.neighbourhood
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    obs = torch.from_numpy(wl.obs).to(dev)
    kw = wl.params(inertia=args.inertia)
    kw.pop("height")
    kw.pop("width")
    levels = kw.pop("levels")
    stream = torch.cuda.current_stream()
    N = wl.height * wl.width

    def job(timing):
        s = Sampler(obs, levels=levels, **kw)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        s.sweep(wl.sweeps)
        ev1.record(stream)
        mean = s.posterior_mean()
        mpm = s.marginal_map() if wl.tally_stride > 0 else None
        timing.append((ev0, ev1))
        return s, mean, mpm

    spl = 1
    for _ in range(args.warmup):
        s, _, _ = job([])
        s.sync()
        spl = s.sweeps_per_launch()
        s.close()
    torch.cuda.synchronize()

    timing = []
    samplers = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s, mean, mpm = job(timing)
        samplers.append(s)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for s in samplers:
        s.sync()
        s.close()

    # event time over the job's sweeps per kernel launch (one launch advances spl sweeps on
    # small lattices with few levels; the time then includes the gaps between launches)
    sweep_ms = [a.elapsed_time(b) for a, b in timing]
    launches = -(-wl.sweeps // spl)
    per_launch = wl.sweeps / launches  # sweeps per launch, on average over the job
    avg_launch_s = (sum(sweep_ms) / len(sweep_ms)) / 1e3 / launches
    su_total = wl.site_updates * args.steps
    value = su_total / elapsed

    ops_per_su = valu_ops_per_site_update(wl.levels, wl.chains, args.inertia, wl.neighbourhood)
    launch_ops = ops_per_su * N * wl.chains * per_launch
    achieved = launch_ops / avg_launch_s / 1e12
    # the committed counter summary is for the default c3 job (1000 sweeps, 250 of them burn-in)
    default_job = (args.inertia == 0 and wl.name == "c3" and args.sweeps is None and args.q is None
                   and args.neighbourhood is None and args.share is None)
    traffic = measured_traffic(N * wl.chains) if default_job else None
    hbm_alg = hbm_bytes_per_launch(wl) * per_launch
    out = {
        "metric": "site-updates/s",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": workload_label(wl, args.inertia),
            "inertia": args.inertia,
            "height": wl.height, "width": wl.width, "levels": wl.levels, "chains": wl.chains,
            "sweeps": wl.sweeps, "site_updates_per_step": wl.site_updates,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_VALU_TOPS,
            "unit": "TOP/s",
            "frac": achieved / PEAK_VALU_TOPS,
            "traffic": traffic,
            "kernel": "sweep_kernel" if spl == 1 else "tb_sweep_kernel",
            "sweeps_per_launch": spl,
            "ops_per_site_update": ops_per_su,
            "ops_model": "dense-equivalent: every level of every chain counted as a full evaluation (levels "
                         "where no chain of a wave is near a neighbour's level, which the kernel handles with "
                         "one fma per chain, are counted in full)",
            "avg_launch_ms": avg_launch_s * 1e3,
            "peak_note": peak_note(wl, args.inertia, spl),
        },
        "hbm": {
            "algorithmic_bytes_per_launch": hbm_alg,
            "achieved_GBs": hbm_alg / avg_launch_s / 1e9,
            "peak_GBs": PEAK_HBM_GBS,
            "frac": hbm_alg / avg_launch_s / 1e9 / PEAK_HBM_GBS,
            "model_bytes_per_site_update": model_bytes_per_site_update(wl.chains),
            "frac_at_model_bytes": model_bytes_per_site_update(wl.chains) * N * wl.chains * per_launch
                                   / avg_launch_s / 1e9 / PEAK_HBM_GBS,
        },
        "level_evaluations_per_s": value * wl.levels,
    }
    # one more job with the observation starting in host memory and the mean and mode
    # ending there: the end-to-end time a caller holding host arrays sees (not `value`)
    obs_host = wl.obs.copy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = Sampler(torch.from_numpy(obs_host).to(dev), levels=levels, **kw)
    s.sweep(wl.sweeps)
    s.posterior_mean().cpu()
    if wl.tally_stride > 0:
        s.marginal_map().cpu()
    torch.cuda.synchronize()
    e2e = time.perf_counter() - t0
    s.close()
    out["end_to_end"] = {"ms_per_job": e2e * 1e3, "site_updates_per_s": wl.site_updates / e2e,
                         "includes": "observation upload from host memory, the job, mean and mode download"}
    same_kernel_work = (wl.name == "c3" and args.inertia == 0 and wl.neighbourhood == 4 and args.q is None
                        and args.share is None)
    issue = measured_valu_per_site_update() if same_kernel_work else None
    if issue is not None:
        # instructions the kernel issued (rocprofv3 SQ_INSTS_VALU x 64 lanes, same kernel source)
        lane_insts = issue * N * wl.chains * per_launch
        out["roofline"]["measured_issue"] = {
            "valu_instructions_per_site_update": issue,
            "achieved": lane_insts / avg_launch_s / 1e12,
            "frac": lane_insts / avg_launch_s / 1e12 / PEAK_VALU_TOPS,
            "source": os.path.relpath(COUNTERS_FILE, ROOT),
        }
    out["quality"] = quality(wl, mean.cpu().numpy(), None if mpm is None else mpm.cpu().numpy())
    if share:
        out["shard"] = share
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds, args.inertia)
        if wl.name == "c1" and args.inertia == 0:
            out["cpu_baseline"]["gibbs"] = gibbs_comparison(wl)
        elif args.inertia == 0:
            out["cpu_baseline"]["gibbs"] = gibbs_rate(wl, args.cpu_seconds / 2)
        threads = min(16, len(os.sched_getaffinity(0)))
        if threads > 1:
            out["cpu_baseline_all_cores"] = cpu_baseline(wl, args.cpu_seconds, args.inertia, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
