#!/usr/bin/env python3
"""Benchmark of the gauged Gaussian fermionic PEPS Monte Carlo on one MI355X.

Default run (the headline): effective samples per second of the plaquette,
estimated at a fixed observable error, of the learned block proposal with
float32 updates and float64 refresh on the 32x32 Z2 K=2 workload (256
chains), against the plain float64 single-link sampler on the same 256 chains
and against the same block moves with an untrained (uniform) proposal.  A
step is one block sweep of every chain (a Metropolis-Hastings move on each of
the 64 4x4-site patches) followed by the plaquette / 2x2 Wilson loop / density
measurement.  Effective samples come from the spread of the chain means
(256 independent chains; ESS = var(O) / SE(mean)^2), which needs no estimate
of the autocorrelation time; tau_int is reported beside it with its window and
its flags (clamped at 1/2, series too short).

Sub-records: the plain float64 sampler on the 8x8 Z2 K=1 workload (4096
chains; proposals/s, the HBM roofline of its window flush), the CPU oracle
timed on bounded samples of both workloads (with the definitional per-proposal
determinant mode), and the oracle's float64 observables of sampled final
configurations against the float32 path.

Other workloads: --workload c2 | c3 | c4 | c5 (one JSON line each).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="north", choices=["north", "c2", "c3", "c4", "c5"],
                    help="north (default): the c5 comparison with the c2 plain float64 leg and the CPU oracle; "
                         "c2: 8x8 Z2 K=1 4096 chains float64; "
                         "c3: 16x16 Z2 K=3 2048 chains float32 + float64 refresh; "
                         "c4: 8192 chains, L in {6,8,12,16,20}, K in {1,2,4}, Z2/Z3, float32 + refresh, "
                         "graph-replayed autotuned sweeps; "
                         "c5: 32x32 Z2 K=2 256 chains, learned 4x4-patch block proposal trained online on the "
                         "plain sampler, float32 + float64 refresh, vs the plain float64 single-link sampler")
    ap.add_argument("--train-chains", type=int, default=32, help="c5: chains of the plain sampler the net trains on")
    ap.add_argument("--train-sweeps", type=int, default=3, help="c5: plain-sampler sweeps of online training")
    ap.add_argument("--train-steps", type=int, default=40, help="c5: Adam steps after each training sweep")
    ap.add_argument("--plain-chains", type=int, default=None,
                    help="c5: chains of the float64 single-link comparison (default: the learned sampler's)")
    ap.add_argument("--plain-steps", type=int, default=5, help="c5: timed sweeps of the float64 single-link comparison")
    ap.add_argument("--untrained", type=int, default=1,
                    help="c5: also time the block moves with an untrained (uniform) proposal (1 = yes)")
    ap.add_argument("--block-pend", type=int, default=-1,
                    help="c5: largest combined rank of pending block moves (-1 = library default, 0 = apply "
                         "each accepted move at once)")
    ap.add_argument("--bond-gradient", type=int, default=1,
                    help="c5: time the gradient with respect to the patch bond states on the final "
                         "configurations (1 = yes)")
    ap.add_argument("--autotune", type=int, default=0, help="sweeps per autotuner candidate (0 = off)")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--chains", type=int, default=None)
    ap.add_argument("--L", type=int, default=None)
    ap.add_argument("--K", type=int, default=None)
    ap.add_argument("--group", type=int, default=None)
    ap.add_argument("--precision", type=int, default=None)
    ap.add_argument("--refresh", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--graph", type=int, default=None, help="1 = replay each sweep as a captured hipGraph")
    ap.add_argument("--balance", type=int, default=None,
                    help="1 = balanced sweeps (every chain steps its own link cursor; uneven batches)")
    ap.add_argument("--delay", type=int, default=None,
                    help="window of delayed updates in link steps (0 = one rank-4 pass per accepted flip; "
                         "default: the library's)")
    ap.add_argument("--flush-grid", type=int, default=0, help="workgroups of the window flush (0 = library default)")
    ap.add_argument("--update-grid", type=int, default=0)
    ap.add_argument("--update-tiles", type=int, default=0)
    ap.add_argument("--update-nt", type=int, default=1)
    ap.add_argument("--traffic-json", default=os.path.join(HERE, "profiles", "k_update_traffic.json"),
                    help="measured HBM traffic of the update kernel (from rocprofv3 counters)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (counter calibration) and exit")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="derive the update kernel's HBM bytes per launch from rocprofv3 --pmc CSVs, "
                         "write --traffic-json and exit (no GPU needed)")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30, help="size of the calibration copy (--traffic-from)")
    ap.add_argument("--block-traffic-from", nargs=5,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV", "BENCH_JSON"),
                    help="derive the block update's HBM bytes per accepted move from rocprofv3 --pmc CSVs of a "
                         "--workload c5 run and that run's JSON line, write profiles/k_block_traffic.json and exit")
    ap.add_argument("--lambda-iters", type=int, default=0,
                    help="after the timed sweeps, rounds of the variational optimisation of lambda (K > 1 "
                         "workloads; --lambda-sweeps sweeps per round), reported under 'lambda_opt'")
    ap.add_argument("--lambda-sweeps", type=int, default=2)
    ap.add_argument("--gamma-iters", type=int, default=0,
                    help="after the timed sweeps, rounds of gradient descent on Gamma_A (--lambda-sweeps "
                         "sweeps per round, --gamma-step), reported under 'gamma_opt'")
    ap.add_argument("--gamma-step", type=float, default=0.01)
    ap.add_argument("--electric-traffic-from", nargs=4,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="derive the electric measurement kernel's HBM bytes per launch from rocprofv3 --pmc "
                         "CSVs, write profiles/k_electric_traffic.json and exit (no GPU needed)")
    args = ap.parse_args()
    presets = {
        # float64 refactorisation every 131072 changed links (about 130 block sweeps): after 135 block
        # sweeps without one the float32 drift of every observable is at most 4.3e-7 and of log N 5.6e-7
        # (bench float32_drift with --steps 130 --refresh 0), inside the 1e-6 target
        "north": dict(steps=20, warmup=5, chains=256, L=32, K=2, group=2, precision=32, refresh=131072, delay=16),
        "c2": dict(steps=20, warmup=3, chains=4096, L=8, K=1, group=2, precision=64, refresh=16384, delay=16,
                   graph=1),
        "c3": dict(steps=3, warmup=1, chains=2048, L=16, K=3, group=2, precision=32, refresh=64, delay=16),
        "c4": dict(steps=2, warmup=1, chains=8192, L=0, K=0, group=0, precision=32, refresh=64, delay=16,
                   graph=1, balance=1),
        "c5": dict(steps=20, warmup=5, chains=256, L=32, K=2, group=2, precision=32, refresh=131072, delay=16),
    }
    for k, v in presets[args.workload].items():
        if getattr(args, k) is None:
            setattr(args, k, v)
    for k in ("graph", "balance"):
        if getattr(args, k) is None:
            setattr(args, k, 0)
    if args.plain_chains is None:
        args.plain_chains = args.chains
    return args


def c2_args(args):
    """The plain float64 8x8 leg of the default run (fixed counts: 20 timed sweeps after 3)."""
    import copy
    a = copy.copy(args)
    a.workload = "c2"
    for k, v in dict(steps=20, warmup=3, chains=4096, L=8, K=1, group=2, precision=64, refresh=16384,
                     delay=16, graph=1, balance=0).items():
        setattr(a, k, v)
    return a


def ess_between_chains(series):
    """Effective samples of the grand mean of series[t, c] (independent chains c): the variance of
    one sample over the squared standard error of the mean, the latter from the spread of the chain
    means.  Returns (ess, standard error of the mean, variance of one sample)."""
    x = np.asarray(series, np.float64)
    n_t, n_c = x.shape
    se2 = x.mean(axis=0).var(ddof=1) / n_c
    var = x.var(ddof=1)
    return (var / se2 if se2 > 0 else float("inf")), float(np.sqrt(se2)), float(var)


def statistics(series, elapsed):
    """ESS/s, the standard error after one second of sampling, and tau_int with its flags."""
    from paper_2412_01737_amd.ggf import autocorr_time, TAU_FLOOR, TAU_SHORT
    ess, se, var = ess_between_chains(series)
    rec = {"effective_samples_per_s": ess / elapsed, "ess": ess, "samples": int(series.size),
           "mean": float(np.mean(series)), "se_mean": se, "se_at_1s": float(np.sqrt(var * elapsed / ess))
           if ess > 0 else None}
    if series.shape[0] >= 2:
        tau, err, w, fl = autocorr_time(series, with_flags=True)
        rec.update(tau_int=tau, tau_int_err=err, tau_window=w, tau_at_floor=bool(fl & TAU_FLOOR),
                   tau_series_too_short=bool(fl & TAU_SHORT))
    return rec


def traffic_from(args):
    """HBM bytes per k_update launch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch).

    Each counter is scaled by bytes_known / counter_read for a plain copy of
    --copy-bytes bytes (FETCH_SIZE reads half the bytes of 128-byte requests on
    this part, WRITE_SIZE reads them in full)."""
    import csv

    def per_kernel(path, counter, match):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                if r["Counter_Name"] == counter and match in r["Kernel_Name"]]
        return sum(vals) / len(vals), len(vals)

    kernel = "k_window_flush" if args.delay > 0 else "k_update"
    if args.delay > 0:
        # the window flush: k_window_gemm, after k_window_snap when the context has K > 1
        # (with K = 1 the link steps copy P = G[A,:])
        fetch, write, nf, nw = 0.0, 0.0, 0, 0
        pairs = args.K > 1 or args.workload == "c4"
        for k in ("k_window_snap", "k_window_gemm") if pairs else ("k_window_gemm",):
            f_, n_ = per_kernel(args.traffic_from[0], "FETCH_SIZE", k)
            w_, m_ = per_kernel(args.traffic_from[1], "WRITE_SIZE", k)
            fetch, write, nf, nw = fetch + f_, write + w_, n_, m_
    else:
        fetch, nf = per_kernel(args.traffic_from[0], "FETCH_SIZE", kernel)
        write, nw = per_kernel(args.traffic_from[1], "WRITE_SIZE", kernel)
    cfetch, _ = per_kernel(args.traffic_from[2], "FETCH_SIZE", "probe_copy")
    cwrite, _ = per_kernel(args.traffic_from[3], "WRITE_SIZE", "probe_copy")
    known_kib = args.copy_bytes / 1024.0
    sf, sw = known_kib / cfetch, known_kib / cwrite
    rec = {"bytes_per_launch": (fetch * sf + write * sw) * 1024.0,
           "read_bytes_per_launch": fetch * sf * 1024.0, "write_bytes_per_launch": write * sw * 1024.0,
           "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write, "dispatches": [nf, nw],
           "fetch_scale": sf, "write_scale": sw, "kernel": kernel,
           "source_digest": source_digest(KERNEL_SOURCE[kernel])}
    key = traffic_key(args)
    try:
        with open(args.traffic_json) as f:
            tj = json.load(f)
    except (OSError, ValueError):
        tj = {}
    tj[key] = rec
    with open(args.traffic_json, "w") as f:
        json.dump(tj, f, indent=1)
    print(json.dumps({key: rec}))


ELECTRIC_TRAFFIC_JSON = os.path.join(HERE, "profiles", "k_electric_traffic.json")


def electric_kernel(args) -> str:
    return "k_electric1" if (args.workload != "c4" and args.K == 1) else "k_electric"


def electric_traffic_from(args):
    """HBM bytes per electric measurement launch from FETCH_SIZE / WRITE_SIZE, scaled by the
    plain-copy calibration as for the update kernels."""
    import csv
    kernel = electric_kernel(args)

    def per_kernel(path, counter, match):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                if r["Counter_Name"] == counter and match + "<" in r["Kernel_Name"]]
        return sum(vals) / len(vals), len(vals)

    fetch, nf = per_kernel(args.electric_traffic_from[0], "FETCH_SIZE", kernel)
    write, nw = per_kernel(args.electric_traffic_from[1], "WRITE_SIZE", kernel)
    cfetch, _ = per_kernel(args.electric_traffic_from[2], "FETCH_SIZE", "probe_copy")
    cwrite, _ = per_kernel(args.electric_traffic_from[3], "WRITE_SIZE", "probe_copy")
    known_kib = args.copy_bytes / 1024.0
    sf, sw = known_kib / cfetch, known_kib / cwrite
    rec = {"bytes_per_launch": (fetch * sf + write * sw) * 1024.0,
           "read_bytes_per_launch": fetch * sf * 1024.0, "write_bytes_per_launch": write * sw * 1024.0,
           "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write, "dispatches": [nf, nw],
           "fetch_scale": sf, "write_scale": sw, "kernel": kernel, "source_digest": source_digest()}
    try:
        with open(ELECTRIC_TRAFFIC_JSON) as f:
            tj = json.load(f)
    except (OSError, ValueError):
        tj = {}
    tj[traffic_key(args)] = rec
    with open(ELECTRIC_TRAFFIC_JSON, "w") as f:
        json.dump(tj, f, indent=1)
    print(json.dumps({traffic_key(args): rec}))


def block_traffic_from(args):
    """HBM bytes per block update of G (k_window_snap + k_window_gemm), from FETCH_SIZE / WRITE_SIZE.

    Counters are scaled by the copy calibration as in traffic_from; the number of
    updates of G per launch comes from the profiled run's own JSON line."""
    import csv

    def per_kernel(path, counter, match):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter and match in r["Kernel_Name"]]
        if rows and "Dispatch_Id" in rows[0]:
            rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return [float(r["Counter_Value"]) for r in rows]

    f_csv, w_csv, cf_csv, cw_csv, bench_json = args.block_traffic_from
    cfetch = sum(per_kernel(cf_csv, "FETCH_SIZE", "probe_copy")) / len(per_kernel(cf_csv, "FETCH_SIZE", "probe_copy"))
    cwrite = sum(per_kernel(cw_csv, "WRITE_SIZE", "probe_copy")) / len(per_kernel(cw_csv, "WRITE_SIZE", "probe_copy"))
    known_kib = args.copy_bytes / 1024.0
    sf, sw = known_kib / cfetch, known_kib / cwrite
    rec = None
    for line in open(bench_json):
        if line.startswith("{") and '"learned"' in line:
            rec = json.loads(line)
    learned = rec["learned"]
    updates_per_launch = learned["updates_of_G"] / learned["update_launches"]
    # only the learned sampler's timed block sweeps: the last update_launches dispatches of each
    # kernel (run with --untrained 0 --plain-steps 0, so nothing dispatches them afterwards; the
    # training context's block sweeps of the output-scale trials come earlier)
    last = int(learned["update_launches"])
    out = {"source_digest": source_digest(BLOCK_SOURCES), "updates_per_launch": updates_per_launch,
           "moves_per_update": learned["moves_per_update"], "fetch_scale": sf, "write_scale": sw}
    total = 0.0
    tname = "float" if rec["config"]["precision"] == 32 else "double"
    # block moves only: k_window_snap and the <T, 8, true, *> instances of k_window_gemm (the
    # training sampler's window flushes run <T, 4, false, *>)
    for k in (f"k_window_snap<{tname}>", f"k_window_gemm<{tname}, 8, true,"):
        fv, wv = per_kernel(f_csv, "FETCH_SIZE", k)[-last:], per_kernel(w_csv, "WRITE_SIZE", k)[-last:]
        rd = sum(fv) / len(fv) * sf * 1024.0
        wr = sum(wv) / len(wv) * sw * 1024.0
        out[k.split("<")[0]] = {"read_bytes_per_launch": rd, "write_bytes_per_launch": wr,
                                "dispatches": [len(fv), len(wv)]}
        total += rd + wr
    n = rec["config"]["n"]
    esz = 4 if rec["config"]["precision"] == 32 else 8
    out["bytes_per_update"] = total / updates_per_launch
    out["algorithmic_bytes_per_update"] = (n * (n + 1) / 2 + n * n) * esz
    key = f"L{rec['config']['L']}_K{rec['config']['K']}_Z{rec['config']['group']}_p{rec['config']['precision']}"
    path = os.path.join(HERE, "profiles", "k_block_traffic.json")
    try:
        with open(path) as f:
            tj = json.load(f)
    except (OSError, ValueError):
        tj = {}
    tj[key] = out
    with open(path, "w") as f:
        json.dump(tj, f, indent=1)
    print(json.dumps({key: out}))


def copy_probe(nbytes: int):
    """Project stream probes (ggf_stream_probe) on a buffer of known size.

    Calibrates FETCH_SIZE / WRITE_SIZE per byte moved and measures the
    achievable copy and read-modify-write bandwidth the update kernel is
    compared with."""
    import ctypes
    import torch
    from paper_2412_01737_amd.ggf import load
    lib = load()
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    s = torch.cuda.current_stream()
    out = {"bytes": nbytes}
    for mode, name, moved in ((0, "copy", 2), (1, "copy_nt", 2), (2, "rmw", 2), (3, "rmw_nt", 2),
                              (4, "copy_unrolled", 2), (5, "rmw_unrolled", 2), (6, "read_unrolled", 1),
                              (7, "write_unrolled", 1)):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st = lib.ggf_stream_probe(mode, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), nbytes, 0,
                                  ctypes.c_void_p(s.cuda_stream))
        assert st == 0
        reps = 5
        ev0.record(s)
        for _ in range(reps):
            lib.ggf_stream_probe(mode, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), nbytes, 0,
                                 ctypes.c_void_p(s.cuda_stream))
        ev1.record(s)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        out[name + "_GBps"] = moved * nbytes / (ms * 1e-3) / 1e9
    print(json.dumps(out))


KERNEL_SOURCE = {"k_update": ("ggf_sweep.hip",), "k_window_flush": ("ggf_block.inc", "ggf_window.inc")}
BLOCK_SOURCES = ("ggf_block.inc", "ggf_window.inc")   # block moves: decision in the first, update in the second


def traffic_key(args) -> str:
    key = f"L{args.L}_K{args.K}_Z{args.group}_p{args.precision}_c{args.chains}"
    return key + (f"_flush{args.delay}" if args.delay > 0 else "")


def source_digest(names=("ggf_sweep.hip",)) -> str:
    """Digest of a kernel's source files; traffic counters are only reported for the kernel they measured."""
    import hashlib
    h = hashlib.sha256()
    for name in ([names] if isinstance(names, str) else names):
        with open(os.path.join(HERE, "paper_2412_01737_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def float32_drift(ctx, stream):
    """Drift of every observable slot of a maintained float32 state: the measurement before and after a
    float64 refactorisation of every chain (largest |difference| / max(1, |value|) over chains)."""
    from paper_2412_01737_amd.ggf import OBS_ALL
    before = ctx.measure(OBS_ALL)
    ctx.refresh_all(stream=stream)
    after = ctx.measure(OBS_ALL)
    rel = np.abs(before - after) / np.maximum(1.0, np.abs(after))
    names = ["plaquette", "wilson2x2", "density", "log_n"] + [f"meson_{r}" for r in range(1, 17)] + ["electric"]
    return {"what": "largest |maintained - refactorised| / max(1, |value|) over chains, after the timed sweeps",
            "per_observable": {nm: float(rel[:, q].max()) for q, nm in enumerate(names) if np.any(after[:, q] != 0)}}


def refresh_rates(st0, st1, steps: int, refresh: int):
    """Mean refactorisations per chain over `steps` sweeps: (at the true rate, counted).

    st0, st1: per-chain state dicts ("accepts", "refreshes") before and after the
    sweeps.  A chain is refactorised at the first sweep end after `refresh`
    accepted flips, i.e. every ceil(refresh / accepted flips per sweep) sweeps."""
    import math
    expected, actual = [], []
    for a, b in zip(st0, st1):
        fps = (b["accepts"] - a["accepts"]) / steps
        period = math.ceil(refresh / fps) if refresh > 0 and fps > 0 else 0
        expected.append(steps / period if period > 0 else 0.0)
        actual.append(b["refreshes"] - a["refreshes"])
    return float(np.mean(expected)), float(np.mean(actual))


def refresh_correction(ctx, args, st0, stream, st1=None):
    """Float64 refactorisations charged at their true rate.

    A chain is refactorised at the first sweep end after refresh_every accepted
    flips, i.e. every ceil(refresh_every / flips per sweep) sweeps.  The timed
    sweeps contain however many refactorisations their alignment gives; the
    difference to the true rate is charged (or credited) at the measured cost
    of refactorising all chains, timed here after the timed region."""
    import torch
    if st1 is None:
        st1 = [ctx.get_state(c)[1] for c in range(args.chains)]
    exp_mean, act_mean = refresh_rates(st0, st1, args.steps, args.refresh)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.refresh_all(stream=stream)
    torch.cuda.synchronize()
    ms_all = (time.perf_counter() - t) * 1e3
    return {"every_accepted_flips": args.refresh, "per_chain_in_timed_sweeps": act_mean,
            "per_chain_at_true_rate": exp_mean, "ms_all_chains": ms_all,
            "correction_ms": (exp_mean - act_mean) * ms_all if args.refresh > 0 else 0.0}


def host_info():
    """CPU model and core count of the host, and the worker processes the oracle legs use (at most 16:
    one GPU's share of the host)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    return {"cpu_model": model, "nproc": nproc, "workers": max(1, min(16, nproc))}


def cpu_baseline(args, budget_s: float):
    """The oracle on host cores, bounded in time: its Woodbury chain (one chain per worker process, one
    BLAS thread each), and its definitional mode (a fresh determinant per proposal) on one core."""
    import multiprocessing as mp
    info = host_info()
    workers = info["workers"]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers, initializer=_cpu_init) as pool:
        res = pool.starmap(_cpu_chain, [(args.L, args.K, args.group, c, budget_s, False) for c in range(workers)])
        dres = pool.starmap(_cpu_chain, [(args.L, args.K, args.group, 0, min(budget_s, 5.0), True)])
    wall = time.perf_counter() - t0 - min(budget_s, 5.0)
    props = sum(r[0] for r in res)
    sweeps = sum(r[1] for r in res)
    rec = {"value": props / (wall if wall > 0 else budget_s), "unit": "proposals/s", "cores": workers,
           "kind": "oracle",
           "sample": f"{workers} chains x {min(r[1] for r in res)}-{max(r[1] for r in res)} sweeps of L={args.L} "
                     f"K={args.K} Z{args.group} (Woodbury-mode oracle, float64, 1 BLAS thread per process), "
                     f"{wall:.1f} s wall",
           "o_def_proposals_per_s": dres[0][0] / dres[0][2],
           "o_def_sample": f"1 chain, {dres[0][0]} proposals, each from a fresh determinant, {dres[0][2]:.1f} s"}
    rec.update(info)
    return rec


def _cpu_init():
    try:
        import threadpoolctl
        threadpoolctl.threadpool_limits(1)
    except Exception:
        pass


def _cpu_chain(L, K, group, chain, budget_s, definitional):
    import synth
    from oracle.chain import DefinitionChain, WoodburyChain
    from oracle.lattice import Lattice
    from oracle.model import Ansatz
    spec = synth.make_tensor(L, K=K, group=group)
    an = Ansatz(Lattice(L, L), spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k, spec.c)
    ch = (DefinitionChain(an, synth.SEED_CHAIN, chain) if definitional
          else WoodburyChain(an, synth.SEED_CHAIN, chain, refresh_every=1024))
    t0 = time.perf_counter()
    sweeps = props = 0
    if definitional:
        # proposals one at a time (a sweep of the definitional chain can outlast the budget)
        from oracle import philox
        from oracle.chain import propose
        ell = 0
        while time.perf_counter() - t0 < budget_s or props == 0:
            u, step = philox.draw(ch.seed, ch.chain, ch.sweep_idx, ell, an.group)
            knew = ch.k.copy()
            knew[ell] = propose(int(ch.k[ell]), int(step), an.group)
            ln_new = ch._logn(knew)
            if float(u) < np.exp(ln_new - ch.logn):
                ch.k, ch.logn = knew, ln_new
            props += 1
            ell = (ell + 1) % an.lat.n_links
        return props, sweeps, time.perf_counter() - t0
    while time.perf_counter() - t0 < budget_s or sweeps == 0:
        ch.sweep()
        sweeps += 1
    return ch.proposals, sweeps, time.perf_counter() - t0


def cpu_baseline_c5(args, budget_s: float, c5: dict):
    """The oracle on the 32x32 K=2 learned-proposal workload, bounded in time, in one process with every
    BLAS thread of one GPU's share of the host: hot start of chain 0, then block moves of the same
    network (fresh LU factorisations of M(G) and M(G') per move) until the budget is spent.  Effective
    samples per second = block sweeps per second / (2 tau), tau the GPU run's plaquette tau_int (at
    least 1/2).  Also: the oracle's float64 observables of the GPU's final configuration of chain 0,
    from a fresh inverse, against the float32 path's values."""
    import threadpoolctl
    info = host_info()
    with threadpoolctl.threadpool_limits(info["workers"]):
        return _cpu_baseline_c5(args, budget_s, c5, info)


def _cpu_baseline_c5(args, budget_s, c5, info):
    import synth
    from oracle import nn
    from oracle.chain import WoodburyChain, block_move, hot_links
    from oracle.lattice import Lattice
    from oracle.model import Ansatz
    L, K, group, P = args.L, args.K, args.group, 4
    spec = synth.make_tensor(L, K=K, group=group)
    an = Ansatz(Lattice(L, L), spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k, spec.c)
    t0 = time.perf_counter()
    learned = c5["learned"]
    k_gpu = np.array(learned["final_chain0"]["links"], np.int8)
    G = np.linalg.inv(an.assemble_M(k_gpu))
    ref = an.observables_from_inverse(k_gpu, G)
    del G
    gobs = np.array(learned["final_chain0"]["obs"])
    err = np.abs(gobs - ref) / np.maximum(1.0, np.abs(ref))
    t_check = time.perf_counter() - t0
    params = c5.pop("_params", None)
    if params is None:
        params = nn.init_params(NN_SEED).astype(np.float32)
    t0 = time.perf_counter()
    ch = WoodburyChain(an, synth.SEED_CHAIN, 0, hot_links(synth.SEED_CHAIN, 0, an.lat.n_links, group))
    moves = 0
    npatch = (L // P) ** 2
    while time.perf_counter() - t0 < budget_s or moves == 0:
        block_move(ch, params, P, moves % npatch, route="patch")
        moves += 1
    wall = time.perf_counter() - t0
    tau = max(0.5, learned["plaquette"].get("tau_int") or 0.5)
    rec = {"value": moves / npatch / wall / (2.0 * tau), "unit": "effective samples/s", "cores": info["workers"],
           "kind": "oracle",
           "sample": f"1 chain of {L}x{L} Z{group} K={K}: hot start and {moves} learned block moves "
                     f"({moves / npatch:.3f} block sweeps; fresh LU factorisations of M per move, "
                     f"{info['workers']} BLAS threads) in {wall:.1f} s, divided by 2 tau_int "
                     f"(tau = {tau:.3f} from the GPU run)",
           "oracle_check": {"what": "float64 oracle observables of the float32 path's final configuration of "
                                    "chain 0 (fresh inverse) against the path's values, |d| / max(1, |x|)",
                            "max_error": float(err.max()), "worst_slot": int(err.argmax()),
                            "errors": err.tolist(), "seconds": t_check}}
    rec.update(info)
    return rec


NN_SEED = 7
BETAS = (0.0, 0.25, 0.5, 0.75, 1.0)     # candidate scales of the network's output layer
N_LAST = 2 * 32 * 9 + 2                 # output layer: W4 [2][32][3][3] and b4 [2], the last parameters
RHOS = (1.0, 0.5, 0.25, 0.125)         # candidate move rates of the block proposal
MFMA_PEAK_F32_TFLOPS = 157.3


def run_c5(args):
    """Learned block proposal (4x4-site patches) vs the plain float64 single-link sampler, one GPU.

    1. Online training: a plain float32 single-link sampler on --train-chains
       chains; after each of its sweeps the network takes --train-steps Adam
       steps on (window, patch) examples of its current link fields.
    2. The learned sampler: --chains chains, one block sweep = one
       Metropolis-Hastings block move on every patch, float32 inverse with a
       float64 refactorisation every --refresh changed links (charged at its
       true rate); the plaquette and the density are measured after every sweep.
       The output scale, then the move rate, are chosen on the training chains
       (the most changed links of accepted moves per block sweep).
    3. The same block moves with an untrained network (all weights and biases
       zero: every patch link proposed with probability 1/2, move rate 1), same
       chains.
    4. The plain float64 single-link sampler on the same GPU (--plain-chains
       chains, delayed updates, no refactorisation: its drift is negligible,
       --plain-steps sweeps), measured the same way.
    Effective samples per second from the spread of the chain means (see
    ess_between_chains), for the plaquette and the density."""
    import torch
    import synth
    from paper_2412_01737_amd.ggf import Context, OBS_LINK, OBS_DENSITY, GGF_NOBS, load

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    L, K, group, P = args.L, args.K, args.group, 4
    n = 8 * L * L
    spec = synth.make_tensor(L, K=K, group=group)
    nparams = load().ggf_nn_nparams()

    t0 = time.perf_counter()
    tr = Context(0)
    tr.set_option("delay", args.delay)
    tid = tr.set_tensor_spec(spec)
    tr.init_chains([L] * args.train_chains, tid, synth.SEED_CHAIN + 1, init=1, precision=32,
                   refresh_every=args.refresh, stream=stream)
    tr.nn_init(P, NN_SEED)
    losses = []
    for sw in range(args.train_sweeps):
        tr.sweep(1, stream=stream)
        losses.append(tr.nn_train(args.train_steps, 512, 3e-3, NN_SEED + 1 + sw, stream=stream))
        log(f"c5 training sweep {sw + 1}/{args.train_sweeps}: loss {losses[-1]:.4f} nats/patch")
    trained = tr.nn_params()
    # adaptation of the proposal's sharpness during burn-in, then frozen: the last layer scaled by
    # beta (beta = 0 is the uniform proposal), beta chosen to maximise the links that accepted block
    # moves change per block sweep on the training chains
    scale_trials = []
    for beta in BETAS:
        p = trained.copy()
        p[-N_LAST:] *= beta
        tr.nn_params(p)
        st0 = np.array([tr.block_stats(c) for c in range(args.train_chains)])
        tr.block_sweep(2, stream=stream)
        st1 = np.array([tr.block_stats(c) for c in range(args.train_chains)])
        d = st1 - st0
        scale_trials.append({"beta": beta, "acceptance": float(d[:, 1].sum() / max(1, d[:, 0].sum())),
                             "accepted_links_per_sweep": float(d[:, 2].sum() / 2.0 / args.train_chains)})
        log(f"c5 proposal scale {beta}: {scale_trials[-1]}")
    best = max(scale_trials, key=lambda t: t["accepted_links_per_sweep"])
    beta = best["beta"]
    params = trained.copy()
    params[-N_LAST:] *= beta
    # then the move rate at that scale (rho = 1 redraws every patch link; rho < 1 keeps each with
    # probability 1 - rho), chosen the same way
    tr.nn_params(params)
    rate_trials = [{"rho": 1.0, "acceptance": best["acceptance"],
                    "accepted_links_per_sweep": best["accepted_links_per_sweep"]}]
    for rho in RHOS[1:]:
        tr.set_option("block_rho", int(round(rho * 65536)))
        st0 = np.array([tr.block_stats(c) for c in range(args.train_chains)])
        tr.block_sweep(2, stream=stream)
        st1 = np.array([tr.block_stats(c) for c in range(args.train_chains)])
        d = st1 - st0
        rate_trials.append({"rho": rho, "acceptance": float(d[:, 1].sum() / max(1, d[:, 0].sum())),
                            "accepted_links_per_sweep": float(d[:, 2].sum() / 2.0 / args.train_chains)})
        log(f"c5 move rate {rho}: {rate_trials[-1]}")
    rho_best = max(rate_trials, key=lambda t: t["accepted_links_per_sweep"])["rho"]
    tr.close()
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0

    def sampler(name, chains, precision, refresh, net, steps, warmup, rho=1.0):
        ctx = Context(0)
        ctx.set_option("delay", args.delay)
        ctx.set_option("block_rho", int(round(rho * 65536)))
        if args.block_pend >= 0:
            ctx.set_option("block_pend", args.block_pend)
        if args.update_grid:
            ctx.set_option("update_grid", args.update_grid)
        tid = ctx.set_tensor_spec(spec)
        ti = time.perf_counter()
        ctx.init_chains([L] * chains, tid, synth.SEED_CHAIN, init=1, precision=precision,
                        refresh_every=refresh, stream=stream)
        if net is not None:
            ctx.nn_init(P, NN_SEED)
            ctx.nn_params(net)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - ti
        block = net is not None
        step = (lambda: ctx.block_sweep(1, stream=stream)) if block else (lambda: ctx.sweep(1, stream=stream))
        for w in range(warmup):
            step()
            torch.cuda.synchronize()
            log(f"c5 {name} warmup sweep {w + 1}/{warmup}")
        before = [ctx.block_stats(c) for c in range(chains)] if block else None
        st_before = [ctx.get_state(c)[1] for c in range(chains)]
        acc_before = sum(st["accepts"] for st in st_before) if not block else 0
        ctx.set_option("time_update", 1)
        obs = torch.zeros((steps, chains, GGF_NOBS), dtype=torch.float64, device=dev)
        upd_ms, launches, changed = 0.0, 0, 0
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for s_ in range(steps):
            step()
            ms, la, fl = ctx.update_timing()
            upd_ms, launches, changed = upd_ms + ms, launches + la, changed + fl
            ctx.measure(OBS_LINK | OBS_DENSITY, obs[s_], stream=stream)
            log(f"c5 {name} sweep {s_ + 1}/{steps}")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - ts
        # float64 refactorisations charged at their true rate: a chain is refactorised at the first
        # sweep end after `refresh` changed links (accepted flips for the single-link sampler), i.e.
        # every ceil(refresh / changed links per sweep) sweeps; the timed sweeps hold however many
        # their alignment gives, and the difference is charged (or credited) at the measured cost
        # of refactorising all chains, timed here after the timed region
        st_after = [ctx.get_state(c)[1] for c in range(chains)]
        if block:
            moved = [ctx.block_stats(c)[2] - before[c][2] for c in range(chains)]
        else:
            moved = [b_["accepts"] - a_["accepts"] for a_, b_ in zip(st_before, st_after)]
        expected = [steps / math.ceil(refresh / (mv / steps)) if refresh > 0 and mv > 0 else 0.0 for mv in moved]
        actual = [b_["refreshes"] - a_["refreshes"] for a_, b_ in zip(st_before, st_after)]
        series = obs.cpu().numpy()
        final0 = ctx.measure()[0]                  # every slot of chain 0's final configuration
        refreshes = float(np.mean([st["refreshes"] for st in st_after]))
        drift = float32_drift(ctx, stream) if precision == 32 else None
        bond = None
        if block and name == "learned" and K > 1 and args.bond_gradient:
            # gradient of <H> with respect to the patch bond states on the sampled configurations
            from paper_2412_01737_amd.ggf import bond_gradient
            torch.cuda.synchronize()
            tb = time.perf_counter()
            er = ctx.measure_energy(BENCH_COUPLINGS, stream=stream)
            tr = time.perf_counter()
            br = ctx.measure_bond_rows(BENCH_COUPLINGS, stream=stream)
            tg = time.perf_counter()
            gb = bond_gradient(spec, BENCH_COUPLINGS, er, br)
            te = time.perf_counter()
            bond = {"what": "d<H>/d theta for the six rotation generators of the patch bond, over the chains' "
                            "final configurations", "couplings": BENCH_COUPLINGS, "mean_energy": float(er[:, 0].mean()),
                    "grad": gb.tolist(), "energy_rows_s": tr - tb, "bond_rows_s": tg - tr, "host_gradient_s": te - tg}
            log(f"c5 bond gradient: {te - tb:.3f} s")
        # the refactorisation of all chains, timed after the drift and the final-state readings
        torch.cuda.synchronize()
        tr0 = time.perf_counter()
        ctx.refresh_all(stream=stream)
        torch.cuda.synchronize()
        ms_all = (time.perf_counter() - tr0) * 1e3
        refresh_rec = {"every_changed_links" if block else "every_accepted_flips": refresh,
                       "per_chain_in_timed_sweeps": float(np.mean(actual)),
                       "per_chain_at_true_rate": float(np.mean(expected)), "ms_all_chains": ms_all,
                       "correction_ms": (float(np.mean(expected)) - float(np.mean(actual))) * ms_all}
        timed_s = elapsed
        elapsed = elapsed + refresh_rec["correction_ms"] * 1e-3
        rec = {"chains": chains, "sweeps": steps, "warmup": warmup, "s_per_sweep": elapsed / steps,
               "timed_s": timed_s, "refresh": refresh_rec,
               "init_s": t_init, "precision": precision, "refresh_every": refresh,
               "plaquette": statistics(series[:, :, 0], elapsed), "density": statistics(series[:, :, 2], elapsed),
               "update_ms_total": upd_ms, "update_launches": launches, "links_changed": changed,
               "final_chain0": {"links": ctx.get_state(0)[0].tolist(), "obs": final0.tolist()},
               "refreshes_per_chain": refreshes, "float32_drift": drift}
        if bond is not None:
            rec["bond_gradient"] = bond
        if block:
            after = [ctx.block_stats(c) for c in range(chains)]
            prop = sum(a[0] - b[0] for a, b in zip(after, before))
            acc = sum(a[1] - b[1] for a, b in zip(after, before))
            upd = sum(a[3] - b[3] for a, b in zip(after, before))
            rec.update(acceptance=acc / max(prop, 1), links_per_accepted_move=changed / max(acc, 1),
                       accepted_moves=acc, updates_of_G=upd, moves_per_update=acc / max(upd, 1),
                       link_proposals_per_s=chains * steps * 2 * L * L / elapsed)
        else:
            acc = sum(ctx.get_state(c)[1]["accepts"] for c in range(chains)) - acc_before
            rec.update(acceptance=acc / (chains * steps * 2 * L * L),
                       link_proposals_per_s=chains * steps * 2 * L * L / elapsed)
        ctx.close()
        torch.cuda.synchronize()
        return rec

    learned = sampler("learned", args.chains, args.precision, args.refresh, params, args.steps, args.warmup,
                      rho=rho_best)
    untrained = (sampler("untrained", args.chains, args.precision, args.refresh, np.zeros(nparams, np.float32),
                         args.steps, args.warmup) if args.untrained else None)
    # the float64 comparison leg needs no refactorisation over its sweeps (float64 Woodbury
    # drift: 2e-14 in log W over 128 sweeps), so it runs without one
    plain = (sampler("plain", args.plain_chains, 64, 0, None, args.plain_steps, 1)
             if args.plain_steps > 0 else None)
    # block update G -= G[:,U] W G[U,:] per update of G (one accepted move, or several pending ones
    # combined: rank r = 4 x their changed links), on the upper triangle of the antisymmetric G and
    # mirrored: algorithmic bytes = the upper triangle read and all of G written
    # ((n (n + 1) / 2 + n^2) * 4), flops = n^2 r
    esz = 4 if args.precision == 32 else 8
    upd_s = learned["update_ms_total"] * 1e-3
    bytes_moved = (n * (n + 1) / 2 + n * n) * esz * learned["updates_of_G"]
    flops = n * n * 4.0 * learned["links_changed"]
    achieved = bytes_moved / upd_s / 1e9 if upd_s > 0 else 0.0
    tflops = flops / upd_s / 1e12 if upd_s > 0 else 0.0
    traffic = None
    try:
        with open(os.path.join(HERE, "profiles", "k_block_traffic.json")) as f:
            tj = json.load(f).get(f"L{L}_K{K}_Z{group}_p{args.precision}")
        if tj and tj["source_digest"] == source_digest(BLOCK_SOURCES):
            # measured bytes per update of G x updates per launch of this run
            traffic = tj["bytes_per_update"] * learned["updates_of_G"] / learned["update_launches"]
    except (OSError, ValueError, KeyError):
        pass

    def ratio(a, b, obs_name="plaquette"):
        if not a or not b:
            return None
        return a[obs_name]["effective_samples_per_s"] / b[obs_name]["effective_samples_per_s"]

    return {
        "metric": "link-update proposals/sec and effective samples/sec at fixed obs. error, 1 MI355X",
        "value": learned["plaquette"]["effective_samples_per_s"],
        "unit": "effective samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": learned["s_per_sweep"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"Z{group} {L}x{L} periodic, K={K}, {args.chains} chains, learned 4x4-patch block "
                                f"proposal (4-layer 3x3 conv, 32 channels, bf16 weights), float32 inverse, float64 "
                                f"refresh every {args.refresh} changed links; effective samples of the plaquette "
                                f"from the spread of the chain means; vs the plain float64 single-link sampler "
                                f"(delayed updates, window {args.delay}) on {args.plain_chains} chains and the "
                                f"untrained block proposal"),
                   "name": "c5", "L": L, "K": K, "group": group, "chains": args.chains, "n": n, "patch": P,
                   "precision": args.precision, "refresh_every": args.refresh},
        "learned": learned,
        "untrained_block": untrained,
        "plain_f64_single_link": plain,
        "ess_ratio_learned_vs_plain": ratio(learned, plain),
        "ess_ratio_learned_vs_plain_density": ratio(learned, plain, "density"),
        "ess_ratio_learned_vs_untrained": ratio(learned, untrained),
        "training": {"chains": args.train_chains, "sweeps": args.train_sweeps, "adam_steps_per_sweep": args.train_steps,
                     "loss_nats_per_patch": losses, "uniform_loss_nats_per_patch": 32 * float(np.log(2.0)),
                     "output_scale_trials": scale_trials, "output_scale": beta,
                     "move_rate_trials": rate_trials, "move_rate": rho_best, "seconds": t_train},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_window_snap + k_window_gemm (block moves)",
                     "algorithmic_bytes_per_launch": bytes_moved / max(learned["update_launches"], 1),
                     "bytes_per_update": (n * (n + 1) / 2 + n * n) * esz,
                     "tflops": tflops, "mfma_peak_tflops": MFMA_PEAK_F32_TFLOPS,
                     "flops_per_changed_link": 4.0 * n * n},
        "cpu_baseline": None,
        "_params": params,
    }


def electric_measurement(ctx, args, Lc, stream, reps=20):
    """Electric-field observable f_E (Sec. 5.3) of every chain's final configuration: the
    electric-only measurement kernel (k_electric1 when every chain has K = 1, else k_electric;
    one workgroup per chain) timed with HIP events
    on its launch stream, after the timed sweeps.  Algorithmic bytes per link: the six distinct
    entries of the antisymmetric 4x4 block of G on the link's Majoranas (for K > 1 each pair
    of the superposition also reads G on the link rows and the pair's patch columns, not
    counted)."""
    import torch
    from paper_2412_01737_amd.ggf import OBS_ELECTRIC, GGF_NOBS
    out = torch.zeros((args.chains, GGF_NOBS), dtype=torch.float64, device=stream.device)
    ctx.measure(OBS_ELECTRIC, out, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        ctx.measure(OBS_ELECTRIC, out, stream=stream)
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    links = int((2 * Lc.astype(np.int64) ** 2).sum())
    esz = 8 if args.precision == 64 else 4
    nbytes = links * 6 * esz
    achieved = nbytes / (us * 1e-6) / 1e9
    kernel = electric_kernel(args)
    traffic = None
    try:
        with open(ELECTRIC_TRAFFIC_JSON) as f:
            rec = json.load(f).get(traffic_key(args))
        if rec and rec.get("kernel") == kernel and rec.get("source_digest") == source_digest():
            traffic = rec["bytes_per_launch"]
    except (OSError, ValueError):
        pass
    return {"kernel": kernel, "bound": "hbm", "us_per_launch": us, "links_per_s": links / (us * 1e-6),
            "algorithmic_bytes_per_launch": nbytes, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "mean_final": float(out[:, 20].mean().item())}


BENCH_COUPLINGS = dict(t=1.0, mu=0.0, m=0.5, kb=-1.0, ke=1.0)


def energy_measurement(ctx, args, stream, reps=5):
    """Local energy of the gauged Hamiltonian (Sec. 2, 2.3; estimators of Sec. 5.2, 5.3) and the
    pair matrices of the linear step for lambda, for every chain's final configuration: k_energy
    (one workgroup per chain) timed with HIP events on its launch stream after the timed sweeps."""
    import torch
    from paper_2412_01737_amd.ggf import GGF_ENERGY_STRIDE
    out = torch.zeros((args.chains, GGF_ENERGY_STRIDE), dtype=torch.float64, device=stream.device)
    ctx.measure_energy(BENCH_COUPLINGS, out, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        ctx.measure_energy(BENCH_COUPLINGS, out, stream=stream)
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    res = {"kernel": "k_energy", "bound": "latency", "us_per_launch": us, "couplings": BENCH_COUPLINGS,
           "mean_local_energy": float(out[:, 0].mean().item())}
    if args.workload != "c4" and args.L <= (32 if args.K == 1 else 8):
        # sensitivities to the on-site covariance (gradient of <H> with respect to Gamma_A)
        from paper_2412_01737_amd.ggf import GGF_SENS_STRIDE, gamma_gradient
        sens = torch.zeros((args.chains, GGF_SENS_STRIDE), dtype=torch.float64, device=stream.device)
        ctx.measure_sensitivity(BENCH_COUPLINGS, sens, stream=stream)
        e0.record(stream)
        for _ in range(reps):
            ctx.measure_sensitivity(BENCH_COUPLINGS, sens, stream=stream)
        e1.record(stream)
        e1.synchronize()
        g = gamma_gradient(synth_gamma_loc(args), out.cpu().numpy(), sens.cpu().numpy())
        if args.K == 1:
            res["sensitivity"] = {"kernel": "k_sens", "bound": "latency",
                                  "us_per_launch": e0.elapsed_time(e1) * 1e3 / reps,
                                  "gradient_norm": float(np.abs(g).max())}
        else:
            # one call: k_energy, then per pair k_form_pair (M_ab^-1 of every chain) and k_sens_pair,
            # between a device allocation of the pair inverses and a stream synchronisation
            res["sensitivity"] = {"kernel": "k_form_pair + k_sens_pair", "bound": "latency",
                                  "us_per_call": e0.elapsed_time(e1) * 1e3 / reps,
                                  "gradient_norm": float(np.abs(g).max())}
    return res


def synth_gamma_loc(args):
    import synth
    return synth.make_tensor(args.L, K=args.K, group=args.group).gamma_loc


def run_plain(args, with_cpu=True):
    """Single-link sweeps of the c2 / c3 / c4 workloads: one JSON record."""
    import torch
    import synth
    from paper_2412_01737_amd.ggf import Context, autocorr_time, OBS_LINK, OBS_DENSITY, GGF_NOBS

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    L, K, group = args.L, args.K, args.group
    ctx = Context(0)
    if args.workload == "c4":
        Ls, Ks, groups = synth.mixed_batch(args.chains)
        ids = {}
        keys = list(zip(Ls.tolist(), Ks.tolist(), groups.tolist()))
        for key in sorted(set(keys)):
            # one ansatz per (L, K, group), its patch links drawn on its own lattice
            ids[key] = ctx.set_tensor_spec(synth.make_tensor(key[0], K=key[1], group=key[2]))
        Lc = Ls
        tids = np.array([ids[key] for key in keys], np.int32)
    else:
        Lc = np.full(args.chains, L, np.int32)
        tids = ctx.set_tensor_spec(synth.make_tensor(L, K=K, group=group))
    n_c = 8 * Lc.astype(np.int64) ** 2
    n = int(n_c.max())
    t_init = time.perf_counter()
    ctx.init_chains(Lc, tids, synth.SEED_CHAIN, init=1, precision=args.precision,
                    refresh_every=args.refresh, stream=stream)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t_init
    ctx.set_option("delay", args.delay)
    if args.update_grid:
        ctx.set_option("update_grid", args.update_grid)
    if args.update_tiles:
        ctx.set_option("update_tiles", args.update_tiles)
    if args.flush_grid:
        ctx.set_option("flush_grid", args.flush_grid)
    ctx.set_option("update_nt", args.update_nt)
    tuned = None
    if args.autotune:
        # after the delay window is set: the tuner times the launch shapes of the path that runs
        tuned = ctx.autotune(args.autotune, os.path.join(HERE, "paper_2412_01737_amd", "autotune_cache.txt"),
                             stream=stream)
    ctx.set_option("graph", args.graph)
    ctx.set_option("balance", args.balance)
    mask = OBS_LINK | OBS_DENSITY
    obs = torch.zeros((args.warmup + args.steps, args.chains, GGF_NOBS), dtype=torch.float64, device=dev)
    for w in range(args.warmup):
        ctx.sweep(1, stream=stream)
        ctx.measure(mask, obs[w], stream=stream)
    st0 = [ctx.get_state(c)[1] for c in range(args.chains)]
    # per-kernel HIP events are recorded only on eager launches: with graph replay the timed sweeps
    # run as graphs (timed by the host clock) and the kernel times come from eager sweeps afterwards
    ctx.set_option("time_update", 0 if args.graph else 1)
    upd_ms, upd_launches, upd_flips = 0.0, 0, 0
    rat_ms, rat_launches = 0.0, 0
    acc0 = sum(st["accepts"] for st in st0)

    def timings():
        nonlocal upd_ms, upd_launches, upd_flips, rat_ms, rat_launches
        ms, la, fl = ctx.update_timing()
        upd_ms += ms
        upd_launches += la
        upd_flips += fl
        ms, la = ctx.ratio_timing()
        rat_ms += ms
        rat_launches += la

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ctx.sweep(1, stream=stream)
        if not args.graph:
            timings()
        ctx.measure(mask, obs[args.warmup + s], stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st1 = [ctx.get_state(c)[1] for c in range(args.chains)]
    drift = float32_drift(ctx, stream) if args.precision == 32 else None
    refresh = refresh_correction(ctx, args, st0, stream, st1)
    kernel_sweeps = args.steps
    kernel_flips = upd_flips                   # accepted flips of the sweeps whose kernels were timed
    if args.graph:
        # graph replays are timed with host clocks; the kernels of two further eager sweeps with
        # HIP events (their flips, not the timed sweeps', go with their launches)
        upd_flips_timed = sum(ctx.get_state(c)[1]["accepts"] for c in range(args.chains)) - acc0
        ctx.set_option("time_update", 1)
        kernel_sweeps = 2
        upd_flips = 0
        for _ in range(kernel_sweeps):
            ctx.sweep(1, stream=stream)
            timings()
        kernel_flips = upd_flips
        upd_flips = upd_flips_timed
    electric = electric_measurement(ctx, args, Lc, stream)
    energy = energy_measurement(ctx, args, stream)
    lambda_opt = None
    if args.lambda_iters > 0 and args.workload != "c4" and args.K > 1:
        torch.cuda.synchronize()
        t_opt = time.perf_counter()
        en_, eo_, lam_ = ctx.optimise_lambda(int(tids), BENCH_COUPLINGS, args.lambda_iters, args.lambda_sweeps,
                                             args.K, stream=stream)
        t_opt = time.perf_counter() - t_opt
        lambda_opt = {"rounds": args.lambda_iters, "sweeps_per_round": args.lambda_sweeps,
                      "s_per_round": t_opt / args.lambda_iters, "energy_per_round": en_.tolist(),
                      "optimum_per_round": eo_.tolist(), "lambda_re": lam_.real.tolist(),
                      "lambda_im": lam_.imag.tolist(), "couplings": BENCH_COUPLINGS}
    gamma_opt = None
    if args.gamma_iters > 0 and args.workload != "c4":
        torch.cuda.synchronize()
        t_opt = time.perf_counter()
        en_, gn_, _ = ctx.optimise_gamma(int(tids), BENCH_COUPLINGS, args.gamma_iters, args.lambda_sweeps,
                                         args.gamma_step, stream=stream)
        t_opt = time.perf_counter() - t_opt
        gamma_opt = {"rounds": args.gamma_iters, "sweeps_per_round": args.lambda_sweeps, "step": args.gamma_step,
                     "s_per_round": t_opt / args.gamma_iters, "energy_per_round": en_.tolist(),
                     "grad_norm_per_round": gn_.tolist(), "couplings": BENCH_COUPLINGS}
    timed_s = elapsed
    elapsed = elapsed + refresh["correction_ms"] * 1e-3
    # with balanced sweeps every chain proposes a link at every one of the max_links link steps
    per_sweep = (int(2 * Lc.astype(np.int64).max() ** 2) * args.chains if args.balance
                 else int((2 * Lc.astype(np.int64) ** 2).sum()))
    proposals = per_sweep * args.steps
    value = proposals / elapsed
    series = obs[args.warmup:].cpu().numpy()
    plaq_stats = statistics(series[:, :, 0], elapsed)
    dens_stats = statistics(series[:, :, 2], elapsed)
    acceptance = upd_flips / proposals
    esz = 8 if args.precision == 64 else 4
    if args.workload == "c4":
        # flips per chain are not tracked by the timer: weight each chain's bytes by its accepted flips
        acc = np.array([ctx.get_state(c)[1]["accepts"] for c in range(args.chains)], np.float64)
        bytes_per_flip = float((acc * 2.0 * n_c.astype(np.float64) ** 2 * esz).sum() / max(acc.sum(), 1.0))
    else:
        bytes_per_flip = 2.0 * n * n * esz
    F = args.delay
    if F > 0:
        # delayed updates: the dominant kernel is the window flush (the matrix-core k_window_gemm
        # on the upper triangle, mirrored): per chain with a pending flip in the window (at these
        # acceptances, every window it has link steps in) the upper triangle of G read once,
        # n (n + 1) / 2 elements, and all of G written once, n^2; the reads of P = G[A,:] (r n
        # elements, copied by the link steps) are not counted
        nl_c = 2 * Lc.astype(np.int64) ** 2
        windows = -(-int(nl_c.max()) // F)
        # the fraction of windows in which a chain has link steps (all of them with balanced sweeps)
        share = np.ones(len(nl_c)) if args.balance else np.minimum(-(-nl_c // F), windows) / windows
        nf_ = n_c.astype(np.float64)
        bytes_per_launch = float((share * (nf_ * (nf_ + 1) / 2 + nf_ ** 2) * esz).sum())
        kernel = "k_window_flush"
    else:
        bytes_per_launch = kernel_flips * bytes_per_flip / max(upd_launches, 1)
        kernel = "k_update"
    achieved = bytes_per_launch / (upd_ms / upd_launches * 1e-3) / 1e9 if upd_ms > 0 else 0.0
    traffic = None
    try:
        with open(args.traffic_json) as f:
            tj = json.load(f)
        key = traffic_key(args)
        if key in tj and tj[key].get("source_digest") == source_digest(KERNEL_SOURCE[kernel]):
            traffic = tj[key]["bytes_per_launch"]
    except (OSError, ValueError):
        pass
    cpu = None
    if with_cpu and not args.no_cpu and args.workload != "c4":
        cpu = cpu_baseline(args, args.cpu_seconds)
    mean_obs = obs[args.warmup:].mean(dim=(0, 1)).cpu().numpy()
    out = {
        "metric": "link-update proposals/sec and effective samples/sec at fixed obs. error, 1 MI355X",
        "value": value,
        "unit": "proposals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 64 else "f32",
        "data": "synthetic",
        "config": {"workload": (f"Z{group} {L}x{L} periodic, K={K}, {args.chains} chains, single-link Metropolis, "
                                f"float{args.precision} inverse, float64 refresh every {args.refresh} accepted flips")
                   if args.workload != "c4" else
                   (f"{args.chains} chains, L in {{6,8,12,16,20}}, K in {{1,2,4}}, Z2/Z3 (uniform from seed), "
                    f"single-link Metropolis, float{args.precision} inverse, float64 refresh every {args.refresh} "
                    f"accepted flips"),
                   "name": args.workload, "L": L, "K": K, "group": group, "chains": args.chains, "n_max": n,
                   "precision": args.precision, "refresh_every": args.refresh, "graph": args.graph,
                   "balance": args.balance,
                   "delay_window": F, "autotuned": list(tuned) if tuned else None},
        "effective_samples_per_s": plaq_stats["effective_samples_per_s"],
        "plaquette": plaq_stats,
        "density": dens_stats,
        "acceptance": acceptance,
        "observables_mean": {"plaquette": float(mean_obs[0]), "wilson2x2": float(mean_obs[1]),
                             "density": float(mean_obs[2])},
        "init_s": t_init,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "algorithmic_bytes_per_launch": bytes_per_launch,
                     "update_ms_total": upd_ms, "update_launches": upd_launches, "flips": upd_flips,
                     "kernel_timed_flips": kernel_flips},
        "kernels_ms_per_step": {kernel: upd_ms / kernel_sweeps, "k_ratio": rat_ms / kernel_sweeps},
        "timed_s": timed_s,
        "refresh": refresh,
        "float32_drift": drift,
        "electric": electric,
        "energy": energy,
        "lambda_opt": lambda_opt,
        "gamma_opt": gamma_opt,
        "cpu_baseline": cpu,
    }
    return out


def run_north(args):
    """The default run: the c5 comparison (headline), the c2 plain float64 leg, the CPU oracle legs."""
    import torch

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    a2 = c2_args(args)
    log("north: 8x8 plain float64 leg")
    c2 = run_plain(a2, with_cpu=False)
    torch.cuda.synchronize()
    log("north: 32x32 learned-proposal comparison")
    out = run_c5(args)
    params = out.pop("_params", None)
    cpu = None
    if not args.no_cpu:
        log("north: CPU oracle legs")
        c2["cpu_baseline"] = cpu_baseline(a2, args.cpu_seconds)
        out["_params"] = params
        cpu = cpu_baseline_c5(args, 2.0 * args.cpu_seconds, out)
        out.pop("_params", None)
    for rec in (out.get("learned"), out.get("untrained_block"), out.get("plain_f64_single_link")):
        if rec:
            rec.pop("final_chain0", None)
    out["cpu_baseline"] = cpu
    out["plain_f64_c2"] = c2
    print(json.dumps(out))


def main():
    args = parse()
    if args.traffic_from:
        traffic_from(args)
        return
    if args.electric_traffic_from:
        electric_traffic_from(args)
        return
    if args.block_traffic_from:
        block_traffic_from(args)
        return
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: --gpus {args.gpus} is not supported (chains are independent and "
              "would shard by contiguous ranges of chains with one reduction of the observables, but that "
              "path is not built)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "north":
        run_north(args)
        return
    if args.workload == "c5":
        out = run_c5(args)
        out.pop("_params", None)
        for rec in (out.get("learned"), out.get("untrained_block"), out.get("plain_f64_single_link")):
            if rec:
                rec.pop("final_chain0", None)
        print(json.dumps(out))
        return
    print(json.dumps(run_plain(args)))


if __name__ == "__main__":
    main()
