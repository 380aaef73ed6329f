#!/usr/bin/env python3
"""Benchmark: single-link Metropolis sweeps of gauged Gaussian fermionic PEPS on one MI355X.

Workload (default): Z2 gauge field on an 8x8 periodic lattice (128 links,
n = 512 virtual Majoranas), the seeded Haar on-site Gaussian tensor, K = 1,
4096 independent chains, float64 inverse with a float64 refactorisation every
16384 accepted flips per chain (about 130 sweeps; the float64 drift over such
an interval is below 1e-13 in log W).  Refactorisations are charged at their
true rate: the timed sweeps are corrected by the difference between the
refactorisations they contain and that rate, at the measured cost of one.  A step is one sweep of every chain (128
proposals each: ratio and Metropolis decision on the current inverse, the
Woodbury factors of an accepted flip kept pending, and one matrix-core flush
of the pending flips per window of 16 link steps) followed by the plaquette /
2x2 Wilson loop / density measurement.

Prints one JSON line: link-update proposals per second (value), effective
samples per second of the lattice-mean plaquette, the HBM roofline of the
dominant kernel (the window flush: per window, every chain's upper triangle of
G read once and all of G written once, since G is antisymmetric; time: HIP
events around every flush launch on its stream; with
--delay 0 the rank-4 update, 2 n^2 * 8 bytes per accepted flip), the time of
the ratio kernels, and the CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
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
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5"],
                    help="c2: 8x8 Z2 K=1 4096 chains float64 (default, the headline workload); "
                         "c3: 16x16 Z2 K=3 2048 chains float32 + float64 refresh; "
                         "c4: 8192 chains, L in {6,8,12,16,20}, K in {1,2,4}, Z2/Z3, float32 + refresh, "
                         "graph-replayed autotuned sweeps; "
                         "c5: 32x32 Z2 K=2 256 chains, learned 4x4-patch block proposal trained online on the "
                         "plain sampler, float32 + float64 refresh, vs the plain float64 single-link sampler")
    ap.add_argument("--train-chains", type=int, default=32, help="c5: chains of the plain sampler the net trains on")
    ap.add_argument("--train-sweeps", type=int, default=3, help="c5: plain-sampler sweeps of online training")
    ap.add_argument("--train-steps", type=int, default=40, help="c5: Adam steps after each training sweep")
    ap.add_argument("--plain-chains", type=int, default=64, help="c5: chains of the float64 single-link comparison")
    ap.add_argument("--plain-steps", type=int, default=4, help="c5: timed sweeps of the float64 single-link comparison")
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
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--delay", type=int, default=None,
                    help="window of delayed updates in link steps (0 = one rank-4 pass per accepted flip; "
                         "default: the library's)")
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
                    help="after the timed sweeps, rounds of gradient descent on Gamma_A (L <= 16 for K = 1, "
                         "L <= 8 for K > 1; --lambda-sweeps sweeps per round, --gamma-step), reported under "
                         "'gamma_opt'")
    ap.add_argument("--gamma-step", type=float, default=0.01)
    ap.add_argument("--electric-traffic-from", nargs=4,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="derive the electric measurement kernel's HBM bytes per launch from rocprofv3 --pmc "
                         "CSVs, write profiles/k_electric_traffic.json and exit (no GPU needed)")
    args = ap.parse_args()
    presets = {
        "c2": dict(steps=20, warmup=3, chains=4096, L=8, K=1, group=2, precision=64, refresh=16384, delay=16),
        "c3": dict(steps=3, warmup=1, chains=2048, L=16, K=3, group=2, precision=32, refresh=64, delay=16),
        "c4": dict(steps=2, warmup=1, chains=8192, L=0, K=0, group=0, precision=32, refresh=64, delay=16),
        "c5": dict(steps=8, warmup=1, chains=256, L=32, K=2, group=2, precision=32, refresh=4096, delay=16),
    }
    for k, v in presets[args.workload].items():
        if getattr(args, k) is None:
            setattr(args, k, v)
    return args


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
    """HBM bytes per accepted block move of k_window_snap + k_window_gemm, from FETCH_SIZE / WRITE_SIZE.

    Counters are scaled by the copy calibration as in traffic_from; the number of
    accepted moves per launch comes from the profiled run's own JSON line."""
    import csv

    def per_kernel(path, counter, match):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                if r["Counter_Name"] == counter and match in r["Kernel_Name"]]
        return vals

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
    moves_per_launch = learned["accepted_moves"] / learned["update_launches"]
    out = {"source_digest": source_digest(BLOCK_SOURCES), "moves_per_launch": moves_per_launch,
           "fetch_scale": sf, "write_scale": sw}
    total = 0.0
    tname = "float" if rec["config"]["precision"] == 32 else "double"
    # block moves only: k_window_snap and the <T, 8, true> instance of k_window_gemm (the training
    # sampler's window flushes run <T, 4, false>)
    for k in (f"k_window_snap<{tname}>", f"k_window_gemm<{tname}, 8, true>"):
        fv, wv = per_kernel(f_csv, "FETCH_SIZE", k), per_kernel(w_csv, "WRITE_SIZE", k)
        rd = sum(fv) / len(fv) * sf * 1024.0
        wr = sum(wv) / len(wv) * sw * 1024.0
        out[k.split("<")[0]] = {"read_bytes_per_launch": rd, "write_bytes_per_launch": wr,
                                "dispatches": [len(fv), len(wv)]}
        total += rd + wr
    n = rec["config"]["n"]
    esz = 4 if rec["config"]["precision"] == 32 else 8
    out["bytes_per_accepted_move"] = total / moves_per_launch
    out["algorithmic_bytes_per_accepted_move"] = (n * (n + 1) / 2 + n * n) * esz
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
    for mode, name, moved in ((0, "copy", 2), (1, "copy_nt", 2), (2, "rmw", 2), (3, "rmw_nt", 2)):
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


def refresh_correction(ctx, args, st0, stream):
    """Float64 refactorisations charged at their true rate.

    A chain is refactorised at the first sweep end after refresh_every accepted
    flips, i.e. every ceil(refresh_every / flips per sweep) sweeps.  The timed
    sweeps contain however many refactorisations their alignment gives; the
    difference to the true rate is charged (or credited) at the measured cost
    of refactorising all chains, timed here after the timed region."""
    import torch
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


def cpu_baseline(args, budget_s: float):
    """The oracle's Woodbury chain on host cores, one chain per worker process, bounded in time."""
    import multiprocessing as mp
    workers = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers, initializer=_cpu_init) as pool:
        res = pool.starmap(_cpu_chain, [(args.L, args.K, args.group, c, budget_s) for c in range(workers)])
    wall = time.perf_counter() - t0
    props = sum(r[0] for r in res)
    sweeps = sum(r[1] for r in res)
    return {"value": props / wall, "unit": "proposals/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} chains x {sweeps // workers}-{max(r[1] for r in res)} sweeps of L={args.L} "
                      f"K={args.K} Z{args.group} (Woodbury-mode oracle, float64, 1 BLAS thread per process), "
                      f"{wall:.1f} s wall"}


def _cpu_init():
    try:
        import threadpoolctl
        threadpoolctl.threadpool_limits(1)
    except Exception:
        pass


def _cpu_chain(L, K, group, chain, budget_s):
    import synth
    from oracle.chain import WoodburyChain
    from oracle.lattice import Lattice
    from oracle.model import Ansatz
    spec = synth.make_tensor(L, K=K, group=group)
    an = Ansatz(Lattice(L, L), spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k, spec.c)
    ch = WoodburyChain(an, synth.SEED_CHAIN, chain, refresh_every=1024)
    t0 = time.perf_counter()
    sweeps = 0
    while time.perf_counter() - t0 < budget_s or sweeps == 0:
        ch.sweep()
        sweeps += 1
    return ch.proposals, sweeps


NN_SEED = 7
MFMA_PEAK_F32_TFLOPS = 157.3


def run_c5(args):
    """Learned block proposal (4x4-site patches) vs the plain float64 single-link sampler, one GPU.

    1. Online training: a plain float32 single-link sampler on --train-chains
       chains; after each of its sweeps the network takes --train-steps Adam
       steps on (window, patch) examples of its current link fields.
    2. The learned sampler: --chains chains, one block sweep = one
       Metropolis-Hastings block move on every patch, float32 inverse with a
       float64 refactorisation every --refresh changed links; the plaquette
       is measured after every sweep.
    3. The plain float64 single-link sampler on the same GPU (--plain-chains
       chains, --plain-steps sweeps), measured the same way.
    Effective samples per second = chains * sweeps / (2 tau_int) / wall time."""
    import torch
    import synth
    from paper_2412_01737_amd.ggf import Context, autocorr_time, OBS_LINK, GGF_NOBS

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    L, K, group, P = args.L, args.K, args.group, 4
    n = 8 * L * L
    spec = synth.make_tensor(L, K=K, group=group)

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
    params = tr.nn_params()
    tr.close()
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0

    def sampler(chains, precision, refresh, learned, steps, warmup):
        ctx = Context(0)
        ctx.set_option("delay", args.delay)
        tid = ctx.set_tensor_spec(spec)
        ti = time.perf_counter()
        ctx.init_chains([L] * chains, tid, synth.SEED_CHAIN, init=1, precision=precision,
                        refresh_every=refresh, stream=stream)
        if learned:
            ctx.nn_init(P, NN_SEED)
            ctx.nn_params(params)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - ti
        step = (lambda: ctx.block_sweep(1, stream=stream)) if learned else (lambda: ctx.sweep(1, stream=stream))
        for w in range(warmup):
            step()
            torch.cuda.synchronize()
            log(f"c5 {'learned' if learned else 'plain'} warmup sweep {w + 1}/{warmup}")
        before = [ctx.block_stats(c) for c in range(chains)] if learned else None
        acc_before = sum(ctx.get_state(c)[1]["accepts"] for c in range(chains)) if not learned else 0
        ctx.set_option("time_update", 1)
        obs = torch.zeros((steps, chains, GGF_NOBS), dtype=torch.float64, device=dev)
        upd_ms, launches, changed = 0.0, 0, 0
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for s in range(steps):
            step()
            ms, la, fl = ctx.update_timing()
            upd_ms, launches, changed = upd_ms + ms, launches + la, changed + fl
            ctx.measure(OBS_LINK, obs[s], stream=stream)
            log(f"c5 {'learned' if learned else 'plain'} sweep {s + 1}/{steps}")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - ts
        series = obs[:, :, 0].cpu().numpy()
        tau, tau_err = autocorr_time(series)[:2] if steps >= 2 else (float("nan"), float("nan"))
        rec = {"chains": chains, "sweeps": steps, "s_per_sweep": elapsed / steps, "init_s": t_init,
               "tau_int_plaquette": tau, "tau_int_err": tau_err,
               "effective_samples_per_s": steps * chains / (2.0 * tau) / elapsed,
               "plaquette_mean": float(series.mean()), "update_ms_total": upd_ms, "update_launches": launches,
               "links_changed": changed}
        if learned:
            after = [ctx.block_stats(c) for c in range(chains)]
            prop = sum(a[0] - b[0] for a, b in zip(after, before))
            acc = sum(a[1] - b[1] for a, b in zip(after, before))
            rec.update(acceptance=acc / max(prop, 1), links_per_accepted_move=changed / max(acc, 1), accepted_moves=acc,
                       link_proposals_per_s=chains * steps * 2 * L * L / elapsed)
        else:
            acc = sum(ctx.get_state(c)[1]["accepts"] for c in range(chains)) - acc_before
            rec.update(acceptance=acc / (chains * steps * 2 * L * L),
                       link_proposals_per_s=chains * steps * 2 * L * L / elapsed)
        ctx.close()
        torch.cuda.synchronize()
        return rec

    learned = sampler(args.chains, args.precision, args.refresh, True, args.steps, args.warmup)
    plain = sampler(args.plain_chains, 64, 1024, False, args.plain_steps, 1) if args.plain_steps > 0 else None
    # block update G -= G[:,U] W G[U,:] per accepted move of m changed links (rank r = 4 m), on the
    # upper triangle of the antisymmetric G and mirrored: algorithmic bytes = the upper triangle read
    # and all of G written ((n (n + 1) / 2 + n^2) * 4), flops = n^2 r
    esz = 4 if args.precision == 32 else 8
    upd_s = learned["update_ms_total"] * 1e-3
    bytes_moved = (n * (n + 1) / 2 + n * n) * esz * learned["accepted_moves"]
    flops = n * n * 4.0 * learned["links_changed"]
    achieved = bytes_moved / upd_s / 1e9 if upd_s > 0 else 0.0
    tflops = flops / upd_s / 1e12 if upd_s > 0 else 0.0
    traffic = None
    try:
        with open(os.path.join(HERE, "profiles", "k_block_traffic.json")) as f:
            tj = json.load(f).get(f"L{L}_K{K}_Z{group}_p{args.precision}")
        if tj and tj["source_digest"] == source_digest(BLOCK_SOURCES):
            # measured bytes per accepted move x accepted moves per launch of this run
            traffic = tj["bytes_per_accepted_move"] * learned["accepted_moves"] / learned["update_launches"]
    except (OSError, ValueError, KeyError):
        pass
    out = {
        "metric": "link-update proposals/sec and effective samples/sec at fixed obs. error, 1 MI355X",
        "value": learned["effective_samples_per_s"],
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
                                f"refresh every {args.refresh} changed links; vs the plain float64 single-link "
                                f"sampler (delayed updates, window {args.delay}) on {args.plain_chains} chains"),
                   "name": "c5", "L": L, "K": K, "group": group, "chains": args.chains, "n": n, "patch": P,
                   "precision": args.precision, "refresh_every": args.refresh},
        "learned": learned,
        "plain_f64_single_link": plain,
        "ess_ratio_learned_vs_plain": (learned["effective_samples_per_s"] / plain["effective_samples_per_s"]
                                       if plain else None),
        "training": {"chains": args.train_chains, "sweeps": args.train_sweeps, "adam_steps_per_sweep": args.train_steps,
                     "loss_nats_per_patch": losses, "seconds": t_train},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_window_snap + k_window_gemm (block moves)",
                     "algorithmic_bytes_per_launch": bytes_moved / max(learned["update_launches"], 1),
                     "bytes_per_accepted_move": (n * (n + 1) / 2 + n * n) * esz,
                     "tflops": tflops, "mfma_peak_tflops": MFMA_PEAK_F32_TFLOPS,
                     "flops_per_changed_link": 4.0 * n * n},
        "cpu_baseline": None,
    }
    print(json.dumps(out))


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
    if args.workload != "c4" and args.L <= (16 if args.K == 1 else 8):
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
    if args.workload == "c5":
        run_c5(args)
        return
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
        for kk in synth.MIX_K:
            for gg in synth.MIX_GROUP:
                # patch links drawn on the smallest lattice exist on every lattice of the batch
                ids[(kk, gg)] = ctx.set_tensor_spec(synth.make_tensor(min(synth.MIX_L), K=int(kk), group=int(gg)))
        Lc = Ls
        tids = np.array([ids[(int(k), int(g))] for k, g in zip(Ks, groups)], np.int32)
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
    tuned = None
    if args.autotune:
        tuned = ctx.autotune(args.autotune, os.path.join(HERE, "paper_2412_01737_amd", "autotune_cache.txt"),
                             stream=stream)
    if args.update_grid:
        ctx.set_option("update_grid", args.update_grid)
    if args.update_tiles:
        ctx.set_option("update_tiles", args.update_tiles)
    ctx.set_option("graph", args.graph)
    ctx.set_option("delay", args.delay)
    if not args.autotune:
        ctx.set_option("update_nt", args.update_nt)
    mask = OBS_LINK | OBS_DENSITY
    obs = torch.zeros((args.warmup + args.steps, args.chains, GGF_NOBS), dtype=torch.float64, device=dev)
    for w in range(args.warmup):
        ctx.sweep(1, stream=stream)
        ctx.measure(mask, obs[w], stream=stream)
    st0 = [ctx.get_state(c)[1] for c in range(args.chains)]
    ctx.set_option("time_update", 1)
    upd_ms, upd_launches, upd_flips = 0.0, 0, 0
    rat_ms, rat_launches = 0.0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ctx.sweep(1, stream=stream)
        ms, la, fl = ctx.update_timing()
        upd_ms += ms
        upd_launches += la
        upd_flips += fl
        ms, la = ctx.ratio_timing()
        rat_ms += ms
        rat_launches += la
        ctx.measure(mask, obs[args.warmup + s], stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    refresh = refresh_correction(ctx, args, st0, stream)
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
    if args.gamma_iters > 0 and args.workload != "c4" and args.L <= (16 if args.K == 1 else 8):
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
    proposals = int((2 * Lc.astype(np.int64) ** 2).sum()) * args.steps
    value = proposals / elapsed
    series = obs[args.warmup:, :, 0].cpu().numpy()
    if series.shape[0] >= 2:
        tau, tau_err, window = autocorr_time(series)
        ess_per_s = series.shape[0] * series.shape[1] / (2.0 * tau) / elapsed
    else:
        tau = tau_err = ess_per_s = None
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
        share = np.minimum(-(-nl_c // F), windows) / windows
        nf_ = n_c.astype(np.float64)
        bytes_per_launch = float((share * (nf_ * (nf_ + 1) / 2 + nf_ ** 2) * esz).sum())
        kernel = "k_window_flush"
    else:
        bytes_per_launch = upd_flips * bytes_per_flip / max(upd_launches, 1)
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
    if not args.no_cpu and args.workload != "c4":
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
                   "delay_window": F, "autotuned": list(tuned) if tuned else None},
        "effective_samples_per_s": ess_per_s,
        "tau_int_plaquette": tau,
        "tau_int_err": tau_err,
        "acceptance": acceptance,
        "observables_mean": {"plaquette": float(mean_obs[0]), "wilson2x2": float(mean_obs[1]),
                             "density": float(mean_obs[2])},
        "init_s": t_init,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "algorithmic_bytes_per_launch": bytes_per_launch,
                     "update_ms_total": upd_ms, "update_launches": upd_launches, "flips": upd_flips},
        "kernels_ms_per_step": {kernel: upd_ms / args.steps, "k_ratio": rat_ms / args.steps},
        "timed_s": timed_s,
        "refresh": refresh,
        "electric": electric,
        "energy": energy,
        "lambda_opt": lambda_opt,
        "gamma_opt": gamma_opt,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
