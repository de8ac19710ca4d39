"""Throughput benchmark of the REWL hot path on one MI355X.

A step is one REWL cycle over the whole batch: rewl_run_sweeps(F) (every
walker makes F Wang-Landau attempts), rewl_merge (flatness test and in-window
merge) and rewl_exchange (one replica-exchange round).  The workload is the
2D Ising L=32 REWL configuration (16 windows x 8 walkers, 75 % overlap,
flatness 0.8, exchange every 10^4 flips, FP64 ln g) replicated R times as
independent instances so that the chip is filled; each copy carries its
instance index in every random-number counter.  The launch shape is chosen
by rewl_autotune after the warm-up steps, on the state the timed steps start
from (untimed; it saves the whole state first and restores it).

Printed: one JSON line with spin-flip attempts/s, the sweep kernel's
roofline position (kernel time from HIP events recorded on the library's
stream); after the timed region, the time to converge of 8 Ising L=8
instances and of 8 Ising L=32 instances to ln f = 1e-8 in FP64 and in
two-float FP32 (the same instances, on the balanced split), each with its
error against the exact density of states, the autotuned throughput of
the batched 64-instance mix; and the CPU oracle's
attempts/s on a bounded sample, on one pinned core (Ising L=32, and q=10
Potts L=20 in FP64 and FP32) and on every host core (one independent
instance per process).  Progress lines go to stderr.

--workload potts10 (q=10 Potts L=20, filled with copies) or mix (the batched
64-instance mix) measures the other forms; --precision fp32c the two-float
FP32 ln g.

--converge --config {ising8,ising32,potts10,potts10-both} [--schedule
halving|1t] runs R
copies of a configuration to ln f <= ln f_final and reports time to
convergence and the C_V peak (Potts); potts10-both runs the q=10 Potts instances in
FP64 and in two-float FP32 and compares them (progress lines precede the
JSON line).  --balanced first plans run-time balanced windows (Fig. 1b)
from a first-iteration pre-run (--replan: again from a second pre-run on
those windows).  --save keeps the normalised ln g and
jackknife errors for scoring against exact results by
tests/converge_report.py.
"""
import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures used for the roofline: 256 compute units at 2.4 GHz.
N_CU = 256
CLOCK_HZ = 2.4e9
VALU_LANE_OPS_PER_CLK_PER_CU = 64          # 4 SIMD x 16 lanes, full-rate 32-bit / FP64 ops
PEAK_VALU = N_CU * VALU_LANE_OPS_PER_CLK_PER_CU * CLOCK_HZ   # 3.93e13 lane-op/s
# Algorithmic VALU work of one attempt in full-rate lane-op slots:
# Philox4x32-10 60 (20 32x32->64 multiplies, one slot each since the wide
# multiply issues at the full rate on gfx950, see --alu-rate, and 40
# two-input xors), site and neighbour indexing 24, energy change and window
# test 8, acceptance with the exponential 26, update 8.
VALU_SLOTS_PER_ATTEMPT = 126
# Algorithmic LDS bytes of one attempt (Ising L=32): three 4-byte lattice rows
# read, 8 B ln g read, 8 B ln g written, 4 B histogram read-modify-write
# (counted 8), 4 B lattice row written on acceptance (~0.5).
LDS_BYTES_PER_ATTEMPT = 38.0
PEAK_LDS = N_CU * 128 * CLOCK_HZ            # 128 B/clk/CU
PROFILE = os.path.join(ROOT, "profiles", "k_sweep_ising_L32_pmc.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--replicas", type=int, default=None,
                    help="instances (default: 1024 for the throughput run, 8 for --converge, "
                         "32 per h for --speedup)")
    ap.add_argument("--flips", type=int, default=10000)
    ap.add_argument("--precision", choices=["fp64", "fp32c"], default="fp64")
    ap.add_argument("--workload", choices=["ising32", "potts10", "mix"], default="ising32",
                    help="throughput run: Ising L=32 (default), q=10 Potts L=20, or the "
                         "64-instance batched mix")
    ap.add_argument("--page-bins", type=int, default=0,
                    help="fixed ln g page size for the sweep (0: autotune)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--solo", type=int, default=0,
                    help="--workload mix: also time this many instances alone")
    ap.add_argument("--no-ttc", action="store_true",
                    help="skip the time-to-converge run (Ising L=8) after the throughput run")
    ap.add_argument("--no-ttc32", action="store_true",
                    help="skip the Ising L=32 time to ln f = 1e-8 (FP64 and FP32C, ~3 minutes)")
    ap.add_argument("--converge", action="store_true")
    ap.add_argument("--config", choices=["ising8", "ising32", "potts10", "potts10-both"],
                    default="ising32")
    ap.add_argument("--max-minutes", type=float, default=50.0)
    ap.add_argument("--schedule", choices=["halving", "1t"], default="halving")
    ap.add_argument("--speedup", action="store_true")
    ap.add_argument("--L", type=int, default=32, help="lattice size (--speedup)")
    ap.add_argument("--q", type=int, default=2, help="--speedup: q > 2 runs q-state Potts")
    ap.add_argument("--hs", default="1,2,4,8,16,32", help="window counts (--speedup)")
    ap.add_argument("--walkers", type=int, default=None,
                    help="walkers per window (--speedup: default 1; --converge: the config's)")
    ap.add_argument("--alpha", type=float, default=2.0, help="cost exponent of the balanced split")
    ap.add_argument("--lnf-final", type=float, default=0.0,
                    help="override ln f_final of the configuration (--converge)")
    ap.add_argument("--save", default="", help="npz for ln g and jackknife errors (--converge)")
    ap.add_argument("--balanced", action="store_true",
                    help="--converge on the run-time balanced split planned from a pre-run")
    ap.add_argument("--replan", action="store_true",
                    help="--balanced: plan again from a second pre-run on the planned windows")
    ap.add_argument("--copy-reference", action="store_true",
                    help="only copy a 512 MiB device buffer 3 times (HBM counter calibration)")
    ap.add_argument("--alu-rate", action="store_true",
                    help="only measure the issue cost of the VALU forms the sweep uses")
    return ap.parse_args()


def progress(**kw):
    """A progress line on stderr (the JSON result line alone goes to stdout)."""
    print(json.dumps(kw), file=sys.stderr, flush=True)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo where it exists)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


ORACLE_CONFIGS = {"ising32": ("ISING_L32", "Ising L=32 REWL (16 windows x 8 walkers)"),
                  "potts10": ("POTTS_Q10_L20", "q=10 Potts L=20 REWL (32 windows x 16 walkers)"),
                  "potts10_fp32c": ("POTTS_Q10_L20_FP32C",
                                    "q=10 Potts L=20 REWL (32 windows x 16 walkers), two-float FP32")}


def _oracle_worker(args):
    """Cycles of one oracle instance for `seconds` (pinned to `core` when
    given); returns attempts made, the time taken and the core it ran on."""
    name, inst, flips, seconds, core = args
    if core is not None:
        os.sched_setaffinity(0, {core})
    from oracle import oracle as O
    from paper_1402_2328_amd import workloads as WL
    c = getattr(WL, ORACLE_CONFIGS[name][0])
    sim = O.Sim(model=c["model"], L=c["L"], q=c["q"], n_windows=c["n_windows"],
                walkers_per_window=c["walkers_per_window"], lnf_final=c["lnf_final"],
                flips_per_exchange=flips, seed=c["seed"], precision=c["precision"], instance=inst)
    W = c["n_windows"] * c["walkers_per_window"]
    cycles = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        sim.sweep(flips)
        sim.merge()
        sim.exchange()
        cycles += 1
    return cycles * W * flips, time.perf_counter() - t0, sorted(os.sched_getaffinity(0)), cycles


def cpu_baseline(flips, seconds):
    """The oracle on one host core (a child process pinned to the last core
    this process may use), on the Ising L=32 workload and, as context, on
    q=10 Potts L=20 in FP64 and in two-float FP32."""
    import multiprocessing as mp
    core = sorted(os.sched_getaffinity(0))[-1]
    rates = {}
    with mp.get_context("spawn").Pool(1) as pool:
        for name in ORACLE_CONFIGS:
            sec = seconds if name == "ising32" else 2.0 * seconds / 3.0
            att, dt, aff, cycles = pool.apply(_oracle_worker, ((name, 0, flips, sec, core),))
            assert aff == [core]
            rates[name] = (att / dt, dt, cycles)
    v, dt, cycles = rates["ising32"]
    return {"value": v, "unit": "attempts/s", "cores": 1, "kind": "oracle",
            "sample": f"{ORACLE_CONFIGS['ising32'][1]}, {cycles} cycles of {flips} attempts per "
                      f"walker from a fresh start, one thread pinned to core {core}, {dt:.1f} s",
            "cpu": cpu_model(), "host_cpus": os.cpu_count(), "pinned_core": core,
            "other_workloads": {n: {"value": r[0], "unit": "attempts/s", "seconds": r[1],
                                    "cycles": r[2], "workload": ORACLE_CONFIGS[n][1]}
                                for n, r in rates.items() if n != "ising32"}}


def cpu_baseline_all_cores(flips, seconds, max_procs=16):
    """The oracle on every host core at once: independent Ising L=32 instances, one
    process each (at most max_procs, the host share of one GPU)."""
    import multiprocessing as mp
    n = max(1, min(max_procs, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(n) as pool:
        res = pool.map(_oracle_worker, [("ising32", i, flips, seconds, None) for i in range(n)])
    wall = time.perf_counter() - t0
    att = sum(r[0] for r in res)
    span = max(r[1] for r in res)
    return {"value": att / span, "unit": "attempts/s", "cores": n, "kind": "oracle",
            "sample": f"{n} independent Ising L=32 REWL instances (16 windows x 8 walkers), one "
                      f"process each, {seconds:.0f} s of cycles of {flips} attempts per walker "
                      f"from a fresh start ({wall:.1f} s wall with start-up)"}


def traffic_from_profile(R, flips, page):
    """HBM bytes per sweep launch from the committed rocprofv3 counters, if
    they were taken on the current kernel sources and workload (else None)."""
    try:
        prof = json.load(open(PROFILE))
    except (OSError, ValueError):
        return None
    csrc = os.path.join(ROOT, "paper_1402_2328_amd", "csrc")
    for key, name in (("source_sha256", "rewl_sweep.hip"), ("device_h_sha256", "rewl_device.h")):
        if prof.get(key) != hashlib.sha256(open(os.path.join(csrc, name), "rb").read()).hexdigest():
            return None
    if prof.get("replicas") != R or prof.get("flips") != flips or prof.get("page_bins") != page:
        return None
    return (prof["fetch_kib"] * prof["fetch_scale"] + prof["write_kib"] * prof["write_scale"]) * 1024


def run_to_convergence(ctx, R, flips, max_s, tag, quiet=False):
    """Cycles until every instance is finished or has failed (or max_s);
    returns the wall time at which each instance finished.  A failed
    instance (an error code in its status) stops advancing; it is reported
    on stderr and not waited for."""
    import torch
    t0 = time.perf_counter()
    cycles = 0
    done_at = {}
    failed = {}
    while True:
        ctx.run_cycles(100, flips, use_graph=True)
        cycles += 100
        torch.cuda.synchronize()
        now = time.perf_counter() - t0
        st = [ctx.status(i) for i in range(R)]
        for i, s in enumerate(st):
            if s["error"] and i not in failed:
                failed[i] = int(s["error"])
                progress(run=tag, instance=i, failed=failed[i])
            elif s["done"] and i not in done_at:
                done_at[i] = now
        if not quiet and (cycles % 1000 == 0 or len(done_at) == R):
            stages = np.array([s["stage"].min() for s in st])
            print(json.dumps({"run": tag, "cycles": cycles, "t": round(now, 1), "done": len(done_at),
                              "stage_min": int(stages.min()),
                              "stage_med": float(np.median(stages))}), flush=True)
        if len(done_at) + len(failed) == R or now > max_s:
            return done_at, cycles, now


def exact_ising_lng(L):
    """ln g(E) of the periodic L x L Ising model, E = -2N + 4k, from the
    stored exact table (tests/golden, Kaufman's closed form)."""
    path = os.path.join(ROOT, "tests", "golden", f"ising_dos_L{L}.txt")
    vals = [int(x) for x in open(path) if not x.startswith("#")]
    return np.array([math.log(v) if v else -np.inf for v in vals])


def time_to_converge_ising8(R=8):
    """Ising L=8 REWL (4 windows x 1 walker, halving to ln f = 1e-6, F=1000)
    run R times to convergence: wall time per instance and its max |ln g
    error| against the exact density of states."""
    from paper_1402_2328_amd import rewl
    from paper_1402_2328_amd import workloads as WL
    cfg = WL.ISING_L8
    F = cfg["flips_per_exchange"]
    ctx = rewl.Context([WL.rewl_params_of(cfg)] * R)
    ctx.autotune(F)
    done_at, cycles, wall = run_to_convergence(ctx, R, F, 120, "ising8", quiet=True)
    exact = exact_ising_lng(cfg["L"])
    fin = np.isfinite(exact)
    errs = [float(np.max(np.abs(ctx.get_lng(i)[0][fin] - exact[fin]))) for i in sorted(done_at)]
    ctx.close()
    return {"config": "Ising L=8, 4 windows x 1 walker, ln f 1 -> 1e-6 by halving, F=1000",
            "instances": R, "finished": len(done_at),
            "wall_s_median": float(np.median(list(done_at.values()))) if done_at else None,
            "wall_s_all": wall, "max_abs_err_vs_exact": errs,
            "max_abs_err_median": float(np.median(errs)) if errs else None}


def time_to_converge_ising32(R=8, max_s=420.0):
    """The Ising L=32 REWL configuration (16 windows x 8 walkers, halving to
    ln f = 1e-8, F = 10^4) run to convergence by R instances in FP64 and the
    same R instances (same seeds and instance indices, so the same initial
    states) in two-float FP32, on the run-time balanced split (Fig. 1b)
    planned from a first-iteration pre-run of R other seeds.  The two
    precisions are separate contexts on separate streams, so they sweep side
    by side (each fills only a few of the compute units), and each advances
    at its own pace: a context gets its next 100 cycles as soon as its
    stream has finished the last ones, so neither waits for the other.  Per
    precision: wall time at which each instance finished, and its max |ln g
    error| against the exact density of states."""
    import torch
    from paper_1402_2328_amd import rewl
    from paper_1402_2328_amd import workloads as WL
    base = WL.ISING_L32
    F = base["flips_per_exchange"]
    t_pre = time.perf_counter()
    progress(phase="balanced-split pre-run, Ising L=32", instances=R)
    windows, pre = balanced_split(base, R, 2.0, 60.0, quiet=True)
    pre["wall_s_total"] = time.perf_counter() - t_pre
    runs = {}
    for tag, prec in (("fp64", WL.FP64), ("fp32c", WL.FP32C)):
        stream = torch.cuda.Stream()
        ctx = rewl.Context([WL.rewl_params_of(dict(base, precision=prec))] * R, windows=windows,
                           stream=stream)
        # three sweeps per candidate: with one, the choice between plans
        # within a few per cent of each other is left to chance
        plan = ctx.autotune(F, repeats=3)
        runs[tag] = {"ctx": ctx, "stream": stream, "plan": plan, "done_at": {}, "failed": {},
                     "cycles": 0, "over": False}
    exact = exact_ising_lng(base["L"])
    fin = np.isfinite(exact)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in runs.values():
        r["ctx"].run_cycles(100, F, use_graph=True)
    next_report = 20.0
    while not all(r["over"] for r in runs.values()):
        idle = True
        for r in runs.values():
            if r["over"] or not r["stream"].query():
                continue
            idle = False
            now = time.perf_counter() - t0
            r["cycles"] += 100
            for i in range(R):
                if i in r["done_at"] or i in r["failed"]:
                    continue
                st = r["ctx"].status(i)
                if st["error"]:
                    r["failed"][i] = int(st["error"])   # stops advancing; reported below
                elif st["done"]:
                    r["done_at"][i] = now
            if len(r["done_at"]) + len(r["failed"]) == R or now > max_s:
                r["over"] = True
            else:
                r["ctx"].run_cycles(100, F, use_graph=True)
        if time.perf_counter() - t0 >= next_report:
            next_report += 20.0
            progress(phase="time to converge, Ising L=32", t=round(time.perf_counter() - t0, 1),
                     **{tag: {"cycles": r["cycles"], "done": len(r["done_at"])}
                        for tag, r in runs.items()})
        if idle:
            time.sleep(0.002)
    out = {"config": "Ising L=32, 16 windows x 8 walkers, ln f 1 -> 1e-8 by halving, F=10^4, "
                     "balanced split (Fig. 1b)",
           "instances": R, "balanced_prerun": pre,
           "cycles_polled": {tag: r["cycles"] for tag, r in runs.items()}}
    for tag, r in runs.items():
        ctx, done = r["ctx"], r["done_at"]
        errs = [float(np.max(np.abs(ctx.get_lng(i)[0][fin] - exact[fin]))) for i in sorted(done)]
        out[tag] = {"finished": len(done), "failed": r["failed"], "launch": r["plan"],
                    "wall_s_median": float(np.median(list(done.values()))) if done else None,
                    "wall_s_all": float(max(done.values())) if len(done) == R else None,
                    "cycles_to_converge": [int(ctx.status(i)["done_merge"]) + 1 for i in sorted(done)],
                    "max_abs_err_vs_exact": errs,
                    "max_abs_err_median": float(np.median(errs)) if errs else None}
        ctx.close()
    return out


def mix_throughput(flips, steps=10, warmup=2, repeats=5):
    """The 64-instance batched mix (Ising L 16-64 and q-state Potts q 2-10,
    8-48 windows x 4-16 walkers) in one context: autotuned launch plan
    (median of `repeats` sweeps per candidate), then `steps` timed cycles
    (sweep, merge, exchange)."""
    import torch
    from paper_1402_2328_amd import rewl
    from paper_1402_2328_amd import workloads as WL
    cfgs = [dict(c, flips_per_exchange=flips) for c in WL.batched_mix()]
    ctx = rewl.Context([WL.rewl_params_of(c) for c in cfgs])
    W = sum(c["n_windows"] * c["walkers_per_window"] for c in cfgs)
    for _ in range(warmup):
        ctx.run_cycles(1, flips)
    t0 = time.perf_counter()
    plan = ctx.autotune(flips, repeats=repeats)
    tune_s = time.perf_counter() - t0
    ctx.run_cycles(1, flips)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run_cycles(steps, flips)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    return {"workload": "batched mix of 64 Ising/Potts REWL instances (L 16-64, q 2-10, 8-48 "
                        f"windows x 4-16 walkers), F={flips}", "walkers": W, "steps": steps,
            "attempts_per_s": W * flips * steps / dt, "ms_per_cycle": dt / steps * 1e3,
            "launch": plan, "autotune_s": tune_s, "autotune_repeats": repeats}


def solo_vs_batch(cfgs, n_sample, flips, batch_cycle_s):
    """Time a cycle of n_sample instances of the batch run alone (each in a
    context of its own, autotuned like the batch) and compare the sum over
    the whole batch, estimated from that sample, with the batched cycle."""
    import torch
    from paper_1402_2328_amd import rewl
    from paper_1402_2328_amd import workloads as WL
    rng = np.random.Generator(np.random.PCG64(11))
    pick = sorted(rng.choice(len(cfgs), size=min(n_sample, len(cfgs)), replace=False).tolist())
    solo = []
    for i in pick:
        ctx = rewl.Context([WL.rewl_params_of(cfgs[i])])
        ctx.autotune(flips)
        ctx.run_cycles(1, flips)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.run_cycles(3, flips)
        torch.cuda.synchronize()
        solo.append((time.perf_counter() - t0) / 3)
        ctx.close()
    est = float(np.mean(solo)) * len(cfgs)
    return {"instances_timed_alone": pick, "solo_cycle_s": solo,
            "sequential_cycle_s_estimate": est, "batched_cycle_s": batch_cycle_s,
            "speedup": est / batch_cycle_s}


def cv_peak(ctx, i, T):
    """Peak of C_V(T) per spin on the grid T, refined by a parabola."""
    E, C = ctx.thermo(T, instance=i)
    k = int(np.argmax(C))
    k = min(max(k, 1), len(T) - 2)
    y0, y1, y2 = C[k - 1], C[k], C[k + 1]
    den = y0 - 2 * y1 + y2
    off = 0.5 * (y0 - y2) / den if den != 0 else 0.0
    h = T[1] - T[0]
    return float(T[k] + off * h), float(y1 - 0.25 * (y0 - y2) * off)


def balanced_split(cfg, R, alpha, max_s, quiet=False, replan=False):
    """Run-time balanced windows (Fig. 1b) for `cfg`: a pre-run of R
    instances with the equal split, other seeds, stopped after the first WL
    iteration (ln f_final = ln f_0 / 2), gives each window's first-iteration
    steps; rewl_balanced_windows turns their mean into window edges.  With
    replan, a second pre-run on those windows (again other seeds) adds its
    windows and steps, and the edges are planned again from both.
    Returns ([(lo, hi)] * R, pre-run summary)."""
    from paper_1402_2328_amd import rewl
    from paper_1402_2328_amd import workloads as WL
    F = cfg["flips_per_exchange"]

    def pre_run(windows, seed_offset, tag):
        pre_cfg = dict(cfg, lnf_final=cfg["lnf_init"] / 2, seed=cfg["seed"] + seed_offset,
                       schedule=WL.HALVING)
        ctx = rewl.Context([WL.rewl_params_of(pre_cfg)] * R, windows=windows)
        ctx.autotune(F)
        done_at, cycles, wall = run_to_convergence(ctx, R, F, max_s, tag, quiet=quiet)
        steps = []
        for i in sorted(done_at):
            _, sm = ctx.get_schedule(i)
            steps.append((sm[:, 0] + 1) * F)
        g = ctx.geometry[0]
        ctx.close()
        return g, np.mean(np.array(steps, float), axis=0), {"instances": len(steps), "cycles": cycles,
                                                            "wall_s": wall}

    g, mean, info = pre_run(None, 1000, "balanced pre-run")
    lo, hi = rewl.balanced_windows(g["nbins"], g["h"], g["lo"], g["hi"], mean,
                                   overlap=tuple(cfg["overlap"]), alpha=alpha)
    pre = dict(info, first_iteration_steps_mean=[float(x) for x in mean])
    if replan:
        g2, mean2, info2 = pre_run([(lo, hi)] * R, 2000, "balanced second pre-run")
        lo, hi = rewl.balanced_windows(g["nbins"], g["h"], np.concatenate([g["lo"], g2["lo"]]),
                                       np.concatenate([g["hi"], g2["hi"]]),
                                       np.concatenate([mean, mean2]),
                                       overlap=tuple(cfg["overlap"]), alpha=alpha)
        pre["second"] = dict(info2, first_iteration_steps_mean=[float(x) for x in mean2])
    return [(lo, hi)] * R, pre


def converge(a):
    """Runs R instances of a configuration to ln f <= lnf_final and reports
    time to convergence, C_V peaks (Potts) and, for --config potts10-both, the
    two-float FP32 form against FP64 on the same instances.  The normalised
    ln g and jackknife errors of every finished instance are saved to
    --save (an .npz); tests/converge_report.py scores them against exact
    results."""
    from paper_1402_2328_amd import rewl
    from paper_1402_2328_amd import workloads as WL
    name = a.config
    R = a.replicas
    runs = {"ising8": [("fp64", WL.ISING_L8)], "ising32": [("fp64", WL.ISING_L32)],
            "potts10": [("fp64", WL.POTTS_Q10_L20)],
            "potts10-both": [("fp64", WL.POTTS_Q10_L20), ("fp32c", WL.POTTS_Q10_L20_FP32C)]}[name]
    sched = WL.ONE_OVER_T if a.schedule == "1t" else WL.HALVING
    out = {"metric": "time to ln f <= ln f_final", "config": name, "schedule": a.schedule,
           "instances": R, "walkers_per_window": a.walkers, "balanced": a.balanced, "runs": {}}
    out["note"] = ("saved jackknife errors come from the m pieces per window, which share their "
                   "history up to the last merge, so they understate the error; use the spread "
                   "between the independent instances instead")
    saved = {}
    lng_by_run = {}
    for tag, cfg in runs:
        cfg = dict(cfg, schedule=sched)
        if a.lnf_final > 0:
            cfg["lnf_final"] = a.lnf_final
        if a.walkers:
            cfg["walkers_per_window"] = a.walkers
        windows, pre = None, None
        if a.balanced:
            windows, pre = balanced_split(cfg, R, a.alpha, a.max_minutes * 60, replan=a.replan)
        ctx = rewl.Context([WL.rewl_params_of(cfg)] * R, windows=windows)
        plan = ctx.autotune(cfg["flips_per_exchange"], repeats=3)
        done_at, cycles, wall = run_to_convergence(ctx, R, cfg["flips_per_exchange"],
                                                   a.max_minutes * 60 / len(runs), tag)
        g = ctx.geometry[0]
        N = g["N"]
        res = {"precision": tag, "lnf_final": cfg["lnf_final"], "launch": plan,
               "windows_lo": [int(x) for x in g["lo"]], "balanced_prerun": pre,
               "converged": len(done_at), "cycles_run": cycles, "wall_s_all": wall,
               "wall_s_median": float(np.median(list(done_at.values()))) if done_at else None,
               "cycles_to_converge": sorted(int(ctx.status(i)["done_merge"]) for i in done_at)}
        ids = sorted(done_at)
        lngs = {i: ctx.get_lng(i)[0] for i in ids}
        lng_by_run[tag] = lngs
        if ids:
            saved[f"{tag}_instances"] = np.array(ids)
            saved[f"{tag}_lng"] = np.array([lngs[i] for i in ids])
            if cfg["walkers_per_window"] > 1:
                saved[f"{tag}_jk_err"] = np.array([ctx.jackknife(i)[1] for i in ids])
        if cfg["model"] == WL.POTTS and ids:
            T = np.arange(0.60, 0.80, 1e-4)
            res["cv_peak_T_and_height_per_spin"] = [
                (lambda tp: (tp[0], tp[1] / N))(cv_peak(ctx, i, T)) for i in ids]
        out["runs"][tag] = res
        ctx.close()
    if "fp32c" in lng_by_run and "fp64" in lng_by_run:
        a64, a32 = lng_by_run["fp64"], lng_by_run["fp32c"]
        common = sorted(set(a64) & set(a32))
        d = []
        for i in common:
            fin = np.isfinite(a64[i]) & np.isfinite(a32[i])
            d.append(float(np.max(np.abs(a64[i][fin] - a32[i][fin]))))
        # the same statistic between independent FP64 instances sets the scale
        ids = sorted(a64)
        dd = []
        for x, y in zip(ids[::2], ids[1::2]):
            fin = np.isfinite(a64[x]) & np.isfinite(a64[y])
            dd.append(float(np.max(np.abs(a64[x][fin] - a64[y][fin]))))
        out["fp32c_vs_fp64_max_abs_diff"] = d
        out["fp64_vs_fp64_independent_max_abs_diff"] = dd
    if a.save:
        os.makedirs(os.path.dirname(os.path.abspath(a.save)), exist_ok=True)
        np.savez(a.save, config=name, model=runs[0][1]["model"], L=runs[0][1]["L"],
                 q=runs[0][1]["q"], **saved)
        out["saved"] = a.save
    return out


def speedup(a):
    """Speed-up s_o(h, m) = N_single / N_o(h, m) (Eq. for the speed-up in
    Sec. 4): N is the number of MC steps per walker the slowest window needs
    to finish its first WL iteration.  Ising L x L (default 32), or
    q-state Potts with --q, m walkers per window, overlap 75 %, exchange
    every F flips.  Every h runs as R independent instances in one batched
    context; N(h) is their median.  N_single is one walker on the whole
    range (with m > 1 it gets a run of its own).
    Then the run-time balanced split (Fig. 1b) is planned per h from the
    equal-split runs (rewl_balanced_windows on the mean per-window first
    iteration steps) and measured on R other seeds; a third pass re-plans
    from both runs' data."""
    import torch
    from paper_1402_2328_amd import rewl
    from paper_1402_2328_amd import workloads as WL
    hs = [int(x) for x in a.hs.split(",")]
    R, F, m = a.replicas, a.flips, (a.walkers or 1)
    model = WL.POTTS if a.q > 2 else WL.ISING
    base = WL.config(model, a.L, q=a.q, n_windows=1, walkers_per_window=m, lnf_final=0.5, flips=F)
    what = f"2D q={a.q} Potts L={a.L}" if model == WL.POTTS else f"2D Ising L={a.L}"

    def measure(tag, split, seed0, mm=m):
        cfgs, windows = [], []
        for h in split:
            for r in range(R):
                cfgs.append(dict(base, n_windows=h, walkers_per_window=mm, seed=seed0 + r))
                windows.append(split[h])
        explicit = windows[0] is not None
        assert all((w is not None) == explicit for w in windows)
        ctx = rewl.Context([WL.rewl_params_of(c) for c in cfgs], windows=windows if explicit else None)
        ctx.autotune(F)
        t0 = time.perf_counter()
        done_at, cycles, wall = run_to_convergence(ctx, len(cfgs), F, a.max_minutes * 60, tag)
        torch.cuda.synchronize()
        res = {}
        i = 0
        for h in split:
            steps, per_window = [], []
            for r in range(R):
                st = ctx.status(i)
                _, sm = ctx.get_schedule(i)
                if st["done"]:
                    steps.append((st["done_merge"] + 1) * F)
                    per_window.append((sm[:, 0] + 1) * F)
                i += 1
            g = ctx.geometry[i - 1]
            res[h] = {"N_median": float(np.median(steps)) if steps else None, "finished": len(steps),
                      "per_window_mean": np.mean(np.array(per_window, float), axis=0) if per_window else None,
                      "lo": g["lo"].copy(), "hi": g["hi"].copy(), "nbins": g["nbins"]}
        ctx.close()
        return res, time.perf_counter() - t0

    eq, t_eq = measure("equal", {h: None for h in hs}, 1)
    if m == 1:
        N1 = eq[hs[0]]["N_median"] if hs[0] == 1 else None
    else:
        # N_single is one walker on the whole range (h = m = 1)
        single, _ = measure("single walker", {1: None}, 1 + 3 * R, mm=1)
        N1 = single[1]["N_median"]

    def plan(runs, h):
        lo = np.concatenate([r[h]["lo"] for r in runs])
        hi = np.concatenate([r[h]["hi"] for r in runs])
        S = np.concatenate([r[h]["per_window_mean"] for r in runs])
        return rewl.balanced_windows(runs[0][h]["nbins"], h, lo, hi, S, alpha=a.alpha)

    multi = [h for h in hs if h > 1]
    bal, t_bal = measure("balanced", {h: plan([eq], h) for h in multi}, 1 + R)
    ref, t_ref = measure("balanced_refined", {h: plan([eq, bal], h) for h in multi}, 1 + 2 * R)

    def summary(res):
        out = {}
        for h, r in res.items():
            s_ = N1 / r["N_median"] if (N1 and r["N_median"]) else None
            out[str(h)] = {"N_slowest_median": r["N_median"], "speedup": s_, "finished": r["finished"],
                           "windows_lo": [int(x) for x in r["lo"]]}
        pts = [(h, v["speedup"]) for h, v in ((int(k), v) for k, v in out.items()) if v["speedup"]]
        if N1 and m == 1:
            pts = [(1, 1.0)] + [p for p in pts if p[0] != 1]
        slope = None
        if len(pts) >= 2:
            x = np.array([p[0] for p in pts], float)
            y = np.array([p[1] for p in pts], float)
            slope = float(np.polyfit(x, y, 1)[0])
        return out, slope

    out = {"metric": "speed-up s(h) = N_single / N_slowest(h), first WL iteration",
           "config": {"workload": f"{what}, m={m} walkers/window, overlap 75%, "
                                  f"F={F} flips per exchange, flatness 0.8, {R} instances per h",
                      "hs": hs, "alpha": a.alpha}}
    for name, res, t in (("equal", eq, t_eq), ("balanced", bal, t_bal), ("balanced_refined", ref, t_ref)):
        per_h, slope = summary(res)
        out[name] = {"per_h": per_h, "slope": slope, "wall_s": t}
    return out


def alu_rate(iters=4096):
    """Issue cost of the instruction forms of the sweep, in full-rate slots
    (ns per wavefront step per SIMD, divided by that of a one-slot op)."""
    import ctypes
    path = os.path.join(ROOT, "paper_1402_2328_amd", "libalurate.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    lib.alu_rate.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_int32]
    lib.alu_rate.restype = ctypes.c_int
    out = (ctypes.c_double * 5)()
    rc = lib.alu_rate(iters, out, 5)
    if rc != 0:
        raise RuntimeError(f"alu_rate failed ({rc})")
    ns = list(out)
    forms = ["v_xad_u32", "v_mad_u64_u32 + v_xor_b32", "v_mul_lo_u32 + v_mul_hi_u32 + v_xor_b32",
             "v_fma_f64", "v_bitop3_b32"]
    one = ns[0]
    clock_ghz = 4.0 / one
    lib.lds_rate.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_int32]
    lib.lds_rate.restype = ctypes.c_int
    lds = (ctypes.c_double * 3)()
    rc = lib.lds_rate(iters, lds, 3)
    if rc != 0:
        raise RuntimeError(f"lds_rate failed ({rc})")
    lforms = ["4 B per lane (ds_read2st64_b32)", "8 B per lane (ds_read2st64_b64)",
              "16 B per lane (ds_read_b128)"]
    return {"metric": "VALU issue cost per wavefront step, 8 waves per SIMD; LDS read bandwidth",
            "ns_per_wave_step": dict(zip(forms, ns)),
            "slots": dict(zip(forms, [v / one for v in ns])),
            "clock_ghz_if_one_slot_is_4_cycles": clock_ghz,
            "lds_read_TBps": dict(zip(lforms, [v / 1e12 for v in lds])),
            "lds_read_B_per_clk_per_cu_at_that_clock":
                dict(zip(lforms, [v / (N_CU * clock_ghz * 1e9) for v in lds]))}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures the single-GPU path only (got --gpus {a.gpus}); REWL across "
              "several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1402_2328_amd import rewl
    from paper_1402_2328_amd import workloads as WL

    torch.cuda.set_device(0)
    if a.replicas is None and (a.converge or a.speedup):
        a.replicas = 8 if a.converge else 32
    if a.converge:
        print(json.dumps(converge(a)), flush=True)
        return
    if a.speedup:
        print(json.dumps(speedup(a)), flush=True)
        return
    if a.alu_rate:
        print(json.dumps(alu_rate()), flush=True)
        return
    if a.copy_reference:
        x = torch.empty(128 * 2 ** 20, dtype=torch.float32, device="cuda")
        x.fill_(1.0)
        for _ in range(3):
            y = x.clone()
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes": 4 * x.numel(), "copies": 3, "check": float(y[0])}))
        return
    prec = WL.FP64 if a.precision == "fp64" else WL.FP32C
    if a.workload == "ising32":
        cfg = dict(WL.ISING_L32, precision=prec, flips_per_exchange=a.flips)
        R = a.replicas or 1024
        cfgs = [cfg] * R
        name = (f"2D Ising L=32 REWL, 16 windows x 8 walkers, 75% overlap, flatness 0.8, "
                f"F={a.flips} flips per exchange, x{R} independent instances")
    elif a.workload == "potts10":
        cfg = dict(WL.POTTS_Q10_L20, precision=prec, flips_per_exchange=a.flips)
        R = a.replicas or WL.bench_replicas(cfg)
        cfgs = [cfg] * R
        name = (f"2D q=10 Potts L=20 REWL, 32 windows x 16 walkers, 75% overlap, flatness 0.8, "
                f"F={a.flips} flips per exchange, x{R} independent instances")
    else:
        R = a.replicas or 1
        cfgs = [dict(c, flips_per_exchange=a.flips) for c in WL.batched_mix(precision=prec)] * R
        name = (f"batched mix of 64 Ising/Potts REWL instances (L 16-64, q 2-10, 8-48 windows x "
                f"4-16 walkers), F={a.flips} flips per exchange, x{R}")
    ctx = rewl.Context([WL.rewl_params_of(c) for c in cfgs])
    if a.page_bins > 0:
        plan = ctx.set_launch(page_bins=a.page_bins)
    W = sum(c["n_windows"] * c["walkers_per_window"] for c in cfgs)
    stream = ctx.stream

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        ctx.run_sweeps(a.flips)
        if ev is not None:
            ev[1].record(stream)
        ctx.merge()
        ctx.exchange()

    progress(phase="throughput", workload=name)
    for _ in range(a.warmup):
        step()
    if a.page_bins <= 0:
        # tuned on the state the timed steps start from (tuning restores it)
        plan = ctx.autotune(a.flips, repeats=5 if a.workload == "mix" else 3)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(a.steps)]
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(evs[i])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sweep_ms = float(np.mean([s.elapsed_time(e) for s, e in evs]))
    attempts = W * a.flips * a.steps
    value = attempts / dt
    sweep_rate = W * a.flips / (sweep_ms * 1e-3)
    achieved_valu = sweep_rate * VALU_SLOTS_PER_ATTEMPT
    st = ctx.status(0)
    out = {
        "metric": "spin-flip attempts/s (REWL sweep + merge + exchange cycles)",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == WL.FP64 else "f32x2",
        "data": "synthetic (seeded Philox initial lattices)",
        "config": {"workload": name, "replicas": R, "walkers": W, "flips": a.flips,
                   "precision": a.precision, "launch": plan},
        "roofline": {"bound": "alu", "achieved": achieved_valu / 1e12, "peak": PEAK_VALU / 1e12,
                     "unit": "Tlane-op/s", "frac": achieved_valu / PEAK_VALU,
                     "traffic": traffic_from_profile(R, a.flips,
                                                     plan.get("ising_L<=32", {}).get("page_bins")),
                     "kernel": "k_sweep", "kernel_ms": sweep_ms,
                     "valu_slots_per_attempt": VALU_SLOTS_PER_ATTEMPT,
                     "lds_achieved_TBps": sweep_rate * LDS_BYTES_PER_ATTEMPT / 1e12,
                     "lds_frac": sweep_rate * LDS_BYTES_PER_ATTEMPT / PEAK_LDS},
        "sweep_attempts_per_s": sweep_rate,
        "stage_of_instance0": int(np.max(st["stage"])),
    }
    if a.workload != "ising32" or prec != WL.FP64:
        # the algorithmic slot count above is that of the FP64 Ising attempt
        out["roofline"] = None
        out["kernel_ms"] = sweep_ms
    progress(phase="throughput done", attempts_per_s=value)
    if a.workload == "ising32" and prec == WL.FP64 and not a.no_ttc:
        progress(phase="time to converge, Ising L=8")
        out["time_to_converge"] = time_to_converge_ising8()
        if not a.no_ttc32:
            out["time_to_converge_ising32"] = time_to_converge_ising32()
        progress(phase="batched 64-instance mix")
        out["batched_mix"] = mix_throughput(a.flips)
    if a.workload == "mix" and a.solo > 0:
        out["batching"] = solo_vs_batch(cfgs, a.solo, a.flips, dt / a.steps)
    if not a.no_cpu and a.workload == "ising32":
        progress(phase="CPU oracle baseline, one pinned core")
        out["cpu_baseline"] = cpu_baseline(a.flips, a.cpu_seconds)
        progress(phase="CPU oracle baseline, every core")
        out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(a.flips, a.cpu_seconds)
        ttc = out.get("time_to_converge_ising32", {}).get("fp64", {})
        if ttc.get("cycles_to_converge"):
            # the oracle's trajectory is the GPU's bit for bit, so it would need
            # the same attempts: CPU time = attempts / the pinned oracle rate
            W = WL.ISING_L32["n_windows"] * WL.ISING_L32["walkers_per_window"]
            est = [c * W * a.flips / out["cpu_baseline"]["value"] for c in ttc["cycles_to_converge"]]
            out["cpu_time_to_converge_ising32_estimate"] = {
                "method": "attempts of each FP64 instance's GPU run to ln f = 1e-8 / single-thread "
                          "oracle rate (cpu_baseline.value)",
                "seconds": est, "seconds_median": float(np.median(est)),
                "gpu_wall_s_median": ttc["wall_s_median"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
