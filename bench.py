"""Throughput benchmark of the REWL hot path on one MI355X.

A step is one REWL cycle over the whole batch: rewl_run_sweeps(F) (every
walker does F Wang-Landau attempts), rewl_merge (flatness test and in-window
merge) and rewl_exchange (one replica-exchange round).  The workload is the
2D Ising L=32 REWL configuration (16 windows x 8 walkers, 75 % overlap,
flatness 0.8, exchange every 10^4 flips, FP64 ln g) replicated R times as
independent instances so that the chip is filled; each copy carries its
instance index in every random-number counter.

Printed: one JSON line with spin-flip attempts/s, the sweep kernel's
roofline position (timed with HIP events on the library's stream) and the
single-threaded CPU oracle's attempts/s on a bounded sample.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures used for the roofline ("Roofline").
N_CU = 256
CLOCK_HZ = 2.4e9
VALU_LANE_OPS_PER_CLK_PER_CU = 64          # 4 SIMD x 16 lanes, full-rate 32-bit/FP64 ops
PEAK_VALU = N_CU * VALU_LANE_OPS_PER_CLK_PER_CU * CLOCK_HZ   # 3.93e13 lane-ops/s
# Algorithmic VALU work of one attempt, in full-rate lane-op slots:
# Philox4x32-10 100, site/neighbour indexing 28, dE + window 8, WL test and
# exp 32, update 8.
VALU_SLOTS_PER_ATTEMPT = 176
# Algorithmic LDS bytes of one attempt: 5 spin bytes read, 8 B ln g read,
# 8 B ln g write, 4 B H read + 4 B H write, spin write (1 B x acceptance ~ 0.5)
LDS_BYTES_PER_ATTEMPT = 29.5
PEAK_LDS = N_CU * 128 * CLOCK_HZ            # 128 B/clk/CU


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--replicas", type=int, default=0, help="instances of the L=32 config (0: fill chip)")
    ap.add_argument("--flips", type=int, default=10000)
    ap.add_argument("--precision", choices=["fp64", "fp32c"], default="fp64")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def cpu_baseline(flips, seconds):
    from oracle import oracle as O
    from paper_1402_2328_amd import workloads as WL
    c = WL.CFG2
    sim = O.Sim(model=c["model"], L=c["L"], n_windows=c["n_windows"],
                walkers_per_window=c["walkers_per_window"], lnf_final=c["lnf_final"],
                flips_per_exchange=flips, seed=c["seed"])
    W = c["n_windows"] * c["walkers_per_window"]
    cycles = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        sim.sweep(flips)
        sim.merge()
        sim.exchange()
        cycles += 1
    dt = time.perf_counter() - t0
    return {"value": cycles * W * flips / dt, "unit": "attempts/s", "cores": 1, "kind": "oracle",
            "sample": f"Ising L=32 REWL (16 windows x 8 walkers), {cycles} cycles of {flips} "
                      f"attempts per walker from a fresh start, single thread, {dt:.1f} s",
            "cpu": platform.processor() or platform.machine()}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); multi-GPU REWL is a design "
              "note, not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1402_2328_amd import rewl
    from paper_1402_2328_amd import workloads as WL

    torch.cuda.set_device(0)
    prec = WL.FP64 if a.precision == "fp64" else WL.FP32C
    cfg = dict(WL.CFG2, precision=prec, flips_per_exchange=a.flips)
    one = [WL.rewl_params_of(cfg)]
    R = a.replicas if a.replicas > 0 else WL.bench_replicas(cfg)
    params = one * R
    ctx = rewl.Context(params)
    plan = ctx.set_launch()
    W = R * cfg["n_windows"] * cfg["walkers_per_window"]
    stream = ctx.stream

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        ctx.run_sweeps(a.flips)
        if ev is not None:
            ev[1].record(stream)
        ctx.merge()
        ctx.exchange()

    for _ in range(a.warmup):
        step()
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
        "metric": "spin-flip attempts/s (REWL sweep+merge+exchange cycles)",
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
        "config": {"workload": f"2D Ising L=32 REWL, 16 windows x 8 walkers, 75% overlap, "
                               f"flatness 0.8, F={a.flips} flips per exchange, x{R} independent "
                               f"instances", "replicas": R, "walkers": W, "flips": a.flips,
                   "precision": a.precision, "launch": plan},
        "roofline": {"bound": "alu", "achieved": achieved_valu / 1e12, "peak": PEAK_VALU / 1e12,
                     "unit": "Tlane-op/s", "frac": achieved_valu / PEAK_VALU, "traffic": None,
                     "kernel": "k_sweep", "kernel_ms": sweep_ms,
                     "lds_achieved_TBps": sweep_rate * LDS_BYTES_PER_ATTEMPT / 1e12,
                     "lds_frac": sweep_rate * LDS_BYTES_PER_ATTEMPT / PEAK_LDS},
        "sweep_attempts_per_s": sweep_rate,
        "stage_of_instance0": int(np.max(st["stage"])),
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(a.flips, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
