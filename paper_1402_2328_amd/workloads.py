"""Seeded synthetic workloads (parameter sets only; none of the method's arithmetic).

The configurations below are the REWL runs this library is measured on: 2D
Ising and q-state Potts models on periodic lattices with equal-size windows
of 75 % overlap (Fig. 1a of the paper), flatness 0.8 and ln f halving.  The
batched mix is drawn with numpy's PCG64 generator so that both the GPU path
and the test oracle receive the same list of instances.
"""
import numpy as np

ISING, POTTS = 0, 1
FP64, FP32C = 0, 1
HALVING, ONE_OVER_T = 0, 1


def config(model, L, q=2, n_windows=1, walkers_per_window=1, lnf_final=1e-8, flips=10000,
           seed=1, precision=FP64, flat=(4, 5), overlap=(3, 4), lnf_init=1.0, schedule=HALVING):
    return dict(model=model, L=L, q=q, n_windows=n_windows, walkers_per_window=walkers_per_window,
                lnf_final=lnf_final, flips_per_exchange=flips, seed=seed, precision=precision,
                flat=flat, overlap=overlap, lnf_init=lnf_init, schedule=schedule)


# Ising L=8: 4 windows x 1 walker, ln f 1 -> 1e-6, exchange every 1000 flips
ISING_L8 = config(ISING, 8, n_windows=4, walkers_per_window=1, lnf_final=1e-6, flips=1000)
# Ising L=32: 16 windows x 8 walkers, ln f 1 -> 1e-8, exchange every 10^4 flips
ISING_L32 = config(ISING, 32, n_windows=16, walkers_per_window=8, lnf_final=1e-8, flips=10000)
# Potts q=10 L=20: 32 windows x 16 walkers
POTTS_Q10_L20 = config(POTTS, 20, q=10, n_windows=32, walkers_per_window=16, lnf_final=1e-8, flips=10000)
# the same with two-float FP32 ln g
POTTS_Q10_L20_FP32C = dict(POTTS_Q10_L20, precision=FP32C)


def bench_replicas(cfg, n_cu=256):
    """Copies of `cfg` that fill every compute unit with resident sweep
    workgroups once, for the default launch plan."""
    from . import rewl
    ctx = rewl.Context([rewl_params_of(cfg)])
    (plan,) = ctx.set_launch(rng_producer=0, potts_nibbles=1).values()
    ctx.close()
    per_cu = max(1, (160 * 1024) // plan["lds_bytes"])
    return max(1, (n_cu * per_cu) // plan["workgroups"])


def replicated(cfg, copies):
    """`copies` independent instances of one configuration.  They share the
    seed and differ by their instance index, which every random-number
    counter carries, so copy 0 is the single-instance run."""
    return [dict(cfg) for _ in range(copies)]


def batched_mix(n=64, seed=5, precision=FP64):
    """Uneven mix of independent instances: Ising with L in {16,24,32,48,64}
    or q-Potts with q in 2..10 and even L in 16..32; 8-48 windows; 4-16
    walkers per window; instance i uses seed i+1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        if rng.integers(0, 2) == 0:
            c = config(ISING, int(rng.choice([16, 24, 32, 48, 64])))
        else:
            c = config(POTTS, int(rng.choice(np.arange(16, 33, 2))), q=int(rng.integers(2, 11)))
        c["n_windows"] = int(rng.integers(8, 49))
        c["walkers_per_window"] = int(rng.integers(4, 17))
        c["seed"] = i + 1
        c["precision"] = precision
        out.append(c)
    return out


def rewl_params_of(cfg):
    """C-ABI parameter struct for a configuration dict."""
    from . import rewl
    return rewl.make_params(model=cfg["model"], L=cfg["L"], q=cfg["q"],
                            n_windows=cfg["n_windows"], overlap=tuple(cfg["overlap"]),
                            walkers_per_window=cfg["walkers_per_window"], flat=tuple(cfg["flat"]),
                            precision=cfg["precision"], lnf_init=cfg["lnf_init"],
                            lnf_final=cfg["lnf_final"], flips_per_exchange=cfg["flips_per_exchange"],
                            seed=cfg["seed"], schedule=cfg.get("schedule", HALVING))
