"""Helpers for GPU-vs-oracle parity tests: build the same REWL instance on
both sides and compare their complete logical state."""
import hashlib
import math
import os

import numpy as np

from oracle import oracle as O
from paper_1402_2328_amd import workloads


def oracle_sim(cfg, instance=0, windows=None):
    return O.Sim(windows=windows, model=cfg["model"], L=cfg["L"], q=cfg["q"], n_windows=cfg["n_windows"],
                 overlap=tuple(cfg["overlap"]), walkers_per_window=cfg["walkers_per_window"],
                 flat=tuple(cfg["flat"]), lnf_init=cfg["lnf_init"], lnf_final=cfg["lnf_final"],
                 flips_per_exchange=cfg["flips_per_exchange"], seed=cfg["seed"],
                 precision=cfg["precision"], instance=instance,
                 schedule=cfg.get("schedule", O.HALVING))


def gpu_context(cfgs, windows=None):
    from paper_1402_2328_amd import rewl
    return rewl.Context([workloads.rewl_params_of(c) for c in cfgs], windows=windows)


def oracle_cycle(sim, flips):
    sim.sweep(flips)
    sim.merge()
    sim.exchange()


def compare_state(ctx, instance, sim, slots=None, windows=True):
    """Assert the GPU instance and the oracle hold identical state.

    Walker-level: spins of the carried configuration, energy, H, ln g bits
    (FP64, or both two-float parts), attempt counter, configuration identity.
    Window-level: ln f, stage, schedule phase, iteration-end merges, frozen
    flag, visited union, and the frozen pieces of its walkers.  Instance-level:
    finished flag, merge and round counters, exchange statistics.
    """
    g = ctx.geometry[instance]
    W = g["h"] * g["m"]
    slots = range(W) if slots is None else slots
    for slot in slots:
        a, b = ctx.get_walker(instance, slot), sim.walker(slot)
        tag = f"instance {instance} slot {slot}"
        assert a["E"] == b["E"], tag
        assert a["attempts"] == b["attempts"], tag
        assert a["config"] == b["config"], tag
        assert np.array_equal(a["spins"], b["spins"]), tag
        assert np.array_equal(a["H"], b["H"]), tag
        if "lng_hi" in a:
            assert np.array_equal(a["lng_hi"].view(np.uint32), b["lng_hi"].view(np.uint32)), tag
            assert np.array_equal(a["lng_lo"].view(np.uint32), b["lng_lo"].view(np.uint32)), tag
        else:
            assert np.array_equal(a["lng"].view(np.uint64), b["lng"].view(np.uint64)), tag
    if not windows:
        return
    st = ctx.status(instance)
    os_ = sim.status()
    assert st["done"] == os_["done"]
    assert st["merges"] == os_["merges"] and st["rounds"] == os_["rounds"]
    assert st["done_merge"] == os_["done_merge"]
    phase, sm = ctx.get_schedule(instance)
    for w in range(g["h"]):
        ow = sim.window(w)
        assert st["stage"][w] == ow["stage"] and st["frozen"][w] == ow["frozen"], w
        assert st["lnf"][w] == ow["lnf"], w
        assert phase[w] == ow["phase"], w
        assert np.array_equal(sm[w], ow["stage_merge"]), w
        assert np.array_equal(ctx.get_visited(instance, w), ow["U"]), w
        for k in range(g["m"]):
            slot = w * g["m"] + k
            assert np.array_equal(ctx.get_piece(instance, slot).view(np.uint64),
                                  sim.piece(slot).view(np.uint64)), (w, k)
    t, r, a = ctx.get_exchange_stats(instance)
    ot, orr, oa = sim.exchange_stats()
    assert np.array_equal(t, ot) and np.array_equal(r, orr) and np.array_equal(a, oa)


# the stored q=10 Potts L=20 runs (FP64 and two-float FP32) stop at this
# ln f: ten merges per window, then every window freezes and is joined
POTTS_RUN_LNF_FINAL = 1e-3


def golden_potts_q10_L20_run(tag):
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        f"oracle_potts_q10_L20_h32_m16_seed1_{tag}.txt")


GOLDEN_ISING_L32_RUN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                    "oracle_ising_L32_h16_m8_seed1.txt")


def load_golden_ising_L32_run():
    """The stored oracle run: metadata (done_merge, cycles, joins) and the
    joined and normalised ln g per bin."""
    return load_golden_run(GOLDEN_ISING_L32_RUN)


def _digest(walkers, windows):
    """SHA-256 over the logical state of an instance, in slot then window
    order: per walker energy, attempts, configuration identity, spins, H and
    the bits of ln g (both two-float parts for FP32C); per window ln f bits,
    stage, frozen flag and visited union."""
    h = hashlib.sha256()
    for wk in walkers:
        h.update(np.array([wk["E"], wk["config"]], np.int64).tobytes())
        h.update(np.array([wk["attempts"]], np.uint64).tobytes())
        h.update(np.ascontiguousarray(wk["spins"], np.int8).tobytes())
        h.update(np.ascontiguousarray(wk["H"], np.uint32).tobytes())
        if "lng_hi" in wk:
            h.update(np.ascontiguousarray(wk["lng_hi"], np.float32).tobytes())
            h.update(np.ascontiguousarray(wk["lng_lo"], np.float32).tobytes())
        else:
            h.update(np.ascontiguousarray(wk["lng"], np.float64).tobytes())
    for lnf, stage, frozen, U in windows:
        h.update(np.array([lnf], np.float64).tobytes())
        h.update(np.array([stage, frozen], np.int64).tobytes())
        h.update(np.ascontiguousarray(U, np.uint8).tobytes())
    return h.hexdigest()


def oracle_digest(sim):
    W, h = sim.info.W, sim.info.h
    wins = [sim.window(w) for w in range(h)]
    return _digest((sim.walker(s) for s in range(W)),
                   [(x["lnf"], x["stage"], x["frozen"], x["U"]) for x in wins])


def gpu_digest(ctx, instance):
    g = ctx.geometry[instance]
    st = ctx.status(instance)
    return _digest((ctx.get_walker(instance, s) for s in range(g["h"] * g["m"])),
                   [(st["lnf"][w], st["stage"][w], st["frozen"][w], ctx.get_visited(instance, w))
                    for w in range(g["h"])])


def load_golden_run(path):
    """A stored oracle run: metadata lines '# key v1 v2 ..' and per bin the
    joined ln g and the normalised ln g (hexadecimal floats, or -inf)."""
    meta, raw, norm = {}, [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                parts = line[1:].split()
                if parts and parts[0] in ("done_merge", "cycles", "joins"):
                    meta[parts[0]] = [int(p) for p in parts[1:]]
                elif parts and parts[0] == "digest":
                    meta["digest"] = parts[1]
                continue
            a, b = line.split()
            raw.append(-math.inf if a == "-inf" else float.fromhex(a))
            norm.append(-math.inf if b == "-inf" else float.fromhex(b))
    return meta, np.array(raw), np.array(norm)
