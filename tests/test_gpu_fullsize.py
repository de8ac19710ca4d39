"""Full-size GPU parity on the q=10 Potts L=20 geometry (32 windows x 16
walkers, F = 10^4), FP64 and two-float FP32: one instance run by the GPU
until every window is frozen (halving from ln f = 1 to 1e-3: ten merges per
window of 16 walkers, the freeze, the join over 32 windows) must reproduce
the oracle's stored run bit for bit: the merge at which the last window
froze, the join bins, the joined ln g, and the SHA-256 of the final state of
all 512 walkers and 32 windows (spins, energies, histograms, ln g bits,
attempt counters, configuration identities, ln f, stages, visited unions).
The normalised ln g agrees within 1e-12 (platform exp and log).

The stored runs (tests/golden/oracle_potts_q10_L20_h32_m16_seed1_*.txt) were
written by tests/golden/make_oracle_potts_q10_L20_runs.py, which calls only
the oracle.  The FP64 run uses the benchmark's launch shape for this
workload (page of 32 bins, nibble lattices, no RNG producer), the FP32C run
the library's default shape for one instance (with the producer).
"""
import os

import numpy as np
import pytest

from paper_1402_2328_amd import workloads as WL
from tests.parity import (POTTS_RUN_LNF_FINAL, golden_potts_q10_L20_run, gpu_context, gpu_digest,
                          load_golden_run)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tag,precision,shape", [
    ("fp64", WL.FP64, dict(page_bins=32, rng_producer=0, potts_nibbles=1)),
    ("fp32c", WL.FP32C, None)])
def test_potts_q10_L20_run_to_freeze_matches_stored_oracle_run(tag, precision, shape):
    path = golden_potts_q10_L20_run(tag)
    meta, raw, norm = load_golden_run(path)
    assert len(raw) == 801
    cfg = dict(WL.POTTS_Q10_L20, precision=precision, lnf_final=POTTS_RUN_LNF_FINAL)
    ctx = gpu_context([cfg])
    if shape:
        print(f"[parity] Potts q=10 L=20 {tag}: plan {ctx.set_launch(**shape)}", flush=True)
    F = cfg["flips_per_exchange"]
    cycles = 0
    while ctx.running() and cycles < 2 * meta["cycles"][0]:
        ctx.run_cycles(250, F, use_graph=True)
        cycles += 250
        print(f"[parity] Potts q=10 L=20 {tag}: {cycles} cycles, lowest stage "
              f"{int(ctx.status(0)['stage'].min())}", flush=True)
    st = ctx.status(0)
    assert st["error"] == 0
    assert st["done"] and st["done_merge"] == meta["done_merge"][0]
    g_raw, joins = ctx.get_lng(0, normalise=False)
    g_norm, _ = ctx.get_lng(0)
    assert list(joins) == meta["joins"]
    fin = np.isfinite(raw)
    assert np.array_equal(np.isfinite(g_raw), fin) and np.array_equal(np.isfinite(g_norm), fin)
    assert np.array_equal(g_raw[fin].view(np.uint64), raw[fin].view(np.uint64))
    assert np.max(np.abs(g_norm[fin] - norm[fin])) <= 1e-12
    assert gpu_digest(ctx, 0) == meta["digest"]
