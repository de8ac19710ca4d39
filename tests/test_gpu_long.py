"""Full-length GPU parity: one 2D Ising L=32 REWL instance (16 windows x 8
walkers, ln f 1 -> 1e-8 by halving, F = 10^4) run to the end on the GPU must
reproduce the oracle's stored run bit for bit: the merge at which the last
window froze, the join bins and the joined ln g; the normalised ln g within
1e-12 (it goes through the platform's exp and log).

The stored run (tests/golden/oracle_ising_L32_h16_m8_seed1.txt) was written
by tests/golden/make_oracle_ising_L32_run.py, which calls only the oracle.
The GPU run takes about five minutes.  It is cut into four tests of at most
20 000 cycles each on one context, so that a quiet test runner still reports
progress every minute or so; REWL_SKIP_LONG=1 skips them.
"""
import os

import numpy as np
import pytest

from paper_1402_2328_amd import workloads as WL
from tests.parity import gpu_context, load_golden_ising_L32_run

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("REWL_SKIP_LONG") == "1",
                                 reason="REWL_SKIP_LONG=1: skips the five-minute run to ln f = 1e-8")]

CYCLES_PER_PART = 20000
PARTS = 4


@pytest.fixture(scope="module")
def long_run():
    meta, raw, norm = load_golden_ising_L32_run()
    assert len(raw) == 1025
    assert meta["cycles"][0] <= PARTS * CYCLES_PER_PART
    return {"ctx": gpu_context([WL.ISING_L32]), "cycles": 0, "meta": meta, "raw": raw, "norm": norm}


@pytest.mark.parametrize("part", range(PARTS))
def test_ising_L32_full_run_part(long_run, part):
    """Cycles [part, part + 1) x 20 000 of the run (fewer once it is done)."""
    ctx = long_run["ctx"]
    F = WL.ISING_L32["flips_per_exchange"]
    while ctx.running() and long_run["cycles"] < (part + 1) * CYCLES_PER_PART:
        ctx.run_cycles(2000, F, use_graph=True)
        long_run["cycles"] += 2000
        print(f"[parity] Ising L=32 full run: {long_run['cycles']} cycles, lowest stage "
              f"{int(ctx.status(0)['stage'].min())}", flush=True)
    assert ctx.status(0)["error"] == 0


def test_ising_L32_full_run_matches_stored_oracle_run(long_run):
    ctx, meta, raw, norm = long_run["ctx"], long_run["meta"], long_run["raw"], long_run["norm"]
    st = ctx.status(0)
    print(f"[parity] Ising L=32 full run: {long_run['cycles']} cycles, done_merge {st['done_merge']}",
          flush=True)
    assert st["done"] and st["done_merge"] == meta["done_merge"][0]
    g_raw, joins = ctx.get_lng(0, normalise=False)
    g_norm, _ = ctx.get_lng(0)
    assert list(joins) == meta["joins"]
    fin = np.isfinite(raw)
    assert np.array_equal(np.isfinite(g_raw), fin) and np.array_equal(np.isfinite(g_norm), fin)
    assert np.array_equal(g_raw[fin].view(np.uint64), raw[fin].view(np.uint64))
    assert np.max(np.abs(g_norm[fin] - norm[fin])) <= 1e-12
