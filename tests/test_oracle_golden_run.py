"""The stored oracle runs checked against what does not come from the
oracle.  The full Ising L=32 run (16 windows x 8 walkers, halving to
ln f = 1e-8; tests/golden/oracle_ising_L32_h16_m8_seed1.txt): the exact
density of states (Kaufman's formula, stored table) and the normalisation
Sum g = 2^N; its GPU side is tests/test_gpu_long.py.  The q=10 Potts L=20
runs to ln f = 1e-3 (FP64 and two-float FP32): the exact set of empty
energies and the normalisation; their GPU side is
tests/test_gpu_fullsize.py."""
import math
import os

import numpy as np
import pytest

from oracle import exact_dos as X
from tests.parity import GOLDEN_ISING_L32_RUN, load_golden_ising_L32_run
from tests.test_oracle_exact import load_ising_table


def test_stored_run_is_a_converged_ising_L32_density_of_states():
    assert os.path.exists(GOLDEN_ISING_L32_RUN)
    meta, raw, norm = load_golden_ising_L32_run()
    N = 32 * 32
    assert len(raw) == len(norm) == N + 1
    # one join bin per neighbouring window pair, inside the energy range (with
    # 75 % overlap consecutive join points need not increase)
    assert len(meta["joins"]) == 15 and all(0 < j < N for j in meta["joins"])
    assert meta["done_merge"][0] + 1 == meta["cycles"][0]
    exact = X.ln_g(load_ising_table(32))
    # bins that never occur (E = -2N + 4 and 2N - 4) are empty, all others filled
    assert np.array_equal(np.isfinite(norm), np.isfinite(exact))
    assert np.array_equal(np.isfinite(raw), np.isfinite(exact))
    fin = np.isfinite(exact)
    # normalised: log-sum-exp = N ln 2
    top = norm[fin].max()
    lse = top + math.log(np.exp(norm[fin] - top).sum())
    assert abs(lse - N * math.log(2.0)) < 1e-9
    # the joined ln g differs from the normalised one by one constant
    shift = norm[fin] - raw[fin]
    assert np.ptp(shift) < 1e-9
    # halving to 1e-8 with flatness 0.8 leaves an error of order 0.1 (R22);
    # far below the 700-unit range of ln g
    err = np.abs(norm[fin] - exact[fin])
    assert err.max() < 0.2
    assert np.sqrt(np.mean(err ** 2)) < 0.1


@pytest.mark.parametrize("tag", ["fp64", "fp32c"])
def test_stored_potts_runs_are_joined_normalised_q10_L20_estimates(tag):
    """The stored q=10 Potts L=20 runs (32 windows x 16 walkers, halving to
    ln f = 1e-3; tests/golden/oracle_potts_q10_L20_h32_m16_seed1_*.txt) are
    parity fixtures for the GPU: ten WL iterations are far from converged,
    so only what holds at any stage is pinned here -- exactly the energies
    that cannot occur (one spin differing from a ground state breaks 4
    bonds, so E_min + 1, 2, 3 and 5 are empty; every other energy up to
    E = 0 occurs and was visited), the normalisation g(E_min) = q, one
    constant between the joined and the normalised ln g, and one join per
    neighbouring window pair inside their overlap."""
    from oracle import oracle as O
    from tests.parity import POTTS_RUN_LNF_FINAL, golden_potts_q10_L20_run, load_golden_run
    meta, raw, norm = load_golden_run(golden_potts_q10_L20_run(tag))
    N, q = 400, 10
    assert len(raw) == len(norm) == 2 * N + 1
    assert meta["done_merge"][0] + 1 == meta["cycles"][0]
    assert len(meta["digest"]) == 64
    empty = np.flatnonzero(~np.isfinite(norm))
    assert list(empty) == [1, 2, 3, 5]
    assert np.array_equal(np.isfinite(raw), np.isfinite(norm))
    # the shift log q - R[0] is added to R[0] ~ 1e5, a few of its ulps
    assert abs(norm[0] - math.log(q)) <= 4 * np.spacing(abs(raw[0]))
    fin = np.isfinite(norm)
    assert np.ptp(norm[fin] - raw[fin]) < 1e-9
    lo, hi = O.equal_windows(2 * N + 1, 32)
    assert len(meta["joins"]) == 31
    for w, j in enumerate(meta["joins"]):
        assert lo[w + 1] + 2 <= j <= hi[w] - 2, (w, j)
    assert POTTS_RUN_LNF_FINAL == 1e-3
