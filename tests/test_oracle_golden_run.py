"""The stored full oracle run (2D Ising L=32, 16 windows x 8 walkers, halving
to ln f = 1e-8; tests/golden/oracle_ising_L32_h16_m8_seed1.txt) checked
against what does not come from the oracle: the exact density of states
(Kaufman's formula, stored table) and the normalisation Sum g = 2^N.  The
GPU side of the same run is in tests/test_gpu_long.py."""
import math
import os

import numpy as np

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
