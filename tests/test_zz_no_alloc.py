"""The allocation-free jackknife (rewl_jackknife_noalloc) against
rewl_jackknife and the oracle (GPU).

Two calls in a row on the GPU's one scratch array, the second for a smaller
instance (fewer bins, fewer walkers), so that whatever the first call left
in the array is still there: both must equal rewl_jackknife bit for bit and
the oracle's jackknife within 1e-12 on the mean and 1e-8 relative on the
error (the normalisation goes through the platform's exp and log).
"""
import numpy as np
import pytest

from paper_1402_2328_amd import workloads as WL
from tests.parity import gpu_context, oracle_sim

pytestmark = pytest.mark.gpu

LARGER = WL.config(WL.ISING, 12, n_windows=3, walkers_per_window=5, lnf_final=1e-4, flips=1000,
                   seed=2)
SMALLER = WL.config(WL.ISING, 8, n_windows=4, walkers_per_window=2, lnf_final=1e-6, flips=500,
                    seed=3)


def _finished(cfg):
    ctx = gpu_context([cfg])
    ctx.run_to_convergence(cfg["flips_per_exchange"], cycles_per_check=200)
    assert ctx.status(0)["done"] == 1
    sim = oracle_sim(cfg)
    sim.run(10 ** 8)
    return ctx, sim


def test_noalloc_jackknife_matches_the_workspace_jackknife_twice():
    runs = [_finished(LARGER), _finished(SMALLER)]
    assert runs[0][0].geometry[0]["nbins"] > runs[1][0].geometry[0]["nbins"]
    for ctx, sim in runs:
        mean_n, err_n = ctx.jackknife_noalloc(0)
        mean_w, err_w = ctx.jackknife(0)
        assert np.array_equal(mean_n, mean_w) and np.array_equal(err_n, err_w)
        mean_o, err_o = sim.jackknife()
        fin = np.isfinite(mean_o)
        assert np.array_equal(np.isfinite(mean_n), fin)
        assert np.max(np.abs(mean_n[fin] - mean_o[fin])) < 1e-12
        np.testing.assert_allclose(err_n, err_o, rtol=1e-8, atol=1e-12)


def test_noalloc_jackknife_error_paths():
    from paper_1402_2328_amd import rewl
    ctx = gpu_context([SMALLER, WL.config(WL.ISING, 8, n_windows=2, walkers_per_window=1)])
    ctx.run_cycles(2, 500)
    for inst in (0, 1):               # unfinished; single walker per window
        with pytest.raises(rewl.RewlError) as e:
            ctx.jackknife_noalloc(inst)
        assert e.value.code == -6
    # q = 3 Potts L = 64 with 64 walkers per window: 66 rows of 8193 bins
    # exceed the 2^19-double array, which is refused before anything runs
    big = gpu_context([WL.config(WL.POTTS, 64, q=3, n_windows=2, walkers_per_window=64)])
    with pytest.raises(rewl.RewlError) as e:
        big.jackknife_noalloc(0)
    assert e.value.code == -2
    with pytest.raises(rewl.RewlError) as e:
        big.jackknife(0)              # the workspace form has no such limit
    assert e.value.code == -6
