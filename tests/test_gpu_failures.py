"""Failure paths of the HIP library, forced from the host (GPU).

Faults are written into the device workspace through torch, at the offsets
rewl_locate_walker reports; every kernel still runs normally and in bounds.
Each case must raise its REWL_E_* code in the instance's status, the failed
instance must stop advancing (no further attempts, merges or exchange
rounds), and a healthy instance in the same batch must carry on exactly as
the oracle does.
"""
import numpy as np
import pytest

from paper_1402_2328_amd import workloads as WL
from tests.parity import compare_state, gpu_context, oracle_cycle, oracle_sim

pytestmark = pytest.mark.gpu

F = 500
# flatness 0/1: every window is flat at every check, so it merges every cycle
BAD = WL.config(WL.ISING, 8, n_windows=4, walkers_per_window=2, lnf_final=1e-6, flips=F, seed=3,
                flat=(0, 1))
GOOD = WL.config(WL.POTTS, 8, q=3, n_windows=3, walkers_per_window=2, flips=F, seed=6)


def poke(ctx, offset, values):
    """Overwrite workspace bytes [offset, offset + nbytes(values))."""
    import torch
    raw = np.ascontiguousarray(values).view(np.uint8)
    src = torch.from_numpy(raw.copy()).to(ctx.workspace.device)
    torch.cuda.synchronize()
    ctx.workspace[offset:offset + raw.size].copy_(src)
    torch.cuda.synchronize()


def frozen_after_error(ctx, code):
    """The failed instance (0) keeps its code and does not advance."""
    st = ctx.status(0)
    assert st["error"] == code, st
    before = (st["attempts"], st["merges"], st["rounds"])
    ctx.run_cycles(3, F)
    st = ctx.status(0)
    assert st["error"] == code
    assert (st["attempts"], st["merges"], st["rounds"]) == before
    assert ctx.running() == 1          # only the healthy instance runs


def healthy_instance_matches_oracle(ctx, cycles):
    sim = oracle_sim(GOOD, instance=1)
    for _ in range(cycles):
        oracle_cycle(sim, F)
    compare_state(ctx, 1, sim)


@pytest.mark.parametrize("precision", [WL.FP64, WL.FP32C])
def test_non_finite_lng_is_reported_at_the_merge(precision):
    bad, good = dict(BAD, precision=precision), dict(GOOD, precision=precision)
    ctx = gpu_context([bad, good])
    ctx.run_cycles(2, F)
    assert ctx.status(0)["error"] == 0
    loc = ctx.locate_walker(0, 1)
    nan = np.full(loc["n_bins"], np.nan, np.float64 if precision == WL.FP64 else np.float32)
    poke(ctx, loc["lng"], nan)
    ctx.run_cycles(1, F)
    frozen_after_error(ctx, -4)
    if precision == WL.FP64:
        healthy_instance_matches_oracle(ctx, 6)


def test_histogram_near_two_to_the_31_is_reported_as_overflow():
    ctx = gpu_context([BAD, GOOD])
    ctx.run_cycles(1, F)
    loc = ctx.locate_walker(0, 2)
    # every bin one count short of 2^31: whatever the walker visits next
    # crosses it
    poke(ctx, loc["H"], np.full(loc["n_bins"], 0x7FFFFFFF, np.uint32))
    ctx.run_cycles(1, F)
    frozen_after_error(ctx, -5)
    healthy_instance_matches_oracle(ctx, 5)


def test_energy_outside_the_window_is_reported_by_the_sweep():
    ctx = gpu_context([BAD, GOOD])
    ctx.run_cycles(1, F)
    g = ctx.geometry[0]
    loc = ctx.locate_walker(0, 0)
    # window 0 ends at bin hi[0]; put the walker's energy far above it
    e_bad = g["emin"] + (int(g["hi"][0]) + 10) * g["binw"]
    poke(ctx, loc["energy"], np.array([e_bad], np.int32))
    ctx.run_sweeps(F)
    ctx.merge()
    ctx.exchange()
    frozen_after_error(ctx, -6)
    healthy_instance_matches_oracle(ctx, 5)
