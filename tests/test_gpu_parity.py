"""GPU parity: the HIP path (through the C-ABI) against the oracle, bit for bit.

Integer state (spins, energies, histograms, counters, configuration
identities) and ln g bits must be identical after every checked segment; the
joined ln g before normalisation must be identical too; after normalisation
(which uses the platform's exp/log) it must agree to 1e-12 absolute.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1402_2328_amd import workloads as WL
from tests.parity import compare_state, gpu_context, oracle_cycle, oracle_sim

pytestmark = pytest.mark.gpu

SMALL = {
    "ising_L8_h4_m2": WL.config(WL.ISING, 8, n_windows=4, walkers_per_window=2, lnf_final=1e-6,
                                flips=500, seed=3),
    "ising_L6_h3_m3": WL.config(WL.ISING, 6, n_windows=3, walkers_per_window=3,
                                    lnf_final=1e-5, flips=250, seed=11),
    "ising_L16_h5_m4": WL.config(WL.ISING, 16, n_windows=5, walkers_per_window=4, flips=2000,
                                 seed=2),
    "ising_L12_h1_m1": WL.config(WL.ISING, 12, n_windows=1, walkers_per_window=1, flips=3000,
                                 seed=9),
    "potts_q5_L12_h9_m7_ragged": WL.config(WL.POTTS, 12, q=5, n_windows=9, walkers_per_window=7,
                                           flips=1500, seed=12),
    "potts_q10_L8_h4_m4": WL.config(WL.POTTS, 8, q=10, n_windows=4, walkers_per_window=4,
                                    flips=1000, seed=4),
    "ising_L40_h6_m2_tworow": WL.config(WL.ISING, 40, n_windows=6, walkers_per_window=2,
                                        flips=3000, seed=8),
    # L = 32: one word per row, neighbours by word rotation (its own loop copy)
    "ising_L32_h4_m2": WL.config(WL.ISING, 32, n_windows=4, walkers_per_window=2, flips=1000,
                                 seed=14),
    "ising_L32_h3_m3_fp32c": WL.config(WL.ISING, 32, n_windows=3, walkers_per_window=3,
                                       flips=800, seed=15, precision=WL.FP32C),
    "potts_q2_L8_h3_m2": WL.config(WL.POTTS, 8, q=2, n_windows=3, walkers_per_window=2,
                                   flips=700, seed=5),
    "potts_q3_L10_h6_m3": WL.config(WL.POTTS, 10, q=3, n_windows=6, walkers_per_window=3,
                                    flips=900, seed=6),
    # q > 16: Potts spins kept as bytes rather than nibbles in LDS
    "potts_q20_L7_h3_m2": WL.config(WL.POTTS, 7, q=20, n_windows=3, walkers_per_window=2,
                                    flips=600, seed=13),
    "ising_L8_fp32c": WL.config(WL.ISING, 8, n_windows=4, walkers_per_window=2, lnf_final=1e-6,
                                flips=500, seed=3, precision=WL.FP32C),
    "potts_q10_L8_fp32c": WL.config(WL.POTTS, 8, q=10, n_windows=4, walkers_per_window=4,
                                    flips=1000, seed=4, precision=WL.FP32C),
    "ising_L8_h4_m2_1t": WL.config(WL.ISING, 8, n_windows=4, walkers_per_window=2, lnf_final=1e-4,
                                   flips=500, seed=3, schedule=WL.ONE_OVER_T),
    # its oracle run is pinned to the exact q=3 L=6 density of states
    "potts_q3_L6_h3_m4": WL.config(WL.POTTS, 6, q=3, n_windows=3, walkers_per_window=4,
                                   lnf_final=1e-6, flips=300, seed=1),
    "potts_q3_L6_h3_m3_1t_fp32c": WL.config(WL.POTTS, 6, q=3, n_windows=3, walkers_per_window=3,
                                            lnf_final=1e-4, flips=400, seed=6,
                                            precision=WL.FP32C, schedule=WL.ONE_OVER_T),
}


@pytest.mark.parametrize("prod", [0, 1])
@pytest.mark.parametrize("name", list(SMALL))
def test_initial_state_and_segments_match(name, prod):
    """Segments of 1, 2, 10 and 40 cycles, with the random numbers made by
    the walkers' own wavefront (prod = 0) or by a producer wavefront."""
    cfg = SMALL[name]
    ctx = gpu_context([cfg])
    ctx.set_launch(rng_producer=prod)
    sim = oracle_sim(cfg)
    print(f"[parity] {name} prod={prod}: init", flush=True)
    compare_state(ctx, 0, sim)
    F = cfg["flips_per_exchange"]
    for seg in (1, 2, 10, 40):
        for _ in range(seg):
            ctx.run_sweeps(F)
            ctx.merge()
            ctx.exchange()
            oracle_cycle(sim, F)
        print(f"[parity] {name}: +{seg} cycles", flush=True)
        compare_state(ctx, 0, sim)


@pytest.mark.parametrize("name", ["ising_L8_h4_m2", "potts_q2_L8_h3_m2", "ising_L8_fp32c",
                                  "ising_L8_h4_m2_1t", "potts_q3_L6_h3_m4",
                                  "potts_q3_L6_h3_m3_1t_fp32c"])
def test_full_run_to_convergence_matches(name):
    cfg = SMALL[name]
    ctx = gpu_context([cfg])
    sim = oracle_sim(cfg)
    F = cfg["flips_per_exchange"]
    n = ctx.run_to_convergence(F, cycles_per_check=200)
    ocycles = sim.run(10 ** 8)
    st = ctx.status(0)
    assert st["done"] == 1 and sim.status()["done"] == 1
    assert st["done_merge"] == sim.status()["done_merge"]
    assert n >= ocycles
    compare_state(ctx, 0, sim)
    raw_g, joins_g = ctx.get_lng(0, normalise=False)
    raw_o, joins_o = sim.join(normalise=False)
    assert np.array_equal(joins_g, joins_o)
    assert np.array_equal(raw_g.view(np.uint64), raw_o.view(np.uint64))
    nrm_g, _ = ctx.get_lng(0)
    nrm_o, _ = sim.join()
    fin = np.isfinite(nrm_o)
    assert np.array_equal(np.isfinite(nrm_g), fin)
    assert np.max(np.abs(nrm_g[fin] - nrm_o[fin])) < 1e-12
    # jackknife over the frozen pieces (compared bitwise by compare_state):
    # the leave-one-out joins share the normalisation's platform exp/log
    mean_g, err_g = ctx.jackknife(0)
    mean_o, err_o = sim.jackknife()
    fin = np.isfinite(mean_o)
    assert np.array_equal(np.isfinite(mean_g), fin)
    assert np.max(np.abs(mean_g[fin] - mean_o[fin])) < 1e-12
    np.testing.assert_allclose(err_g, err_o, rtol=1e-8, atol=1e-12)


def test_jackknife_rejects_unfinished_runs_and_single_walkers():
    from paper_1402_2328_amd import rewl
    ctx = gpu_context([SMALL["ising_L8_h4_m2"], SMALL["ising_L12_h1_m1"]])
    ctx.run_cycles(2, 500)
    for inst in (0, 1):
        with pytest.raises(rewl.RewlError) as e:
            ctx.jackknife(inst)
        assert e.value.code == -6


def test_instances_in_a_batch_match_standalone_oracles():
    cfgs = [SMALL["ising_L8_h4_m2"], SMALL["ising_L16_h5_m4"], SMALL["potts_q10_L8_h4_m4"],
            SMALL["potts_q2_L8_h3_m2"], SMALL["ising_L8_h4_m2"]]
    ctx = gpu_context(cfgs)
    sims = [oracle_sim(c, instance=i) for i, c in enumerate(cfgs)]
    F = 800
    for _ in range(12):
        ctx.run_sweeps(F)
        ctx.merge()
        ctx.exchange()
        for s in sims:
            oracle_cycle(s, F)
    for i, s in enumerate(sims):
        compare_state(ctx, i, s)


def test_graph_replay_equals_eager():
    cfg = SMALL["potts_q10_L8_h4_m4"]
    a, b = gpu_context([cfg]), gpu_context([cfg])
    a.run_cycles(37, 1000, use_graph=False)
    for _ in range(3):          # replays with eager work and syncs in between
        b.run_cycles(12, 1000, use_graph=True)
        b.status(0)
    b.run_cycles(1, 1000, use_graph=False)
    sim = oracle_sim(cfg)
    for _ in range(37):
        oracle_cycle(sim, 1000)
    compare_state(a, 0, sim)
    compare_state(b, 0, sim)


def test_checkpoint_restore_continues_bit_exactly():
    cfg = SMALL["ising_L16_h5_m4"]
    a = gpu_context([cfg])
    a.run_cycles(10, 2000)
    blob = a.checkpoint()
    a.run_cycles(10, 2000)
    b = gpu_context([cfg])
    b.restore(blob)
    b.run_cycles(10, 2000)
    for slot in range(20):
        x, y = a.get_walker(0, slot), b.get_walker(0, slot)
        assert np.array_equal(x["spins"], y["spins"]) and np.array_equal(x["lng"], y["lng"])
        assert np.array_equal(x["H"], y["H"]) and x["attempts"] == y["attempts"]
    # a blob from another configuration is refused
    c = gpu_context([SMALL["ising_L8_h4_m2"]])
    with pytest.raises(Exception):
        c.restore(blob)


def test_thermo_matches_oracle():
    cfg = SMALL["ising_L8_h4_m2"]
    ctx = gpu_context([cfg])
    sim = oracle_sim(cfg)
    ctx.run_to_convergence(500, cycles_per_check=200)
    sim.run(10 ** 8)
    T = np.linspace(1.0, 4.0, 61)
    Eg, Cg = ctx.thermo(T)
    R, _ = sim.join()
    Eo, Co = O.thermo(R, -128, 4, T)
    assert np.allclose(Eg, Eo, rtol=1e-11, atol=1e-9)
    assert np.allclose(Cg, Co, rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("prod", [0, 1])
def test_flips_not_a_multiple_of_the_rng_chunk(prod):
    """Sweeps of 1, 15, 17 and 1001 attempts (the producer hands over 16 at
    a time) with and without the producer wavefront."""
    cfg = SMALL["ising_L8_h4_m2"]
    ctx = gpu_context([cfg])
    ctx.set_launch(rng_producer=prod)
    sim = oracle_sim(cfg)
    for F in (1, 15, 17, 1001):
        ctx.run_sweeps(F)
        ctx.merge()
        ctx.exchange()
        oracle_cycle(sim, F)
        compare_state(ctx, 0, sim)


def test_zero_flips_is_a_no_op_and_negative_is_rejected():
    cfg = SMALL["ising_L8_h4_m2"]
    ctx = gpu_context([cfg])
    sim = oracle_sim(cfg)
    ctx.run_sweeps(0)
    compare_state(ctx, 0, sim)
    with pytest.raises(Exception):
        ctx.run_sweeps(-1)


def test_unreachable_window_is_reported_on_both_sides():
    # odd L = 5: frustration caps the Ising energy at +30, so a window over
    # E in [34, 50] (bins 21..25) can never be entered
    cfg = WL.config(WL.ISING, 5, n_windows=3, walkers_per_window=1, flips=100, seed=1)
    win = ([0, 10, 21], [12, 22, 25])
    sim = oracle_sim(cfg, windows=win)
    assert not sim.warm_ok
    ctx = gpu_context([cfg], windows=[win])
    assert ctx.status(0)["error"] == -7
    ctx.run_cycles(3, 100)             # a failed instance is never advanced
    st = ctx.status(0)
    assert st["merges"] == 0 and st["rounds"] == 0 and st["attempts"] == 0
    assert ctx.running() == 0


@pytest.mark.parametrize("name,page,group,prod,nib", [
    ("ising_L16_h5_m4", 16, 0, 0, -1), ("ising_L16_h5_m4", 0, 5, 1, -1),
    ("ising_L16_h5_m4", 64, 0, 1, -1),
    ("potts_q5_L12_h9_m7_ragged", 32, 13, 1, 1), ("potts_q5_L12_h9_m7_ragged", 64, 0, 0, 0),
    ("potts_q5_L12_h9_m7_ragged", 32, 0, 0, 2), ("potts_q10_L8_h4_m4", 32, 0, 1, 2),
    ("potts_q10_L8_h4_m4", 32, 3, 0, 1),
    ("potts_q20_L7_h3_m2", 32, 0, 0, 1),
    ("ising_L40_h6_m2_tworow", 16, 0, 1, -1),
    ("ising_L32_h4_m2", 16, 5, 0, -1), ("ising_L32_h4_m2", 16, 0, 1, -1),
    ("ising_L32_h4_m2", 1024, 3, 0, -1), ("ising_L32_h3_m3_fp32c", 16, 7, 1, -1),
    ("ising_L8_fp32c", 16, 0, 1, -1),
    ("potts_q10_L8_fp32c", 32, 7, 0, 1), ("potts_q10_L8_fp32c", 32, 0, 1, 0)])
def test_page_size_and_group_shape_do_not_change_results(name, page, group, prod, nib):
    """Pages much smaller than the windows make the page follow the walker
    through device memory at almost every move; with prod = 1 a second
    wavefront supplies the random numbers; nib picks the Potts lattice
    format (1: nibbles with the neighbour table, 2: nibbles without, 0:
    bytes; nibbles need q <= 16, so q = 20 keeps bytes).  Results must not
    change."""
    cfg = SMALL[name]
    ctx = gpu_context([cfg])
    plan = ctx.set_launch(page_bins=page, walkers_per_group=group, rng_producer=prod,
                          potts_nibbles=nib)
    print(f"[parity] {name}: plan {plan}", flush=True)
    (p,) = plan.values()
    assert p["page_bins"] & (p["page_bins"] - 1) == 0 and p["rng_producer"] == prod
    if nib >= 0 and cfg["model"] == WL.POTTS:
        assert p["potts_nibbles"] == (nib if cfg["q"] <= 16 else 0)
    if page:
        assert p["page_bins"] == page
    sim = oracle_sim(cfg)
    F = cfg["flips_per_exchange"]
    for seg in (3, 30):
        ctx.run_cycles(seg, F)
        for _ in range(seg):
            oracle_cycle(sim, F)
        compare_state(ctx, 0, sim)


@pytest.mark.parametrize("cfg_name,replicas,sample,page,nib", [
    ("ISING_L32", 0, (0, 1, -1), 16, -1),
    ("POTTS_Q10_L20", 3, (0, 2), 32, 1),
    ("POTTS_Q10_L20_FP32C", 2, (1,), 32, 1)])
def test_full_size_configs_sampled(cfg_name, replicas, sample, page, nib):
    """Full-size workloads in the launch shape the benchmark's autotuner
    picks (page bins, Potts nibbles, no RNG producer); sampled instances are
    checked walker by walker against the oracle."""
    cfg = getattr(WL, cfg_name)
    R = replicas or WL.bench_replicas(cfg)
    ctx = gpu_context([cfg] * R)
    plan = ctx.set_launch(page_bins=page, rng_producer=0, potts_nibbles=nib)
    print(f"[parity] {cfg_name} x{R}: plan {plan}", flush=True)
    F = cfg["flips_per_exchange"]
    cycles = 2
    ctx.run_cycles(cycles, F)
    for i in sample:
        i = i % R
        print(f"[parity] {cfg_name} x{R}: instance {i}", flush=True)
        sim = oracle_sim(cfg, instance=i)
        for _ in range(cycles):
            oracle_cycle(sim, F)
        compare_state(ctx, i, sim)


BATCH = ["potts_q5_L12_h9_m7_ragged", "ising_L16_h5_m4", "ising_L40_h6_m2_tworow", "ising_L32_h4_m2"]


@pytest.mark.parametrize("fused,splits,order,prod", [
    (0, 3, 0, -1), (1, 1, 0, 0), (1, 2, 1, 1), (1, 1, 2, 0), (1, 4, 2, 1)])
def test_batching_does_not_change_results(fused, splits, order, prod):
    """Every kernel class in one batch (Ising L <= 32 with and without the
    L = 32 rotation loop, Ising L = 40, Potts), swept per class on forked
    streams or in one fused launch in each workgroup order, in 1 to 4
    launches per sweep, with or without the RNG producer."""
    cfgs = [SMALL[n] for n in BATCH]
    ctx = gpu_context(cfgs)
    if prod >= 0:
        ctx.set_launch(rng_producer=prod)
    plan = ctx.set_batching(fused=fused, splits=splits, order=order)
    print(f"[parity] batching plan {plan}", flush=True)
    assert plan.get("batching", {"fused": 0, "splits": 1, "order": 0}) == \
        {"fused": fused, "splits": splits, "order": order}
    sims = [oracle_sim(c, instance=i) for i, c in enumerate(cfgs)]
    F = 1000
    for seg in (3, 10):
        ctx.run_cycles(seg, F, use_graph=seg > 5)
        for sim in sims:
            for _ in range(seg):
                oracle_cycle(sim, F)
        for i, sim in enumerate(sims):
            compare_state(ctx, i, sim)


def test_fused_batching_needs_one_producer_setting():
    from paper_1402_2328_amd import rewl
    ctx = gpu_context([SMALL[n] for n in BATCH])
    ctx.set_launch(cls=0, rng_producer=1)
    ctx.set_launch(cls=2, rng_producer=0)
    with pytest.raises(rewl.RewlError) as e:
        ctx.set_batching(fused=1)
    assert e.value.code == -1
    ctx.set_launch(rng_producer=0)
    assert ctx.set_batching(fused=1)["batching"]["fused"] == 1
    # a class change that splits the producer setting un-fuses the batch
    plan = ctx.set_launch(cls=1, rng_producer=1)
    assert "batching" not in plan


def test_ising_L32_balanced_split_in_the_time_to_converge_launch():
    """The benchmark's time-to-converge form of Ising L=32: 16 run-time
    balanced windows (planned here from first-iteration step counts of the
    shape a pre-run measures), 8 instances, each whole window in LDS, 24
    walkers per workgroup with the RNG producer; every instance checked in
    full after 3 cycles."""
    from paper_1402_2328_amd import rewl
    cfg = WL.ISING_L32
    lo0, hi0 = O.equal_windows(1025, 16)
    steps = [7.2e6, 2.4e6, 1.7e6, 1.2e6, 9.4e5, 6.8e5, 4.8e5, 2.7e5, 2.7e5, 4.7e5, 6.9e5, 9.2e5,
             1.2e6, 1.7e6, 2.4e6, 7.1e6]
    lo, hi = rewl.balanced_windows(1025, 16, lo0, hi0, steps)
    R = 8
    ctx = gpu_context([cfg] * R, windows=[(lo, hi)] * R)
    plan = ctx.set_launch(page_bins=1024, walkers_per_group=24, rng_producer=1)
    print(f"[parity] Ising L=32 balanced x{R}: windows {list(lo)}, plan {plan}", flush=True)
    F = cfg["flips_per_exchange"]
    ctx.run_cycles(3, F, use_graph=True)
    for i in range(R):
        sim = oracle_sim(cfg, instance=i, windows=(lo, hi))
        for _ in range(3):
            oracle_cycle(sim, F)
        compare_state(ctx, i, sim)


def test_autotune_changes_nothing_but_speed():
    """The tuner's final runs whole cycles (sweeps, merges, exchanges) from
    the saved state; afterwards every counter and the trajectory are those
    of a run that was never tuned."""
    cfg = SMALL["potts_q5_L12_h9_m7_ragged"]
    ctx = gpu_context([cfg, SMALL["ising_L16_h5_m4"], SMALL["ising_L40_h6_m2_tworow"]])
    ctx.run_cycles(4, 1500)
    keys = ("attempts", "merges", "rounds", "done", "error")
    before = [{k: ctx.status(i)[k] for k in keys} for i in range(3)]
    stages = [ctx.status(i)["stage"].copy() for i in range(3)]
    plan = ctx.autotune(1500, repeats=3)
    print(f"[parity] autotune plan {plan}", flush=True)
    for i in range(3):
        st = ctx.status(i)
        assert {k: st[k] for k in keys} == before[i]
        assert np.array_equal(st["stage"], stages[i])
    ctx.run_cycles(6, 1500)
    sims = [oracle_sim(c, instance=i) for i, c in
            enumerate([cfg, SMALL["ising_L16_h5_m4"], SMALL["ising_L40_h6_m2_tworow"]])]
    for i, sim in enumerate(sims):
        for _ in range(10):
            oracle_cycle(sim, 1500)
        compare_state(ctx, i, sim)


def test_batched_mix_all_instances():
    """The uneven 64-instance batch (Ising L up to 64, Potts q = 2..10) in one
    context, hipGraph replay; every instance checked in full."""
    mix = WL.batched_mix()
    ctx = gpu_context(mix)
    F = 10000
    cycles = 2
    ctx.run_cycles(cycles, F, use_graph=True)
    for i in range(len(mix)):
        print(f"[parity] batched mix instance {i}: {mix[i]['model']} L={mix[i]['L']}", flush=True)
        sim = oracle_sim(mix[i], instance=i)
        for _ in range(cycles):
            oracle_cycle(sim, F)
        compare_state(ctx, i, sim)


def test_batched_mix_fp32c_autotuned_sampled():
    """The 64-instance mix with two-float FP32 ln g, in the plan the
    autotuner picks for it; instances of every class checked in full."""
    mix = WL.batched_mix(precision=WL.FP32C)
    ctx = gpu_context(mix)
    F = 10000
    print(f"[parity] mix fp32c: {ctx.autotune(F, repeats=2)}", flush=True)
    ctx.run_cycles(2, F, use_graph=True)
    for i in (1, 2, 4, 6, 33, 63):
        print(f"[parity] mix fp32c instance {i}: {mix[i]['model']} L={mix[i]['L']}", flush=True)
        sim = oracle_sim(mix[i], instance=i)
        for _ in range(2):
            oracle_cycle(sim, F)
        compare_state(ctx, i, sim)


def test_batched_mix_fused_launch_sampled():
    """The 64-instance mix in one fused launch per part, the sweep cut into
    two launches, workgroups of the classes interleaved; instances of every
    class checked in full."""
    mix = WL.batched_mix()
    ctx = gpu_context(mix)
    ctx.set_launch(rng_producer=0)
    print(f"[parity] mix fused: {ctx.set_batching(fused=1, splits=2, order=2)}", flush=True)
    F = 10000
    ctx.run_cycles(2, F, use_graph=True)
    for i in (0, 2, 3, 4, 6, 13, 33, 63):
        print(f"[parity] mix fused instance {i}: {mix[i]['model']} L={mix[i]['L']}", flush=True)
        sim = oracle_sim(mix[i], instance=i)
        for _ in range(2):
            oracle_cycle(sim, F)
        compare_state(ctx, i, sim)


def test_balanced_split_pipeline_matches_oracle():
    """Equal-split pre-run (first WL iteration only) -> per-window first
    iteration steps from rewl_get_schedule -> rewl_balanced_windows -> run on
    the balanced split; every step against the oracle."""
    from oracle.balance import balanced_windows as oracle_balanced
    from paper_1402_2328_amd import rewl
    F, h = 1000, 8
    cfgs = [WL.config(WL.ISING, 16, n_windows=h, walkers_per_window=1, lnf_final=0.5, flips=F,
                      seed=s) for s in (1, 2, 3, 4)]
    ctx = gpu_context(cfgs)
    ctx.run_to_convergence(F, cycles_per_check=100)
    steps = []
    for i, c in enumerate(cfgs):
        sim = oracle_sim(c, instance=i)
        sim.run(10 ** 6)
        compare_state(ctx, i, sim)
        _, sm = ctx.get_schedule(i)
        steps.append((sm[:, 0] + 1) * F)
    g = ctx.geometry[0]
    mean = np.mean(np.array(steps, float), axis=0)
    lo, hi = rewl.balanced_windows(g["nbins"], h, g["lo"], g["hi"], mean)
    olo, ohi = oracle_balanced(g["nbins"], h, (3, 4), list(g["lo"]), list(g["hi"]), list(mean))
    assert list(lo) == olo and list(hi) == ohi
    later = [dict(c, seed=c["seed"] + 4) for c in cfgs]
    windows = [(lo, hi)] * len(later)
    ctx2 = gpu_context(later, windows=windows)
    ctx2.run_to_convergence(F, cycles_per_check=100)
    for i, c in enumerate(later):
        sim = oracle_sim(c, instance=i, windows=(lo, hi))
        sim.run(10 ** 6)
        compare_state(ctx2, i, sim)
