"""Pins for the oracle's REWL algorithm (CPU only).

The method is an iteration, so its pins are properties fixed by the
mathematics: convergence to exact densities of states (brute force, Kaufman),
Potts sum rules and low-energy counts, the stationary distribution implied by
detailed balance for fixed ln g (WL acceptance and exchange Eq. 1 together),
bookkeeping invariants, exact recovery by the joining procedure (Eq. 2) and
canonical averages (Sec. 5, Eqs. 7-8) against direct high-precision sums.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import exact_dos as X
from oracle import oracle as O
from tests.test_oracle_exact import load_ising_table, load_potts_table


def _err_vs_exact(R, exact):
    m = np.isfinite(exact)
    assert np.all(np.isfinite(R) == m), "accessible bins differ from exact"
    return float(np.max(np.abs(R[m] - exact[m])))


# ------------------------------------------------------------ bookkeeping
@pytest.mark.parametrize("model,L,q,h,m", [(O.ISING, 8, 2, 4, 2), (O.POTTS, 6, 10, 6, 2),
                                            (O.POTTS, 6, 2, 3, 3)])
def test_energy_and_histogram_bookkeeping(model, L, q, h, m):
    s = O.Sim(model=model, L=L, q=q, n_windows=h, walkers_per_window=m, flips_per_exchange=300,
              seed=5)
    assert s.warm_ok
    binw = s.info.binw
    for _ in range(30):
        s.run(1)
        for slot in range(s.info.W):
            wk = s.walker(slot)
            assert wk["E"] == O.energy(model, L, q, wk["spins"])
            w = slot // m
            b = (wk["E"] - s.info.emin) // binw
            assert s.lo[w] <= b <= s.hi[w]
            if model == O.ISING:
                assert set(np.unique(wk["spins"])) <= {-1, 1}
            else:
                assert wk["spins"].min() >= 0 and wk["spins"].max() < q
    # every configuration is carried by exactly one walker
    ids = sorted(s.walker(k)["config"] for k in range(s.info.W))
    assert ids == list(range(s.info.W))


def test_histogram_counts_attempts_and_merge_semantics():
    s = O.Sim(model=O.ISING, L=8, n_windows=4, walkers_per_window=3, flips_per_exchange=500,
              seed=11)
    s.sweep(500)
    for slot in range(s.info.W):
        assert int(s.walker(slot)["H"].sum()) == 500       # one H entry per attempt
    # run until the first merge in some window and check its effect
    before = None
    for _ in range(2000):
        before = [s.window(w)["stage"] for w in range(4)]
        s.sweep(500)
        pre = [s.walker(k) for k in range(s.info.W)]
        s.merge()
        after = [s.window(w) for w in range(4)]
        merged = [w for w in range(4) if after[w]["stage"] > before[w]]
        if merged:
            break
        s.exchange()
    assert merged
    for w in merged:
        assert after[w]["lnf"] == 0.5
        ls = [s.walker(w * 3 + k)["lng"] for k in range(3)]
        expect = ((pre[w * 3]["lng"] + pre[w * 3 + 1]["lng"]) + pre[w * 3 + 2]["lng"]) / 3.0
        for k in range(3):
            assert np.array_equal(ls[k], expect)
            assert s.walker(w * 3 + k)["H"].sum() == 0
        # flatness held for every walker over the visited union
        U = after[w]["U"].astype(bool)
        for k in range(3):
            H = pre[w * 3 + k]["H"]
            assert 5 * U.sum() * H[U].min() >= 4 * H.sum()


def test_determinism_and_instance_streams():
    a = O.Sim(model=O.ISING, L=8, n_windows=4, walkers_per_window=2, flips_per_exchange=200, seed=3)
    b = O.Sim(model=O.ISING, L=8, n_windows=4, walkers_per_window=2, flips_per_exchange=200, seed=3)
    c = O.Sim(model=O.ISING, L=8, n_windows=4, walkers_per_window=2, flips_per_exchange=200, seed=3,
              instance=1)
    for s in (a, b, c):
        s.run(20)
    wa, wb, wc = a.walker(5), b.walker(5), c.walker(5)
    assert np.array_equal(wa["spins"], wb["spins"]) and np.array_equal(wa["lng"], wb["lng"])
    assert not np.array_equal(wa["spins"], wc["spins"])


def test_warm_up_reaches_every_window_potts_q10():
    # low windows of q=10 Potts need the extreme-state restart
    s = O.Sim(model=O.POTTS, L=20, q=10, n_windows=32, walkers_per_window=1, seed=1)
    assert s.warm_ok
    for slot in range(32):
        E = s.walker(slot)["E"]
        assert s.lo[slot] <= E + 800 <= s.hi[slot]


# ------------------------------------------------------------ detailed balance
@pytest.mark.parametrize("precision", [O.FP64, O.FP32C])
def test_fixed_lng_stationary_distribution_with_exchanges(precision):
    """With ln g frozen at exact + a per-walker tilt a_i * b, WL moves plus
    exchanges (Eq. 1) must leave walker i with marginal P_i(b) ~ exp(-a_i b)
    over the accessible bins of its window."""
    L, h, m = 4, 2, 2
    exact = X.ln_g(X.brute_ising(L))
    s = O.Sim(model=O.ISING, L=L, n_windows=h, walkers_per_window=m, flips_per_exchange=16,
              lnf_init=1e-300, lnf_final=1e-301, flat=(1, 1), seed=21, precision=precision)
    tilts = [0.15, -0.12, 0.2, -0.25]
    for slot in range(h * m):
        w = slot // m
        b = np.arange(s.lo[w], s.hi[w] + 1)
        ex = np.where(np.isfinite(exact[b]), exact[b], 0.0)
        s.set_lng(slot, ex + tilts[slot] * b)
    s.run(60000)
    tries, inr, acc = s.exchange_stats()
    assert 0 < acc[0] < inr[0]
    for slot in range(h * m):
        w = slot // m
        b = np.arange(s.lo[w], s.hi[w] + 1)
        ok = np.isfinite(exact[b])
        H = s.walker(slot)["H"].astype(float)
        assert np.all(H[~ok] == 0)
        p = np.exp(-tilts[slot] * b[ok])
        p /= p.sum()
        emp = H[ok] / H[ok].sum()
        assert np.max(np.abs(emp / p - 1)) < 0.05, (slot, emp / p)


def test_exact_lng_accepts_every_in_range_exchange():
    L = 8
    exact = X.ln_g(load_ising_table(L))
    s = O.Sim(model=O.ISING, L=L, n_windows=4, walkers_per_window=3, flips_per_exchange=50,
              lnf_init=1e-300, lnf_final=1e-301, flat=(1, 1), seed=2)
    for slot in range(12):
        w = slot // 3
        b = np.arange(s.lo[w], s.hi[w] + 1)
        s.set_lng(slot, np.where(np.isfinite(exact[b]), exact[b], 0.0))
    s.run(8000)
    tries, inr, acc = s.exchange_stats()
    assert inr[:3].sum() > 1000
    assert np.array_equal(inr, acc)
    # with exact ln g every walker samples its window uniformly in energy
    for slot in range(12):
        w = slot // 3
        b = np.arange(s.lo[w], s.hi[w] + 1)
        ok = np.isfinite(exact[b])
        H = s.walker(slot)["H"][ok].astype(float)
        assert H.min() > 0.8 * H.mean()


# ------------------------------------------------------------ convergence
def test_rewl_ising_L4_matches_brute_force():
    exact = X.ln_g(X.brute_ising(4))
    errs = []
    for seed in (1, 2, 3):
        s = O.Sim(model=O.ISING, L=4, n_windows=2, walkers_per_window=4, flips_per_exchange=200,
                  lnf_final=1e-6, seed=seed)
        s.run(10 ** 7)
        assert s.status()["done"]
        R, _ = s.join()
        errs.append(_err_vs_exact(R, exact))
    # tolerance: 1.3 x the largest error over 12 seeds (0.098)
    assert max(errs) < 0.13, errs


def test_ising_L8_h4_m1_matches_exact():
    """Ising L=8, 4 windows, 1 walker, F=1000, ln f 1 -> 1e-6."""
    exact = X.ln_g(load_ising_table(8))
    errs = []
    for seed in range(1, 9):
        s = O.Sim(model=O.ISING, L=8, n_windows=4, walkers_per_window=1, flips_per_exchange=1000,
                  lnf_final=1e-6, seed=seed)
        s.run(10 ** 7)
        R, joins = s.join()
        errs.append(_err_vs_exact(R, exact))
    # m = 1 with 0.8 flatness saturates at a few tenths (WL's known floor);
    # over 12 seeds the largest error was 0.46
    assert max(errs) < 0.6, errs
    assert np.median(errs) < 0.4, errs


def test_more_walkers_per_window_reduce_error():
    """In-window merging reduces the error like 1/sqrt(m) (Sec. 2)."""
    exact = X.ln_g(load_ising_table(8))
    e1, e8 = [], []
    for seed in (1, 2):
        for m, acc in ((1, e1), (8, e8)):
            s = O.Sim(model=O.ISING, L=8, n_windows=4, walkers_per_window=m,
                      flips_per_exchange=1000, lnf_final=1e-5, seed=seed)
            s.run(10 ** 7)
            acc.append(_err_vs_exact(s.join()[0], exact))
    assert np.mean(e8) < 0.6 * np.mean(e1), (e1, e8)
    assert max(e8) < 0.15, e8


def test_rewl_potts_q3_L4_matches_brute_force():
    g = X.brute_potts(3, 4)
    exact = X.ln_g(g)
    errs = []
    for seed in (1, 2):
        s = O.Sim(model=O.POTTS, L=4, q=3, n_windows=3, walkers_per_window=4,
                  flips_per_exchange=200, lnf_final=1e-6, seed=seed)
        s.run(10 ** 7)
        R, _ = s.join()
        errs.append(_err_vs_exact(R, exact))
    # tolerance: 1.3 x the largest error over 12 seeds (0.134)
    assert max(errs) < 0.18, errs


def test_rewl_potts_q3_L6_matches_transfer_matrix():
    """q=3 Potts L=6 (3^36 states, beyond brute force) against the exact
    transfer-matrix density of states: FP64 halving to ln f = 1e-6, and the
    two-float FP32, 1/t configuration that the GPU's full-run parity test
    uses, so that the GPU result, bitwise equal to this one, is tied to
    exact values as well."""
    from paper_1402_2328_amd import workloads as WL
    from tests.parity import oracle_sim
    exact = X.ln_g(load_potts_table(3, 6))
    errs = []
    for seed in (1, 2):
        # seed 1 is also a GPU full-run parity case
        s = oracle_sim(WL.config(WL.POTTS, 6, q=3, n_windows=3, walkers_per_window=4,
                                 lnf_final=1e-6, flips=300, seed=seed))
        s.run(10 ** 8)
        assert s.status()["done"]
        errs.append(_err_vs_exact(s.join()[0], exact))
    # tolerance: 1.3 x the largest error over 12 seeds (0.122)
    assert max(errs) < 0.16, errs
    gpu_case = WL.config(WL.POTTS, 6, q=3, n_windows=3, walkers_per_window=3, lnf_final=1e-4,
                         flips=400, seed=6, precision=WL.FP32C, schedule=WL.ONE_OVER_T)
    s = oracle_sim(gpu_case)
    s.run(10 ** 8)
    assert s.status()["done"]
    # ln f stops at 1e-4: 1.3 x the largest error over 12 seeds (0.426)
    assert _err_vs_exact(s.join()[0], exact) < 0.55


def test_rewl_potts_q10_sum_rule_and_ground_counts():
    L, q = 8, 10
    N = L * L
    s = O.Sim(model=O.POTTS, L=L, q=q, n_windows=6, walkers_per_window=4,
              flips_per_exchange=2000, lnf_final=1e-5, seed=4)
    s.run(10 ** 7)
    assert s.status()["done"]
    R, _ = s.join()
    fin = np.isfinite(R)
    # normalised to g(ground) = q; sum rule sum g = q^N is then a check
    assert R[0] == pytest.approx(math.log(q), abs=1e-12)
    lse = np.max(R[fin]) + math.log(np.exp(R[fin] - np.max(R[fin])).sum())
    assert abs(lse - N * math.log(q)) < 0.15
    low = X.potts_low_energy(q, L)
    for j, v in low.items():
        if v == 0:
            assert not fin[j]
        else:
            assert abs(R[j] - math.log(v)) < 0.15, (j, R[j], math.log(v))


def test_fp32_compensated_mode_converges_like_fp64():
    exact = X.ln_g(load_ising_table(8))
    e64, e32 = [], []
    for seed in (1, 2):
        for prec, acc in ((O.FP64, e64), (O.FP32C, e32)):
            s = O.Sim(model=O.ISING, L=8, n_windows=4, walkers_per_window=4,
                      flips_per_exchange=1000, lnf_final=1e-6, seed=seed, precision=prec)
            s.run(10 ** 7)
            assert s.status()["done"]
            acc.append(_err_vs_exact(s.join()[0], exact))
    # m = 8 over 8 seeds: FP64 max 0.113, FP32C max 0.092; m = 4 is noisier
    assert max(e32) < 0.2 and max(e64) < 0.2, (e64, e32)


# ------------------------------------------------------------ joining, normalisation
@pytest.mark.parametrize("h", [3, 8, 16])
def test_stitch_recovers_exact_from_offset_pieces(h):
    L = 16
    exact = X.ln_g(load_ising_table(L))
    nb = len(exact)
    lo, hi = O.equal_windows(nb, h)
    rng = np.random.default_rng(h)
    pieces, masks = [], []
    for w in range(h):
        b = np.arange(lo[w], hi[w] + 1)
        ok = np.isfinite(exact[b])
        pieces.append(np.where(ok, exact[b], 0.0) + rng.uniform(-500, 500))
        masks.append(ok.astype(np.uint8))
    R, joins = O.stitch(lo, hi, pieces, masks, nb)
    for w in range(1, h):
        assert lo[w] + 2 <= joins[w - 1] <= hi[w - 1] - 2
    fin = np.isfinite(exact)
    assert np.array_equal(np.isfinite(R), fin)
    d = R[fin] - exact[fin]
    assert np.max(np.abs(d - d[0])) < 1e-9
    Rn = O.normalise(O.ISING, L * L, 2, R)
    assert np.max(np.abs(Rn[fin] - exact[fin])) < 1e-9


def test_stitch_join_point_is_where_derivatives_agree():
    # two pieces with equal curvature everywhere except a kink: the join must
    # avoid the kink region and land where the 5-point slopes coincide
    nb = 41
    lo, hi = np.array([0, 10]), np.array([30, 40])
    b = np.arange(nb, dtype=float)
    f = -(b - 20.0) ** 2 / 50.0
    p0 = f[0:31].copy()
    p1 = f[10:41].copy() + 7.0
    p1[: 14 - 10] += np.linspace(0.3, 0.0, 4)                  # distort the lower overlap of piece 1
    p0[26:31] += np.array([0.0, 0.1, 0.3, 0.6, 1.0])           # distort the upper overlap of piece 0
    R, joins = O.stitch(lo, hi, [p0, p1], [np.ones(31, np.uint8)] * 2, nb)
    assert 16 <= joins[0] <= 22
    assert np.allclose(R - R[0], f - f[0], atol=1e-12)


def test_normalise_potts_ground_state():
    R = np.array([0.0, -np.inf, 3.0, 5.0])
    out = O.normalise(O.POTTS, 4, 7, R)
    assert out[0] == pytest.approx(math.log(7)) and out[3] - out[2] == pytest.approx(2.0)


# ------------------------------------------------------------ thermodynamics
def test_thermo_matches_direct_sums():
    L = 16
    g = load_ising_table(L)
    lng = X.ln_g(g)
    T = np.array([1.5, 2.0, 2.269, 2.5, 3.5])
    Em, Cv = O.thermo(lng, -2 * L * L, 4, T)
    with mp.workdps(50):
        for i, t in enumerate(T):
            Z = E1 = E2 = mp.mpf(0)
            for k, v in enumerate(g):
                if v:
                    E = -2 * L * L + 4 * k
                    wgt = mp.mpf(int(v)) * mp.exp(-mp.mpf(E) / mp.mpf(t))
                    Z += wgt
                    E1 += wgt * E
                    E2 += wgt * E * E
            em = E1 / Z
            cv = (E2 / Z - em ** 2) / mp.mpf(t) ** 2
            assert Em[i] == pytest.approx(float(em), rel=1e-10)
            assert Cv[i] == pytest.approx(float(cv), rel=1e-9)
