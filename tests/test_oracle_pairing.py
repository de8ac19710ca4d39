"""Pins for the oracle's exchange pairing (CPU only).

Sec. 2: a walker of window w swaps configurations with a walker of the
neighbouring window chosen at random.  The oracle pairs walker k of window w
with walker pi(k) of window w+1, pi a random permutation drawn per round and
window pair.  The pins below hold for that reading whatever the random
stream: pi must be uniform over all m! permutations (chi-square over every
permutation for m = 3 and 4, and over every (k, pi(k)) cell for m = 7), and
the exchange round must actually pair walkers by that pi.  The detailed
balance and exact-ln g pins elsewhere hold for any pairing that does not look
at the state, so they cannot tell a uniform shuffle from, say, Sattolo's
(cyclic permutations only) or a shuffle that skips its last swap.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import exact_dos as X
from oracle import oracle as O
from tests.test_oracle_exact import load_ising_table

# the chi-square statistic of a correct shuffle exceeds this quantile with
# probability 1e-6; the inputs are fixed, so the test is deterministic
P_FAIL = 1e-6


def _perm_counts(m, draws, seed=1, instance=0):
    perms = {p: 0 for p in itertools.permutations(range(m))}
    n = 0
    for t in itertools.count():
        for w in range(4):
            pi = O.exchange_pairing(seed, instance, t, w, m)
            perms[tuple(int(x) for x in pi)] += 1
            n += 1
            if n == draws:
                return perms


@pytest.mark.parametrize("m,draws,seed,instance", [(3, 30000, 1, 0), (4, 48000, 1, 0),
                                                   (4, 24000, 7, 3)])
def test_pairing_is_uniform_over_all_permutations(m, draws, seed, instance):
    counts = _perm_counts(m, draws, seed, instance)
    obs = np.array(list(counts.values()), float)
    assert len(obs) == math.factorial(m)
    assert obs.min() > 0, "some permutations never occur"
    exp = draws / len(obs)
    chi2 = float(np.sum((obs - exp) ** 2 / exp))
    assert chi2 < stats.chi2.isf(P_FAIL, len(obs) - 1), (chi2, counts)


def test_pairing_marginals_are_uniform_for_larger_windows():
    m, draws = 7, 35000
    tab = np.zeros((m, m))
    for t in range(draws // 5):
        for w in range(5):
            pi = O.exchange_pairing(3, 1, t, w, m)
            assert sorted(pi) == list(range(m))
            tab[np.arange(m), pi] += 1
    exp = draws / m
    chi2 = float(np.sum((tab - exp) ** 2 / exp))
    # (m - 1)^2 degrees of freedom for a table with fixed row and column sums
    assert chi2 < stats.chi2.isf(P_FAIL, (m - 1) ** 2), chi2


def test_pairing_depends_on_round_window_seed_and_instance():
    base = O.exchange_pairing(1, 0, 5, 2, 16)
    assert sorted(base) == list(range(16))
    assert np.array_equal(base, O.exchange_pairing(1, 0, 5, 2, 16))
    for args in ((1, 0, 6, 2), (1, 0, 5, 3), (2, 0, 5, 2), (1, 1, 5, 2)):
        assert not np.array_equal(base, O.exchange_pairing(*args, 16)), args
    assert list(O.exchange_pairing(1, 0, 0, 0, 1)) == [0]


def test_exchange_round_pairs_walkers_by_the_pairing():
    """With every walker's ln g set to the exact ln g, Eq. (1) gives
    ln P = 0, so every in-range proposal is accepted: after round t the
    configuration carried by walker (w, k) must be the one that walker
    (w+1, pi(k)) carried, when both energies lie in the partner windows,
    and unchanged otherwise (w = t mod 2)."""
    L, h, m = 8, 4, 5
    exact = X.ln_g(load_ising_table(L))
    s = O.Sim(model=O.ISING, L=L, n_windows=h, walkers_per_window=m, flips_per_exchange=40,
              lnf_init=1e-300, lnf_final=1e-301, flat=(1, 1), seed=9, instance=2)
    for slot in range(h * m):
        w = slot // m
        b = np.arange(s.lo[w], s.hi[w] + 1)
        s.set_lng(slot, np.where(np.isfinite(exact[b]), exact[b], 0.0))
    swaps = 0
    for t in range(40):
        s.sweep(40)
        s.merge()
        before = [s.walker(k) for k in range(h * m)]
        assert s.status()["rounds"] == t
        s.exchange()
        after = [s.walker(k) for k in range(h * m)]
        moved = set()
        for w in range(t % 2, h - 1, 2):
            pi = O.exchange_pairing(9, 2, t, w, m)
            for k in range(m):
                i, j = w * m + k, (w + 1) * m + int(pi[k])
                bi = (before[i]["E"] - s.info.emin) // s.info.binw
                bj = (before[j]["E"] - s.info.emin) // s.info.binw
                inr = s.lo[w] <= bj <= s.hi[w] and s.lo[w + 1] <= bi <= s.hi[w + 1]
                if inr:
                    assert after[i]["config"] == before[j]["config"]
                    assert after[j]["config"] == before[i]["config"]
                    assert after[i]["E"] == before[j]["E"] and after[j]["E"] == before[i]["E"]
                    moved |= {i, j}
                    swaps += 1
        for k in range(h * m):
            if k not in moved:
                assert after[k]["config"] == before[k]["config"], (t, k)
    assert swaps > 100
