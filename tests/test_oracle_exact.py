"""Pins for the exact densities of states the oracle is checked against (CPU).

Brute force, a transfer matrix, Kaufman's torus formula and Onsager's bulk
free energy are independent routes; they are checked against each other and
against sum rules and exact low-energy counts.
"""
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import exact_dos as X

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_ising_table(L):
    with open(os.path.join(GOLD, f"ising_dos_L{L}.txt")) as f:
        return np.array([int(x) for x in f if not x.startswith("#")], dtype=object)


def load_potts_table(q, L):
    """Counts of E = -2N + j, j = 0..2N (tests/golden/make_exact_potts.py)."""
    with open(os.path.join(GOLD, f"potts_dos_q{q}_L{L}.txt")) as f:
        return np.array([int(x) for x in f if not x.startswith("#")], dtype=object)


def test_three_routes_agree_L4():
    b = X.brute_ising(4)
    t = X.transfer_ising(4)
    k, worst = X.kaufman_ising(4)
    assert list(b) == list(t) == list(k)
    assert worst < 1e-30
    assert [v for v in b if v] == [2, 32, 64, 424, 1728, 6688, 13568, 20524, 13568,
                                   6688, 1728, 424, 64, 32, 2]


def test_kaufman_equals_transfer_matrix_L6():
    k, _ = X.kaufman_ising(6)
    assert list(k) == list(X.transfer_ising(6))


@pytest.mark.parametrize("L", [8, 16, 24, 32])
def test_stored_ising_tables(L):
    g = load_ising_table(L)
    N = L * L
    assert len(g) == N + 1
    assert sum(g) == 2 ** N
    assert list(g) == list(g[::-1])                      # E -> -E (bipartite lattice)
    assert g[0] == 2 and g[1] == 0                       # ground states; no E = -2N + 4
    assert g[2] == 2 * N and g[3] == 4 * N               # one flipped spin; adjacent pair
    assert all(v >= 0 for v in g)


def test_stored_L8_table_equals_live_kaufman():
    k, _ = X.kaufman_ising(8)
    assert list(k) == list(load_ising_table(8))


@pytest.mark.parametrize("L", [16, 24, 32])
@pytest.mark.parametrize("K", [0.2, 0.8])
def test_tables_approach_onsager(L, K):
    # away from K_c = 0.4407 the finite-size correction to ln Z / N is
    # exponentially small (correlation length < 1 here); in the ordered phase
    # the two ground-state sectors add exactly ln 2 to ln Z
    g = load_ising_table(L)
    N = L * L
    with mp.workdps(60):
        lnz = X.lnZ_from_dos(g, L, K)
        bulk = X.onsager_lnZ_per_site(K) * N
        if K > 0.4407:
            bulk += mp.log(2)
        assert abs(lnz - bulk) < 1e-6


def test_potts_brute_equals_transfer_and_low_energy_counts():
    b = X.brute_potts(3, 4)
    t = X.transfer_potts(3, 4)
    assert list(b) == list(t)
    assert sum(b) == 3 ** 16
    assert list(b[:9]) == [3, 0, 0, 0, 96, 0, 192, 192, 1800]
    low = X.potts_low_energy(3, 4)
    for j, v in low.items():
        assert b[j] == v


def test_potts_q2_is_ising():
    # delta(s,s') = (1 + sigma sigma')/2  =>  E_Potts = -N + E_Ising / 2
    p = X.transfer_potts(2, 4)
    g = X.brute_ising(4)
    N = 16
    for k, v in enumerate(g):
        EI = -2 * N + 4 * k
        EP = -N + EI // 2
        assert p[EP + 2 * N] == v


def test_potts_low_energy_counts_q4_L4_transfer():
    # q^L row states: q = 4, L = 4 keeps the transfer matrix small
    t = X.transfer_potts(4, 4)
    low = X.potts_low_energy(4, 4)
    for j, v in low.items():
        assert t[j] == v
    assert sum(t) == 4 ** 16


def test_stored_potts_q3_L6_table():
    """The q=3 L=6 table (3^36 states, beyond brute force) against what does
    not come from the transfer matrix: the sum rule, the exact low-energy
    counts, and the first three moments of E over all states.  With every
    configuration equally likely, each bond's indicator delta(s_i, s_j) is
    Bernoulli(1/q), and any three distinct bonds are independent (the
    shortest cycle of the square lattice has four bonds), so the mean,
    variance and third central moment of E = -sum delta are those of a sum of
    2N independent Bernoulli(1/q) variables."""
    q, L = 3, 6
    N = L * L
    c = load_potts_table(q, L)
    assert len(c) == 2 * N + 1
    total = sum(c)
    assert total == q ** N
    for j, v in X.potts_low_energy(q, L).items():
        assert c[j] == v, j
    E = [mp.mpf(-2 * N + j) for j in range(2 * N + 1)]
    with mp.workdps(80):
        m1 = mp.fsum(mp.mpf(int(v)) * e for v, e in zip(c, E)) / total
        m2 = mp.fsum(mp.mpf(int(v)) * (e - m1) ** 2 for v, e in zip(c, E)) / total
        m3 = mp.fsum(mp.mpf(int(v)) * (e - m1) ** 3 for v, e in zip(c, E)) / total
        p = mp.mpf(1) / q
        nb = 2 * N
        assert abs(m1 - (-nb * p)) < mp.mpf("1e-60")
        assert abs(m2 - nb * p * (1 - p)) < mp.mpf("1e-60")
        # E = -sum delta, so its third central moment is minus that of the sum
        assert abs(m3 - (-nb * p * (1 - p) * (1 - 2 * p))) < mp.mpf("1e-60")
