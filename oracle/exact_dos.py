"""Exact densities of states for the 2D Ising and q-state Potts models.

TEST INFRASTRUCTURE ONLY.  These are the pins for the oracle's converged
ln g(E): the paper validates REWL on the 2D Ising model against exact results
(Sec. 4); the Potts checks are sum rules and exact low-energy counts.

Four independent routes:
  * brute-force enumeration of every configuration (small L);
  * a row-to-row transfer matrix with polynomial weights (small L);
  * Kaufman's exact partition function of the periodic L x L Ising model
    (Phys. Rev. 76, 1232 (1949)), whose integer coefficients are extracted the
    way Beale did (Phys. Rev. Lett. 76, 78 (1996)): evaluate the partition
    function as a polynomial in x = exp(-4K) at points on the unit circle in
    high precision and invert the discrete Fourier transform;
  * Onsager's bulk free energy, which ln Z / N approaches exponentially fast
    in L away from the critical point.

Energies: Ising E = -sum s_i s_j = -2N + 4k (k = 0..N); Potts
E = -sum delta(s_i, s_j) = -2N + j (j = 0..2N).
"""
import itertools

import mpmath as mp
import numpy as np


# --------------------------------------------------------------------------
# brute force
# --------------------------------------------------------------------------
def _bond_pairs(L):
    pairs = []
    for y in range(L):
        for x in range(L):
            s = y * L + x
            pairs.append((s, y * L + (x + 1) % L))
            pairs.append((s, ((y + 1) % L) * L + x))
    return np.array(pairs)


def brute_ising(L):
    """g_k, k = 0..N, by enumerating all 2^N configurations (N <= 20)."""
    N = L * L
    assert N <= 20
    idx = np.arange(1 << N, dtype=np.int64)
    spins = (((idx[:, None] >> np.arange(N)) & 1) * 2 - 1).astype(np.int8)
    pr = _bond_pairs(L)
    E = -(spins[:, pr[:, 0]].astype(np.int32) * spins[:, pr[:, 1]]).sum(axis=1)
    k = (E + 2 * N) // 4
    return np.bincount(k, minlength=N + 1).astype(object)


def brute_potts(q, L):
    """counts c_j of E = -2N + j, j = 0..2N, by full enumeration.

    Every configuration is visited; configurations are indexed by their L row
    states so the energy of all q^N of them is one broadcast sum of in-row and
    row-to-row bond counts (q^N <= 5e7).
    """
    N = L * L
    assert q ** N <= 5 * 10 ** 7
    rows = np.array(list(itertools.product(range(q), repeat=L)))
    a = (rows != np.roll(rows, -1, axis=1)).sum(axis=1).astype(np.int16)
    b = (rows[:, None, :] != rows[None, :, :]).sum(axis=2).astype(np.int16)
    R = len(rows)
    shape = [R] * L
    bad = np.zeros(shape, dtype=np.int16)
    for i in range(L):
        ai = a.reshape([R if d == i else 1 for d in range(L)])
        j = (i + 1) % L
        bi = b.reshape([R if d in (i, j) else 1 for d in range(L)] if i < j else
                       [R if d in (i, j) else 1 for d in range(L)])
        if i > j:  # wrap-around pair (row L-1, row 0): b is symmetric
            bi = b.T.reshape([R if d in (i, j) else 1 for d in range(L)])
        bad = bad + ai + bi
    counts = np.bincount(bad.reshape(-1), minlength=2 * N + 1)
    return counts.astype(object)


# --------------------------------------------------------------------------
# transfer matrix (rows of L spins, periodic in both directions)
# --------------------------------------------------------------------------
def transfer_counts(q, L):
    """counts of 'bad' bonds (unequal neighbours), index 0..2N, via Tr(T^L).

    For Ising (q = 2) the energy is E = -2N + 2 * bad; for Potts
    E = -2N + bad.
    """
    N = L * L
    states = list(itertools.product(range(q), repeat=L))
    S = len(states)
    arr = np.array(states)
    a = (arr != np.roll(arr, -1, axis=1)).sum(axis=1)           # in-row bad bonds
    b = (arr[:, None, :] != arr[None, :, :]).sum(axis=2)         # b[s, s'] vertical
    D = 2 * N + 1
    dt = np.int64 if q ** N < 2 ** 62 else object
    v = np.zeros((S, S, D), dtype=dt)                            # [start, current, degree]
    for s in range(S):
        v[s, s, a[s]] = 1
    for _ in range(L - 1):
        nv = np.zeros_like(v)
        for sp in range(S):
            for sh in np.unique(b[:, sp]):
                src = v[:, b[:, sp] == sh, :].sum(axis=1)
                tot = sh + a[sp]
                nv[:, sp, tot:] += src[:, : D - tot]
        v = nv
    Z = np.zeros(D, dtype=object)
    for s0 in range(S):
        for s in range(S):
            sh = b[s, s0]
            Z[sh:] += v[s0, s, : D - sh].astype(object)
    return Z


def transfer_ising(L):
    bad = transfer_counts(2, L)
    N = L * L
    return np.array([bad[2 * k] for k in range(N + 1)], dtype=object)


def transfer_potts(q, L):
    return transfer_counts(q, L)


# --------------------------------------------------------------------------
# Kaufman / Beale: exact Ising DOS for even L
# --------------------------------------------------------------------------
def _cheb(n, c):
    t0, t1 = mp.mpf(1), c
    if n == 0:
        return t0
    for _ in range(n - 1):
        t0, t1 = t1, 2 * c * t1 - t0
    return t1


def kaufman_Z(L, z):
    """Kaufman's torus partition function as a function of z = exp(2K).

    Z = 1/2 (2 sinh 2K)^{N/2} (Z1 + Z2 + Z3 + Z4) with
    cosh(gamma_l) = cosh 2K coth 2K - cos(l pi / L), e^{gamma_0} = e^{2K} tanh K,
    e^{gamma_L} = e^{2K} coth K.  Products over gamma_l = gamma_{2L-l} pairs are
    written as polynomials of cosh(gamma_l) through Chebyshev T_L, so the
    expression has no branch ambiguity at complex z.
    """
    assert L % 2 == 0
    N = L * L
    C = (z * z + 1) ** 2 / (2 * z * (z * z - 1))
    Z1 = Z2 = Z3 = Z4 = mp.mpf(1)
    for l in range(1, L, 2):
        T = _cheb(L, C - mp.cospi(mp.mpf(l) / L))
        Z1 *= 2 + 2 * T
        Z2 *= 2 * T - 2
    for l in range(2, L, 2):
        T = _cheb(L, C - mp.cospi(mp.mpf(l) / L))
        Z3 *= 2 + 2 * T
        Z4 *= 2 * T - 2
    A0 = (z * (z - 1) / (z + 1)) ** (L // 2)
    AL = (z * (z + 1) / (z - 1)) ** (L // 2)
    Z3 *= (A0 + 1 / A0) * (AL + 1 / AL)
    Z4 *= (A0 - 1 / A0) * (AL - 1 / AL)
    pre = (z - 1 / z) ** (N // 2)
    return pre * (Z1 + Z2 + Z3 + Z4) / 2


def kaufman_ising(L, dps=None):
    """Integer g_k (E = -2N + 4k), k = 0..N, from Kaufman's formula.

    P(x) = Z z^{-N} = sum_k g_k x^k with x = z^{-2}; P is sampled at
    x_j = exp(2 pi i (j + 1/2)/(N+1)) (half-step shift keeps z away from the
    poles of the individual factors at z = +-1) and the coefficients are
    recovered by the inverse DFT and rounded.  Returns (g, max distance of the
    raw coefficients from the nearest integer).
    """
    N = L * L
    M = N + 1
    if dps is None:
        dps = int(N * 0.30103 * 1.6) + 80
    with mp.workdps(dps):
        P = []
        for j in range(M):
            th = mp.mpf(j) + mp.mpf(1) / 2
            z = mp.expjpi(-th / M)                      # z = x^{-1/2}
            P.append(kaufman_Z(L, z) * z ** (-N))
        roots = [mp.expjpi(mp.mpf(-2 * n) / M) for n in range(M)]
        g = []
        worst = mp.mpf(0)
        for k in range(M):
            acc = mp.mpc(0)
            for j in range(M):
                acc += P[j] * roots[(j * k) % M]
            c = acc * mp.expjpi(mp.mpf(-k) / M) / M
            n = int(mp.nint(c.real))
            worst = max(worst, abs(c.real - n), abs(c.imag))
            g.append(n)
    return np.array(g, dtype=object), float(worst)


def onsager_lnZ_per_site(K):
    """Onsager's bulk -beta f of the square-lattice Ising model."""
    K = mp.mpf(K)
    kap = 2 * mp.sinh(2 * K) / mp.cosh(2 * K) ** 2
    f = lambda th: mp.log((1 + mp.sqrt(1 - kap ** 2 * mp.sin(th) ** 2)) / 2)
    return mp.log(2 * mp.cosh(2 * K)) + mp.quad(f, [0, mp.pi]) / (2 * mp.pi)


def lnZ_from_dos(g, L, K, model="ising", q=2):
    """ln sum_E g(E) exp(-K E) for an integer DOS table."""
    N = L * L
    K = mp.mpf(K)
    acc = mp.mpf(0)
    for i, gi in enumerate(g):
        if gi:
            E = -2 * N + (4 * i if model == "ising" else i)
            acc += mp.mpf(int(gi)) * mp.exp(-K * E)
    return mp.log(acc)


def ln_g(g):
    """FP64 natural logs of a non-negative integer table (-inf for zero)."""
    out = np.empty(len(g))
    for i, v in enumerate(g):
        out[i] = float(mp.log(int(v))) if v else -np.inf
    return out


# --------------------------------------------------------------------------
# Potts: what is exact at any size
# --------------------------------------------------------------------------
def potts_low_energy(q, L):
    """Exact counts at E = -2N + j for j = 0..7 (periodic L >= 4).

    j=0: q uniform ground states; j=4: one spin differs (N q (q-1));
    j=6: an adjacent pair differs with equal values (2N q (q-1));
    j=7: an adjacent pair with two distinct new values (2N q (q-1)(q-2));
    j=1,2,3,5: impossible.
    """
    N = L * L
    return {0: q, 1: 0, 2: 0, 3: 0, 4: N * q * (q - 1), 5: 0,
            6: 2 * N * q * (q - 1), 7: 2 * N * q * (q - 1) * (q - 2)}
