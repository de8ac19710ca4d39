"""Pins for the oracle's building blocks (CPU only).

Each check compares the oracle with something other than itself: an
independent library implementation, libm / mpmath, exact rational arithmetic,
brute-force enumeration or a closed form.
"""
import math
import os
import shutil
import subprocess
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------- Philox
@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("kat") / "kat"
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950",
                           os.path.join(HERE, "rocrand_philox_kat.cpp"), "-o", str(out)],
                          stderr=subprocess.DEVNULL)
    return str(out)


def test_philox_matches_rocrand(rocrand_kat):
    rng = np.random.default_rng(1234)
    rows = []
    for i in range(400):
        c = rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        k = rng.integers(0, 2 ** 32, 2, dtype=np.uint64).astype(np.uint32)
        c[1] &= 0x3FFFFFFF
        if i < 3:
            c[:] = [0, 0, 0, 0][:4] if i == 0 else c
            k[:] = [0, 0] if i == 0 else k
        rows.append((c, k))
    inp = "\n".join(" ".join(f"{int(v):x}" for v in [*c, *k]) for c, k in rows) + "\n"
    res = subprocess.run([rocrand_kat], input=inp, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().split("\n")
    assert len(lines) == len(rows)
    for (c, k), line in zip(rows, lines):
        want = [int(x, 16) for x in line.split()]
        got = [int(v) for v in O.philox(c, k)]
        assert got == want, (c, k)


def test_philox_zero_block_known_answer():
    # All-zero counter and key (the first known-answer vector of the Philox
    # paper's reference distribution); also produced by rocRAND above.
    assert [hex(int(v)) for v in O.philox([0, 0, 0, 0], [0, 0])] == \
        ["0x6627e8d5", "0xe169c58d", "0xbc57ac4c", "0x9b00dbd8"]


# ----------------------------------------------------------------- exp
def _ulp_diff(a, b):
    ia = np.float64(a).view(np.int64)
    ib = np.float64(b).view(np.int64)
    return abs(int(ia) - int(ib))


def test_exp_spec_within_one_ulp_of_libm():
    rng = np.random.default_rng(7)
    xs = np.concatenate([-rng.random(20000) * 40.0, -rng.random(5000) * 1e-3,
                         [-40.0, -1e-300, -5e-324, -0.5, -math.log(2) / 2, -1.0, -39.999]])
    worst = 0
    for x in xs:
        worst = max(worst, _ulp_diff(O.exp_spec(x), math.exp(x)))
    assert worst <= 1


def test_exp_spec_mpmath_error_bound():
    mp.mp.dps = 40
    rng = np.random.default_rng(8)
    for x in -rng.random(300) * 40.0:
        e = O.exp_spec(float(x))
        ref = mp.exp(mp.mpf(float(x)))
        assert abs((mp.mpf(e) - ref) / ref) < 2.5 * 2.0 ** -53


def test_expf_spec_error_bound():
    mp.mp.dps = 30
    rng = np.random.default_rng(9)
    for x in np.float32(-rng.random(3000) * 17.0):
        e = O.expf_spec(float(x))
        ref = mp.exp(mp.mpf(float(x)))
        assert abs((mp.mpf(e) - ref) / ref) < 2.0 * 2.0 ** -24


def test_accept_rule_semantics():
    # min[1, exp(delta)]: delta >= 0 always accepted
    assert O.accept64(2 ** 53 - 1, 0.0) and O.accept64(2 ** 53 - 1, 3.0)
    # u = 0 accepts any finite delta
    assert O.accept64(0, -1000.0)
    # u = 1/2 vs exp(-ln 2 +- tiny)
    half = 1 << 52
    assert not O.accept64(half, -math.log(2) - 1e-9)
    assert O.accept64(half, -math.log(2) + 1e-9)
    # below -40 only u == 0 accepts (exp(-40) < 2^-53)
    assert math.exp(-40.0) < 2.0 ** -53
    assert not O.accept64(1, -40.5)
    assert O.accept64(1, -36.0)
    # fp32 variant
    assert math.exp(-17.0) < 2.0 ** -24
    assert O.accept32(0, -30.0) and not O.accept32(1, -17.5)
    assert O.accept32(1 << 23, -0.69) and not O.accept32(1 << 23, -0.70)


# ----------------------------------------------------------------- two-float
def _df_exact(h, l):
    return Fraction(float(np.float32(h))) + Fraction(float(np.float32(l)))


def test_two_float_add_is_nearly_exact():
    rng = np.random.default_rng(3)
    for _ in range(3000):
        ah = np.float32(rng.uniform(-5000, 5000))
        al = np.float32(rng.uniform(-1, 1) * abs(float(np.spacing(ah))) / 2)
        b = np.float32(2.0 ** -int(rng.integers(0, 30)))
        rh, rl = O.df_add1(float(ah), float(al), float(b))
        exact = _df_exact(ah, al) + Fraction(float(b))
        assert abs(_df_exact(rh, rl) - exact) <= abs(exact) * Fraction(1, 2 ** 44)
        assert abs(rl) <= abs(float(np.spacing(np.float32(rh))))
        bh = np.float32(rng.uniform(-5000, 5000))
        bl = np.float32(rng.uniform(-1, 1) * abs(float(np.spacing(bh))) / 2)
        rh, rl = O.df_add(float(ah), float(al), float(bh), float(bl))
        exact = _df_exact(ah, al) + _df_exact(bh, bl)
        # the non-IEEE ("sloppy") double-float sum is accurate relative to its
        # operands; merge sums only add ln g values of one sign
        scale = abs(_df_exact(ah, al)) + abs(_df_exact(bh, bl))
        assert abs(_df_exact(rh, rl) - exact) <= scale * Fraction(1, 2 ** 44)


def test_two_float_div_by_walker_count():
    rng = np.random.default_rng(4)
    for _ in range(3000):
        ah = np.float32(rng.uniform(0, 40000))
        al = np.float32(rng.uniform(-1, 1) * abs(float(np.spacing(ah))) / 2)
        m = int(rng.integers(1, 17))
        rh, rl = O.df_div_int(float(ah), float(al), m)
        exact = _df_exact(ah, al) / m
        assert abs(_df_exact(rh, rl) - exact) <= max(abs(exact), 1) * Fraction(1, 2 ** 44)


def test_plain_fp32_drops_small_increments_two_float_keeps_them():
    # The reason for the compensated form: ln f ~ 1e-8 vanishes on ln g ~ 1e3.
    x = np.float32(1234.5)
    assert np.float32(x + np.float32(2.0 ** -27)) == x
    h, l = float(x), 0.0
    for _ in range(1000):
        h, l = O.df_add1(h, l, 2.0 ** -27)
    assert _df_exact(h, l) == Fraction(float(x)) + 1000 * Fraction(1, 2 ** 27)


# ----------------------------------------------------------------- model
def _energy_np(model, L, spins):
    s = spins.reshape(L, L).astype(np.int64)
    r, d = np.roll(s, -1, 1), np.roll(s, -1, 0)
    if model == O.ISING:
        return int(-(s * r).sum() - (s * d).sum())
    return int(-(s == r).sum() - (s == d).sum())


@pytest.mark.parametrize("model,L,q", [(O.ISING, 8, 2), (O.ISING, 5, 2), (O.POTTS, 6, 10),
                                       (O.POTTS, 4, 2), (O.POTTS, 7, 3)])
def test_energy_matches_independent_formula(model, L, q):
    rng = np.random.default_rng(L * 31 + q)
    for _ in range(50):
        if model == O.ISING:
            sp = (rng.integers(0, 2, L * L) * 2 - 1).astype(np.int8)
        else:
            sp = rng.integers(0, q, L * L).astype(np.int8)
        assert O.energy(model, L, q, sp) == _energy_np(model, L, sp)


# ----------------------------------------------------------------- windows
def test_equal_windows_cfg_sizes():
    lo, hi = O.equal_windows(65, 4)
    assert list(lo) == [0, 9, 18, 27] and list(hi) == [37, 46, 55, 64]
    lo, hi = O.equal_windows(1025, 16)
    assert lo[0] == 0 and hi[-1] == 1024
    assert set(np.diff(lo)) <= {53, 54, 55}
    assert set((hi - lo + 1).tolist()) <= {216, 217}
    lo, hi = O.equal_windows(801, 32)
    assert set((hi - lo + 1).tolist()) <= {92, 93}


@pytest.mark.parametrize("nbins,h", [(65, 4), (1025, 16), (801, 32), (257, 8), (4097, 48), (101, 1)])
def test_equal_windows_overlap_three_quarters(nbins, h):
    lo, hi = O.equal_windows(nbins, h)
    S = nbins - 1
    W = S / (1 + (h - 1) * 0.25)
    for i in range(h):
        assert abs(lo[i] - i * 0.25 * W) <= 0.5 and abs(hi[i] - (i * 0.25 + 1) * W) <= 0.5
    assert lo[0] == 0 and hi[-1] == S
    for i in range(h - 1):
        ov = (hi[i] - lo[i + 1]) / (hi[i] - lo[i])
        assert abs(ov - 0.75) < 2.5 / (hi[i] - lo[i])
