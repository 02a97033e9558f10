"""Pins for the oracle's random words and acceptance thresholds.

Philox4x32-10 is pinned against an independent implementation (rocRAND's
host-callable engine, compiled and run here as a black box).  The thresholds
are pinned to their closed form thr_k = floor(exp(-4k/T) 2^32) (eq. 9 with the
uint32 floor quantisation), evaluated here in 60-digit decimal arithmetic, by
properties of the exponential and by their limits.
"""
from decimal import Decimal, localcontext
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rr")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_probe.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return exe


def _cases():
    rng = np.random.default_rng(20141120)
    cases = [(0, 0, 0, 0, 0), (1, 0, 0, 0, 0), (0, 1, 0, 0, 0), (0, 0, 1, 0, 0),
             (0, 0, 0, 1, 0), (0, 0, 0, 0, 1), ((1 << 64) - 1, 0xffffffff, (1 << 30) - 1,
                                                0xffffffff, 0xffffffff)]
    for _ in range(200):
        seed = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        c0 = int(rng.integers(0, 1 << 32))
        c1 = int(rng.integers(0, 1 << 30))
        c2 = int(rng.integers(0, 1 << 32))
        c3 = int(rng.integers(0, 1 << 32))
        cases.append((seed, c0, c1, c2, c3))
    return cases


def test_philox_matches_rocrand(oracle_mod, rocrand_probe):
    cases = _cases()
    text = "".join(f"{s} {a} {b} {c} {d}\n" for s, a, b, c, d in cases)
    out = subprocess.run([rocrand_probe], input=text, capture_output=True, text=True, check=True)
    ref = [tuple(int(v) for v in line.split()) for line in out.stdout.strip().splitlines()]
    assert len(ref) == len(cases)
    for (seed, c0, c1, c2, c3), want in zip(cases, ref):
        got = oracle_mod.philox4x32_10([c0, c1, c2, c3], [seed & 0xffffffff, seed >> 32])
        assert tuple(int(v) for v in got) == want, (seed, c0, c1, c2, c3)


def test_site_word_keying(oracle_mod):
    """The site word is word (h & 3) of the block at counter
    (aux, h>>2, tag<<8 | colour<<1 | replica, sample) under key = seed."""
    seed = 0x123456789ABCDEF
    for (sample, tag, aux, colour, rep, h) in [(0, 0, 0, 0, 0, 0), (3, 0, 99, 1, 1, 4097),
                                               (7, 1, 2, 1, 0, 13), (0, 2, 0, 0, 1, 6)]:
        blk = oracle_mod.philox4x32_10([aux, h >> 2, (tag << 8) | (colour << 1) | rep, sample],
                                       [seed & 0xffffffff, seed >> 32])
        assert oracle_mod.site_word(seed, sample, tag, aux, colour, rep, h) == int(blk[h & 3])


def test_site_words_look_uniform(oracle_mod):
    """Words across sites, sweeps and replicas are uniform and uncorrelated
    (chi-square on the top 4 bits, and no agreement between replicas)."""
    n = 4096
    w0 = np.array([oracle_mod.site_word(5, 0, 0, 17, 0, 0, h) for h in range(n)], dtype=np.uint64)
    w1 = np.array([oracle_mod.site_word(5, 0, 0, 17, 0, 1, h) for h in range(n)], dtype=np.uint64)
    w2 = np.array([oracle_mod.site_word(5, 0, 0, 18, 0, 0, h) for h in range(n)], dtype=np.uint64)
    for w in (w0, w1, w2):
        counts = np.bincount((w >> 28).astype(np.int64), minlength=16)
        chi2 = float(((counts - n / 16) ** 2 / (n / 16)).sum())
        assert chi2 < 50.0  # 15 dof; p ~ 1e-5
    assert np.count_nonzero(w0 == w1) == 0 and np.count_nonzero(w0 == w2) == 0


def test_thresholds_limits(oracle_mod):
    assert list(oracle_mod.thresholds(0.0)) == [0, 0, 0]
    assert list(oracle_mod.thresholds(1e300)) == [0xffffffff] * 3
    # monotone in T and in k
    prev = None
    for T in [0.3, 0.5, 0.7, 1.0, 2.0, 5.0]:
        thr = [int(v) for v in oracle_mod.thresholds(T)]
        assert thr[0] > thr[1] >= thr[2] >= 0
        assert thr[1] > thr[2] or thr[1] == 0 or thr[2] == 0
        if prev:
            assert all(a > b or b == a == 0 for a, b in zip(thr, prev))
            assert all(a >= b for a, b in zip(thr, prev))
        prev = thr


@pytest.mark.parametrize("T", [0.5, 0.6, 0.7, 0.8, 1.0, 1.2, 2.0, 4.5])
def test_thresholds_are_powers_of_one_factor(oracle_mod, T):
    """Eq. (9) gives acceptance exp(-dE/T) with dE = 4k, so
    thr_k / 2^32 = a^k for one a in (0,1): thr_2 ~ thr_1^2 / 2^32 and
    thr_3 ~ thr_1 thr_2 / 2^32, each within the floor's rounding."""
    t1, t2, t3 = (int(v) for v in oracle_mod.thresholds(T))
    two32 = float(1 << 32)
    a = (t1 + 0.5) / two32
    # floor loses < 1 unit; propagate that bound through the products
    assert abs(t2 - (t1 / two32) ** 2 * two32) <= 2.5
    assert abs(t3 - (t1 / two32) * (t2 / two32) * two32) <= 2.5
    # and the factor is the Boltzmann weight of dE = 4 at temperature T
    assert abs(math.log(a) * T + 4.0) < 1e-6 * max(1.0, T) or t1 < 1000


# floor(exp(-4k/T) 2^32) for k = 1, 2, 3, worked out in 60-digit decimals
# (eq. 9 for dE = 4, 8, 12 and the floor rule of the uint32 compare).  The
# fractional parts are listed so that the table shows which entries a
# rounding or ceiling rule would change: at T = 0.6 thr_3 is 8.85 -> 8.
EXACT_THRESHOLDS = {
    0.5: (1440801, 483, 0),
    0.6: (5465920, 6956, 8),        # fractions .557 .115 .853
    0.7: (14166974, 46729, 154),    # fractions .347 .846 .139
    0.8: (28939262, 194991, 1313),  # fractions .003 .214 .840
    1.0: (78665070, 1440801, 26389),
    1.2: (153218634, 5465920, 194991),
    0.513: (1764607, 724, 0),       # thr_2 = 724.997
    0.569: (3801220, 3364, 2),      # thr_3 = 2.977
    2.0: (581260615, 78665070, 10646159),
}


def _exact_floor(T: float, k: int) -> tuple[int, float]:
    """floor(exp(-4k/T) 2^32) and its fractional part, in 60-digit decimals
    (T taken as the exact binary value of the double)."""
    with localcontext() as ctx:
        ctx.prec = 60
        v = (Decimal(-4 * k) / Decimal(T)).exp() * Decimal(1 << 32)
        f = int(v)
        return f, float(v - f)


def test_threshold_table_is_the_closed_form():
    """The literal table above is floor(exp(-4k/T) 2^32) (checks the table)."""
    for T, want in EXACT_THRESHOLDS.items():
        assert tuple(_exact_floor(T, k)[0] for k in (1, 2, 3)) == want, T


@pytest.mark.parametrize("T", sorted(EXACT_THRESHOLDS))
def test_thresholds_exact_floor_table(oracle_mod, T):
    """eq. (9): u < thr_k accepts dE = 4k with probability thr_k / 2^32, and
    thr_k = floor(exp(-4k/T) 2^32) exactly -- a round or ceiling rule fails
    at T = 0.6 (thr_3 8.85), 0.7 (thr_2 .846), 0.513 and 0.569."""
    assert tuple(int(v) for v in oracle_mod.thresholds(T)) == EXACT_THRESHOLDS[T]


def test_thresholds_exact_on_a_grid(oracle_mod):
    """The floor rule at 400 temperatures in (0.05, 20], wherever the decimal
    value is not within double rounding (1e-5 units) of an integer."""
    checked = 0
    for i in range(1, 401):
        T = 0.05 * i
        got = [int(v) for v in oracle_mod.thresholds(T)]
        for k in (1, 2, 3):
            f, frac = _exact_floor(T, k)
            if 1e-5 < frac < 1 - 1e-5:
                assert got[k - 1] == min(f, 0xffffffff), (T, k)
                checked += 1
    assert checked > 1000


def test_thresholds_clamp_at_infinite_temperature(oracle_mod):
    """As T -> infinity exp(-4k/T) 2^32 -> 2^32, which does not fit a uint32:
    the threshold clamps to 2^32 - 1 (every uphill move but u = 2^32 - 1
    accepted); just below the clamp the floor still holds."""
    assert list(oracle_mod.thresholds(1e300)) == [0xffffffff] * 3
    assert list(oracle_mod.thresholds(float(1 << 60))) == [0xffffffff] * 3
    T = 1e6
    assert [int(v) for v in oracle_mod.thresholds(T)] == [_exact_floor(T, k)[0] for k in (1, 2, 3)]
    assert all(v < 0xffffffff for v in oracle_mod.thresholds(T))
    assert list(oracle_mod.thresholds(0.0)) == [0, 0, 0]
