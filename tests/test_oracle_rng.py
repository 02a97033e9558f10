"""Pins for the oracle's random words and acceptance thresholds.

Philox4x32-10 is pinned against an independent implementation (rocRAND's
host-callable engine, compiled and run here as a black box).  The thresholds
are pinned by properties of the exponential in eq. (9) and by their limits.
"""
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
