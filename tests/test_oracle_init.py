"""Pins for the oracle's lattice geometry, couplings and initial state
(Sec. II: bimodal couplings with P(J=-1) = p, quench from random spins)."""
import numpy as np
import pytest


@pytest.mark.parametrize("L", [2, 4, 6, 10])
def test_half_index_is_a_bijection_per_colour(oracle_mod, L):
    N = L ** 3
    seen = [set(), set()]
    for s in range(N):
        x, y, z = s % L, (s // L) % L, s // (L * L)
        c = oracle_mod.colour(L, s)
        assert c == (x + y + z) & 1
        seen[c].add(oracle_mod.half_index(L, s))
    assert seen[0] == set(range(N // 2)) and seen[1] == set(range(N // 2))


def test_p_limits_give_uniform_couplings(oracle_mod):
    J0 = oracle_mod.Sim(6, 0.0, 0.8, seed=3).bonds()
    J1 = oracle_mod.Sim(6, 1.0, 0.8, seed=3).bonds()
    assert np.all(J0 == 1) and np.all(J1 == -1)


@pytest.mark.parametrize("p", [0.1, 0.25, 0.5, 0.8])
def test_coupling_fraction_matches_p(oracle_mod, p):
    L = 12
    J = oracle_mod.Sim(L, p, 0.8, seed=11).bonds()
    n = J.size
    frac = np.count_nonzero(J == -1) / n
    assert abs(frac - p) < 5 * np.sqrt(p * (1 - p) / n)


def test_couplings_nested_in_p(oracle_mod):
    """At a fixed seed each bond's word is fixed, so the set of -1 bonds grows
    with p (common random numbers across the p scan)."""
    prev = None
    for p in [0.15, 0.2, 0.25, 0.3, 0.5]:
        neg = oracle_mod.Sim(8, p, 0.7, seed=1).bonds() == -1
        if prev is not None:
            assert np.all(neg[prev])
        prev = neg


def test_initial_spins_random_and_distinct(oracle_mod):
    L = 16
    a = oracle_mod.Sim(L, 0.5, 0.8, seed=1, sample=0)
    b = oracle_mod.Sim(L, 0.5, 0.8, seed=1, sample=1)
    c = oracle_mod.Sim(L, 0.5, 0.8, seed=2, sample=0)
    N = L ** 3
    s0, s1 = a.spins(0), a.spins(1)
    for S in (s0, s1, b.spins(0), c.spins(0)):
        assert abs(np.count_nonzero(S == -1) - N / 2) < 5 * np.sqrt(N / 4)
    # replicas, samples and seeds are independent: overlaps are O(sqrt N)
    for A, B in [(s0, s1), (s0, b.spins(0)), (s0, c.spins(0))]:
        assert abs(int(np.dot(A.astype(np.int64), B))) < 5 * np.sqrt(N)
    # the bonds do not depend on the replica but do on the sample
    assert not np.array_equal(a.bonds(), b.bonds())
    assert np.array_equal(a.bonds(), oracle_mod.Sim(L, 0.5, 1.1, seed=1).bonds())


def test_create_rejects_bad_arguments(oracle_mod):
    for args in [(3, 0.5, 0.8), (0, 0.5, 0.8), (4, -0.1, 0.8), (4, 1.1, 0.8),
                 (4, 0.5, -1.0), (4, 0.5, float("inf")), (4, float("nan"), 0.8)]:
        with pytest.raises(ValueError):
            oracle_mod.Sim(*args, seed=0)
