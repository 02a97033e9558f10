"""Pins for the oracle's shared-noise keying (asynchronous multispin coding,
Sec. III): the samples packed in one word draw one random number per site and
sweep together, and otherwise each follows its own Metropolis chain.

* Copies: two samples given the same couplings and the same spins stay equal
  for ever when they share the noise, and part when they do not (or when their
  shared ids differ) -- the word depends on (seed, id, sweep, colour, replica,
  site) and on nothing of the sample.
* Coupled decisions: at every half-step, each site whose energy change is the
  same in two sharing samples is flipped in both or in neither, also when
  their couplings differ; with a single site in each sample differing, the
  samples agree elsewhere until the difference spreads.
* Each sharing sample is still an exact Metropolis chain: it samples the
  Boltzmann energy distribution of a 2^3 lattice (G-test against full
  enumeration), and sharing leaves couplings and the start untouched.
"""
import math

import numpy as np
import pytest


def _flip_decisions(oracle_mod, sim, half):
    """Sites each replica flipped in one half-step."""
    before = [sim.spins(r).copy() for r in (0, 1)]
    sim.half_step(half)
    return [before[r] != sim.spins(r) for r in (0, 1)]


def test_sharing_keeps_couplings_and_start(oracle_mod):
    a = oracle_mod.Sim(8, 0.4, 0.9, seed=3, sample=5)
    b = oracle_mod.Sim(8, 0.4, 0.9, seed=3, sample=5)
    b.share_noise(17)
    assert np.array_equal(a.bonds(), b.bonds())
    for r in (0, 1):
        assert np.array_equal(a.spins(r), b.spins(r))
    a.sweep(3)
    b.sweep(3)
    assert any(not np.array_equal(a.spins(r), b.spins(r)) for r in (0, 1))


@pytest.mark.parametrize("T", [0.8, 2.0])
def test_copies_sharing_noise_stay_equal(oracle_mod, T):
    L = 8
    a = oracle_mod.Sim(L, 0.5, T, seed=9, sample=0)
    b = oracle_mod.Sim(L, 0.5, T, seed=9, sample=1)
    c = oracle_mod.Sim(L, 0.5, T, seed=9, sample=1)
    d = oracle_mod.Sim(L, 0.5, T, seed=9, sample=2)
    for s in (b, c, d):
        s.set_bonds(a.bonds())
        for r in (0, 1):
            s.set_spins(r, a.spins(r))
    a.share_noise(40)
    b.share_noise(40)
    d.share_noise(41)
    # c keeps per-sample noise
    for step in range(12):
        for s in (a, b, c, d):
            s.sweep(1)
        for r in (0, 1):
            assert np.array_equal(a.spins(r), b.spins(r)), (step, r)
    assert any(not np.array_equal(a.spins(r), c.spins(r)) for r in (0, 1))
    assert any(not np.array_equal(a.spins(r), d.spins(r)) for r in (0, 1))


def test_equal_energy_change_gives_equal_decision(oracle_mod):
    """Two sharing samples with different couplings: every site whose dE is
    the same in both makes the same decision; per-sample noise does not."""
    L, T = 8, 1.1
    a = oracle_mod.Sim(L, 0.5, T, seed=21, sample=0)
    b = oracle_mod.Sim(L, 0.3, T, seed=21, sample=1)
    a.share_noise(5)
    b.share_noise(5)
    c = oracle_mod.Sim(L, 0.3, T, seed=21, sample=1)
    agree_shared = agree_plain = total = 0
    for sweep in range(6):
        for half in (0, 1):
            dEs = {}
            for name, s in (("a", a), ("b", b), ("c", c)):
                Jb = s.bonds()
                dEs[name] = [np.array([oracle_mod.delta_e(L, s.spins(r), Jb, i) for i in range(L ** 3)])
                             for r in (0, 1)]
            fa = _flip_decisions(oracle_mod, a, half)
            fb = _flip_decisions(oracle_mod, b, half)
            fc = _flip_decisions(oracle_mod, c, half)
            for r in (0, 1):
                colour = np.array([oracle_mod.colour(L, i) for i in range(L ** 3)]) == (r ^ half)
                up_ab = colour & (dEs["a"][r] == dEs["b"][r]) & (dEs["a"][r] > 0)
                assert np.array_equal(fa[r][up_ab], fb[r][up_ab]), (sweep, half, r)
                up_ac = colour & (dEs["a"][r] == dEs["c"][r]) & (dEs["a"][r] > 0)
                agree_shared += int(np.count_nonzero(up_ab))
                agree_plain += int(np.count_nonzero(fa[r][up_ac] == fc[r][up_ac]))
                total += int(np.count_nonzero(up_ac))
    assert agree_shared > 500
    # independent noise agrees only by chance on uphill moves
    assert agree_plain < total


@pytest.mark.parametrize("T", [1.0, 3.0])
def test_sharing_chain_samples_exact_energy_distribution(oracle_mod, T):
    L = 2
    sim = oracle_mod.Sim(L, 0.5, T, seed=300 + int(T), sample=4)
    J = sim.bonds()
    if np.all(J == J[0]):
        J[0] = -J[0]
    sim.set_bonds(J)
    sim.share_noise(12)
    idx = np.arange(256)
    states = (1 - 2 * ((idx[:, None] >> np.arange(8)[None, :]) & 1)).astype(np.int8)
    E = np.array([oracle_mod.energy(L, S, J) for S in states], dtype=np.int64)
    levels = np.unique(E)
    w = np.array([np.exp(-(e - E.min()) / T) * np.count_nonzero(E == e) for e in levels])
    p_exact = w / w.sum()
    sim.sweep(50)
    counts = np.zeros(len(levels))
    for _ in range(3000):
        sim.sweep(8)
        for r in (0, 1):
            counts[np.searchsorted(levels, oracle_mod.energy(L, sim.spins(r), J))] += 1
    expected = p_exact * counts.sum()
    keep = expected > 5
    obs = counts[keep]
    exp_ = expected[keep] * obs.sum() / expected[keep].sum()
    g = 2.0 * float(np.sum(np.where(obs > 0, obs * np.log(obs / exp_), 0.0)))
    dof = int(keep.sum()) - 1
    assert g < dof + 6 * math.sqrt(2 * dof) + 10, (g, dof, obs, exp_)


def test_shared_batch_helper(oracle_mod):
    sims = oracle_mod.shared_batch(8, 0.5, 0.8, seed=2, sample0=10, n_samples=3, shared_id=7, n_slots=1)
    assert [s.sample for s in sims] == [10, 11, 12]
    assert all(s.shared == 7 for s in sims)
    ref = oracle_mod.Sim(8, 0.5, 0.8, seed=2, sample=11)
    assert np.array_equal(sims[1].bonds(), ref.bonds())
