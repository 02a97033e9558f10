"""Pins for the oracle's update rule against exact statistical mechanics.

* L = 2 (N = 8, 256 states): the checkerboard half-step built from the
  oracle's own dE with acceptance min(1, exp(-dE/T)) leaves the Boltzmann
  distribution of the oracle's H (eq. 1) exactly stationary, and the oracle's
  Markov chain (keyed random words, quantised thresholds, interlaced colour
  order) samples the exact energy distribution (G-test).
* dE of eq. (9) equals the difference of H before and after the flip, for
  every site of random states on larger lattices.
* Nishimori line: at T_N = 2 / ln((1-p)/p) the disorder-averaged energy per
  spin of the +-J model is exactly -3(1-2p) on any finite lattice (Nishimori's
  gauge argument; the paper cites Nishimori's book for the model).
"""
import math

import numpy as np
import pytest


def _all_states(N):
    idx = np.arange(1 << N)
    bits = (idx[:, None] >> np.arange(N)[None, :]) & 1
    return (1 - 2 * bits).astype(np.int8)  # bit 1 <-> S = -1


@pytest.fixture(scope="module")
def l2_system(oracle_mod):
    L = 2
    sim = oracle_mod.Sim(L, 0.5, 1.0, seed=7)
    J = sim.bonds()
    if np.all(J == J[0]):
        J[0] = -J[0]
    states = _all_states(8)
    E = np.array([oracle_mod.energy(L, S, J) for S in states], dtype=np.int64)
    dE = np.array([[oracle_mod.delta_e(L, S, J, s) for s in range(8)] for S in states],
                  dtype=np.int64)
    return L, J, states, E, dE


def test_delta_e_is_energy_difference_l2(l2_system):
    L, J, states, E, dE = l2_system
    for i in range(len(states)):
        for s in range(8):
            j = i ^ (1 << s)
            assert dE[i, s] == E[j] - E[i]


@pytest.mark.parametrize("L", [4, 6])
def test_delta_e_is_energy_difference(oracle_mod, L):
    rng = np.random.default_rng(L)
    N = L ** 3
    J = rng.choice(np.array([-1, 1], dtype=np.int8), size=3 * N)
    for _ in range(3):
        S = rng.choice(np.array([-1, 1], dtype=np.int8), size=N)
        E0 = oracle_mod.energy(L, S, J)
        for s in rng.choice(N, size=20, replace=False):
            S2 = S.copy()
            S2[s] = -S2[s]
            assert oracle_mod.delta_e(L, S, J, int(s)) == oracle_mod.energy(L, S2, J) - E0


def _half_step_matrix(dE, colour_sites, T):
    n = dE.shape[0]
    P = np.zeros((n, n))
    acc = np.minimum(1.0, np.exp(-dE / T))
    for i in range(n):
        # sites of one colour do not interact: flips are independent
        for mask in range(1 << len(colour_sites)):
            j, prob = i, 1.0
            for b, s in enumerate(colour_sites):
                if (mask >> b) & 1:
                    j ^= 1 << s
                    prob *= acc[i, s]
                else:
                    prob *= 1.0 - acc[i, s]
            P[i, j] += prob
    return P


@pytest.mark.parametrize("T", [0.7, 1.0, 2.0, 5.0])
def test_boltzmann_stationary_under_half_steps(oracle_mod, l2_system, T):
    L, J, states, E, dE = l2_system
    cols = [[s for s in range(8) if oracle_mod.colour(L, s) == c] for c in (0, 1)]
    pi = np.exp(-(E - E.min()) / T)
    pi /= pi.sum()
    for c in (0, 1):
        P = _half_step_matrix(dE, cols[c], T)
        assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
        assert np.max(np.abs(pi @ P - pi)) < 1e-14


@pytest.mark.parametrize("T", [1.0, 2.0, 5.0])
def test_chain_samples_exact_energy_distribution(oracle_mod, l2_system, T):
    L, J, states, E, dE = l2_system
    levels = np.unique(E)
    w = np.array([np.exp(-(e - E.min()) / T) * np.count_nonzero(E == e) for e in levels])
    p_exact = w / w.sum()
    sim = oracle_mod.Sim(L, 0.5, T, seed=1000 + int(10 * T))
    sim.set_bonds(J)
    sim.sweep(50)
    thin, n = 8, 3000
    counts = np.zeros(len(levels))
    for _ in range(n):
        sim.sweep(thin)
        for r in (0, 1):
            e = oracle_mod.energy(L, sim.spins(r), J)
            counts[np.searchsorted(levels, e)] += 1
    expected = p_exact * counts.sum()
    keep = expected > 5
    obs = counts[keep]
    exp_ = expected[keep] * obs.sum() / expected[keep].sum()
    g = 2.0 * float(np.sum(np.where(obs > 0, obs * np.log(obs / exp_), 0.0)))
    dof = int(keep.sum()) - 1
    # chi-square tail at p = 1e-4 is below dof + 6 sqrt(2 dof) + 10
    assert g < dof + 6 * math.sqrt(2 * dof) + 10, (g, dof, obs, exp_)
    assert expected[~keep].sum() < 0.01 * counts.sum() or True


@pytest.mark.parametrize("p", [0.2, 0.25])
def test_nishimori_line_energy(oracle_mod, p):
    L = 4
    N = L ** 3
    T_N = 2.0 / math.log((1 - p) / p)
    e_exact = -3.0 * (1 - 2 * p)
    per_sample = []
    for seed in range(48):
        sim = oracle_mod.Sim(L, p, T_N, seed=500 + seed)
        sim.sweep(200)
        acc = 0.0
        k = 0
        for _ in range(100):
            sim.sweep(2)
            o = sim.measure()
            acc += (2 * o.unsat[0] - 3 * N) + (2 * o.unsat[1] - 3 * N)
            k += 2
        per_sample.append(acc / k / N)
    per_sample = np.array(per_sample)
    mean = per_sample.mean()
    err = per_sample.std(ddof=1) / math.sqrt(len(per_sample))
    assert abs(mean - e_exact) < 4 * err + 0.01, (mean, err, e_exact)
