"""Exact invariances of the oracle's dynamics and observables.

* Gauge invariance: with eps_i = +-1, J'_ij = eps_i J_ij eps_j and
  S'(0) = eps S(0), the keyed dynamics gives S'(t) = eps S(t) exactly, and
  every gauge-invariant observable (unsatisfied bonds, q, C, C4) is equal.
  A misindexed coupling or neighbour breaks this.
* The staggered map eps = (-1)^(x+y+z) turns p = 0 (all J = +1) into p = 1
  (all J = -1): the two runs stay staggered images of each other.
* T = 0: no uphill move, so the energy never rises and the trajectory does
  not depend on the random words.
* Determinism identities: splitting sweeps, resuming from a stored state,
  and permuting the update order inside a colour change nothing.
* Observables: C(t,t) = 1 and C4(0) = 1 (eqs. 3, 7); S4 equals the circular
  autocorrelation of q computed by FFT; q = 1 for identical replicas.
"""
import numpy as np
import pytest


def _coords(L):
    s = np.arange(L ** 3)
    return s % L, (s // L) % L, s // (L * L)


def _gauge_bonds(L, J, eps):
    x, y, z = _coords(L)
    Jg = J.reshape(-1, 3).copy()
    nbs = [((x + 1) % L) + L * (y + L * z), x + L * (((y + 1) % L) + L * z),
           x + L * (y + L * ((z + 1) % L))]
    for d in range(3):
        Jg[:, d] = eps * Jg[:, d] * eps[nbs[d]]
    return Jg.reshape(-1)


@pytest.mark.parametrize("L,p,T", [(4, 0.5, 0.7), (6, 0.3, 0.9), (8, 0.5, 0.8)])
def test_gauge_invariance(oracle_mod, L, p, T):
    rng = np.random.default_rng(L)
    N = L ** 3
    eps = rng.choice(np.array([-1, 1], dtype=np.int8), size=N)
    a = oracle_mod.Sim(L, p, T, seed=21, n_slots=1)
    b = oracle_mod.Sim(L, p, T, seed=21, n_slots=1)
    b.set_bonds(_gauge_bonds(L, a.bonds(), eps))
    for r in (0, 1):
        b.set_spins(r, eps * a.spins(r))
    for step in range(12):
        a.sweep(3)
        b.sweep(3)
        if step == 2:
            a.snapshot(0)
            b.snapshot(0)
        for r in (0, 1):
            assert np.array_equal(b.spins(r), eps * a.spins(r))
        oa, ob = a.measure(), b.measure()
        assert np.array_equal(oa.unsat, ob.unsat)
        assert oa.overlap == ob.overlap
        assert np.array_equal(oa.c4, ob.c4)
        if step >= 2:
            assert np.array_equal(oa.autocorr, ob.autocorr)
    # the dynamics did something
    assert not np.array_equal(a.spins(0), oracle_mod.Sim(L, p, T, seed=21).spins(0))


def test_ferro_antiferro_staggered_map(oracle_mod):
    L, T = 8, 0.9
    x, y, z = _coords(L)
    eps = (1 - 2 * ((x + y + z) & 1)).astype(np.int8)
    fm = oracle_mod.Sim(L, 0.0, T, seed=4)
    afm = oracle_mod.Sim(L, 1.0, T, seed=4)
    for r in (0, 1):
        afm.set_spins(r, eps * fm.spins(r))
    for _ in range(10):
        fm.sweep(2)
        afm.sweep(2)
        for r in (0, 1):
            assert np.array_equal(afm.spins(r), eps * fm.spins(r))
    assert np.array_equal(fm.measure().unsat, afm.measure().unsat)


def test_ferromagnet_orders_below_tc(oracle_mod):
    """At p = 0 (all J = +1, T_FM ~ 4.51) a quench to T = 0.7 grows
    ferromagnetic domains: |M| rises far above sqrt(N), while at p = 1 the
    same happens to the staggered magnetisation instead."""
    L = 12
    N = L ** 3
    x, y, z = _coords(L)
    eps = (1 - 2 * ((x + y + z) & 1)).astype(np.int64)
    fm = oracle_mod.Sim(L, 0.0, 0.7, seed=9)
    afm = oracle_mod.Sim(L, 1.0, 0.7, seed=9)
    fm.sweep(300)
    afm.sweep(300)
    e_fm = (2 * fm.measure().unsat[0] - 3 * N) / N
    assert e_fm < -2.5
    m = abs(int(fm.spins(0).astype(np.int64).sum()))
    m_st = abs(int((eps * afm.spins(0)).sum()))
    m_afm_plain = abs(int(afm.spins(0).astype(np.int64).sum()))
    assert m > 0.5 * N and m_st > 0.5 * N
    assert m_afm_plain < 0.2 * N


def test_zero_temperature_quench(oracle_mod):
    L, N = 8, 512
    a = oracle_mod.Sim(L, 0.5, 0.0, seed=1)
    b = oracle_mod.Sim(L, 0.5, 0.0, seed=999)  # different random words
    b.set_bonds(a.bonds())
    for r in (0, 1):
        b.set_spins(r, a.spins(r))
    J = a.bonds()
    prev = [oracle_mod.energy(L, a.spins(r), J) for r in (0, 1)]
    for _ in range(20):
        for half in (0, 1):
            a.half_step(half)
            b.half_step(half)
            now = [oracle_mod.energy(L, a.spins(r), J) for r in (0, 1)]
            assert all(n <= p for n, p in zip(now, prev))
            prev = now
        for r in (0, 1):
            assert np.array_equal(a.spins(r), b.spins(r))
    assert prev[0] < -N  # well below the random-state energy ~ 0


def test_sweep_splitting_and_resume(oracle_mod):
    L = 6
    a = oracle_mod.Sim(L, 0.5, 0.8, seed=33)
    a.sweep(7)
    a.sweep(5)
    b = oracle_mod.Sim(L, 0.5, 0.8, seed=33)
    b.sweep(12)
    for r in (0, 1):
        assert np.array_equal(a.spins(r), b.spins(r))
    # resume: a fresh run given the state at t = 12 continues identically
    c = oracle_mod.Sim(L, 0.5, 0.8, seed=33)
    for r in (0, 1):
        c.set_spins(r, b.spins(r))
    c.set_time(12)
    b.sweep(9)
    c.sweep(9)
    for r in (0, 1):
        assert np.array_equal(b.spins(r), c.spins(r))
    assert b.time == c.time == 21


def test_update_order_within_colour_is_irrelevant(oracle_mod):
    L = 6
    rng = np.random.default_rng(1)
    a = oracle_mod.Sim(L, 0.5, 0.8, seed=8)
    b = oracle_mod.Sim(L, 0.5, 0.8, seed=8)
    for _ in range(6):
        for half in (0, 1):
            a.half_step(half)
            b.half_step(half, perm=rng.permutation(L ** 3 // 2))
    for r in (0, 1):
        assert np.array_equal(a.spins(r), b.spins(r))


def test_interlaced_colour_order(oracle_mod):
    """Replica r updates colour r first: after half-step 0 only colour-0 sites
    of replica 0 and colour-1 sites of replica 1 may have changed."""
    L = 6
    sim = oracle_mod.Sim(L, 0.5, 2.0, seed=2)
    x, y, z = _coords(L)
    col = (x + y + z) & 1
    before = [sim.spins(r) for r in (0, 1)]
    sim.half_step(0)
    for r in (0, 1):
        changed = before[r] != sim.spins(r)
        assert changed.any()
        assert np.all(col[changed] == r)
    assert sim.time == 0
    sim.half_step(1)
    assert sim.time == 1


def test_observable_identities(oracle_mod):
    L = 8
    N = L ** 3
    sim = oracle_mod.Sim(L, 0.5, 0.8, seed=5, n_slots=2)
    sim.sweep(10)
    sim.snapshot(0)
    o = sim.measure()
    assert list(o.autocorr[:, 0]) == [N, N]          # C(t,t) = 1
    assert list(o.c4[:, 0]) == [N, N, N]              # C4(0) = 1
    for v in [o.overlap, *o.mag]:
        assert abs(v) <= N and (v - N) % 2 == 0
    sim.sweep(5)
    sim.snapshot(1)
    o2 = sim.measure()
    assert list(o2.autocorr[:, 1]) == [N, N]
    assert all(abs(v) < N for v in o2.autocorr[:, 0])
    # identical replicas: q_i = 1 everywhere
    sim.set_spins(1, sim.spins(0))
    o3 = sim.measure()
    assert o3.overlap == N and np.all(o3.c4 == N)
    # reversed replica: q = -N, but C4 is quadratic in q
    sim.set_spins(1, -sim.spins(0))
    o4 = sim.measure()
    assert o4.overlap == -N and np.all(o4.c4 == N)


@pytest.mark.parametrize("L", [4, 6, 10])
def test_c4_is_circular_autocorrelation(oracle_mod, L):
    sim = oracle_mod.Sim(L, 0.5, 0.8, seed=L)
    sim.sweep(3)
    q = (sim.spins(0).astype(np.int64) * sim.spins(1)).reshape(L, L, L)  # [z, y, x]
    o = sim.measure()
    F = np.fft.fftn(q.astype(float))
    for d, axis in enumerate((2, 1, 0)):  # x, y, z
        auto = np.fft.ifft(np.abs(np.fft.fft(q.astype(float), axis=axis)) ** 2, axis=axis).real
        other = tuple(a for a in range(3) if a != axis)
        series = auto.sum(axis=other)
        want = np.rint(series[: L // 2 + 1]).astype(np.int64)
        assert np.array_equal(o.c4[d], want)
    assert abs(F[0, 0, 0].real - o.overlap) < 1e-6


def test_energy_and_magnetisation_special_states(oracle_mod):
    L = 6
    N = L ** 3
    sim = oracle_mod.Sim(L, 0.0, 0.8, seed=1)  # ferromagnet
    sim.set_spins(0, np.ones(N, dtype=np.int8))
    x, y, z = _coords(L)
    sim.set_spins(1, (1 - 2 * ((x + y + z) & 1)).astype(np.int8))
    o = sim.measure()
    assert o.unsat[0] == 0 and o.unsat[1] == 3 * N   # E = -3N and +3N
    assert o.mag[0] == N and o.mag[1] == 0
