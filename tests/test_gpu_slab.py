"""Parity of the plain form's persistent slab path (ea_set_slab_plan):
every replica cut into z-slabs held in LDS with ghost planes, exchanging
boundary planes through device memory once per `ghost` half-steps.  Spins
and every observable are compared bit for bit with the CPU oracle (and,
where the oracle is too slow, with the one-launch-per-half-step path, itself
compared with the oracle here and in test_gpu_plain.py)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _compare_obs(go, oo, ctx):
    assert go.t == oo.t, ctx
    assert list(go.unsat) == list(oo.unsat), ctx
    assert list(go.mag) == list(oo.mag), ctx
    assert go.overlap == oo.overlap, ctx
    if oo.autocorr.size:
        assert np.array_equal(go.autocorr, oo.autocorr), ctx
    assert np.array_equal(go.c4, oo.c4), ctx


def _compare_state(a, b, ctx):
    for r in (0, 1):
        x, y = a.spins(r), b.spins(r)
        if not np.array_equal(x, y):
            bad = np.flatnonzero(x != y)
            raise AssertionError(f"{ctx}: replica {r} differs at {bad.size} sites, first {bad[:8]}")


# (L, words_per_row, slabs, ghost, sweeps): one slab per replica (the ghost
# planes are the slab's own planes wrapped round), even and uneven slabs,
# slabs thinner than the ghost depth (ghosts from several neighbours), every
# ghost depth 1..4, several packings.
PLANS = [
    (8, 1, 1, 1, 30), (8, 1, 8, 3, 30), (16, 2, 5, 2, 20), (16, 1, 16, 4, 20),
    (24, 1, 3, 1, 12), (24, 3, 7, 2, 12), (32, 2, 32, 2, 10),
    (64, 4, 64, 2, 5), (64, 1, 13, 1, 5), (64, 2, 20, 3, 5), (64, 8, 64, 4, 4),
    (72, 3, 9, 1, 3), (96, 2, 48, 2, 2), (128, 2, 25, 1, 2), (128, 4, 100, 2, 2),
]


@pytest.mark.parametrize("L,rw,K,g,sweeps", PLANS)
def test_slab_plans_match_oracle(ea_gpu, oracle_mod, L, rw, K, g, sweeps):
    _say(f"slab L={L} rw={rw} K={K} g={g} sweeps={sweeps}")
    p, T = (0.5, 0.8) if L % 16 else (0.3, 0.6)
    gs = ea_gpu.Sim(L, p, T, seed=11, sample=2, n_slots=1, words_per_row=rw)
    gs.set_slab_plan(K, g)
    assert gs.slab_plan == (K, g)
    o = oracle_mod.Sim(L, p, T, seed=11, sample=2, n_slots=1)
    gs.snapshot(0)
    o.snapshot(0)
    done = 0
    # an odd split of the sweeps: launches of one sweep and of the rest
    for chunk in (1, sweeps - 1):
        gs.sweep(chunk)
        o.sweep(chunk)
        done += chunk
        _compare_state(gs, o, f"L={L} rw={rw} K={K} g={g} t={done}")
    _compare_obs(gs.measure(), o.measure(), f"L={L} K={K} g={g}")
    gs.close()


@pytest.mark.parametrize("L,T", [(16, 0.0), (16, 3.0), (24, 0.7)])
def test_slab_extreme_temperatures_and_couplings(ea_gpu, oracle_mod, L, T):
    for p in (0.0, 1.0, 0.5):
        gs = ea_gpu.Sim(L, p, T, seed=3, sample=0)
        gs.set_slab_plan(L // 2, 2)
        o = oracle_mod.Sim(L, p, T, seed=3, sample=0)
        gs.sweep(15)
        o.sweep(15)
        _compare_state(gs, o, f"L={L} p={p} T={T}")
        _compare_obs(gs.measure(), o.measure(), f"L={L} p={p} T={T}")
        gs.close()


def test_slab_many_launches_and_long_launch(ea_gpu, oracle_mod):
    """Exchange epochs advance across launches: 200 launches of one sweep,
    then one call longer than a launch chunk (16384 sweeps), L = 8 with one
    slab per plane, against the oracle."""
    L = 8
    gs = ea_gpu.Sim(L, 0.5, 0.9, seed=21, sample=4)
    gs.set_slab_plan(8, 1)
    o = oracle_mod.Sim(L, 0.5, 0.9, seed=21, sample=4)
    for i in range(200):
        gs.sweep(1)
    o.sweep(200)
    _compare_state(gs, o, "200 launches")
    gs.set_slab_plan(4, 3)
    gs.sweep(20000)
    o.sweep(20000)
    _compare_state(gs, o, "20200 sweeps")
    _compare_obs(gs.measure(), o.measure(), "20200 sweeps")
    gs.close()


def test_slab_and_half_step_launches_agree_at_size(ea_gpu, oracle_mod):
    """L = 64, 128 and 256 (the largest side): the automatic slab plan and
    the one-launch-per-half-step path give the same spins after 300 sweeps;
    the latter is itself compared with the oracle for its first sweep."""
    for L in (64, 128, 256):
        a = ea_gpu.Sim(L, 0.5, 0.7, seed=1, sample=0)
        b = ea_gpu.Sim(L, 0.5, 0.7, seed=1, sample=0, words_per_row=a.words_per_row)
        b.set_slab_plan(-1, 0)
        assert a.slab_plan[0] > 0 and b.slab_plan == (-1, 0)
        _say(f"L={L} plan {a.slab_plan} rw={a.words_per_row}")
        if L <= 128:
            o = oracle_mod.Sim(L, 0.5, 0.7, seed=1, sample=0)
            b.sweep(1)
            o.sweep(1)
            _compare_state(b, o, f"half-step path L={L} t=1")
            a.sweep(1)
            _compare_state(a, o, f"slab path L={L} t=1")
            a.sweep(299)
            b.sweep(299)
        else:
            a.sweep(300)
            b.sweep(300)
        _compare_state(a, b, f"L={L} t=300")
        oa, ob = a.measure(), b.measure()
        assert list(oa.unsat) == list(ob.unsat) and oa.overlap == ob.overlap
        assert np.array_equal(oa.c4, ob.c4)
        a.close()
        b.close()


def test_half_step_path_matches_oracle(ea_gpu, oracle_mod):
    """The one-launch-per-half-step path (slabs = -1) still runs and is
    bit-exact, at sizes where it is no longer the default."""
    for L, rw in ((16, 1), (64, 4), (96, 3)):
        g = ea_gpu.Sim(L, 0.5, 0.8, seed=9, sample=1, words_per_row=rw)
        g.set_slab_plan(-1, 0)
        o = oracle_mod.Sim(L, 0.5, 0.8, seed=9, sample=1)
        g.sweep(3)
        o.sweep(3)
        _compare_state(g, o, f"half-step path L={L}")
        g.close()


def test_slab_group_matches_oracle(ea_gpu, oracle_mod):
    """The crossover runs' shape: five L = 128 runs (p = 0.5 ... 0.15,
    T = 0.7) advanced by ea_sweep_group in one slab launch, each against the
    oracle after two sweeps, then against its own run alone after 64 more."""
    ps = [0.5, 0.3, 0.25, 0.2, 0.15]
    sims = [ea_gpu.Sim(128, p, 0.7, seed=1, sample=0) for p in ps]
    ea_gpu.sweep_group(sims, 2)
    for p, s in zip(ps, sims):
        o = oracle_mod.Sim(128, p, 0.7, seed=1, sample=0)
        o.sweep(2)
        _compare_state(s, o, f"group p={p} t=2")
    ea_gpu.sweep_group(sims, 64)
    for p, s in zip(ps, sims):
        alone = ea_gpu.Sim(128, p, 0.7, seed=1, sample=0)
        alone.sweep(66)
        _compare_state(s, alone, f"group vs alone p={p} t=66")
        alone.close()
    for s in sims:
        s.close()


def test_slab_resume_and_reset(ea_gpu, oracle_mod):
    """Spins and time restored into a fresh run continue the trajectory; a
    reset run starts over exactly."""
    L = 32
    a = ea_gpu.Sim(L, 0.4, 0.75, seed=8, sample=1)
    a.sweep(37)
    st = [a.spins(0), a.spins(1)]
    b = ea_gpu.Sim(L, 0.4, 0.75, seed=8, sample=1)
    b.set_spins(0, st[0])
    b.set_spins(1, st[1])
    b.set_time(37)
    a.sweep(23)
    b.sweep(23)
    _compare_state(a, b, "resumed")
    a.reset(8, 1)
    c = ea_gpu.Sim(L, 0.4, 0.75, seed=8, sample=1)
    a.sweep(5)
    c.sweep(5)
    _compare_state(a, c, "reset")
    o = oracle_mod.Sim(L, 0.4, 0.75, seed=8, sample=1)
    o.sweep(5)
    _compare_state(a, o, "reset vs oracle")
    for s in (a, b, c):
        s.close()


def test_slab_plan_errors(ea_gpu):
    s = ea_gpu.Sim(64, 0.5, 0.8, seed=1)
    with pytest.raises(ea_gpu.EAError):
        s.set_slab_plan(65, 1)       # more slabs than planes
    with pytest.raises(ea_gpu.EAError):
        s.set_slab_plan(8, 9)        # ghost depth beyond 8
    with pytest.raises(ea_gpu.EAError):
        s.set_slab_plan(-2, 0)
    k, g = s.slab_plan
    assert k > 0 and g > 0           # the default plan is the slab path
    s.set_slab_plan(-1, 0)
    assert s.slab_plan == (-1, 0)
    s.close()
    # 2 x 200 workgroups exceed the compute units
    big = ea_gpu.Sim(256, 0.5, 0.8, seed=1)
    with pytest.raises(ea_gpu.EAError):
        big.set_slab_plan(200, 1)
    big.close()
    # a packing whose plane of one colour exceeds one workgroup's threads
    big = ea_gpu.Sim(256, 0.5, 0.8, seed=1, words_per_row=8)
    assert big.slab_plan == (-1, 0)
    with pytest.raises(ea_gpu.EAError):
        big.set_slab_plan(16, 1)
    big.close()


@pytest.mark.parametrize("T", [0.6, 1.2])
def test_screened_slabs_match_oracle(ea_gpu, oracle_mod, T):
    """Slabs thick enough to give every SIMD four waves per half-step take
    the screened instantiation (rare uphill moves ruled out per word); at
    T = 0.6 the screen applies, at T = 1.2 moves with dE >= 8 are too
    frequent and every word takes the table select."""
    g = ea_gpu.Sim(64, 0.5, T, seed=13, sample=0, words_per_row=4)
    g.set_slab_plan(4, 1)
    o = oracle_mod.Sim(64, 0.5, T, seed=13, sample=0)
    g.sweep(4)
    o.sweep(4)
    _compare_state(g, o, f"screened slabs T={T}")
    _compare_obs(g.measure(), o.measure(), f"screened slabs T={T}")
    g.close()


def test_group_shares_spanning_replicas(ea_gpu, oracle_mod):
    """Three L = 64 runs of different p and T in one group: 384 planes on
    at most 256 workgroups, so shares of one or two planes span the end of
    one replica and the start of the next, sometimes of another run (with
    its own select table); every run against the oracle."""
    params = [(0.5, 0.5), (0.3, 0.9), (0.2, 1.3)]
    sims = [ea_gpu.Sim(64, p, T, seed=17, sample=i, words_per_row=4) for i, (p, T) in enumerate(params)]
    ea_gpu.sweep_group(sims, 1)
    ea_gpu.sweep_group(sims, 4)
    for i, ((p, T), s) in enumerate(zip(params, sims)):
        o = oracle_mod.Sim(64, p, T, seed=17, sample=i)
        o.sweep(5)
        _compare_state(s, o, f"spanning group run {i} p={p} T={T}")
        _compare_obs(s.measure(), o.measure(), f"spanning group run {i}")
    for s in sims:
        s.close()
