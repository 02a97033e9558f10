"""Parity of the plain GPU path (ea_sweep with its default plan: the
persistent slab launches for every lattice whose plane of one colour fits a
workgroup, one launch per checkerboard half-step otherwise) against the CPU
oracle: bit-exact couplings, spins and every integer observable, on the same
seeds and schedules.  test_gpu_slab.py covers explicit slab plans and the
one-launch-per-half-step path."""
import sys

import numpy as np
import pytest

from definitions import axis_c4, unsat_count

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
    if go.c4 is not None:
        assert np.array_equal(go.c4, oo.c4), ctx


def _compare_state(g, o, ctx):
    for r in (0, 1):
        gs, os_ = g.spins(r), o.spins(r)
        if not np.array_equal(gs, os_):
            bad = np.flatnonzero(gs != os_)
            raise AssertionError(f"{ctx}: replica {r} differs at {bad.size} sites, first {bad[:8]}")


# L values chosen to exercise every packed-row shape: W = L/2 for L <= 64
# (one word per row), and multi-word rows for L = 72 (3 x 12), 88 (11 x 4),
# 96 (2 x 24), 128 (2 x 32).
@pytest.mark.parametrize("L", [8, 16, 24, 40, 48, 64, 72, 88, 96, 128])
def test_initial_state_matches_oracle(ea_gpu, oracle_mod, L):
    _say(f"init L={L}")
    for p, seed, sample in [(0.5, 1, 0), (0.23, 77, 3)]:
        g = ea_gpu.Sim(L, p, 0.8, seed=seed, sample=sample)
        o = oracle_mod.Sim(L, p, 0.8, seed=seed, sample=sample)
        assert np.array_equal(g.bonds(), o.bonds()), (L, p)
        _compare_state(g, o, f"L={L} p={p} t=0")


@pytest.mark.parametrize("L,p,T,sweeps", [
    (8, 0.5, 0.8, 40), (16, 0.5, 0.8, 25), (24, 0.3, 0.6, 12), (32, 0.5, 1.0, 10),
    (40, 0.2, 0.7, 6), (48, 0.5, 0.7, 6), (64, 0.25, 0.7, 4), (72, 0.5, 1.2, 3),
    (88, 0.5, 0.5, 2), (96, 0.15, 0.7, 2), (128, 0.5, 0.7, 2),
    (16, 0.0, 0.7, 20), (16, 1.0, 0.7, 20), (16, 0.5, 0.0, 20), (16, 0.5, 3.0, 20),
])
def test_sweeps_match_oracle(ea_gpu, oracle_mod, L, p, T, sweeps):
    _say(f"sweeps L={L} p={p} T={T} n={sweeps}")
    g = ea_gpu.Sim(L, p, T, seed=5, sample=1, n_slots=1)
    o = oracle_mod.Sim(L, p, T, seed=5, sample=1, n_slots=1)
    g.snapshot(0)
    o.snapshot(0)
    done = 0
    for chunk in (1, sweeps - 1):
        if chunk <= 0:
            continue
        g.sweep(chunk)
        o.sweep(chunk)
        done += chunk
        _compare_state(g, o, f"L={L} p={p} T={T} t={done}")
        _compare_obs(g.measure(), o.measure(), f"L={L} t={done}")


def test_small_config_full_run(ea_gpu, oracle_mod):
    """L = 16, p = 0.5, T = 0.8, 1000 sweeps; measure at 10, 100, 1000 with
    t_w = 100 and C4 for r = 0..8 along the three axes."""
    _say("config L=16 1000 sweeps")
    L, p, T = 16, 0.5, 0.8
    g = ea_gpu.Sim(L, p, T, seed=1, n_slots=1)
    o = oracle_mod.Sim(L, p, T, seed=1, n_slots=1)
    t = 0
    for target in (10, 100, 1000):
        g.sweep(target - t)
        o.sweep(target - t)
        t = target
        if t == 100:
            g.snapshot(0)
            o.snapshot(0)
        _compare_obs(g.measure(), o.measure(), f"t={t}")
        _compare_state(g, o, f"t={t}")
    go = g.measure()
    assert go.c4.shape == (3, 9) and np.all(go.c4[:, 0] == L ** 3)


def test_gauge_transformed_run_on_gpu(ea_gpu, oracle_mod):
    """Couplings and spins set through the ABI: a random gauge transform of
    the run gives the transformed trajectory (exact)."""
    L, p, T = 24, 0.5, 0.7
    N = L ** 3
    rng = np.random.default_rng(3)
    eps = rng.choice(np.array([-1, 1], dtype=np.int8), size=N)
    s = np.arange(N)
    x, y, z = s % L, (s // L) % L, s // (L * L)
    nbs = [((x + 1) % L) + L * (y + L * z), x + L * (((y + 1) % L) + L * z),
           x + L * (y + L * ((z + 1) % L))]
    a = ea_gpu.Sim(L, p, T, seed=9)
    b = ea_gpu.Sim(L, p, T, seed=9)
    J = a.bonds().reshape(-1, 3)
    Jg = np.stack([eps * J[:, d] * eps[nbs[d]] for d in range(3)], axis=1).astype(np.int8)
    b.set_bonds(Jg.reshape(-1))
    assert np.array_equal(b.bonds(), Jg.reshape(-1))
    for r in (0, 1):
        b.set_spins(r, eps * a.spins(r))
    a.sweep(30)
    b.sweep(30)
    for r in (0, 1):
        assert np.array_equal(b.spins(r), eps * a.spins(r))
    oa, ob = a.measure(), b.measure()
    assert list(oa.unsat) == list(ob.unsat) and oa.overlap == ob.overlap
    assert np.array_equal(oa.c4, ob.c4)
    # and the untransformed GPU run agrees with the oracle
    o = oracle_mod.Sim(L, p, T, seed=9)
    o.sweep(30)
    for r in (0, 1):
        assert np.array_equal(a.spins(r), o.spins(r))


def test_windowed_parity_mid_size(ea_gpu, oracle_mod):
    """L = 64, p = 0.5, T = 0.7: the oracle, started from the GPU state at
    t0, reproduces the GPU state after a window of sweeps (the random words
    are keyed by the absolute sweep index)."""
    L, p, T = 64, 0.5, 0.7
    g = ea_gpu.Sim(L, p, T, seed=1)
    for t0, k in [(0, 3), (1000, 3), (20000, 2)]:
        g.sweep(t0 - g.time)
        o = oracle_mod.Sim(L, p, T, seed=1)
        for r in (0, 1):
            o.set_spins(r, g.spins(r))
        o.set_time(t0)
        g.sweep(k)
        o.sweep(k)
        _say(f"window L=64 t0={t0} k={k}")
        _compare_state(g, o, f"window t0={t0}")
        _compare_obs(g.measure(), o.measure(), f"window t0={t0}")


def test_resume_and_determinism(ea_gpu):
    L = 32
    a = ea_gpu.Sim(L, 0.5, 0.8, seed=4)
    b = ea_gpu.Sim(L, 0.5, 0.8, seed=4)
    a.sweep(50)
    b.sweep(20)
    b.sweep(30)
    for r in (0, 1):
        assert np.array_equal(a.spins(r), b.spins(r))
    c = ea_gpu.Sim(L, 0.5, 0.8, seed=4)
    for r in (0, 1):
        c.set_spins(r, a.spins(r))
    c.set_time(50)
    a.sweep(25)
    c.sweep(25)
    for r in (0, 1):
        assert np.array_equal(a.spins(r), c.spins(r))


def test_errors_on_gpu(ea_gpu):
    g = ea_gpu.Sim(16, 0.5, 0.8, seed=1, n_slots=2)
    with pytest.raises(ea_gpu.EAError):
        g.snapshot(2)
    with pytest.raises(ea_gpu.EAError):
        g.snapshot(-1)
    g.set_time((1 << 32) - 5)
    with pytest.raises(ea_gpu.EAError):
        g.sweep(5)
    g.sweep(4)
    assert g.time == (1 << 32) - 1
    with pytest.raises(ea_gpu.EAError):
        g.set_spins(0, np.zeros(16 ** 3, dtype=np.int8))


@pytest.mark.parametrize("L,rw", [(24, 1), (24, 3), (64, 1), (64, 2), (64, 4), (64, 8),
                                  (96, 2), (96, 3), (96, 6), (96, 12), (128, 4), (128, 16)])
def test_packings_match_oracle(ea_gpu, oracle_mod, L, rw):
    """Every bit packing of the plain form (W = L/(2 rw) sites per word)
    gives the oracle's trajectory and observables."""
    _say(f"packing L={L} rw={rw}")
    g = ea_gpu.Sim(L, 0.4, 0.8, seed=8, sample=2, n_slots=1, words_per_row=rw)
    assert g.words_per_row == rw
    o = oracle_mod.Sim(L, 0.4, 0.8, seed=8, sample=2, n_slots=1)
    g.snapshot(0)
    o.snapshot(0)
    g.sweep(3)
    o.sweep(3)
    _compare_state(g, o, f"L={L} rw={rw}")
    _compare_obs(g.measure(), o.measure(), f"L={L} rw={rw}")


def test_tune_plain(ea_gpu):
    for L in (32, 64, 96):
        r = ea_gpu.tune_plain(L, force=True)
        _say(f"tune_plain L={L}: {r}")
        assert r["tried"] and all(c["parity_ok"] for c in r["tried"])
        assert r["words_per_row"] in [c["words_per_row"] for c in r["tried"]]
        assert ea_gpu.tune_plain(L)["tried"] == []  # cached
        g = ea_gpu.Sim(L, 0.5, 0.8, seed=1)
        assert g.words_per_row == r["words_per_row"]
    with pytest.raises(ea_gpu.EAError):
        ea_gpu.tune_plain(12)


@pytest.mark.parametrize("p", [0.5, 0.15])
def test_crossover_windows_L128(ea_gpu, oracle_mod, p):
    """L = 128, T = 0.7 across the crossover (nested couplings, seed 1): the
    oracle reproduces the GPU from t = 0 and from the GPU state after 3000
    sweeps, magnetisation included."""
    from paper_1411_5512_amd import workloads as wl
    job = [j for j in wl.crossover_jobs(10_000) if j.p == p][0]
    g = ea_gpu.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample)
    for t0, k in [(0, 2), (3000, 2)]:
        g.sweep(t0 - g.time)
        o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample)
        for r in (0, 1):
            o.set_spins(r, g.spins(r))
        o.set_time(t0)
        g.sweep(k)
        o.sweep(k)
        _say(f"crossover L=128 p={p} window t0={t0}")
        _compare_state(g, o, f"p={p} t0={t0}")
        _compare_obs(g.measure(), o.measure(), f"p={p} t0={t0}")


def _fft_shells(q, L, n_shells):
    f = np.fft.fftn(q.reshape(L, L, L).astype(np.float64))
    corr = np.rint(np.fft.ifftn(np.conj(f) * f).real).astype(np.int64)
    m = np.minimum(np.arange(L), L - np.arange(L)) ** 2
    k = m[:, None, None] + m[None, :, None] + m[None, None, :]
    out = np.zeros(n_shells, dtype=np.int64)
    sel = k < n_shells
    np.add.at(out, k[sel], corr[sel])
    return out


@pytest.mark.parametrize("L,rw", [(8, 0), (16, 0), (16, 1), (24, 0), (32, 2)])
def test_c4_shells_match_oracle(ea_gpu, oracle_mod, L, rw):
    g = ea_gpu.Sim(L, 0.5, 0.8, seed=6, sample=1, words_per_row=rw)
    o = oracle_mod.Sim(L, 0.5, 0.8, seed=6, sample=1)
    g.sweep(9)
    o.sweep(9)
    _say(f"c4 shells L={L} rw={g.words_per_row}")
    for n in (None, 3 * (L // 2) ** 2 + 1, 5):
        assert np.array_equal(g.c4_shells(n), o.c4_shells(n)), (L, n)


@pytest.mark.parametrize("L", [64, 96, 128, 136, 256])
def test_c4_shells_full_size(ea_gpu, L):
    """At full size (no oracle): equal to an FFT autocorrelation of the GPU's
    own q, and the shell identities (r = 0, unit shell = axis C4 at 1, sum of
    every shell = Q^2).  L = 136 and 256 take the rows kernel of three and four
    64-bit words per row."""
    g = ea_gpu.Sim(L, 0.3, 0.7, seed=1)
    g.sweep(50)
    _say(f"c4 shells full size L={L}")
    q = g.spins(0).astype(np.int64) * g.spins(1)
    n_all = 3 * (L // 2) ** 2 + 1
    got = g.c4_shells(n_all)
    assert np.array_equal(got, _fft_shells(q, L, n_all))
    obs = g.measure()
    assert got[0] == L ** 3 and got[1] == 2 * int(obs.c4[:, 1].sum())
    assert int(got.sum()) == obs.overlap ** 2
    assert np.array_equal(g.c4_shells(), got[:(L // 2) ** 2 + 1])


@pytest.mark.parametrize("L", [200, 256])
def test_largest_lattices(ea_gpu, oracle_mod, L):
    """The largest plain-form lattices (L = 256, the maximum, and L = 200,
    not a power of two): couplings, the initial state and the state after
    two sweeps equal the oracle's bit for bit.  The oracle's full measurement
    takes minutes at this size, so the GPU's observables are checked against
    their definitions (unsatisfied bonds of the Hamiltonian, magnetisation,
    overlap, C(t, t_w) of eq. 7, C4 along the axes of eq. 3) evaluated on
    that oracle-checked state."""
    g = ea_gpu.Sim(L, 0.5, 0.7, seed=3, n_slots=1)
    o = oracle_mod.Sim(L, 0.5, 0.7, seed=3)
    _say(f"largest lattices L={L} rw={g.words_per_row}: initial state")
    J = g.bonds()
    assert np.array_equal(J, o.bonds())
    _compare_state(g, o, f"L={L} t=0")
    g.snapshot(0)
    S0 = [g.spins(r) for r in (0, 1)]
    g.sweep(2)
    o.sweep(2)
    _say(f"largest lattices L={L}: after two sweeps")
    _compare_state(g, o, f"L={L} t=2")
    obs = g.measure()
    S = [g.spins(r) for r in (0, 1)]
    assert obs.t == 2
    assert list(obs.unsat) == [unsat_count(S[r], J, L) for r in (0, 1)]
    assert list(obs.mag) == [int(S[r].astype(np.int64).sum()) for r in (0, 1)]
    q = S[0].astype(np.int64) * S[1]
    assert obs.overlap == int(q.sum())
    assert list(obs.autocorr[:, 0]) == [int((S[r].astype(np.int64) * S0[r]).sum()) for r in (0, 1)]
    assert np.array_equal(obs.c4, axis_c4(q, L))


def test_c4_shells_errors(ea_gpu):
    g = ea_gpu.Sim(16, 0.5, 0.8, seed=1)
    for n in (0, 3 * 64 + 2):
        with pytest.raises(ea_gpu.EAError):
            g.c4_shells(n)
    big = ea_gpu.Sim(136, 0.5, 0.8, seed=1)  # beyond 128: the rows kernel
    assert big.c4_shells(10)[0] == 136 ** 3


def test_sweep_group_matches_oracle(ea_gpu, oracle_mod):
    """Grouped launches give each member the oracle's own trajectory: mixed
    p, T, seed, sample and start times, members on separate streams (one of
    them library-owned), group and single sweeps interleaved."""
    L = 24
    params = [(0.5, 0.8, 3, 0), (0.2, 0.6, 3, 1), (0.5, 1.2, 91, 4), (0.0, 0.7, 5, 2)]
    gs = [ea_gpu.Sim(L, p, T, seed=s, sample=k, n_slots=1, use_torch=(i != 2))
          for i, (p, T, s, k) in enumerate(params)]
    os_ = [oracle_mod.Sim(L, p, T, seed=s, sample=k, n_slots=1) for (p, T, s, k) in params]
    for g, o in zip(gs, os_):
        g.snapshot(0)
        o.snapshot(0)
    gs[1].sweep(2)
    os_[1].sweep(2)
    _say("group L=24: 4 runs x 5 sweeps")
    ea_gpu.sweep_group(gs, 5)
    for o in os_:
        o.sweep(5)
    gs[3].sweep(1)
    os_[3].sweep(1)
    ea_gpu.sweep_group(gs[1:], 3)
    for o in os_[1:]:
        o.sweep(3)
    for i, (g, o) in enumerate(zip(gs, os_)):
        _compare_state(g, o, f"group member {i}")
        oo = o.measure()
        assert g.time == oo.t
        _compare_obs(g.measure(), oo, f"group member {i}")


@pytest.mark.parametrize("L,n_runs,rw", [(16, 21, 0), (64, 3, 2), (128, 5, 0)])
def test_sweep_group_equals_single_runs(ea_gpu, L, n_runs, rw):
    """A group of n_runs (more than one launch's 16 members for n_runs = 21)
    reaches bit for bit the spins of the same runs swept one by one."""
    _say(f"group L={L} runs={n_runs} rw={rw}")
    mk = lambda i: ea_gpu.Sim(L, 0.5 if i % 2 else 0.3, 0.7 + 0.05 * (i % 3), seed=11, sample=i,
                              words_per_row=rw)
    grp = [mk(i) for i in range(n_runs)]
    one = [mk(i) for i in range(n_runs)]
    ea_gpu.sweep_group(grp, 4)
    ea_gpu.sweep_group(grp, 0)
    for s in one:
        s.sweep(4)
    for i, (a, b) in enumerate(zip(grp, one)):
        assert a.time == b.time == 4
        for r in (0, 1):
            assert np.array_equal(a.spins(r), b.spins(r)), (L, i, r)


@pytest.mark.parametrize("T", [0.7, 0.88])
def test_screened_group_matches_oracle(ea_gpu, oracle_mod, T):
    """Launches with four or more waves per SIMD (here four runs of L = 128
    in one group) screen the rare uphill moves of dE >= 8 with one minimum
    per word; at T = 0.88 about one wave in five meets such a random word
    and takes the general select for those lanes, at T = 0.7 one in fifty.
    Every member equals its oracle run."""
    L = 128
    params = [(0.5, 3, 0), (0.3, 3, 1), (0.2, 8, 2), (0.5, 9, 5)]
    grp = [ea_gpu.Sim(L, p, T, seed=s, sample=k) for (p, s, k) in params]
    _say(f"screened group L={L} x{len(grp)} T={T}")
    ea_gpu.sweep_group(grp, 2)
    for i, (p, s, k) in enumerate(params):
        o = oracle_mod.Sim(L, p, T, seed=s, sample=k)
        o.sweep(2)
        _compare_state(grp[i], o, f"screened member {i} T={T}")


def test_sweep_group_errors(ea_gpu):
    a = ea_gpu.Sim(16, 0.5, 0.8, seed=1)
    b = ea_gpu.Sim(16, 0.5, 0.8, seed=2)
    c = ea_gpu.Sim(24, 0.5, 0.8, seed=3)
    d = ea_gpu.Sim(64, 0.5, 0.8, seed=3, words_per_row=1)
    e = ea_gpu.Sim(64, 0.5, 0.8, seed=3, words_per_row=2)
    for bad in ([], [a, c], [a, a], [a, b, a], [d, e]):
        with pytest.raises(ea_gpu.EAError):
            ea_gpu.sweep_group(bad, 1)
    b.set_time((1 << 32) - 3)
    with pytest.raises(ea_gpu.EAError):
        ea_gpu.sweep_group([a, b], 3)
    assert a.time == 0 and b.time == (1 << 32) - 3   # nothing advanced
    ea_gpu.sweep_group([a, b], 2)
    assert a.time == 2 and b.time == (1 << 32) - 1


def test_run_group_schedules_match_oracle(ea_gpu, oracle_mod):
    """run_group: runs of one L with different p, T, seeds, lengths and
    schedules advance together and each gives its oracle run's observables
    at its own measurement times."""
    from paper_1411_5512_amd.workloads import Job
    jobs = [Job(24, 0.5, 0.8, seed=3, sample=0, n_sweeps=40, meas_t=[5, 17, 40], tw=[5]),
            Job(24, 0.2, 0.6, seed=4, sample=2, n_sweeps=25, meas_t=[1, 25], tw=[1, 12]),
            Job(24, 0.4, 1.1, seed=5, sample=1, n_sweeps=33, meas_t=[33], tw=[])]
    _say("run_group L=24 x 3")
    res = ea_gpu.run_group(jobs)
    for i, job in enumerate(jobs):
        o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=len(job.tw))
        t, k = 0, 0
        for te, slots, meas in job.events():
            o.sweep(te - t)
            t = te
            for slot in slots:
                o.snapshot(slot)
            if meas:
                _compare_obs(res[i][k], o.measure(), f"job {i} t={te}")
                k += 1
        assert k == len(res[i]) == len(job.meas_t)
