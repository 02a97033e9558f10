"""Late-time oracle windows on the configurations the benchmark times, in
the launch configurations it times them with: the oracle, started from the
GPU's state at t0 near the end of the run (and given the GPU's reference
configurations S(t_w) as its snapshots), reproduces the last sweeps bit for
bit, with every observable of the final measurement (Sec. III's dynamics,
eq. 9; observables of eqs. 1, 2, 3, 7)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(go, oo, ctx, autocorr=True):
    assert go.t == oo.t, ctx
    assert list(go.unsat) == list(oo.unsat), ctx
    assert list(go.mag) == list(oo.mag), ctx
    assert go.overlap == oo.overlap, ctx
    if autocorr:
        assert np.array_equal(go.autocorr, oo.autocorr), ctx
    assert np.array_equal(go.c4, oo.c4), ctx


def _oracle_from(oracle_mod, job, refs, state, t0):
    """An oracle run of `job` holding the GPU's snapshots (refs: list of
    (t_w, [S_0, S_1])) and state at t0."""
    o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=len(job.tw))
    for k, (tw, st) in enumerate(refs):
        for r in (0, 1):
            o.set_spins(r, st[r])
        o.set_time(tw)
        o.snapshot(k)
    for r in (0, 1):
        o.set_spins(r, state[r])
    o.set_time(t0)
    return o


def test_crossover_window_at_one_million_sweeps(ea_gpu, oracle_mod):
    """The five crossover runs (L = 128, p = 0.5 ... 0.15, T = 0.7) grouped as
    the benchmark runs them (ea_sweep_group, slab launches), advanced to
    t0 = 10^6 - 2; the oracle from there gives the GPU's spins at 10^6 and
    the final measurement, C(t, t_w) at t_w = 100 and 10^4 included."""
    from paper_1411_5512_amd import workloads as wl
    jobs = wl.crossover_jobs(1_000_000)
    t_end = jobs[0].n_sweeps
    t0 = t_end - 2
    sims = [ea_gpu.Sim(j.L, j.p, j.T, seed=j.seed, sample=j.sample, n_slots=len(j.tw)) for j in jobs]
    refs = [[] for _ in jobs]
    t = 0
    for k, tw in enumerate(jobs[0].tw):
        ea_gpu.sweep_group(sims, tw - t)
        t = tw
        for i, s in enumerate(sims):
            s.snapshot(k)
            refs[i].append((tw, [s.spins(0), s.spins(1)]))
    _say(f"crossover: snapshots at {jobs[0].tw}, plan {sims[0].slab_plan} (alone)")
    ea_gpu.sweep_group(sims, t0 - t)
    states = [[s.spins(0), s.spins(1)] for s in sims]
    ea_gpu.sweep_group(sims, 2)
    for i, (job, s) in enumerate(zip(jobs, sims)):
        _say(f"crossover window p={job.p}")
        o = _oracle_from(oracle_mod, job, refs[i], states[i], t0)
        o.sweep(2)
        for r in (0, 1):
            assert np.array_equal(s.spins(r), o.spins(r)), (job.p, r)
        _same(s.measure(), o.measure(), f"p={job.p} t={t_end}")
        s.close()


def test_mid_size_window_at_the_end(ea_gpu, oracle_mod):
    """The mid-size plain run (L = 64, p = 0.5, T = 0.7) with its default
    packing and slab plan, as the benchmark runs it: its whole schedule, the
    oracle restarted at t0 = 10^5 - 3 with the GPU's snapshots."""
    from paper_1411_5512_amd import workloads as wl
    job = wl.mid_job(100_000)
    g = ea_gpu.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=len(job.tw))
    _say(f"mid-size: rw={g.words_per_row} plan={g.slab_plan}")
    refs, t, last = [], 0, None
    t0 = job.n_sweeps - 3
    for te, slots, meas in job.events():
        if te > t0 >= t:
            g.sweep(t0 - t)
            t = t0
            state = [g.spins(0), g.spins(1)]
        g.sweep(te - t)
        t = te
        for k in slots:
            g.snapshot(k)
            refs.append((te, [g.spins(0), g.spins(1)]))
        if meas:
            last = g.measure()
    assert t == job.n_sweeps and last.t == job.n_sweeps
    o = _oracle_from(oracle_mod, job, refs, state, t0)
    o.sweep(3)
    for r in (0, 1):
        assert np.array_equal(g.spins(r), o.spins(r)), r
    _same(last, o.measure(), "mid-size t=1e5")
    g.close()


def test_benchmark_batch_window_with_tuned_launches(ea_gpu, oracle_mod):
    """The benchmark's batch (256 jobs, L in {24, 32, 48, 64}, 10^5 sweeps)
    with the autotuned launches, captured and replayed as the benchmark does:
    for the first job of each L (and of each T), the oracle started from that
    job's state at t0 = 99997 (taken from an eager run of the same tuned
    batch stopped there) reproduces the replayed batch's final spins and its
    last measurement, C(t, t_w) included."""
    from paper_1411_5512_amd import workloads as wl
    jobs = wl.batch_jobs(n_jobs=256, n_sweeps=100_000)
    for L in sorted({j.L for j in jobs}):
        _say(f"tune L={L}: {ea_gpu.tune(L)['chosen']}")
    picks = []
    for key in sorted({(j.L, j.T) for j in jobs}):
        picks.append(next(i for i, j in enumerate(jobs) if (j.L, j.T) == key))
    t0 = 99_997
    eager = ea_gpu.Batch(jobs, autotune=True)
    refs = {i: [] for i in picks}
    for tw in jobs[0].tw:
        eager.run(tw)
        for i in picks:
            refs[i].append((tw, [eager.spins(i, 0), eager.spins(i, 1)]))
    eager.run(t0)
    states = {i: [eager.spins(i, 0), eager.spins(i, 1)] for i in picks}
    eager.close()
    bench = ea_gpu.Batch(jobs, autotune=True)
    bench.capture()
    bench.replay()
    for i in picks:
        job = jobs[i]
        _say(f"batch window job {i}: L={job.L} p={job.p} T={job.T}")
        o = _oracle_from(oracle_mod, job, refs[i], states[i], t0)
        o.sweep(3)
        for r in (0, 1):
            assert np.array_equal(bench.spins(i, r), o.spins(r)), (i, r)
        _same(bench.result(i, len(job.meas_t) - 1), o.measure(), f"job {i} t=1e5")
    bench.close()
