"""Parity of the batched form: every job of a batch gives, measurement by
measurement, the same integers as the oracle (and as a plain GPU run) with the
same parameters and schedule, whatever the mix of sizes around it and however
the sweeps are split into launches."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run_schedule(sim, job):
    """Drive a plain (oracle or GPU) run through the job's schedule."""
    res = []
    t = 0
    for te, slots, meas in job.events():
        if te > t:
            sim.sweep(te - t)
            t = te
        for k in slots:
            sim.snapshot(k)
        if meas:
            res.append(sim.measure())
    if job.n_sweeps > t:
        sim.sweep(job.n_sweeps - t)
    return res


def _same_obs(a, b, ctx):
    assert a.t == b.t, ctx
    assert list(a.unsat) == list(b.unsat), ctx
    assert list(a.mag) == list(b.mag), ctx
    assert a.overlap == b.overlap, ctx
    assert np.array_equal(a.autocorr, b.autocorr), ctx
    assert np.array_equal(a.c4, b.c4), ctx


def _mixed_jobs():
    from paper_1411_5512_amd.workloads import Job
    return [
        Job(8, 0.5, 0.8, seed=11, sample=0, n_sweeps=40, meas_t=[0, 1, 5, 17, 40], tw=[0, 5]),
        Job(16, 0.3, 0.6, seed=12, sample=2, n_sweeps=30, meas_t=[3, 10, 30], tw=[10]),
        Job(24, 0.5, 1.0, seed=13, sample=0, n_sweeps=20, meas_t=[20], tw=[]),
        Job(32, 0.2, 0.7, seed=14, sample=1, n_sweeps=16, meas_t=[2, 16], tw=[2, 8]),
        Job(40, 0.5, 0.9, seed=15, sample=0, n_sweeps=10, meas_t=[1, 10], tw=[1]),
        Job(48, 0.25, 0.7, seed=16, sample=0, n_sweeps=8, meas_t=[4, 8], tw=[4]),
        Job(56, 0.5, 1.2, seed=17, sample=0, n_sweeps=6, meas_t=[6], tw=[3]),
        Job(64, 0.5, 0.7, seed=1, sample=0, n_sweeps=6, meas_t=[1, 6], tw=[1]),
        Job(16, 0.0, 0.7, seed=18, sample=0, n_sweeps=25, meas_t=[25], tw=[5]),
        Job(16, 1.0, 0.7, seed=18, sample=0, n_sweeps=25, meas_t=[25], tw=[5]),
        Job(16, 0.5, 0.0, seed=19, sample=0, n_sweeps=25, meas_t=[12, 25], tw=[12]),
        Job(24, 0.5, 0.8, seed=20, sample=0, n_sweeps=0, meas_t=[0], tw=[0]),
    ]


def test_batch_matches_oracle(ea_gpu, oracle_mod):
    jobs = _mixed_jobs()
    b = ea_gpu.Batch(jobs)
    b.run()
    for j, job in enumerate(jobs):
        _say(f"batch job {j}: L={job.L} p={job.p} T={job.T} sweeps={job.n_sweeps}")
        o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=len(job.tw))
        ref = _run_schedule(o, job)
        assert b.time(j) == job.n_sweeps
        for k, want in enumerate(ref):
            _same_obs(b.result(j, k), want, f"job {j} meas {k}")
        for r in (0, 1):
            assert np.array_equal(b.spins(j, r), o.spins(r)), f"job {j} replica {r}"


def test_batch_split_into_spans(ea_gpu):
    jobs = _mixed_jobs()
    whole = ea_gpu.Batch(jobs)
    whole.run()
    parts = ea_gpu.Batch(jobs)
    for t in (0, 1, 7, 13, 13, 29):
        parts.run(t)
    parts.run()
    for j, job in enumerate(jobs):
        for k in range(len(job.meas_t)):
            _same_obs(parts.result(j, k), whole.result(j, k), f"job {j} meas {k}")
        for r in (0, 1):
            assert np.array_equal(parts.spins(j, r), whole.spins(j, r))
    # reset regenerates the same initial state and results
    whole.reset()
    whole.run()
    for j, job in enumerate(jobs):
        for k in range(len(job.meas_t)):
            _same_obs(parts.result(j, k), whole.result(j, k), f"reset job {j} meas {k}")


def test_batch_matches_plain_gpu_runs(ea_gpu):
    """A slice of the 256-job mixed workload (L in {24,32,48,64}, p in
    {0.5,0.3,0.2}, T in {0.6,0.8,1.0}) at 3000 sweeps: every job of the
    batch equals the same job run alone through the plain form."""
    from paper_1411_5512_amd import workloads as wl
    jobs = wl.batch_jobs(n_jobs=256, n_sweeps=3000)[:24]
    b = ea_gpu.Batch(jobs)
    b.run()
    for j, job in enumerate(jobs):
        if j % 3:
            continue
        _say(f"alone job {j}: L={job.L}")
        g = ea_gpu.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=len(job.tw))
        ref = _run_schedule(g, job)
        for k, want in enumerate(ref):
            _same_obs(b.result(j, k), want, f"job {j} meas {k}")
        for r in (0, 1):
            assert np.array_equal(b.spins(j, r), g.spins(r))


def test_batch_windowed_parity_late_times(ea_gpu, oracle_mod):
    """The oracle, started from a batch job's state at t0, reproduces the
    batch after a few more sweeps (late-time window of a long run)."""
    from paper_1411_5512_amd.workloads import Job
    jobs = [Job(64, 0.5, 0.7, seed=1, n_sweeps=20000, meas_t=[20000], tw=[]),
            Job(48, 0.3, 0.6, seed=2, n_sweeps=20000, meas_t=[20000], tw=[])]
    b = ea_gpu.Batch(jobs)
    b.run(15000)
    states = [[b.spins(j, r) for r in (0, 1)] for j in range(2)]
    b.run(15003)
    for j, job in enumerate(jobs):
        o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample)
        for r in (0, 1):
            o.set_spins(r, states[j][r])
        o.set_time(15000)
        o.sweep(3)
        for r in (0, 1):
            assert np.array_equal(b.spins(j, r), o.spins(r)), (j, r)


def test_batch_errors(ea_gpu):
    from paper_1411_5512_amd.workloads import Job
    with pytest.raises(ea_gpu.EAError):
        ea_gpu.Batch([Job(72, 0.5, 0.7, seed=1, n_sweeps=10, meas_t=[10])])
    with pytest.raises(ea_gpu.EAError):
        ea_gpu.Batch([Job(16, 0.5, 0.7, seed=1, n_sweeps=10, meas_t=[5, 5])])
    with pytest.raises(ea_gpu.EAError):
        ea_gpu.Batch([Job(16, 0.5, 0.7, seed=1, n_sweeps=10, meas_t=[11])])
    b = ea_gpu.Batch([Job(16, 0.5, 0.7, seed=1, n_sweeps=10, meas_t=[3, 10], tw=[3])])
    b.run(5)
    b.result(0, 0)
    with pytest.raises(ea_gpu.EAError):
        b.result(0, 1)
    b.run()
    b.result(0, 1)


def test_batch_graph_replays(ea_gpu):
    """The captured reset + run graph gives the eager results on every
    replay, with other eager work on the device in between."""
    jobs = _mixed_jobs()
    eager = ea_gpu.Batch(jobs)
    eager.run()
    g = ea_gpu.Batch(jobs)
    g.capture()
    other = ea_gpu.Sim(16, 0.5, 0.8, seed=3)
    for rep in range(3):
        g.replay()
        for j, job in enumerate(jobs):
            assert g.time(j) == job.n_sweeps
            for k in range(len(job.meas_t)):
                _same_obs(g.result(j, k), eager.result(j, k), f"replay {rep} job {j} meas {k}")
            for r in (0, 1):
                assert np.array_equal(g.spins(j, r), eager.spins(j, r)), (rep, j, r)
        other.sweep(10)
        other.measure()


# ---------------------------------------------------------------------------
# Split replicas: two workgroups per replica exchanging boundary planes.

def _split_jobs():
    from paper_1411_5512_amd.workloads import Job
    return [
        Job(64, 0.5, 0.7, seed=21, sample=0, n_sweeps=12, meas_t=[0, 1, 5, 12], tw=[0, 5]),
        Job(48, 0.3, 0.9, seed=22, sample=1, n_sweeps=10, meas_t=[3, 10], tw=[3]),
        Job(56, 0.5, 1.1, seed=23, sample=0, n_sweeps=8, meas_t=[8], tw=[2]),
        Job(64, 0.2, 0.0, seed=24, sample=0, n_sweeps=6, meas_t=[6], tw=[]),
        Job(16, 0.5, 0.8, seed=25, sample=0, n_sweeps=20, meas_t=[20], tw=[10]),
        Job(48, 0.5, 0.8, seed=26, sample=0, n_sweeps=0, meas_t=[0], tw=[0]),
    ]


def test_split_batch_matches_oracle(ea_gpu, oracle_mod):
    jobs = _split_jobs()
    b = ea_gpu.Batch(jobs, split=ea_gpu.Batch.SPLIT_ALWAYS)
    assert [b.parts(j) for j in range(len(jobs))] == [2, 2, 2, 2, 1, 2]
    b.run()
    for j, job in enumerate(jobs):
        _say(f"split job {j}: L={job.L} p={job.p} T={job.T} sweeps={job.n_sweeps}")
        o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=len(job.tw))
        ref = _run_schedule(o, job)
        assert b.time(j) == job.n_sweeps
        for k, want in enumerate(ref):
            _same_obs(b.result(j, k), want, f"split job {j} meas {k}")
        for r in (0, 1):
            assert np.array_equal(b.spins(j, r), o.spins(r)), f"split job {j} replica {r}"


def test_split_spans_reset_and_graph(ea_gpu):
    jobs = _split_jobs()
    whole = ea_gpu.Batch(jobs, split=ea_gpu.Batch.SPLIT_NEVER)
    whole.run()
    parts = ea_gpu.Batch(jobs, split=ea_gpu.Batch.SPLIT_ALWAYS)
    for t in (0, 1, 4, 4, 9):
        parts.run(t)
    parts.run()

    def same(a, label):
        for j, job in enumerate(jobs):
            for k in range(len(job.meas_t)):
                _same_obs(a.result(j, k), whole.result(j, k), f"{label} job {j} meas {k}")
            for r in (0, 1):
                assert np.array_equal(a.spins(j, r), whole.spins(j, r)), (label, j, r)

    same(parts, "spans")
    parts.reset()
    parts.run()
    same(parts, "reset")
    g = ea_gpu.Batch(jobs, split=ea_gpu.Batch.SPLIT_ALWAYS)
    g.capture()
    other = ea_gpu.Sim(16, 0.5, 0.8, seed=3)
    for rep in range(3):
        g.replay()
        same(g, f"replay {rep}")
        other.sweep(10)
        other.measure()


def test_split_matches_unsplit_full_mix(ea_gpu):
    """The 256-job mixed workload (L in {24,32,48,64}) in one launch with its
    L = 64 replicas split (256 slabs, one per CU) equals the unsplit run,
    every measurement and final state, at 300 sweeps."""
    from paper_1411_5512_amd import workloads as wl
    jobs = wl.batch_jobs(n_jobs=256, n_sweeps=300)
    sp = ea_gpu.Batch(jobs, split=ea_gpu.Batch.SPLIT_ALWAYS)
    split_jobs = [j for j in range(len(jobs)) if sp.parts(j) == 2]
    _say(f"split {len(split_jobs)} jobs, sizes {sorted({jobs[j].L for j in split_jobs})}")
    assert split_jobs and all(jobs[j].L == 64 for j in split_jobs)
    sp.run()
    ref = ea_gpu.Batch(jobs, split=ea_gpu.Batch.SPLIT_NEVER)
    ref.run()
    for j, job in enumerate(jobs):
        for k in range(len(job.meas_t)):
            _same_obs(sp.result(j, k), ref.result(j, k), f"job {j} meas {k}")
        if j in split_jobs[:8]:
            for r in (0, 1):
                assert np.array_equal(sp.spins(j, r), ref.spins(j, r)), (j, r)


def test_split_automatic_choice(ea_gpu):
    """Automatic choice: a few large samples (the run is one replica's
    latency) are split; the 256-job mix (enough work for every CU) is not."""
    from paper_1411_5512_amd import workloads as wl
    from paper_1411_5512_amd.workloads import Job
    few = [Job(64, 0.5, 0.7, seed=40 + i, n_sweeps=50, meas_t=[10, 50], tw=[10]) for i in range(8)]
    a = ea_gpu.Batch(few)
    assert all(a.parts(j) == 2 for j in range(len(few)))
    a.run()
    ref = ea_gpu.Batch(few, split=ea_gpu.Batch.SPLIT_NEVER)
    ref.run()
    for j, job in enumerate(few):
        for k in range(len(job.meas_t)):
            _same_obs(a.result(j, k), ref.result(j, k), f"few job {j} meas {k}")
    mix = ea_gpu.Batch(wl.batch_jobs(n_jobs=256, n_sweeps=100))
    assert all(mix.parts(j) == 1 for j in range(256))


def test_split_windowed_parity_late_times(ea_gpu, oracle_mod):
    from paper_1411_5512_amd.workloads import Job
    jobs = [Job(64, 0.5, 0.7, seed=1, n_sweeps=20000, meas_t=[20000], tw=[]),
            Job(48, 0.3, 0.6, seed=2, n_sweeps=20000, meas_t=[20000], tw=[])]
    b = ea_gpu.Batch(jobs, split=ea_gpu.Batch.SPLIT_ALWAYS)
    assert b.parts(0) == 2 and b.parts(1) == 2
    b.run(15000)
    states = [[b.spins(j, r) for r in (0, 1)] for j in range(2)]
    b.run(15003)
    for j, job in enumerate(jobs):
        o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample)
        for r in (0, 1):
            o.set_spins(r, states[j][r])
        o.set_time(15000)
        o.sweep(3)
        for r in (0, 1):
            assert np.array_equal(b.spins(j, r), o.spins(r)), (j, r)


def test_coherence_length_grows(ea_gpu):
    """Ageing (Sec. IV): the integral estimate xi_1 of the coherence length,
    from the disorder average over 48 samples at p = 0.5, T = 0.7, grows
    between t = 10 and t = 2000 sweeps."""
    from paper_1411_5512_amd import analysis as an
    from paper_1411_5512_amd.workloads import Job
    L = 32
    jobs = [Job(L, 0.5, 0.7, seed=100 + i, n_sweeps=2000, meas_t=[10, 2000]) for i in range(48)]
    b = ea_gpu.Batch(jobs)
    b.run()
    xi = []
    for k in range(2):
        curves = []
        for j in range(len(jobs)):
            r, c = an.c4_of_axes(b.result(j, k).c4, L)
            curves.append(c)
        xi.append(an.xi_k_samples(r, np.array(curves), k=1)[0])
    _say(f"xi_1(t=10) = {xi[0]:.3f}, xi_1(t=2000) = {xi[1]:.3f}")
    assert 0 < xi[0] < xi[1] < L / 2
