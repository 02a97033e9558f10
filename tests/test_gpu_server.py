"""The serving form: jobs submitted while others run are admitted by memory
and slots, interleave on the device, and each one's results equal the same
job run alone (tolerance 0: every observable is an integer)."""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same_obs(a, b, ctx):
    assert a.t == b.t, ctx
    assert list(a.unsat) == list(b.unsat), ctx
    assert list(a.mag) == list(b.mag), ctx
    assert a.overlap == b.overlap, ctx
    assert np.array_equal(a.autocorr, b.autocorr), ctx
    assert np.array_equal(a.c4, b.c4), ctx


def _stream_jobs(n, seed, sweep_range=(20, 400)):
    """A small Poisson-like mix of L in {8..64}, p in [0.1, 0.5],
    T in [0.5, 1.2], log-uniform sweeps, log-spaced schedules."""
    from paper_1411_5512_amd.workloads import Job, log_schedule
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(n):
        L = int(rng.choice([8, 16, 24, 32, 40, 48, 56, 64]))
        nsw = int(round(np.exp(rng.uniform(np.log(sweep_range[0]), np.log(sweep_range[1])))))
        tw = [t for t in (5, 50) if t <= nsw]
        meas = sorted(set(log_schedule(nsw, 6)) | set(tw))
        jobs.append(Job(L, float(rng.uniform(0.1, 0.5)), float(rng.uniform(0.5, 1.2)),
                        seed=7000 + j, sample=j % 3, n_sweeps=nsw, meas_t=meas, tw=tw))
    return jobs


def test_server_mix_equals_alone(ea_gpu):
    jobs = _stream_jobs(40, seed=1)
    # a budget that holds only a few jobs at once, so admission binds
    budget = 3 * max(ea_gpu.Server.footprint(j) for j in jobs)
    srv = ea_gpu.Server(hbm_budget=budget, max_resident=6, epoch_site_sweeps=64 ** 3 * 8)
    srv.start()
    ids = []
    for j in jobs:
        ids.append(srv.submit(j))
        time.sleep(0.002)  # arrivals interleave with running epochs
    srv.drain(300)
    srv.stop()
    st = srv.stats()
    _say(f"server stats {st}")
    assert st["completed"] == len(jobs) and st["pending"] == 0 and st["resident"] == 0
    assert 0 < st["hbm_peak"] <= budget
    assert st["epochs"] > 1 and st["p99_latency_s"] >= st["p50_latency_s"] > 0
    # the reference: every job in a batch of its own (one job, one launch)
    for i, (jid, job) in enumerate(zip(ids, jobs)):
        assert srv.poll(jid) == ea_gpu.JOB_DONE
        alone = ea_gpu.Batch([job])
        alone.run()
        for k in range(len(job.meas_t)):
            _same_obs(srv.result(jid, k), alone.result(0, k), f"job {i} meas {k}")
        alone.close()
        assert srv.latency(jid) > 0


def test_server_step_mode_matches_oracle(ea_gpu, oracle_mod):
    """Driven epoch by epoch on the calling thread, with a tiny epoch so that
    every job is split over many launches."""
    jobs = _stream_jobs(6, seed=2, sweep_range=(10, 60))
    srv = ea_gpu.Server(hbm_budget=1 << 26, max_resident=3, epoch_site_sweeps=16 ** 3 * 3)
    ids = [srv.submit(j) for j in jobs]
    n = 0
    while srv.step():
        n += 1
        assert n < 10000
    for jid, job in zip(ids, jobs):
        o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=len(job.tw))
        t, k = 0, 0
        for te, slots, meas in job.events():
            o.sweep(te - t)
            t = te
            for s in slots:
                o.snapshot(s)
            if meas:
                _same_obs(srv.result(jid, k), o.measure(), f"job {jid} meas {k}")
                k += 1
        srv.release(jid)
        with pytest.raises(ea_gpu.EAError):
            srv.poll(jid)


def test_server_admission_limits(ea_gpu):
    from paper_1411_5512_amd.workloads import Job
    big = Job(64, 0.5, 0.7, seed=1, n_sweeps=5, meas_t=[5])
    fp = ea_gpu.Server.footprint(big)
    srv = ea_gpu.Server(hbm_budget=fp, max_resident=4, max_pending=2)
    with pytest.raises(ea_gpu.EAError):  # larger than the whole budget
        srv.submit(Job(64, 0.5, 0.7, seed=1, n_sweeps=5, meas_t=[1, 2, 3, 4, 5], tw=[1, 2]))
    for L in (100, 264):  # no lattice of that size exists in either form
        with pytest.raises(ea_gpu.EAError):
            srv.submit(Job(L, 0.5, 0.7, seed=1, n_sweeps=5, meas_t=[5]))
    a = srv.submit(big)
    b = srv.submit(big)
    with pytest.raises(ea_gpu.EAError):  # max_pending
        srv.submit(big)
    assert srv.step()
    # only one fits the budget: the first ran, the second waited
    assert srv.poll(a) == ea_gpu.JOB_DONE and srv.poll(b) == ea_gpu.JOB_PENDING
    with pytest.raises(ea_gpu.EAError):
        srv.result(b, 0)
    assert srv.step()
    assert srv.poll(b) == ea_gpu.JOB_DONE
    assert not srv.step()
    _same_obs(srv.result(a, 0), srv.result(b, 0), "identical jobs")


def _alone_plain(ea_gpu, job):
    """The job run alone through the plain form, measurement by measurement."""
    g = ea_gpu.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=len(job.tw))
    res, t = [], 0
    for te, slots, meas in job.events():
        if te > t:
            g.sweep(te - t)
            t = te
        for k in slots:
            g.snapshot(k)
        if meas:
            res.append(g.measure())
    return res


def test_server_streams_large_lattices(ea_gpu):
    """Lattices above 64 (streamed through the plain kernels on a second
    stream) mixed with LDS-resident ones: every job equals its run alone."""
    from paper_1411_5512_amd.workloads import Job
    jobs = [
        Job(96, 0.5, 0.7, seed=31, sample=0, n_sweeps=40, meas_t=[0, 3, 17, 40], tw=[3, 17]),
        Job(16, 0.3, 0.8, seed=32, sample=1, n_sweeps=300, meas_t=[10, 100, 300], tw=[10]),
        Job(128, 0.2, 0.7, seed=33, sample=0, n_sweeps=25, meas_t=[1, 25], tw=[1]),
        Job(64, 0.5, 0.9, seed=34, sample=0, n_sweeps=60, meas_t=[0, 60], tw=[0]),
        Job(72, 0.4, 1.1, seed=35, sample=2, n_sweeps=0, meas_t=[0], tw=[0]),
        Job(256, 0.5, 0.7, seed=36, sample=0, n_sweeps=3, meas_t=[3], tw=[]),
        Job(32, 0.5, 0.6, seed=37, sample=0, n_sweeps=200, meas_t=[50, 200], tw=[50]),
    ]
    srv = ea_gpu.Server(hbm_budget=1 << 28, max_resident=4, epoch_site_sweeps=32 ** 3 * 4)
    srv.start()
    ids = [srv.submit(j) for j in jobs]
    srv.drain(300)
    srv.stop()
    st = srv.stats()
    _say(f"server stats {st}")
    assert st["completed"] == len(jobs)
    for jid, job in zip(ids, jobs):
        _say(f"streamed-mix job L={job.L} sweeps={job.n_sweeps}")
        ref = _alone_plain(ea_gpu, job)
        assert len(ref) == len(job.meas_t)
        for k, want in enumerate(ref):
            _same_obs(srv.result(jid, k), want, f"L={job.L} meas {k}")


def test_server_groups_streamed_jobs_of_one_size(ea_gpu):
    """Several streamed jobs of the same L with different lengths and
    schedules, beside another size and an LDS job, through many epochs:
    every job equals its run alone."""
    from paper_1411_5512_amd.workloads import Job
    jobs = [
        Job(96, 0.5, 0.7, seed=51, sample=0, n_sweeps=37, meas_t=[0, 4, 21, 37], tw=[4]),
        Job(96, 0.3, 0.9, seed=52, sample=1, n_sweeps=12, meas_t=[12], tw=[3]),
        Job(96, 0.2, 0.6, seed=53, sample=0, n_sweeps=50, meas_t=[1, 7, 50], tw=[7, 30]),
        Job(72, 0.5, 0.8, seed=54, sample=0, n_sweeps=29, meas_t=[9, 29], tw=[9]),
        Job(72, 0.4, 1.0, seed=55, sample=2, n_sweeps=18, meas_t=[2, 18], tw=[]),
        Job(24, 0.5, 0.8, seed=56, sample=0, n_sweeps=90, meas_t=[30, 90], tw=[30]),
    ]
    srv = ea_gpu.Server(hbm_budget=1 << 28, max_resident=8, epoch_site_sweeps=24 ** 3 * 5)
    ids = [srv.submit(j) for j in jobs]
    n = 0
    while srv.step():
        n += 1
        assert n < 10000
    for jid, job in zip(ids, jobs):
        _say(f"grouped streamed job L={job.L} sweeps={job.n_sweeps}")
        ref = _alone_plain(ea_gpu, job)
        for k, want in enumerate(ref):
            _same_obs(srv.result(jid, k), want, f"L={job.L} seed={job.seed} meas {k}")


def test_server_streamed_job_matches_oracle(ea_gpu, oracle_mod):
    """One streamed job, split over many epochs, against the oracle."""
    from paper_1411_5512_amd.workloads import Job
    job = Job(80, 0.5, 0.8, seed=41, sample=3, n_sweeps=6, meas_t=[0, 2, 5, 6], tw=[2])
    srv = ea_gpu.Server(hbm_budget=1 << 26, max_resident=2)
    jid = srv.submit(job)
    n = 0
    while srv.step():
        n += 1
        assert n < 1000
    o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=1)
    t, k = 0, 0
    for te, slots, meas in job.events():
        o.sweep(te - t)
        t = te
        for s in slots:
            o.snapshot(s)
        if meas:
            _same_obs(srv.result(jid, k), o.measure(), f"meas {k}")
            k += 1
    assert k == len(job.meas_t)


def test_server_moves_a_long_batched_job_to_slabs(ea_gpu):
    """A long L = 48 job admitted to the batched launch while every worker
    has a streamed job moves to the slab path once a worker is free (its
    state, snapshots and first measurements carried over); an L = 64 job
    admitted to an idle server goes to the slab path at once; every job's
    results equal its run alone."""
    from paper_1411_5512_amd.workloads import Job
    first = [Job(72, 0.5, 0.8, seed=80 + i, sample=i, n_sweeps=30, meas_t=[30], tw=[]) for i in range(5)]
    long48 = Job(48, 0.4, 0.7, seed=90, sample=1, n_sweeps=6000, meas_t=[0, 100, 700, 3000, 6000],
                 tw=[10, 5000])
    small = Job(16, 0.5, 0.9, seed=91, sample=0, n_sweeps=400, meas_t=[400], tw=[50])
    jobs = first + [long48, small]
    srv = ea_gpu.Server(hbm_budget=1 << 28, max_resident=16)
    ids = [srv.submit(j) for j in jobs]
    n = 0
    while srv.step():
        n += 1
        assert n < 100000
    st = srv.stats()
    _say(f"server stats {st}")
    assert st["moved"] >= 1 and st["completed"] == len(jobs)
    for jid, job in zip(ids, jobs):
        alone = ea_gpu.Batch([job]) if job.L <= 64 else None
        if alone is not None:
            alone.run()
            for k in range(len(job.meas_t)):
                _same_obs(srv.result(jid, k), alone.result(0, k), f"L={job.L} meas {k}")
            alone.close()
        else:
            ref = _alone_plain(ea_gpu, job)
            for k, want in enumerate(ref):
                _same_obs(srv.result(jid, k), want, f"L={job.L} meas {k}")
    idle = ea_gpu.Server(hbm_budget=1 << 28, max_resident=4)
    job = Job(64, 0.5, 0.7, seed=92, sample=0, n_sweeps=300, meas_t=[0, 37, 300], tw=[37])
    jid = idle.submit(job)
    while idle.step():
        pass
    assert idle.stats()["streamed_small"] == 1
    alone = ea_gpu.Batch([job])
    alone.run()
    for k in range(len(job.meas_t)):
        _same_obs(idle.result(jid, k), alone.result(0, k), f"idle L=64 meas {k}")
    alone.close()


def test_server_long_jobs_equal_alone(ea_gpu):
    """Long jobs of the serving configuration's sizes (L = 128 for 4 x 10^4
    sweeps, L = 96 for 3 x 10^4, and a long L = 64 job that starts in the
    batched launch and moves to the slab path mid-run) through the worker
    thread: every measurement, late ones included, equals the job run alone."""
    from paper_1411_5512_amd.workloads import Job, log_schedule
    jobs = []
    for i, (L, n) in enumerate([(72, 40), (72, 40), (72, 40), (72, 40), (72, 40),
                                (128, 40_000), (96, 30_000), (64, 20_000)]):
        tw = [t for t in (100, 1000) if t <= n]
        meas = sorted(set(log_schedule(n, 12)) | set(tw))
        jobs.append(Job(L, 0.2 + 0.05 * (i % 5), 0.6 + 0.1 * (i % 4), seed=300 + i, sample=i % 3,
                        n_sweeps=n, meas_t=meas, tw=tw))
    srv = ea_gpu.Server(hbm_budget=1 << 29, max_resident=16)
    ids = [srv.submit(j) for j in jobs]  # all admitted at the first epoch, in this order
    srv.start()
    srv.drain(600)
    srv.stop()
    st = srv.stats()
    _say(f"server stats {st}")
    assert st["completed"] == len(jobs) and st["moved"] >= 1
    for jid, job in zip(ids, jobs):
        if job.L <= 64:
            alone = ea_gpu.Batch([job])
            alone.run()
            ref = [alone.result(0, k) for k in range(len(job.meas_t))]
            alone.close()
        else:
            ref = _alone_plain(ea_gpu, job)
        _say(f"long job L={job.L} sweeps={job.n_sweeps}")
        for k, want in enumerate(ref):
            _same_obs(srv.result(jid, k), want, f"L={job.L} meas {k} t={job.meas_t[k]}")
