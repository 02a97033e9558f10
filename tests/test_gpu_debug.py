"""Race and order debug mode (ea_set_debug).  Within a half-step of the
checkerboard schedule (Sec. III, Fig. 1) every site of one colour depends only
on the other colour, so which workgroup takes which tile, in what order, and
what LDS held before a kernel ran must not change a single bit.  With the
workgroups' tiles reversed and/or rotated and the persistent kernels' LDS
poisoned before they load, every form is compared with the CPU oracle (or,
where the oracle would take minutes, with the same run in the default
mode, itself compared with the oracle in the other GPU tests)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

R, ROT, POI = 1, 2, 4
MODES = [(R, 0), (ROT, 5), (ROT, 77777), (POI, 3), (R | ROT | POI, 12345)]
MODE_IDS = ["reverse", "rotate5", "rotate77777", "poison", "all"]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture
def debug(ea_gpu):
    """Sets a mode for the test and always switches it off afterwards (the
    mode is process-wide)."""
    def set_mode(flags, seed):
        ea_gpu.set_debug(flags, seed)
        assert ea_gpu.get_debug() == (flags, seed)
    yield set_mode
    ea_gpu.set_debug(0, 0)


def _same_obs(a, b, ctx):
    assert a.t == b.t, ctx
    assert list(a.unsat) == list(b.unsat), ctx
    assert list(a.mag) == list(b.mag), ctx
    assert a.overlap == b.overlap, ctx
    assert np.array_equal(a.autocorr, b.autocorr), ctx
    assert np.array_equal(a.c4, b.c4), ctx


def _same_state(a, b, ctx):
    for r in (0, 1):
        assert np.array_equal(a.spins(r), b.spins(r)), (ctx, r)


_ORACLE = {}


def _oracle_run(oracle_mod, L, p, T, seed, sample, sweeps):
    """Oracle state and observables after `sweeps` (snapshot at t = 0),
    cached across the modes."""
    key = (L, p, T, seed, sample, sweeps)
    if key not in _ORACLE:
        o = oracle_mod.Sim(L, p, T, seed=seed, sample=sample, n_slots=1)
        o.snapshot(0)
        o.sweep(sweeps)
        _ORACLE[key] = ([o.spins(0), o.spins(1)], o.measure())
    return _ORACLE[key]


def _check_plain(g, oracle_mod, L, p, T, seed, sample, sweeps, ctx):
    spins, obs = _oracle_run(oracle_mod, L, p, T, seed, sample, sweeps)
    for r in (0, 1):
        assert np.array_equal(g.spins(r), spins[r]), (ctx, r)
    _same_obs(g.measure(), obs, ctx)


@pytest.mark.parametrize("flags,seed", MODES, ids=MODE_IDS)
def test_half_step_launches_under_debug(ea_gpu, oracle_mod, debug, flags, seed):
    """One launch per half-step (plain and grouped), with the 64-sweep graph
    captured under the mode: against the oracle."""
    debug(flags, seed)
    for L, rw in ((16, 1), (24, 3)):
        _say(f"half-step L={L} rw={rw} mode={flags}/{seed}")
        g = ea_gpu.Sim(L, 0.5, 0.8, seed=4, sample=1, n_slots=1, words_per_row=rw)
        g.set_slab_plan(-1, 0)
        g.snapshot(0)
        g.sweep(70)  # one graph replay of 64 sweeps, then 6 launches
        _check_plain(g, oracle_mod, L, 0.5, 0.8, 4, 1, 70, f"half-step L={L} rw={rw}")
        g.close()
    sims = [ea_gpu.Sim(16, p, 0.7, seed=9, sample=0, n_slots=1) for p in (0.5, 0.2)]
    for s in sims:
        s.set_slab_plan(-1, 0)
        s.snapshot(0)
    ea_gpu.sweep_group(sims, 9)
    for p, s in zip((0.5, 0.2), sims):
        _check_plain(s, oracle_mod, 16, p, 0.7, 9, 0, 9, f"grouped half-step p={p}")
        s.close()


@pytest.mark.parametrize("flags,seed", MODES, ids=MODE_IDS)
def test_slab_launches_under_debug(ea_gpu, oracle_mod, debug, flags, seed):
    """Slab launches with one and several ghost planes, one plane per
    workgroup, and shares spanning two replicas of different runs: against
    the oracle."""
    debug(flags, seed)
    for L, rw, K, gh, sweeps in ((32, 2, 8, 1, 6), (24, 1, 3, 2, 7), (64, 4, 64, 1, 3)):
        _say(f"slab L={L} rw={rw} K={K} g={gh} mode={flags}/{seed}")
        s = ea_gpu.Sim(L, 0.4, 0.75, seed=6, sample=2, n_slots=1, words_per_row=rw)
        s.set_slab_plan(K, gh)
        s.snapshot(0)
        s.sweep(1)
        s.sweep(sweeps - 1)
        _check_plain(s, oracle_mod, L, 0.4, 0.75, 6, 2, sweeps, f"slab L={L} K={K} g={gh}")
        s.close()
    params = [(0.5, 0.5), (0.3, 0.9), (0.2, 1.3)]
    sims = [ea_gpu.Sim(64, p, T, seed=17, sample=i, n_slots=1, words_per_row=4) for i, (p, T) in enumerate(params)]
    for s in sims:
        s.snapshot(0)
    ea_gpu.sweep_group(sims, 3)
    for i, ((p, T), s) in enumerate(zip(params, sims)):
        _check_plain(s, oracle_mod, 64, p, T, 17, i, 3, f"spanning group run {i}")
        s.close()


def _batch_jobs():
    from paper_1411_5512_amd.workloads import Job
    return [
        Job(64, 0.5, 0.7, seed=21, sample=0, n_sweeps=8, meas_t=[0, 1, 5, 8], tw=[0, 5]),
        Job(48, 0.3, 0.9, seed=22, sample=1, n_sweeps=10, meas_t=[3, 10], tw=[3]),
        Job(16, 0.5, 0.8, seed=25, sample=0, n_sweeps=20, meas_t=[20], tw=[10]),
        Job(24, 0.2, 0.6, seed=26, sample=2, n_sweeps=15, meas_t=[4, 15], tw=[4]),
        Job(32, 0.5, 1.1, seed=27, sample=0, n_sweeps=12, meas_t=[12], tw=[]),
        Job(8, 0.5, 0.0, seed=28, sample=0, n_sweeps=30, meas_t=[0, 30], tw=[0]),
    ]


_BATCH_REF = {}


def _batch_reference(oracle_mod):
    """Oracle observables and final spins of every job of _batch_jobs()."""
    if not _BATCH_REF:
        for j, job in enumerate(_batch_jobs()):
            o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=len(job.tw))
            res, t = [], 0
            for te, slots, meas in job.events():
                if te > t:
                    o.sweep(te - t)
                    t = te
                for k in slots:
                    o.snapshot(k)
                if meas:
                    res.append(o.measure())
            _BATCH_REF[j] = (res, [o.spins(0), o.spins(1)])
    return _BATCH_REF


def _check_batch(b, ref, ctx):
    for j, job in enumerate(_batch_jobs()):
        res, spins = ref[j]
        for k, want in enumerate(res):
            _same_obs(b.result(j, k), want, f"{ctx} job {j} meas {k}")
        for r in (0, 1):
            assert np.array_equal(b.spins(j, r), spins[r]), (ctx, j, r)


@pytest.mark.parametrize("flags,seed", MODES, ids=MODE_IDS)
def test_batched_form_under_debug(ea_gpu, oracle_mod, debug, flags, seed):
    """The batched kernel with whole and split replicas (unit order permuted,
    split pairs kept together in front), in spans and as a captured graph
    replayed twice: against the oracle."""
    ref = _batch_reference(oracle_mod)
    debug(flags, seed)
    jobs = _batch_jobs()
    for split in (ea_gpu.Batch.SPLIT_NEVER, ea_gpu.Batch.SPLIT_ALWAYS):
        _say(f"batch split={split} mode={flags}/{seed}")
        b = ea_gpu.Batch(jobs, split=split)
        if split == ea_gpu.Batch.SPLIT_ALWAYS:
            assert [b.parts(j) for j in range(len(jobs))] == [2, 2, 1, 1, 1, 1]
        b.run(3)
        b.run()
        _check_batch(b, ref, f"split={split} spans")
        b.close()
    g = ea_gpu.Batch(jobs, split=ea_gpu.Batch.SPLIT_ALWAYS)
    g.capture()
    for rep in range(2):
        g.replay()
        _check_batch(g, ref, f"graph replay {rep}")
    g.close()


@pytest.mark.parametrize("flags,seed", [MODES[0], MODES[-1]], ids=[MODE_IDS[0], MODE_IDS[-1]])
def test_multispin_batch_under_debug(ea_gpu, debug, flags, seed):
    """The multispin-coded batch (one launch per half-step, its graph captured
    under the mode) equals the same batch in the default mode: every
    sample's spins and every counter."""
    def run():
        m = ea_gpu.Msc(16, 64, 0.5, 0.8, seed=5, n_slots=1)
        m.snapshot(0)
        m.sweep(70)
        out = m.measure(), [m.spins(b, r) for b in (0, 31, 63) for r in (0, 1)]
        m.close()
        return out

    base_obs, base_spins = run()
    debug(flags, seed)
    obs, spins = run()
    for a, b in zip(spins, base_spins):
        assert np.array_equal(a, b)
    assert len(obs) == len(base_obs)
    for k, (a, b) in enumerate(zip(obs, base_obs)):
        _same_obs(a, b, f"msc sample {k}")


def test_serving_form_under_debug(ea_gpu, oracle_mod, debug):
    """The serving form with every debug flag: LDS-resident jobs in batched
    launches and a streamed L = 72 job in slab launches, each against the
    oracle."""
    from paper_1411_5512_amd.workloads import Job
    debug(R | ROT | POI, 99)
    jobs = [
        Job(72, 0.5, 0.8, seed=61, sample=0, n_sweeps=6, meas_t=[0, 2, 6], tw=[2]),
        Job(16, 0.3, 0.7, seed=62, sample=1, n_sweeps=40, meas_t=[5, 40], tw=[5]),
        Job(32, 0.5, 1.0, seed=63, sample=0, n_sweeps=12, meas_t=[12], tw=[]),
        Job(48, 0.2, 0.6, seed=64, sample=0, n_sweeps=5, meas_t=[1, 5], tw=[1]),
    ]
    srv = ea_gpu.Server(hbm_budget=1 << 27, max_resident=4, epoch_site_sweeps=32 ** 3 * 4)
    ids = [srv.submit(j) for j in jobs]
    n = 0
    while srv.step():
        n += 1
        assert n < 10000
    for jid, job in zip(ids, jobs):
        _say(f"served job L={job.L} sweeps={job.n_sweeps}")
        o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample, n_slots=len(job.tw))
        res, t = [], 0
        for te, slots, meas in job.events():
            if te > t:
                o.sweep(te - t)
                t = te
            for k in slots:
                o.snapshot(k)
            if meas:
                res.append(o.measure())
        for k, want in enumerate(res):
            _same_obs(srv.result(jid, k), want, f"served L={job.L} meas {k}")
