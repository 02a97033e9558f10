"""Full-vector C4 (eq. 3 over every displacement, summed by minimum-image
distance shells) of the batched form's published configurations and of the
multispin-coded batch's samples, against the oracle's shells of the same
configuration (tolerance 0: integer sums)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_batch_shells_match_oracle(ea_gpu, oracle_mod):
    """Three jobs of different size, p and T; shells at each measurement
    (every displacement, and the |r| <= L/2 default) equal the oracle's at the
    same time."""
    from paper_1411_5512_amd.workloads import Job
    jobs = [Job(16, 0.5, 0.8, seed=41, sample=0, n_sweeps=20, meas_t=[0, 5, 20], tw=[5]),
            Job(24, 0.3, 0.6, seed=42, sample=1, n_sweeps=12, meas_t=[12], tw=[]),
            Job(32, 0.2, 1.1, seed=43, sample=0, n_sweeps=6, meas_t=[3, 6], tw=[3])]
    b = ea_gpu.Batch(jobs)
    b.run()
    for j, job in enumerate(jobs):
        o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample)
        t = 0
        for k, tm in enumerate(job.meas_t):
            o.sweep(tm - t)
            t = tm
            n_all = 3 * (job.L // 2) ** 2 + 1
            _say(f"batch shells job {j} L={job.L} t={tm}")
            want = o.c4_shells(n_all)
            assert np.array_equal(b.c4_shells(j, k, n_all), want), (j, k)
            assert np.array_equal(b.c4_shells(j, k), want[:(job.L // 2) ** 2 + 1]), (j, k)


def test_batch_shells_errors(ea_gpu):
    from paper_1411_5512_amd.workloads import Job
    b = ea_gpu.Batch([Job(16, 0.5, 0.8, seed=1, n_sweeps=10, meas_t=[4, 10])])
    b.run(5)
    b.c4_shells(0, 0, 5)
    with pytest.raises(ea_gpu.EAError):
        b.c4_shells(0, 1, 5)   # not reached
    with pytest.raises(ea_gpu.EAError):
        b.c4_shells(0, 2, 5)   # no such measurement
    with pytest.raises(ea_gpu.EAError):
        b.c4_shells(1, 0, 5)   # no such job
    with pytest.raises(ea_gpu.EAError):
        b.c4_shells(0, 0, 3 * 64 + 2)


@pytest.mark.parametrize("L,B", [(16, 32), (16, 8), (24, 64)])
def test_msc_shells_match_oracle(ea_gpu, oracle_mod, L, B):
    """Samples of a multispin batch (32 per word; 8 per word in four z-slabs;
    two word sets) against the shared-noise oracle's runs of the same
    samples."""
    m = ea_gpu.Msc(L, B, 0.5, 0.8, seed=5, sample0=3, shared=2)
    om = oracle_mod.shared_batch(L, 0.5, 0.8, seed=5, sample0=3, n_samples=B, shared_id=2)
    m.sweep(7)
    n_all = 3 * (L // 2) ** 2 + 1
    for bi in sorted({0, 1, B // 2 - 1, B - 1}):
        om[bi].sweep(7)
        _say(f"msc shells L={L} B={B} sample {bi}")
        assert np.array_equal(m.c4_shells(bi, n_all), om[bi].c4_shells(n_all)), bi
    with pytest.raises(ea_gpu.EAError):
        m.c4_shells(B, 5)


def test_multifit_error_on_a_multispin_batch(ea_gpu):
    """Sec. IV's error estimate end to end on GPU data (a pipeline check, not
    parity): a 32^3 multispin batch of 64 samples, C4 along the axes from the
    in-run measurement and over every distance from the shells, both
    multifitted over t_w = 20 .. 640; the errors come out finite and the
    exponents inside their fit ranges."""
    from paper_1411_5512_amd import analysis as an
    L, B = 32, 64
    m = ea_gpu.Msc(L, B, 0.5, 0.8, seed=9, sample0=0, shared=4)
    tws = [20, 80, 320, 640]
    r_axis = np.arange(L // 2 + 1, dtype=np.float64)
    n_sh = (L // 2) ** 2 + 1
    r_all, _ = an.c4_of_shells(np.ones(n_sh), L)
    axis, axis_e, allr, allr_e = [], [], [], []
    t = 0
    for tw in tws:
        m.sweep(tw - t)
        t = tw
        per_axis = np.array([o.c4.mean(axis=0) / L ** 3 for o in m.measure(autocorr=False)])
        per_all = np.array([an.c4_of_shells(m.c4_shells(b, n_sh), L)[1] for b in range(B)])
        axis.append(per_axis.mean(0))
        axis_e.append(per_axis.std(0, ddof=1) / np.sqrt(B))
        allr.append(per_all.mean(0))
        allr_e.append(per_all.std(0, ddof=1) / np.sqrt(B))
    res = an.multifit_error(r_axis, np.array(axis), r_all, np.array(allr), axis_errors=np.array(axis_e),
                            all_errors=np.array(allr_e), n_sigma=3.0)
    _say(f"axis: alpha={res['axis']['alpha']:.3f} beta={res['axis']['beta']:.3f} xi={res['axis']['xi']}; "
         f"all r: alpha={res['all_r']['alpha']:.3f} beta={res['all_r']['beta']:.3f}; "
         f"errors {res['alpha_err']:.3f} {res['beta_err']:.3f} {res['xi_err']}")
    assert np.isfinite(res["alpha_err"]) and np.isfinite(res["beta_err"]) and np.all(np.isfinite(res["xi_err"]))
    assert -0.5 <= res["axis"]["alpha"] <= 3.0 and 0.5 <= res["all_r"]["beta"] <= 4.0
