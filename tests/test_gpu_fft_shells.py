"""The FFT route of the full-vector C4 shells (eq. 3 over every displacement,
summed by minimum-image shell; an fp64 3D DFT of q, its squared modulus, the
inverse DFT, each sum rounded to the nearest integer and binned) against the
oracle at small L, against the direct route and numpy's FFT of the GPU's own
q at full size, in all three forms, and on the two spectra that put all of
|F|^2 on one wave vector, where its rounding is stressed most (q = 1
everywhere: k = 0; a checkerboard q: k = (pi, pi, pi)).  Tolerance 0:
integer sums."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture
def ea_route(ea_gpu):
    """The library, with the shell route put back to automatic afterwards."""
    yield ea_gpu
    ea_gpu.set_shell_route(ea_gpu.SHELLS_AUTO)


def _routes(ea, fn):
    """fn() under the FFT route, then under the direct route."""
    ea.set_shell_route(ea.SHELLS_FFT)
    a = fn()
    ea.set_shell_route(ea.SHELLS_DIRECT)
    b = fn()
    ea.set_shell_route(ea.SHELLS_AUTO)
    return a, b


def _min_image_k(L):
    m = np.minimum(np.arange(L), L - np.arange(L)) ** 2
    return m[:, None, None] + m[None, :, None] + m[None, None, :]


def _numpy_shells(q, L, n_shells):
    f = np.fft.fftn(q.reshape(L, L, L).astype(np.float64))
    corr = np.rint(np.fft.ifftn(np.conj(f) * f).real).astype(np.int64)
    k = _min_image_k(L)
    out = np.zeros(n_shells, dtype=np.int64)
    sel = k < n_shells
    np.add.at(out, k[sel], corr[sel])
    return out


@pytest.mark.parametrize("L,rw", [(8, 0), (16, 0), (16, 1), (24, 0), (24, 1), (32, 0), (32, 2)])
def test_fft_shells_match_oracle(ea_route, oracle_mod, L, rw):
    """The sizes the route takes up to 32 (2^k, and 24 = 3 x 8 with its
    radix-3 stage), in several packings: equal to the oracle's shells (every displacement, the |r| <= L/2
    default, and truncations to 5 and 1 shells), and to the direct route."""
    ea = ea_route
    g = ea.Sim(L, 0.5, 0.8, seed=8, sample=2, words_per_row=rw)
    o = oracle_mod.Sim(L, 0.5, 0.8, seed=8, sample=2)
    g.sweep(11)
    o.sweep(11)
    _say(f"fft shells L={L} rw={g.words_per_row}")
    for n in (3 * (L // 2) ** 2 + 1, None, 5, 1):
        want = o.c4_shells(n)
        fft, direct = _routes(ea, lambda: g.c4_shells(n))
        assert np.array_equal(fft, want), (L, n)
        assert np.array_equal(direct, want), (L, n)


@pytest.mark.parametrize("L", [48, 64, 96, 128, 192, 256])
def test_fft_shells_equal_direct_full_size(ea_route, L):
    """At full size (no oracle): the FFT route equals the direct route and
    numpy's FFT of the GPU's own q, over every displacement and |r| <= L/2;
    shell 0 = N, the sum of all shells = Q^2."""
    ea = ea_route
    g = ea.Sim(L, 0.3, 0.7, seed=2)
    g.sweep(30)
    _say(f"fft shells full size L={L}")
    n_all = 3 * (L // 2) ** 2 + 1
    fft, direct = _routes(ea, lambda: g.c4_shells(n_all))
    assert np.array_equal(fft, direct)
    q = g.spins(0).astype(np.int64) * g.spins(1)
    assert np.array_equal(fft, _numpy_shells(q, L, n_all))
    assert fft[0] == L ** 3 and int(fft.sum()) == int(q.sum()) ** 2
    ea.set_shell_route(ea.SHELLS_FFT)
    assert np.array_equal(g.c4_shells(), fft[:(L // 2) ** 2 + 1])


@pytest.mark.parametrize("L", [8, 24, 64, 96, 256])
def test_fft_shells_extreme_spectra(ea_route, L):
    """q = 1 everywhere (replica 1 a copy of replica 0): shell k = N times the
    number of displacements in it.  q = (-1)^(x+y+z): every product
    q(x) q(x + r) is (-1)^(rx+ry+rz), so shell k = N times the signed count.
    Both put all of |F|^2 (N^2) on one wave vector."""
    ea = ea_route
    g = ea.Sim(L, 0.5, 0.9, seed=4)
    g.sweep(3)
    N = L ** 3
    n_all = 3 * (L // 2) ** 2 + 1
    k = _min_image_k(L).ravel()
    a = np.arange(L)
    parity = ((a[:, None, None] + a[None, :, None] + a[None, None, :]) & 1).ravel()
    S0 = g.spins(0)
    for name, S1, sign in (("q = 1", S0, np.ones(N, dtype=np.int64)),
                           ("checkerboard q", (S0 * (1 - 2 * parity)).astype(np.int8), 1 - 2 * parity)):
        g.set_spins(1, S1)
        _say(f"fft shells L={L}: {name}")
        want = N * np.bincount(k, weights=sign, minlength=n_all).astype(np.int64)
        fft, direct = _routes(ea, lambda: g.c4_shells(n_all))
        assert np.array_equal(fft, want), name
        assert np.array_equal(direct, want), name


def test_fft_shells_batch_and_msc(ea_route, oracle_mod):
    """The batched form's published configurations (L = 16, 24, 32) and
    multispin samples (L = 32, two word sets) by the FFT route against the
    oracle's shells of the same runs; an L = 48 job and a multispin L = 64
    batch, FFT against direct."""
    ea = ea_route
    from paper_1411_5512_amd.workloads import Job
    jobs = [Job(16, 0.5, 0.8, seed=51, sample=0, n_sweeps=9, meas_t=[4, 9], tw=[]),
            Job(32, 0.25, 0.7, seed=52, sample=3, n_sweeps=7, meas_t=[7], tw=[7]),
            Job(24, 0.4, 0.9, seed=53, sample=1, n_sweeps=5, meas_t=[5], tw=[]),
            Job(48, 0.3, 0.6, seed=54, sample=2, n_sweeps=4, meas_t=[4], tw=[])]
    b = ea.Batch(jobs)
    b.run()
    for j, job in enumerate(jobs):
        if job.L > 32:  # beyond the oracle's brute-force shells in test time
            _say(f"fft shells batch job {j} L={job.L}: FFT against direct")
            fft, direct = _routes(ea, lambda: b.c4_shells(j, 0, 3 * (job.L // 2) ** 2 + 1))
            assert np.array_equal(fft, direct) and fft[0] == job.L ** 3, j
            continue
        o = oracle_mod.Sim(job.L, job.p, job.T, seed=job.seed, sample=job.sample)
        t = 0
        n_all = 3 * (job.L // 2) ** 2 + 1
        for kk, tm in enumerate(job.meas_t):
            o.sweep(tm - t)
            t = tm
            _say(f"fft shells batch job {j} L={job.L} t={tm}")
            fft, direct = _routes(ea, lambda: b.c4_shells(j, kk, n_all))
            want = o.c4_shells(n_all)
            assert np.array_equal(fft, want), (j, kk)
            assert np.array_equal(direct, want), (j, kk)
    L, B = 32, 64
    m = ea.Msc(L, B, 0.5, 0.8, seed=6, sample0=1, shared=3)
    om = oracle_mod.shared_batch(L, 0.5, 0.8, seed=6, sample0=1, n_samples=B, shared_id=3)
    m.sweep(5)
    n_all = 3 * (L // 2) ** 2 + 1
    for bi in (0, 37, B - 1):
        om[bi].sweep(5)
        _say(f"fft shells msc L={L} sample {bi}")
        ea.set_shell_route(ea.SHELLS_FFT)
        assert np.array_equal(m.c4_shells(bi, n_all), om[bi].c4_shells(n_all)), bi
    m64 = ea.Msc(64, 32, 0.3, 0.7, seed=7)
    m64.sweep(4)
    for bi in (0, 31):
        _say(f"fft shells msc L=64 sample {bi}")
        fft, direct = _routes(ea, lambda: m64.c4_shells(bi, 3 * 32 ** 2 + 1))
        assert np.array_equal(fft, direct), bi
