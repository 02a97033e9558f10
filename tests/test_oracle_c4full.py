"""Pins of the oracle's full-vector four-point correlation (eq. 3 over every
displacement, summed by minimum-image distance shells): an independent FFT
autocorrelation of q, and identities that any correct implementation obeys."""
import numpy as np
import pytest


def _shells_by_fft(q, L, n_shells):
    """sum_x q(x) q(x + r) for every r by the Wiener-Khinchin theorem, binned
    by minimum-image |r|^2."""
    field = q.reshape(L, L, L).astype(np.float64)  # [z][y][x], s = x + L (y + L z)
    f = np.fft.fftn(field)
    corr = np.rint(np.fft.ifftn(np.conj(f) * f).real).astype(np.int64)
    m = np.minimum(np.arange(L), L - np.arange(L)) ** 2
    k = m[:, None, None] + m[None, :, None] + m[None, None, :]
    out = np.zeros(n_shells, dtype=np.int64)
    sel = k < n_shells
    np.add.at(out, k[sel], corr[sel])
    return out


@pytest.mark.parametrize("L,p,T,sweeps", [(8, 0.5, 0.8, 7), (12, 0.3, 1.1, 4), (6, 0.0, 0.5, 3)])
def test_shells_equal_fft_autocorrelation(oracle_mod, L, p, T, sweeps):
    o = oracle_mod.Sim(L, p, T, seed=9, sample=1)
    o.sweep(sweeps)
    q = o.spins(0).astype(np.int64) * o.spins(1)
    n = 3 * (L // 2) ** 2 + 1  # every shell
    got = o.c4_shells(n)
    assert np.array_equal(got, _shells_by_fft(q, L, n))


def test_shell_identities(oracle_mod):
    L = 10
    o = oracle_mod.Sim(L, 0.5, 0.9, seed=4)
    o.sweep(6)
    N = L ** 3
    q = o.spins(0).astype(np.int64) * o.spins(1)
    full = o.c4_shells(3 * (L // 2) ** 2 + 1)
    assert full[0] == N                          # r = 0: q^2 = 1 at every site
    assert full.sum() == int(q.sum()) ** 2       # sum over all r of the autocorrelation = Q^2
    obs = o.measure()
    # the six unit displacements are the axis correlation at rho = 1, both directions
    assert full[1] == 2 * int(obs.c4[:, 1].sum())
    # the default range stops at |r| = L/2 and agrees with the full list there
    part = o.c4_shells()
    assert len(part) == (L // 2) ** 2 + 1 and np.array_equal(part, full[:len(part)])
    # shells that no displacement reaches stay zero (7 is not a sum of three squares)
    assert full[7] == 0 and full[15] == 0


def test_equal_replicas_give_shell_counts(oracle_mod):
    """q = 1 everywhere: every displacement contributes N, so shell k holds N
    times the number of lattice vectors of minimum-image length^2 k."""
    L = 8
    o = oracle_mod.Sim(L, 0.5, 0.8, seed=2)
    o.set_spins(1, o.spins(0))
    got = o.c4_shells(3 * (L // 2) ** 2 + 1)
    m = np.minimum(np.arange(L), L - np.arange(L)) ** 2
    k = (m[:, None, None] + m[None, :, None] + m[None, None, :]).ravel()
    counts = np.bincount(k, minlength=len(got))
    assert np.array_equal(got, L ** 3 * counts)
