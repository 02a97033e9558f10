"""The host-side estimators: shell bookkeeping and the integral estimators
of the coherence length (eqs. 5, 6) against closed forms."""
import numpy as np
import pytest

from paper_1411_5512_amd import analysis as an


def test_shell_counts():
    for L in (4, 8, 10):
        c = an.shell_counts(L)
        assert c.sum() == L ** 3
        assert c[0] == 1 and c[1] == 6 and c[2] == 12 and c[3] == 8
        assert c[7] == 0  # no sum of three squares
    # L = 4: the image at distance 2 along an axis is single (min(2, 2) = 2)
    assert an.shell_counts(4)[4] == 3


def test_c4_of_shells_and_axes():
    L = 8
    n = L ** 3
    cnt = an.shell_counts(L, 17)
    r, c = an.c4_of_shells(n * cnt, L)  # C4 = 1 on every displacement
    assert np.allclose(c, 1.0) and r[0] == 0.0 and np.isclose(r[1], 1.0)
    ax = np.tile(np.arange(5) * n, (3, 1))
    r, c = an.c4_of_axes(ax, L)
    assert np.allclose(c, np.arange(5)) and np.array_equal(r, np.arange(5))


def _exp_integrals(xi, R, k):
    """Closed form of int_0^R r^k exp(-r/xi) dr for k = 1, 2."""
    u = R / xi
    if k == 1:
        return xi ** 2 * (1 - np.exp(-u) * (1 + u))
    return 2 * xi ** 3 * (1 - np.exp(-u) * (1 + u + u * u / 2))


def test_integral_estimator_closed_form():
    xi, R = 3.0, 40.0
    r = np.linspace(0, R, 20001)
    c = np.exp(-r / xi)
    assert an.integral(r, c, 1) == pytest.approx(_exp_integrals(xi, R, 1), rel=1e-7)
    want = _exp_integrals(xi, R, 2) / _exp_integrals(xi, R, 1)
    assert an.xi_k(r, c, 1) == pytest.approx(want, rel=1e-7)
    # cut-off: integrals stop at r_cut
    assert an.xi_k(r, c, 1, r_cut=10.0) == pytest.approx(
        _exp_integrals(xi, 10.0, 2) / _exp_integrals(xi, 10.0, 1), rel=1e-6)


def test_samples_cutoff_and_tail():
    rng = np.random.default_rng(0)
    r = np.arange(0, 33, dtype=np.float64)
    amp, alpha, xi, beta = 1.0, 0.5, 4.0, 1.5
    truth = np.where(r > 0, an.c4_form(np.maximum(r, 1e-9), amp, alpha, xi, beta), 1.0)
    noise = 0.002
    curves = truth + rng.normal(0, noise, size=(400, r.size))
    est, r_cut, params = an.xi_k_samples(r, curves, k=1)
    # the cut sits where the signal is no longer 3 standard errors above zero
    se = noise / np.sqrt(400)
    assert truth[int(r_cut)] >= 3 * se * 0.5 and r_cut < 32
    assert params is not None and params[2] == pytest.approx(xi, rel=0.1)
    # against the noiseless integrals to L/2 (trapezoid on the integer grid)
    want = an.xi_k(r, truth, 1)
    assert est == pytest.approx(want, rel=0.03)
    # without the tail the estimate is biased low but stays close for a cut far out
    est_no_tail, _, _ = an.xi_k_samples(r, curves, k=1, tail=False)
    assert est_no_tail <= est * 1.001
