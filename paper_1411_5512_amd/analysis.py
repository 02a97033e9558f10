"""Host-side analysis of the measured integer series: the four-point
correlation as a function of distance and the integral estimators of the
coherence length (eqs. 5 and 6 of the paper, after Belletti et al.).

Everything here works on the integers the library returns (axis sums
``Obs.c4`` or full-vector shell sums ``Sim.c4_shells``); nothing runs on the
GPU and nothing here is on the simulation path.
"""
from __future__ import annotations

import numpy as np


def shell_counts(L: int, n_shells: int | None = None) -> np.ndarray:
    """Number of displacements r in Z_L^3 whose minimum-image squared length
    is k, for k = 0 .. n_shells - 1 (default: every shell)."""
    n = 3 * (L // 2) ** 2 + 1 if n_shells is None else int(n_shells)
    m = np.minimum(np.arange(L), L - np.arange(L)) ** 2
    k = (m[:, None, None] + m[None, :, None] + m[None, None, :]).ravel()
    return np.bincount(k[k < n], minlength=n)[:n]


def c4_of_shells(shell_sums, L: int):
    """(r, C4(r)) from full-vector shell sums: the average of C4 over all
    displacements of length r = sqrt(k), for every shell that has one."""
    s = np.asarray(shell_sums, dtype=np.float64)
    cnt = shell_counts(L, len(s))
    keep = cnt > 0
    k = np.nonzero(keep)[0]
    return np.sqrt(k), s[keep] / (cnt[keep] * float(L) ** 3)


def c4_of_axes(c4_sums, L: int):
    """(r, C4(r)) at integer distances r = 0 .. L/2 along the lattice axes,
    averaged over the three axes, from ``Obs.c4`` ([3][L/2 + 1] sums)."""
    c = np.asarray(c4_sums, dtype=np.float64).reshape(3, -1)
    return np.arange(c.shape[1], dtype=np.float64), c.mean(axis=0) / float(L) ** 3


def integral(r, c4, k: int, r_cut: float | None = None) -> float:
    """I_k = integral of r^k C4(r) dr from 0 to r_cut (default: the last
    point), by the trapezoid rule over the given points (eq. 5)."""
    r = np.asarray(r, dtype=np.float64)
    c = np.asarray(c4, dtype=np.float64)
    if r_cut is not None:
        m = r <= r_cut
        r, c = r[m], c[m]
    f = r ** k * c
    return float(np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(r)))


def xi_k(r, c4, k: int = 1, r_cut: float | None = None) -> float:
    """Integral estimator xi_k = I_{k+1} / I_k (eq. 6)."""
    return integral(r, c4, k + 1, r_cut) / integral(r, c4, k, r_cut)


def c4_form(r, amp, alpha, xi, beta):
    """The functional form of eq. 4 with a stretched exponential g:
    amp r^-alpha exp(-(r/xi)^beta)."""
    r = np.asarray(r, dtype=np.float64)
    return amp * r ** (-alpha) * np.exp(-(r / xi) ** beta)


def xi_k_samples(r, curves, k: int = 1, n_sigma: float = 3.0, tail: bool = True,
                 r_max: float | None = None):
    """xi_k from C4(r) curves of many disorder samples (rows of `curves`).

    The integrals run over the sample mean up to the first distance where it
    falls below n_sigma times its standard error; beyond that, if `tail`,
    they are completed with eq. 4 fitted to the points before the cut (r >= 1)
    and integrated up to r_max (default: the last distance given).  Returns
    (xi_k, r_cut, fit parameters or None)."""
    from scipy import integrate, optimize

    r = np.asarray(r, dtype=np.float64)
    c = np.asarray(curves, dtype=np.float64)
    mean = c.mean(axis=0)
    err = c.std(axis=0, ddof=1) / np.sqrt(c.shape[0]) if c.shape[0] > 1 else np.zeros_like(mean)
    below = np.nonzero(mean < n_sigma * err)[0]
    i_cut = int(below[0]) if below.size else len(r)
    r_cut = r[i_cut - 1]
    r_end = r[-1] if r_max is None else float(r_max)
    ik = integral(r[:i_cut], mean[:i_cut], k)
    ik1 = integral(r[:i_cut], mean[:i_cut], k + 1)
    params = None
    if tail and r_end > r_cut:
        m = (r >= 1.0) & (r <= r_cut)
        if m.sum() >= 4:
            p0 = (max(mean[m][0], 1e-12), 0.5, max(r_cut / 2, 1.0), 1.5)
            import warnings
            try:
                with warnings.catch_warnings():
                    warnings.simplefilter("ignore", optimize.OptimizeWarning)
                    params, _ = optimize.curve_fit(c4_form, r[m], mean[m], p0=p0, maxfev=20000)
            except RuntimeError:
                params = None
        if params is not None:
            ik += integrate.quad(lambda x: x ** k * c4_form(x, *params), r_cut, r_end)[0]
            ik1 += integrate.quad(lambda x: x ** (k + 1) * c4_form(x, *params), r_cut, r_end)[0]
    return ik1 / ik, r_cut, params
