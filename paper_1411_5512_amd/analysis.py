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
    # a fit may probe parameters where the form is undefined (xi <= 0): NaN there
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
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


# ---------------------------------------------------------------------------
# The paper's fitted-exponent analysis (Sec. IV): a multifit of eq. 4 over all
# waiting times, the growth exponent z of the coherence length, the
# equilibrium exponent x of the autocorrelation (eq. 8) and the collapse of
# C(t, t_w) with xi(t_w + t) / xi(t_w).  Host-side, on measured series.

def multifit_c4(r, curves, r_min: float = 3.0, errors=None, p0=(0.5, 1.5), n_sigma: float | None = None,
                alpha_range=(-0.5, 3.0), beta_range=(0.5, 4.0)):
    """Fit eq. 4, C4(r, t_w) = A(t_w) r^-alpha exp(-(r / xi(t_w))^beta), to
    several waiting times at once: alpha and beta shared by all curves, the
    amplitude and xi one per curve (Sec. IV).  `curves` is [n_tw][len(r)];
    only points with r >= r_min and C4 > 0 enter; `errors` (same shape)
    weights them, and with n_sigma each curve is cut, as for the integral
    estimator, before the first distance where it is below n_sigma errors.
    alpha and beta are kept inside the given ranges.  Returns dict(alpha,
    beta, xi[n_tw], amp[n_tw], cost)."""
    from scipy import optimize

    r = np.asarray(r, dtype=np.float64)
    c = np.atleast_2d(np.asarray(curves, dtype=np.float64))
    n = c.shape[0]
    e = np.ones_like(c) if errors is None else np.atleast_2d(np.asarray(errors, dtype=np.float64))
    masks = []
    for i in range(n):
        m = (r >= r_min) & (c[i] > 0) & (e[i] > 0)
        if n_sigma is not None and errors is not None:
            below = np.nonzero(c[i] <= n_sigma * e[i])[0]
            if below.size:
                m &= np.arange(len(r)) < below[0]
        masks.append(m)
    # start: xi from the integral estimator of each curve, amplitude from its first point
    xi0, a0 = [], []
    for i in range(n):
        m = masks[i]
        if m.sum() < 2:
            raise ValueError(f"curve {i} has fewer than two usable points")
        xi0.append(max(xi_k(np.r_[0.0, r[m]], np.r_[c[i][m][0], c[i][m]], 1), r[m][0] / 2))
        a0.append(c[i][m][0] * r[m][0] ** p0[0])

    def resid(v):
        alpha, beta = v[0], v[1]
        out = []
        for i in range(n):
            m = masks[i]
            model = np.exp(v[2 + n + i]) * r[m] ** (-alpha) * np.exp(-(r[m] / np.exp(v[2 + i])) ** beta)
            out.append((c[i][m] - model) / e[i][m])
        return np.concatenate(out)

    x0 = np.r_[p0[0], p0[1], np.log(xi0), np.log(a0)]
    lo = np.r_[alpha_range[0], beta_range[0], np.full(n, np.log(1e-2)), np.full(n, -50.0)]
    hi = np.r_[alpha_range[1], beta_range[1], np.full(n, np.log(1e6)), np.full(n, 50.0)]
    res = optimize.least_squares(resid, np.clip(x0, lo + 1e-9, hi - 1e-9), bounds=(lo, hi),
                                 x_scale="jac", max_nfev=20000)
    v = res.x
    # statistical errors from the curvature of the cost: cov = (J^T J)^-1 for
    # residuals weighted by true errors; unweighted, scaled by the residual
    # variance.  xi is fitted as log xi, so sigma_xi = xi sigma_log_xi.
    J = res.jac
    n_pts, n_par = J.shape
    cov = np.linalg.pinv(J.T @ J)
    if errors is None:
        cov *= 2.0 * res.cost / max(n_pts - n_par, 1)
    sig = np.sqrt(np.clip(np.diag(cov), 0.0, None))
    xi = np.exp(v[2:2 + n])
    return {"alpha": float(v[0]), "beta": float(v[1]), "xi": xi,
            "amp": np.exp(v[2 + n:]), "cost": float(res.cost),
            "alpha_err": float(sig[0]), "beta_err": float(sig[1]), "xi_err": xi * sig[2:2 + n]}


def multifit_error(r_axis, axis_curves, r_all, all_curves, axis_errors=None, all_errors=None,
                   r_min: float = 3.0, **kw):
    """The error estimate of Sec. IV: the eq. 4 multifit over the points at
    integer distances (along the lattice axes, from ``Obs.c4``) and over
    every distance r >= r_min (shell averages, from the full-vector shells);
    the error of alpha, beta and each xi is the difference of the two results
    plus both fits' statistical errors.  Returns dict(axis, all_r, alpha_err,
    beta_err, xi_err)."""
    a = multifit_c4(r_axis, axis_curves, r_min=r_min, errors=axis_errors, **kw)
    b = multifit_c4(r_all, all_curves, r_min=r_min, errors=all_errors, **kw)
    return {"axis": a, "all_r": b,
            "alpha_err": abs(a["alpha"] - b["alpha"]) + a["alpha_err"] + b["alpha_err"],
            "beta_err": abs(a["beta"] - b["beta"]) + a["beta_err"] + b["beta_err"],
            "xi_err": np.abs(a["xi"] - b["xi"]) + a["xi_err"] + b["xi_err"]}


def fit_growth(tw, xi, const: bool = True):
    """Power-law growth of the coherence length, xi(t_w) = a t_w^(1/z) (+ c,
    the constant the paper adds to absorb the early bend).  Returns
    dict(z, a, c)."""
    from scipy import optimize

    tw = np.asarray(tw, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    # start from the log-log slope of the last decade
    sl = np.polyfit(np.log(tw), np.log(xi), 1)[0]
    z0 = 1.0 / max(sl, 1e-3)
    a0 = xi[-1] / tw[-1] ** (1.0 / z0)
    if const:
        f = lambda t, a, inv_z, c: a * t ** inv_z + c
        p, _ = optimize.curve_fit(f, tw, xi, p0=(a0, 1.0 / z0, 0.0), maxfev=50000)
        return {"z": float(1.0 / p[1]), "a": float(p[0]), "c": float(p[2])}
    f = lambda t, a, inv_z: a * t ** inv_z
    p, _ = optimize.curve_fit(f, tw, xi, p0=(a0, 1.0 / z0), maxfev=50000)
    return {"z": float(1.0 / p[1]), "a": float(p[0]), "c": 0.0}


def fit_log_growth(tw, xi):
    """Logarithmic growth, xi(t_w) = a log(t_w / t0)^zt (the alternative the
    paper tries at the transition).  Returns dict(zt, t0, a)."""
    from scipy import optimize

    tw = np.asarray(tw, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)

    def f(t, a, log_t0, zt):
        return a * np.maximum(np.log(t) - log_t0, 1e-12) ** zt

    log_t0 = min(np.log(tw[0]) - 1.0, 0.0)
    p, _ = optimize.curve_fit(f, tw, xi, p0=(xi[-1] / (np.log(tw[-1]) - log_t0), log_t0, 1.0),
                              bounds=([0.0, -50.0, 0.01], [np.inf, np.log(tw[0]) - 1e-6, 50.0]), maxfev=50000)
    return {"zt": float(p[2]), "t0": float(np.exp(p[1])), "a": float(p[0])}


def fit_x(t, C, t_lo: float = 100.0, t_hi: float | None = None, tw: float | None = None):
    """Equilibrium exponent of eq. 8, C_eq(t) ~ t^-x: least-squares slope of
    log C against log t over t in [t_lo, t_hi] (default t_hi = t_w / 1000,
    the paper's smallest window).  Returns x."""
    t = np.asarray(t, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    if t_hi is None:
        if tw is None:
            raise ValueError("give t_hi or tw")
        t_hi = tw / 1000.0
    m = (t >= t_lo) & (t <= t_hi) & (C > 0)
    if m.sum() < 2:
        raise ValueError(f"fewer than two points in t in [{t_lo}, {t_hi}]")
    return float(-np.polyfit(np.log(t[m]), np.log(C[m]), 1)[0])


def collapse_spread(x, curves, xi_of):
    """Quality of the collapse C(t, t_w) / t^-x against xi(t_w + t) / xi(t_w)
    (Sec. IV, multiplicative decomposition): `curves` is a list of (t_w, t[],
    C[]); `xi_of` maps times to xi.  Each curve is put on the abscissa
    u = xi(t_w + t) / xi(t_w) - 1 and the spread is the mean squared
    difference of log(C t^x) between curves where their u ranges overlap
    (lower is better)."""
    pts = []
    for tw, t, C in curves:
        t = np.asarray(t, dtype=np.float64)
        C = np.asarray(C, dtype=np.float64)
        m = (t > 0) & (C > 0)
        u = np.asarray(xi_of(tw + t[m]), dtype=np.float64) / float(xi_of(np.array([tw]))[0]) - 1.0
        y = np.log(C[m]) + x * np.log(t[m])
        o = np.argsort(u)
        pts.append((u[o], y[o]))
    total, count = 0.0, 0
    for i in range(len(pts)):
        for j in range(i + 1, len(pts)):
            ui, yi = pts[i]
            uj, yj = pts[j]
            lo, hi = max(ui[0], uj[0]), min(ui[-1], uj[-1])
            if hi <= lo:
                continue
            grid = np.linspace(lo, hi, 32)
            d = np.interp(grid, ui, yi) - np.interp(grid, uj, yj)
            total += float(np.sum(d * d))
            count += grid.size
    return total / count if count else float("inf")


def best_collapse_x(curves, xi_of, x_range=(0.0, 0.1), n: int = 201):
    """The x that minimises `collapse_spread` on a grid over x_range."""
    xs = np.linspace(x_range[0], x_range[1], n)
    s = [collapse_spread(x, curves, xi_of) for x in xs]
    return float(xs[int(np.argmin(s))])


def fit_peak(p, z, offset: bool = True):
    """The transition estimate of Sec. IV: a Gaussian a exp(-(p - p_c)^2 /
    (2 w^2)) (+ b) fitted to the peak of the growth exponent z(p).  Returns
    dict(p_c, width, amp, offset)."""
    from scipy import optimize

    p = np.asarray(p, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    i = int(np.argmax(z))
    base = float(np.min(z)) if offset else 0.0
    w0 = max((p.max() - p.min()) / 6.0, 1e-3)
    if offset:
        f = lambda x, a, pc, w, b: a * np.exp(-(x - pc) ** 2 / (2 * w * w)) + b
        q, _ = optimize.curve_fit(f, p, z, p0=(z[i] - base, p[i], w0, base), maxfev=50000)
        return {"p_c": float(q[1]), "width": float(abs(q[2])), "amp": float(q[0]), "offset": float(q[3])}
    f = lambda x, a, pc, w: a * np.exp(-(x - pc) ** 2 / (2 * w * w))
    q, _ = optimize.curve_fit(f, p, z, p0=(z[i], p[i], w0), maxfev=50000)
    return {"p_c": float(q[1]), "width": float(abs(q[2])), "amp": float(q[0]), "offset": 0.0}
