"""Scaling analysis of the structure factor (host side, numpy).

Eq. (1) of the paper states the self-similar evolution near a non-thermal
fixed point, S(t, k) = (t/t_ref)^alpha f_s((t/t_ref)^beta k), separately in an
infrared and an ultraviolet window of momenta; in the infrared, alpha = d beta
keeps the momentum integral of S conserved (Sec. 2.1, Fig. 2).

``fit_scaling`` finds the exponents that collapse a series of spectra onto the
reference spectrum: every S(t, .) is rescaled by the trial exponents,
interpolated in log k onto the reference momenta inside the window, and the
squared log-deviation from S(t_ref, .) is summed.  For a fixed beta the best
alpha is a closed-form least-squares slope, so the search runs over beta alone
(a scan followed by a golden-section refinement).  ``bootstrap_scaling``
resamples the Wigner runs to give standard errors.
"""
import math

import numpy as np

_GOLDEN = (math.sqrt(5.0) - 1.0) / 2.0


def _log_interp(logk_src, logs_src, logk_dst):
    """log S at logk_dst by linear interpolation in (log k, log S); NaN outside."""
    out = np.interp(logk_dst, logk_src, logs_src, left=np.nan, right=np.nan)
    return out


def _collapse_terms(beta, tau, logk, logs, ref, mask_ref):
    """Per time: the log-deviation vectors (before the alpha term) on the reference
    momenta kept by the window and covered by the rescaled spectrum."""
    lk_ref = logk[mask_ref]
    terms = []
    for i, ti in enumerate(tau):
        if ti == 0.0:
            continue
        # S(t, k) = e^{alpha tau} f(e^{beta tau} k): at reference momentum kappa,
        # f(kappa) = e^{-alpha tau} S(t, kappa e^{-beta tau})
        src = _log_interp(logk, logs[i], lk_ref - beta * ti)
        dev = src - logs[ref][mask_ref]
        ok = np.isfinite(dev)
        if ok.any():
            terms.append((ti, dev[ok]))
    return terms


def _residual_and_alpha(beta, tau, logk, logs, ref, mask_ref, alpha_per_beta):
    terms = _collapse_terms(beta, tau, logk, logs, ref, mask_ref)
    if not terms:
        return math.inf, math.nan, 0
    if alpha_per_beta is not None:
        alpha = alpha_per_beta * beta
    else:
        # minimise sum (dev - alpha tau)^2 over alpha
        num = sum(ti * d.sum() for ti, d in terms)
        den = sum(ti * ti * d.size for ti, d in terms)
        alpha = num / den
    res = sum(float(np.sum((d - alpha * ti) ** 2)) for ti, d in terms)
    npts = sum(d.size for _, d in terms)
    return res / npts, alpha, npts


def fit_scaling(t, k, S, t_ref, k_window, beta_range=(-1.0, 1.0), alpha_per_beta=None, scan=201, tol=1e-10):
    """Exponents (alpha, beta) of Eq. (1) from spectra S[i, b] at times t[i] and
    momenta k[b] (k > 0, increasing), reference time t_ref (one of t), momentum
    window k_window = (k_lo, k_hi) of the reference spectrum.  alpha_per_beta:
    None fits alpha freely; a number d imposes alpha = d beta (the infrared
    relation in d dimensions).  Returns a dict with alpha, beta, the mean
    squared log-deviation of the collapse and the number of points used."""
    t = np.asarray(t, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    if S.shape != (t.size, k.size):
        raise ValueError("S must have shape (len(t), len(k))")
    if np.any(k <= 0) or np.any(np.diff(k) <= 0):
        raise ValueError("k must be positive and increasing")
    if np.any(S <= 0):
        raise ValueError("S must be positive (log-log collapse)")
    hits = np.nonzero(np.isclose(t, t_ref, rtol=0, atol=1e-12 * max(1.0, abs(t_ref))))[0]
    if hits.size != 1:
        raise ValueError("t_ref must be one of the times")
    ref = int(hits[0])
    tau = np.log(t / t_ref)
    logk = np.log(k)
    logs = np.log(S)
    mask_ref = (k >= k_window[0]) & (k <= k_window[1])
    if mask_ref.sum() < 2:
        raise ValueError("the momentum window holds fewer than two momenta")

    def f(beta):
        return _residual_and_alpha(beta, tau, logk, logs, ref, mask_ref, alpha_per_beta)[0]

    lo, hi = beta_range
    grid = np.linspace(lo, hi, scan)
    vals = np.array([f(b) for b in grid])
    j = int(np.argmin(vals))
    a, b = grid[max(j - 1, 0)], grid[min(j + 1, scan - 1)]
    # golden-section refinement inside the bracketing scan cells
    c, d = b - _GOLDEN * (b - a), a + _GOLDEN * (b - a)
    fc, fd = f(c), f(d)
    while b - a > tol:
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - _GOLDEN * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + _GOLDEN * (b - a)
            fd = f(d)
    beta = 0.5 * (a + b)
    res, alpha, npts = _residual_and_alpha(beta, tau, logk, logs, ref, mask_ref, alpha_per_beta)
    return {"alpha": float(alpha), "beta": float(beta), "residual": float(res), "points": int(npts)}


def bootstrap_scaling(t, k, S_samples, t_ref, k_window, n_boot=100, seed=0, **kw):
    """Fit on the sample mean of S_samples[i, s, b] (time, Wigner run, momentum)
    and on n_boot resamplings of the runs (with replacement); returns the fit
    of the mean with the bootstrap standard errors alpha_se, beta_se."""
    S_samples = np.asarray(S_samples, dtype=np.float64)
    nt, ns, nk = S_samples.shape
    best = fit_scaling(t, k, S_samples.mean(axis=1), t_ref, k_window, **kw)
    rng = np.random.default_rng(seed)
    al, be = [], []
    for _ in range(n_boot):
        pick = rng.integers(0, ns, size=ns)
        r = fit_scaling(t, k, S_samples[:, pick, :].mean(axis=1), t_ref, k_window, **kw)
        al.append(r["alpha"])
        be.append(r["beta"])
    best["alpha_se"] = float(np.std(al, ddof=1)) if n_boot > 1 else math.nan
    best["beta_se"] = float(np.std(be, ddof=1)) if n_boot > 1 else math.nan
    return best
