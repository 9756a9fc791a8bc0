"""Gaussian fit of a CCF (oracle, test infrastructure only).

Section 4.1: the RV is the mean of a Gaussian profile fitted to the CCF.  The
reading used here: unweighted least squares of

    g(v) = c0 - a * exp(-(v - mu)^2 / (2 sigma^2))

over every velocity point, solved with a library Levenberg-Marquardt
(scipy ``least_squares``, method "lm") to its tolerance floor.  Start:
c0 = max CCF, a = c0 - min CCF, mu = v at the minimum, sigma from the
half-depth width.  RV = mu, FWHM = 2 sqrt(2 ln 2) |sigma|.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import least_squares

FWHM_PER_SIGMA = 2.0 * np.sqrt(2.0 * np.log(2.0))


def gaussian(v, c0, a, mu, sigma):
    return c0 - a * np.exp(-((v - mu) ** 2) / (2.0 * sigma * sigma))


def initial_guess(v, y):
    v = np.asarray(v, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    c0 = float(np.max(y))
    k = int(np.argmin(y))
    a = c0 - float(y[k])
    half = c0 - 0.5 * a
    below = np.nonzero(y <= half)[0]
    width = float(v[below[-1]] - v[below[0]]) if len(below) > 1 else float(v[1] - v[0])
    sigma = max(width, float(v[1] - v[0])) / FWHM_PER_SIGMA
    return np.array([c0, a, float(v[k]), sigma])


def gauss_fit(v, y):
    """Returns dict(c0, a, mu, sigma, rv_kms, fwhm_kms, chi2)."""
    v = np.asarray(v, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    p0 = initial_guess(v, y)

    def res(p):
        return gaussian(v, *p) - y

    r = least_squares(res, p0, method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=20000)
    c0, a, mu, sigma = r.x
    return dict(
        c0=c0,
        a=a,
        mu=mu,
        sigma=abs(sigma),
        rv_kms=mu,
        fwhm_kms=FWHM_PER_SIGMA * abs(sigma),
        chi2=float(np.sum(res(r.x) ** 2)),
    )
