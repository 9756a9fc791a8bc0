"""Active-region size evolution (oracle, test infrastructure only).

Section 4.2.1: the size of an active region can follow
  i)   a linear growing phase,
  ii)  a linear decaying phase, or
  iii) a growing and decaying phase shaped as an asymmetric Gaussian
       (after Murakozy et al. 2014),
with sizes in millionths of the solar hemisphere (MSH); 10000 MSH is 1% of
the visible hemisphere.  The paper prints the parameters of its example (peak
10000 MSH, FWHM 10 days, asymmetry factor 0.09; linear rate 400 MSH/day) but
not the formulas, so the readings below are this implementation's:

* time t = phase x rotation period (days);
* linear growth: A(t) = A0 + r (t - t0) for t >= t0, A0 before;
* linear decay:  A(t) = max(0, A0 - r (t - t0)) for t >= t0, A0 before;
* asymmetric Gaussian: A(t) = A0 exp(-(t - t0)^2 / (2 w(t)^2)) with a width
  that grows through the event, w(t) = sigma (1 + a (t - t0)),
  sigma = FWHM / (2 sqrt(2 ln 2)) (a > 0: fast growth, slow decay), and
  A = 0 where w(t) <= 0;
* size to cap: an area of A MSH covers the fraction f = A 1e-6 of the
  hemisphere, a spherical cap with 1 - cos(alpha) = f, so the region radius
  sin(alpha) = sqrt(f (2 - f)); A <= 0 means no region at that time.

The region list of each phase is then the static list with these radii
(regions of zero size dropped), integrated as in Algorithm 5.
"""
from __future__ import annotations

import math

import numpy as np

NONE, LINEAR_GROWTH, LINEAR_DECAY, ASYM_GAUSS = 0, 1, 2, 3


def size_msh(mode: int, t_days, t0_days: float, size0_msh: float, rate_msh_day: float = 0.0,
             fwhm_days: float = 1.0, asym_per_day: float = 0.0):
    """Region size A(t) in MSH for the evolution law ``mode``."""
    t = np.asarray(t_days, dtype=np.float64)
    d = t - t0_days
    if mode == NONE:
        return np.full(t.shape, float(size0_msh))
    if mode == LINEAR_GROWTH:
        return np.where(d >= 0.0, size0_msh + rate_msh_day * d, size0_msh)
    if mode == LINEAR_DECAY:
        return np.where(d >= 0.0, np.maximum(0.0, size0_msh - rate_msh_day * d), size0_msh)
    if mode == ASYM_GAUSS:
        sigma = fwhm_days / (2.0 * math.sqrt(2.0 * math.log(2.0)))
        w = sigma * (1.0 + asym_per_day * d)
        with np.errstate(divide="ignore", invalid="ignore"):
            a = size0_msh * np.exp(-(d * d) / (2.0 * w * w))
        return np.where(w > 0.0, a, 0.0)
    raise ValueError(f"unknown evolution mode {mode}")


def cap_radius(size_msh_):
    """sin(alpha) of the cap covering size_msh millionths of the hemisphere
    (1 - cos alpha = f), 0 for non-positive sizes."""
    f = np.asarray(size_msh_, dtype=np.float64) * 1e-6
    f = np.clip(f, 0.0, 1.0)
    return np.sqrt(f * (2.0 - f))


def regions_at(regions, laws, phase: float, prot_days: float):
    """Region list at one phase: each region keeps its type, position and
    contrast and takes the radius of its law's size at t = phase x PROT;
    regions of zero size are left out.  ``laws`` holds, per region, a dict of
    size_msh's keyword arguments (mode, t0_days, size0_msh, ...)."""
    t = phase * prot_days
    out = []
    for reg, law in zip(regions, laws):
        a = float(size_msh(law["mode"], t, law["t0_days"], law["size0_msh"], law.get("rate_msh_day", 0.0),
                           law.get("fwhm_days", 1.0), law.get("asym_per_day", 0.0)))
        if a <= 0.0:
            continue
        rho = float(cap_radius(a))
        out.append(type(reg)(reg.type, reg.lat_deg, reg.lon_deg, rho, reg.contrast))
    return out
