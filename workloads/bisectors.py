"""Depth-dependent line bisectors per mu bin, injected into local spectra.

Section 4.3.2 gives the local spectra of each mu bin the line asymmetry of
convection at that centre-to-limb angle: every point of a normalised
spectrum is Doppler shifted by a velocity that depends on its normalised
depth, v(d, mu), so that each line's bisector at depth d sits at v(d, mu).
The paper's bisector shapes come from solar observations (quiet Sun: cubic
fits for mu >= 0.5 and straight lines below; active regions: a straight line
below depth 0.5 and a fifth-order polynomial above, with convection fully
inhibited), which are not available here.  This module stands in for them
with synthetic shapes of the same kind:

* quiet photosphere: a C shape, most blueshifted at depth 0.58,
  v_q(d, mu) = cb(mu) (1 - k (d - 0.58)^2), cb(mu) the bin's convective
  blueshift (negative) and k = 1.5, so the bisector curves back towards the
  red at the continuum and in the line core;
* active regions: a straight line through zero at depth 0.58 (convection
  inhibited at every mu), v_a(d) = s (d - 0.58) with a small slope s.

The injection itself: normalised depth d_m = 1 - S_m at each pixel; the
pixel moves to m + atanh(v(d_m) / c) / dln (the Doppler shift of Eq. 6 on the
log grid), and the moved samples are resampled onto the grid by linear
interpolation.  Continuum points (d = 0) move by v(0); a bisector function
that is zero leaves the spectrum unchanged.  This is input preparation, not
part of the synthesis: the kernels and the oracle receive the injected
spectra like any other local spectra.
"""
from __future__ import annotations

import numpy as np

C_MS = 299792458.0
DEPTH_MAX_SHIFT = 0.58
K_CURVE = 1.5


def quiet_bisector_ms(depth, cb_ms):
    """v_q(d) = cb (1 - K (d - 0.58)^2), cb < 0 for a blueshift."""
    d = np.asarray(depth, dtype=np.float64)
    return cb_ms * (1.0 - K_CURVE * (d - DEPTH_MAX_SHIFT) ** 2)


def active_bisector_ms(depth, slope_ms=60.0):
    """v_a(d) = slope (d - 0.58): no shift at depth 0.58."""
    d = np.asarray(depth, dtype=np.float64)
    return slope_ms * (d - DEPTH_MAX_SHIFT)


def inject(spectrum, dln, v_of_depth):
    """Shift every point of a normalised spectrum (continuum 1) by the
    velocity its normalised depth calls for, then resample onto the grid."""
    s = np.asarray(spectrum, dtype=np.float64)
    d = np.clip(1.0 - s, 0.0, 1.0)
    v = np.asarray(v_of_depth(d), dtype=np.float64)
    pos = np.arange(len(s), dtype=np.float64) + np.arctanh(v / C_MS) / dln
    if np.any(np.diff(pos) <= 0.0):
        raise ValueError("bisector too steep for the grid: moved samples overtake each other")
    return np.interp(np.arange(len(s), dtype=np.float64), pos, s)


def measure_bisector_ms(spectrum, ln0, dln, centre_a, levels):
    """Bisector of the line nearest centre_a: for each flux level F, the
    midpoint (as a velocity relative to centre_a) of the two points where the
    linearly interpolated profile crosses F on either side of the minimum."""
    s = np.asarray(spectrum, dtype=np.float64)
    pc = (np.log(centre_a) - ln0) / dln
    lo = max(0, int(pc) - 200)
    hi = min(len(s), int(pc) + 200)
    seg = s[lo:hi]
    k = lo + int(np.argmin(seg))
    out = []
    for f in levels:
        i = k
        while i > 0 and s[i] < f:
            i -= 1
        left = i + (f - s[i]) / (s[i + 1] - s[i])
        j = k
        while j < len(s) - 1 and s[j] < f:
            j += 1
        right = (j - 1) + (f - s[j - 1]) / (s[j] - s[j - 1])
        mid = 0.5 * (left + right)
        out.append(np.tanh((mid - pc) * dln) * C_MS)
    return np.array(out)


def inject_star(star, cb_ms_per_bin, active_slope_ms=60.0):
    """A copy of ``star``'s spectra with bisectors injected per mu bin: the
    quiet rows get v_q with their bin's blueshift, the spot and facula rows
    the active line.  The spectra should carry no convective shift of their
    own (their lines symmetric), as after the paper's bisector removal."""
    out = []
    for t, arr in enumerate(star.spectra):
        if arr is None:
            out.append(None)
            continue
        rows = []
        for b in range(arr.shape[0]):
            if t == 0:
                f = lambda d, cb=cb_ms_per_bin[b]: quiet_bisector_ms(d, cb)  # noqa: E731
            else:
                f = lambda d: active_bisector_ms(d, active_slope_ms)  # noqa: E731
            rows.append(inject(arr[b], star.dln_lambda, f))
        out.append(np.stack(rows).astype(arr.dtype))
    return out
