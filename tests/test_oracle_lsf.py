"""Pins of the resolution lowering (the last step of Algorithms 2 and 5):
the line-spread function's width against the resolving power R = lambda /
FWHM, measured on an unresolved line; variance additivity and flux
conservation, which hold exactly for a discrete convolution; linear
spectra and constants preserved; the end-value hold."""
import math

import numpy as np
import pytest

from oracle import lsf as O

C_KMS = 299792.458


def test_kernel_shape():
    dln = 1.0 / (3.0 * 115000.0)
    w = O.kernel(115000.0, dln)
    s = O.sigma_pixels(115000.0, dln)
    assert s == pytest.approx(3.0 / (2.0 * math.sqrt(2.0 * math.log(2.0))), rel=1e-14)
    assert len(w) == 2 * math.ceil(4 * s) + 1 == 13
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.array_equal(w, w[::-1])
    k = np.arange(len(w)) - (len(w) - 1) // 2
    # a Gaussian sampled at whole pixels and cut at 4 sigma keeps its variance
    # to about 1e-3 (the cut tails)
    assert (w * k * k).sum() == pytest.approx(s * s, rel=2e-3)


def test_unresolved_line_takes_the_instrument_width():
    # 0.2 km/s line on a grid of 0.03 km/s per pixel, lowered to R = 50000:
    # the output FWHM is lambda / R widened in quadrature by the line itself
    dln = 1e-7
    n = 20000
    ln0 = math.log(6000.0)
    lam = np.exp(ln0 + dln * np.arange(n))
    lc = lam[n // 2]
    sig_line = lc * 0.2 / C_KMS
    f = 1.0 - 0.5 * np.exp(-0.5 * ((lam - lc) / sig_line) ** 2)
    out = O.lower_resolution(f, 50000.0, dln)
    a = 1.0 - out
    half = a.max() / 2
    above = np.nonzero(a >= half)[0]
    i0, i1 = above[0], above[-1]
    left = (i0 - 1) + (half - a[i0 - 1]) / (a[i0] - a[i0 - 1])
    right = i1 + (a[i1] - half) / (a[i1] - a[i1 + 1])
    fwhm_a = lc * (math.exp((right - left) * dln) - 1.0)
    fwhm_line = 2.0 * math.sqrt(2.0 * math.log(2.0)) * sig_line
    want = math.hypot(lc / 50000.0, fwhm_line)
    assert fwhm_a == pytest.approx(want, rel=2e-3)


def test_variance_adds_and_flux_is_conserved():
    rng = np.random.default_rng(3)
    n = 3000
    dln = 2.5e-6
    m = np.arange(n)
    c = 1500.3
    line = 0.7 * np.exp(-0.5 * ((m - c) / 4.2) ** 2)
    out = O.lower_resolution(1.0 - line, 115000.0, dln)
    a = 1.0 - out
    w = O.kernel(115000.0, dln)
    k = np.arange(len(w)) - (len(w) - 1) // 2
    mom = lambda x: ((x * m).sum() / x.sum(), (x * (m - (x * m).sum() / x.sum()) ** 2).sum() / x.sum())  # noqa: E731
    c_in, v_in = mom(line)
    c_out, v_out = mom(a)
    assert a.sum() == pytest.approx(line.sum(), rel=1e-13)
    assert c_out == pytest.approx(c_in, abs=1e-9)
    assert v_out == pytest.approx(v_in + (w * k * k).sum(), rel=1e-11)
    # a random spectrum keeps its interior pixel sum up to the edge terms
    g = rng.uniform(0.2, 1.0, n)
    g[:20] = g[20]
    g[-20:] = g[-21]
    assert O.lower_resolution(g, 115000.0, dln).sum() == pytest.approx(g.sum(), rel=1e-13)


def test_linear_and_constant_spectra_unchanged():
    n = 500
    dln = 2.9e-6
    lin = 1.0 + 1e-4 * np.arange(n)
    out = O.lower_resolution(lin, 115000.0, dln)
    assert np.allclose(out[10:-10], lin[10:-10], rtol=0, atol=1e-14)
    const = np.full((2, n), 0.83)
    assert np.allclose(O.lower_resolution(const, 115000.0, dln), 0.83, rtol=0, atol=1e-15)
    # end values held: a step at the left edge is seen as a constant beyond it
    step = np.ones(n)
    step[0] = 0.5
    o = O.lower_resolution(step, 115000.0, dln)
    w = O.kernel(115000.0, dln)
    kmax = (len(w) - 1) // 2
    assert o[0] == pytest.approx(1.0 - 0.5 * w[kmax:].sum(), rel=1e-14)
