"""Pins of the bisector injection used to make mu-dependent local spectra
(section 4.3.2: each point of a spectrum shifted by a velocity that depends
on its normalised depth).  The injected line's bisector is measured back
from the profile and compared with the prescribed one."""
import numpy as np
import pytest

import workloads as W
from workloads import bisectors as BI

C_KMS = 299792.458


def _line(dln, n=4000, depth=0.8, sigma_kms=3.0, lam0=5000.0):
    ln0 = np.log(lam0)
    lam = np.exp(ln0 + dln * np.arange(n))
    lc = np.exp(ln0 + dln * (n // 2))
    sig = lc * sigma_kms / C_KMS
    return ln0, lc, 1.0 - depth * np.exp(-0.5 * ((lam - lc) / sig) ** 2)


def test_zero_bisector_is_identity():
    _, _, s = _line(2e-6, n=1500)
    assert np.array_equal(BI.inject(s, 2e-6, lambda d: np.zeros_like(d)), s)


def test_symmetric_line_has_vertical_bisector():
    dln = 2e-7
    ln0, lc, s = _line(dln)
    b = BI.measure_bisector_ms(s, ln0, dln, lc, np.linspace(0.25, 0.9, 14))
    # a Gaussian in lambda sampled uniformly in ln(lambda) leans by
    # (sigma / c) x sigma ~ 0.1 m/s at most
    assert np.max(np.abs(b)) < 0.1


@pytest.mark.parametrize("cb", [-340.0, -120.0])
def test_injected_quiet_bisector_is_measured_back(cb):
    # 60 m/s per pixel and a 3 km/s line: the linear resampling leaves the
    # measured bisector within 0.5 m/s of the prescribed curve
    dln = 2e-7
    ln0, lc, s = _line(dln)
    f = lambda d: BI.quiet_bisector_ms(d, cb)  # noqa: E731
    inj = BI.inject(s, dln, f)
    levels = np.linspace(0.25, 0.9, 14)
    got = BI.measure_bisector_ms(inj, ln0, dln, lc, levels)
    want = f(1.0 - levels)
    assert np.max(np.abs(got - want)) < 0.5
    # C shape: the most blueshifted point sits at depth 0.58
    fine = np.linspace(0.21, 0.95, 75)
    prof = BI.measure_bisector_ms(inj, ln0, dln, lc, fine)
    assert abs((1.0 - fine[np.argmin(prof)]) - 0.58) < 0.02


def test_injected_active_bisector_is_measured_back():
    dln = 2e-7
    ln0, lc, s = _line(dln, depth=0.9)
    inj = BI.inject(s, dln, BI.active_bisector_ms)
    levels = np.linspace(0.2, 0.9, 15)
    got = BI.measure_bisector_ms(inj, ln0, dln, lc, levels)
    assert np.max(np.abs(got - BI.active_bisector_ms(1.0 - levels))) < 0.5
    assert abs(BI.measure_bisector_ms(inj, ln0, dln, lc, [0.42])[0]) < 0.5  # no shift at depth 0.58


def test_continuum_unchanged_and_too_steep_rejected():
    _, _, s = _line(2e-6, n=1500, sigma_kms=2.0)
    inj = BI.inject(s, 2e-6, lambda d: BI.quiet_bisector_ms(d, -340.0))
    far = np.abs(np.arange(1500) - 750) > 200
    assert np.max(np.abs(inj[far] - 1.0)) < 1e-12
    with pytest.raises(ValueError, match="steep"):
        BI.inject(s, 2e-6, lambda d: 5e5 * d)


def test_bisector_star_rows_differ_per_bin():
    st = W.make_bisector_star(n_pix=3000, n_mu=6)
    q = st.spectra[W.QUIET].astype(np.float64)
    cb = W.stars.cb_law_ms(st.mu_bins)
    # the deepest line of the last bin (no blueshift): at normalised depth
    # 0.58 each bin's bisector sits cb_b from the last bin's; at 3 pixels per
    # resolution element the linear resampling blends the sample at depth
    # 0.58 with neighbours that moved less (the C shape peaks there), which
    # pulls the measured shift in by up to 10%
    k = int(np.argmin(q[-1]))
    assert 1.0 - q[-1, k] > 0.6
    lc = np.exp(st.ln_lambda0 + st.dln_lambda * k)
    v = np.array([BI.measure_bisector_ms(q[b], st.ln_lambda0, st.dln_lambda, lc, [0.42])[0]
                  for b in range(st.n_mu)])
    assert np.all(np.abs((v - v[-1]) - cb) <= 0.1 * np.abs(cb) + 5.0), (v - v[-1], cb)
    assert np.all(np.diff(v) > 0)  # blueshift weakens towards the limb
    assert not np.array_equal(q[0], q[1])
    # active rows share one bisector: identical across bins
    assert np.array_equal(st.spectra[W.SPOT][0], st.spectra[W.SPOT][3])
