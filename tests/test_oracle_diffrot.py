"""Pins of differential rotation in the oracle (section 3.4).

* The reading omega_1 = DIFF_ROT x omega_0 reproduces the paper's solar
  numbers (the printed "DIFF_ROT x PROT" does not).
* The disk-integrated line broadening: for a weak narrow line, the second
  velocity moment of the quiet spectrum's absorption equals the line's own
  variance plus the intensity-weighted mean of v^2 over the visible
  hemisphere, computed here by quadrature in stellar coordinates (latitude,
  longitude: v = omega(theta) R cos(theta) sin(phi) sin i) rather than on the
  projected cell grid.
* Brute force per cell equals the grouped form; the sampled-pixel form
  equals the full spectrum; DIFF_ROT = 0 is solid-body rotation bit for bit.
* A region at latitude theta comes back to its place after 1 / (1 + DIFF_ROT
  sin^2 theta) equatorial rotations; an equatorial one after exactly one.
"""
import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from oracle import disk as D
from oracle import spectrum as S

C_KMS = 299792.458


def test_reading_reproduces_solar_rates(golden):
    g = golden["differential_rotation"]
    w0 = 360.0 / g["prot_days"]
    assert w0 == pytest.approx(g["omega0_deg_day"], abs=g["tolerance_deg_day"])
    assert g["diff_rot"] * w0 == pytest.approx(g["omega1_deg_day"], abs=g["tolerance_deg_day"])
    assert abs(g["diff_rot"] * g["prot_days"] - g["omega1_deg_day"]) > 1.0  # the printed form is off


def _quadrature_v2(vsini, incl_deg, alpha, u1, u2, n=400):
    """<v^2> over the visible hemisphere weighted by I(mu) mu dA, by midpoint
    quadrature in latitude and longitude."""
    inc = math.radians(incl_deg)
    th = (np.arange(n) + 0.5) / n * math.pi - math.pi / 2
    ph = (np.arange(2 * n) + 0.5) / (2 * n) * 2 * math.pi - math.pi
    T, P = np.meshgrid(th, ph, indexing="ij")
    mu = math.sin(inc) * np.cos(T) * np.cos(P) + math.cos(inc) * np.sin(T)
    vis = mu > 0
    inten = 1 - u1 * (1 - mu) - u2 * (1 - mu) ** 2
    v = vsini * (1 + alpha * np.sin(T) ** 2) * np.cos(T) * np.sin(P)
    wgt = np.where(vis, inten * mu * np.cos(T), 0.0)
    return float((wgt * v * v).sum() / wgt.sum())


@pytest.mark.parametrize("incl,alpha", [(90.0, -0.18), (60.0, -0.18), (50.0, 0.3)])
def test_broadening_second_moment_matches_spherical_quadrature(incl, alpha):
    dln = 2e-7  # 60 m/s per pixel
    n_pix = 1200
    ln0 = math.log(5000.0)
    lam = np.exp(ln0 + dln * np.arange(n_pix))
    lc = lam[n_pix // 2]
    sig = lc * 0.5 / C_KMS
    depth = 1e-3
    spec = (1 - depth * np.exp(-0.5 * ((lam - lc) / sig) ** 2))[None, :]
    st = W.StarInputs(n_grid=220, vsini_kms=5.0, incl_deg=incl, ld_u1=0.4, ld_u2=0.25, ln_lambda0=ln0,
                      dln_lambda=dln, n_pix=n_pix, mu_bins=np.array([1.0]), spectra=[spec, None, None])
    st.diff_rot = alpha
    q = S.quiet(st)
    a = q.max() - q
    vel = (np.log(lam) - math.log(lc)) * C_KMS  # velocity per pixel (first order in dln)
    var_line = (a * vel * vel).sum() / a.sum()
    # the line itself: second moment of its own absorption on the same grid
    a0 = spec[0].max() - spec[0]
    var0 = (a0 * vel * vel).sum() / a0.sum()
    want = _quadrature_v2(5.0, incl, alpha, 0.4, 0.25)
    assert var_line - var0 == pytest.approx(want, rel=3e-3)
    # and the solid-body value differs well beyond that
    assert abs(_quadrature_v2(5.0, incl, 0.0, 0.4, 0.25) - want) > 0.02 * want


@pytest.mark.parametrize("seed,incl", [(61, 90.0), (62, 55.0)])
def test_bruteforce_equals_grouped_with_differential_rotation(seed, incl):
    st = W.make_tiny(seed, n_grid=12, n_pix=220, n_mu=3, contrast_mode=seed % 2, incl_deg=incl, vsini_kms=6.0)
    st.diff_rot = -0.3
    for eff in (S.TOT, S.FLUX, S.BCONV):
        for ph in st.phases[:2]:
            a = S.integrated_bruteforce(st, ph, eff)
            b = S.integrated(st, ph, eff)
            assert np.max(np.abs(a - b) / np.abs(a)) < 1e-13


@pytest.mark.parametrize("alpha", [0.0, -0.18])
def test_sampled_pixels_equal_full_spectrum(alpha):
    st = W.make_tiny(63, n_grid=30, n_pix=900, n_mu=4, contrast_mode=W.CONTRAST_PLANCK, incl_deg=70.0)
    st.diff_rot = alpha
    pix = np.array([0, 1, 2, 5, 100, 333, 450, 451, 700, 897, 898, 899])
    for eff in (S.TOT, S.FLUX, S.BCONV):
        ph = st.phases[1]
        full = S.integrated(st, ph, eff)
        got = S.integrated_pixels(st, ph, pix, eff)
        assert np.max(np.abs(got - full[pix]) / np.abs(full[pix])) < 1e-13


def test_zero_differential_rotation_is_solid_body_bit_for_bit():
    st = W.make_tiny(64, n_grid=20, n_pix=300, n_mu=3, incl_deg=75.0)
    dr = dataclasses.replace(st)
    dr.diff_rot = 0.0
    for ph in st.phases[:2]:
        assert np.array_equal(S.integrated(dr, ph, S.TOT), S.integrated(st, ph, S.TOT))
    # and a non-zero value changes the spectrum
    dr.diff_rot = -0.18
    assert not np.allclose(S.integrated(dr, st.phases[0], S.TOT), S.integrated(st, st.phases[0], S.TOT), rtol=1e-9)


@pytest.mark.parametrize("lat", [0.0, 35.0, -70.0])
def test_region_returns_after_its_own_rotation_period(lat):
    alpha = -0.18
    sl = math.sin(math.radians(lat))
    period = 1.0 / (1.0 + alpha * sl * sl)
    a = D.region_centre(lat, 40.0, 0.0, 65.0, alpha)
    b = D.region_centre(lat, 40.0, period, 65.0, alpha)
    assert np.allclose(a, b, atol=1e-12)
    if lat != 0.0:
        c = D.region_centre(lat, 40.0, 1.0, 65.0, alpha)  # one equatorial rotation: it lags
        assert not np.allclose(a, c, atol=1e-3)
