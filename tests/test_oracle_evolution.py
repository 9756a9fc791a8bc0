"""Pins of the active-region size evolution (section 4.2.1): each law against
its closed form, the asymmetric Gaussian's half-maximum points solved by
hand, the MSH-to-cap conversion against the sphere's cap area, and the
library's own size function (host code, no device) against the oracle."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import disk as D
from oracle import evolution as E
from oracle import spectrum as S

L = pytest.importorskip("paper_2301_04259_amd", reason="libsoap.so not built")

# the paper's example (section 4.2.1): peak 10000 MSH, FWHM 10 days,
# asymmetry 0.09; linear rate 400 MSH/day from 10000 MSH
PEAK, FWHM, ASYM, RATE = 10000.0, 10.0, 0.09, 400.0


def test_linear_laws_closed_form():
    t = np.array([-3.0, 0.0, 1.0, 7.5, 30.0])
    g = E.size_msh(E.LINEAR_GROWTH, t, 0.0, PEAK, RATE)
    assert np.array_equal(g, [PEAK, PEAK, PEAK + RATE, PEAK + 7.5 * RATE, PEAK + 30 * RATE])
    d = E.size_msh(E.LINEAR_DECAY, t, 0.0, PEAK, RATE)
    assert np.array_equal(d, [PEAK, PEAK, PEAK - RATE, PEAK - 7.5 * RATE, 0.0])  # gone after 25 days


def test_symmetric_gaussian_half_maximum_at_half_fwhm():
    h = E.size_msh(E.ASYM_GAUSS, np.array([-FWHM / 2, 0.0, FWHM / 2]), 0.0, PEAK, fwhm_days=FWHM, asym_per_day=0.0)
    assert h[1] == PEAK
    assert np.allclose(h[[0, 2]], PEAK / 2, rtol=1e-14)


def test_asymmetric_gaussian_half_maximum_points():
    # A = A0/2 where d^2 / (2 w^2) = ln 2, w = sigma (1 + a d), i.e.
    # |d| = k (1 + a d) with k = sigma sqrt(2 ln 2) = FWHM / 2:
    # after the peak d = k / (1 - a k), before it d = -k / (1 + a k)
    k = FWHM / 2
    d_after = k / (1 - ASYM * k)
    d_before = -k / (1 + ASYM * k)
    h = E.size_msh(E.ASYM_GAUSS, np.array([d_before, d_after]), 0.0, PEAK, fwhm_days=FWHM, asym_per_day=ASYM)
    assert np.allclose(h, PEAK / 2, rtol=1e-13)
    assert d_after > -d_before  # fast growth, slow decay
    # the width reaches zero at d = -1/a: no region before that
    assert E.size_msh(E.ASYM_GAUSS, np.array([-1.0 / ASYM - 1e-9]), 0.0, PEAK, fwhm_days=FWHM,
                      asym_per_day=ASYM)[0] == 0.0


def test_msh_to_cap_radius():
    # a cap of angular radius alpha covers 1 - cos(alpha) of the hemisphere
    # (area 2 pi (1 - cos alpha) of 2 pi)
    for msh in (10.0, 1000.0, 10000.0, 250000.0):
        rho = float(E.cap_radius(msh))
        alpha = math.asin(rho)
        assert (1 - math.cos(alpha)) == pytest.approx(msh * 1e-6, rel=1e-12)
    # 1% of the visible hemisphere: sin(alpha) = sqrt(0.0199)
    assert float(E.cap_radius(10000.0)) == pytest.approx(math.sqrt(0.0199), rel=1e-15)
    assert float(E.cap_radius(0.0)) == 0.0


def test_cap_covers_its_area_on_the_disk():
    # a cap at the disk centre projects to a disk of radius sin(alpha): its
    # cells' summed area approaches pi sin^2(alpha)
    n = 400
    rho = float(E.cap_radius(20000.0))
    _, _, x, y, mu = D.disk_cells(n)
    reg = [W.Region(W.SPOT, 0.0, 0.0, rho, 1.0)]
    own = D.owner_map(x, y, mu, reg, 0.0, 90.0)
    area = (own >= 0).sum() * D.cell_area(n)
    assert area == pytest.approx(math.pi * rho * rho, rel=2e-2)


def test_no_evolution_equals_static_region():
    st = W.make_tiny(41, n_grid=14, n_pix=200, n_mu=3, n_phases=3)
    reg = [W.Region(W.SPOT, 10.0, 30.0, float(E.cap_radius(30000.0)), 0.5)]
    laws = [dict(mode=E.NONE, t0_days=0.0, size0_msh=30000.0)]
    for ph in st.phases:
        a = S.integrated(st, ph, S.TOT, E.regions_at(reg, laws, ph, 25.05))
        b = S.integrated(st, ph, S.TOT, reg)
        assert np.array_equal(a, b)


def test_decayed_region_is_gone():
    st = W.make_tiny(42, n_grid=14, n_pix=200, n_mu=3, n_phases=2)
    reg = [W.Region(W.SPOT, 0.0, 0.0, 0.3, 0.5)]
    laws = [dict(mode=E.LINEAR_DECAY, t0_days=0.0, size0_msh=PEAK, rate_msh_day=RATE)]
    assert E.regions_at(reg, laws, 2.0, 25.05) == []  # t = 50 days
    assert np.array_equal(S.integrated(st, 2.0, S.TOT, E.regions_at(reg, laws, 2.0, 25.05)), S.quiet(st))


@pytest.mark.parametrize("mode", [E.NONE, E.LINEAR_GROWTH, E.LINEAR_DECAY, E.ASYM_GAUSS])
def test_library_size_function_matches_oracle(mode):
    law = dict(mode=mode, t0_days=3.0, size0_msh=PEAK, rate_msh_day=RATE, fwhm_days=FWHM, asym_per_day=ASYM)
    for t in np.linspace(-20.0, 40.0, 61):
        want = float(E.size_msh(mode, t, 3.0, PEAK, RATE, FWHM, ASYM))
        got = L.soap_evolution_size(law, t)
        assert got == pytest.approx(want, rel=1e-14, abs=1e-9), (mode, t)
    assert math.isnan(L.soap_evolution_size(dict(mode=9, t0_days=0.0, size0_msh=1.0), 0.0))
    assert math.isnan(L.soap_evolution_size(dict(mode=E.NONE, t0_days=0.0, size0_msh=-1.0), 0.0))
