"""Pins of the oracle's per-pixel contrast (section 4.3.1 chromatic contrast,
section 4.3.3 facula limb brightening and the SED factors of Eqs. 12-14).

The Planck function is evaluated here from h, c and k_B (SI 2019 exact
values) in its textbook form 2 h c^2 / lambda^5 / (exp(h c / lambda k T) - 1),
not through the oracle's ratio of expm1 terms, and the facula temperature
excess from the paper's printed coefficients at each bin's own mu.  The two
forms agree to rounding (1e-12); a slip in the temperature, the bin's mu or
the radiation constant's digits moves them by far more.
"""
import numpy as np
import pytest

import workloads as W
from oracle import spectrum as S

H = 6.62607015e-34
C = 299792458.0
KB = 1.380649e-23


def planck(lam_a, t):
    lam = np.asarray(lam_a, dtype=np.float64) * 1e-10
    return 2.0 * H * C * C / lam**5 / np.expm1(H * C / (lam * KB * t))


def _star20(golden, teff=5778.0, dts=663.0):
    st = W.make_tiny(31, n_grid=12, n_pix=300, n_mu=20, contrast_mode=W.CONTRAST_PLANCK)
    st.mu_bins = np.linspace(1.0, 0.1, 20)
    st.teff_k = teff
    st.dt_spot_k = dts
    st.dt_fac_coef = tuple(golden["facula_limb_brightening"]["coef"])
    return st


def test_facula_contrast_every_bin_follows_dtf_at_its_mu(golden):
    st = _star20(golden)
    a0, a1, a2 = golden["facula_limb_brightening"]["coef"]
    lam = S.wavelengths(st.ln_lambda0, st.dln_lambda, st.n_pix)
    dts = []
    for b, mu in enumerate(st.mu_bins):
        dt = a0 + a1 * mu + a2 * mu * mu
        dts.append(dt)
        want = planck(lam, st.teff_k + dt) / planck(lam, st.teff_k)
        got = S.contrast_array(st, W.FACULA, b, lam)
        assert np.max(np.abs(got / want - 1.0)) < 1e-12, b
    # the bins really differ: disk centre 34.1 K, mu = 0.1 212.039 K
    assert dts[0] == pytest.approx(34.1, abs=1e-9)
    assert dts[-1] == pytest.approx(250.9 - 40.77 + 1.909, abs=1e-9)
    c0 = S.contrast_array(st, W.FACULA, 0, lam)
    c19 = S.contrast_array(st, W.FACULA, 19, lam)
    assert np.all(c19 > c0) and np.all(c0 > 1.0)


def test_facula_contrast_uses_the_bin_mu_not_a_neighbour(golden):
    # a plausible slip (every bin at bin 0's mu, or at the next bin's) moves
    # the contrast by far more than rounding
    st = _star20(golden)
    lam = S.wavelengths(st.ln_lambda0, st.dln_lambda, st.n_pix)
    a0, a1, a2 = golden["facula_limb_brightening"]["coef"]
    for b in (3, 11, 17):
        got = S.contrast_array(st, W.FACULA, b, lam)
        for other in (0, b + 1):
            mu = st.mu_bins[other]
            wrong = planck(lam, st.teff_k + a0 + a1 * mu + a2 * mu * mu) / planck(lam, st.teff_k)
            assert np.min(np.abs(got / wrong - 1.0)) > 1e-4


def test_spot_contrast_is_planck_ratio_at_the_spot_temperature(golden):
    st = _star20(golden, teff=5200.0, dts=850.0)
    lam = S.wavelengths(st.ln_lambda0, st.dln_lambda, st.n_pix)
    want = planck(lam, 5200.0 - 850.0) / planck(lam, 5200.0)
    for b in (0, 7, 19):
        got = S.contrast_array(st, W.SPOT, b, lam)
        assert np.max(np.abs(got / want - 1.0)) < 1e-12


def test_scalar_mode_has_no_array():
    st = W.make_tiny(32, n_grid=8, n_pix=120, n_mu=2)
    lam = S.wavelengths(st.ln_lambda0, st.dln_lambda, st.n_pix)
    assert S.contrast_array(st, W.SPOT, 0, lam) is None


# ------------------------------------------------------------ array mode


def _array_star(seed=33, n=14, p=240, b=3):
    return W.make_tiny(seed, n_grid=n, n_pix=p, n_mu=b, contrast_mode=W.CONTRAST_ARRAY, n_phases=3)


def test_array_mode_returns_the_callers_rows():
    st = _array_star()
    lam = S.wavelengths(st.ln_lambda0, st.dln_lambda, st.n_pix)
    for t in (W.SPOT, W.FACULA):
        for b in range(st.n_mu):
            assert np.array_equal(S.contrast_array(st, t, b, lam), st.contrast[t][b])
    # every row differs from every other one
    rows = np.concatenate([st.contrast[1], st.contrast[2]])
    d = np.abs(rows[:, None, :] - rows[None, :, :]).max(axis=2)
    assert np.all(d[~np.eye(len(rows), dtype=bool)] > 1e-3)


@pytest.mark.parametrize("seed", [33, 34])
def test_array_mode_bruteforce_equals_grouped(seed):
    st = _array_star(seed, n=10, p=180)
    for eff in (S.TOT, S.FLUX, S.BCONV):
        for ph in st.phases[:2]:
            a = S.integrated_bruteforce(st, ph, eff)
            b = S.integrated(st, ph, eff)
            assert np.max(np.abs(a - b) / np.abs(a)) < 1e-13


def test_constant_arrays_equal_scalar_contrast():
    # a contrast that is the same number c at every pixel and bin multiplies
    # after the shift exactly as a scalar c multiplies before it
    st = _array_star(35)
    c = 0.62
    for t in (W.SPOT, W.FACULA):
        st.contrast[t] = np.full_like(st.contrast[t], c)
    sc = _array_star(35)
    sc.contrast_mode = W.CONTRAST_SCALAR
    sc.contrast = [None, None, None]
    regs = [W.Region(r.type, r.lat_deg, r.lon_deg, r.radius, c) for r in st.regions]
    for eff in (S.TOT, S.FLUX):
        for ph in st.phases:
            a = S.integrated(st, ph, eff, regs)
            b = S.integrated(sc, ph, eff, regs)
            assert np.max(np.abs(a - b) / np.abs(b)) < 1e-13


def test_one_row_perturbation_touches_only_its_cells():
    # raising one (type, bin) row by eps changes the total-effect spectrum by
    # eps x the summed shifted spectra of exactly the cells of that type and
    # bin: a wrong row or type index moves a different set of cells
    from oracle import disk as D

    st = _array_star(36, n=16, p=260, b=3)
    st.regions = [W.Region(W.FACULA, 10.0, 20.0, 0.5, 1.0), W.Region(W.SPOT, -5.0, 30.0, 0.3, 1.0)]
    ph = 0.05
    base = S.integrated(st, ph, S.TOT)
    lam = S.wavelengths(st.ln_lambda0, st.dln_lambda, st.n_pix)
    _, _, x, y, mu = D.disk_cells(st.n_grid)
    owner = D.owner_map(x, y, mu, st.regions, ph, st.incl_deg)
    bins = D.mu_bin(mu, st.mu_bins)
    inten = D.limb_darkening(mu, st.ld_u1, st.ld_u2)
    area = D.cell_area(st.n_grid)
    eps = 1e-3
    hit = 0
    for t in (W.SPOT, W.FACULA):
        for b in range(st.n_mu):
            sel = np.nonzero((owner >= 0) & (bins == b))[0]
            sel = [c for c in sel if st.regions[owner[c]].type == t]
            pert = _array_star(36, n=16, p=260, b=3)
            pert.regions = st.regions
            pert.contrast[t] = pert.contrast[t].copy()
            pert.contrast[t][b] += eps
            d = S.integrated(pert, ph, S.TOT) - base
            want = np.zeros(st.n_pix)
            for c in sel:
                v = D.los_velocity(x[c], st.vsini_kms)
                want += area * inten[c] * S.shift_spectrum(st.spectra[t][b], lam, v)
            want *= eps
            assert np.max(np.abs(d - want)) < 1e-12 * np.abs(base).max()
            hit += len(sel) > 0
    assert hit >= 3
