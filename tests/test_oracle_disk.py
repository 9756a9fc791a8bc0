"""Pins of the oracle's disk geometry, interpolation and integration.

Each test checks the oracle against something other than itself: a closed
form, a brute-force evaluation, an invariant the mathematics fixes, or a
number the paper prints.
"""
import numpy as np
import pytest

import workloads as W
from oracle import disk as D
from oracle import spectrum as S


def _flat_star(n_grid, n_pix=64, n_mu=3, u1=0.4, u2=0.25, vsini=3.0):
    mu_b = np.linspace(1.0, 0.2, n_mu)
    ones = np.ones((n_mu, n_pix))
    return W.StarInputs(
        n_grid=n_grid, vsini_kms=vsini, incl_deg=90.0, ld_u1=u1, ld_u2=u2,
        ln_lambda0=np.log(5000.0), dln_lambda=3e-6, n_pix=n_pix, mu_bins=mu_b,
        spectra=[ones, ones.copy(), ones.copy()], precision=W.PREC_FP64,
    )


# ---------------------------------------------------------------- geometry


def test_cell_count_matches_quoted_visible_cells(golden):
    g = golden["cell_counts"]
    _, _, x, _, _ = D.disk_cells(g["n_grid"])
    assert abs(len(x) - g["visible_cells_approx"]) <= g["tolerance"]
    # lattice count of the unit disk: pi (N/2)^2 within the boundary term
    assert abs(len(x) - np.pi * (g["n_grid"] / 2) ** 2) < 4 * g["n_grid"]


def test_cell_centres_symmetric_and_inside():
    for n in (2, 3, 7, 100, 301):
        c = D.cell_centres(n)
        assert np.allclose(c, -c[::-1], atol=1e-15)
        assert c.min() > -1 and c.max() < 1
        assert np.allclose(np.diff(c), 2.0 / n)


def test_limb_darkening_integral_closed_form():
    # integral of I over the unit disk = pi (1 - u1/3 - u2/6)
    u1, u2 = 0.4, 0.25
    exact = np.pi * (1 - u1 / 3 - u2 / 6)
    errs = []
    for n in (100, 200, 400):
        _, _, x, y, mu = D.disk_cells(n)
        tot = D.cell_area(n) * D.limb_darkening(mu, u1, u2).sum()
        errs.append(abs(tot - exact) / exact)
    assert errs[-1] < 1e-4
    assert errs[2] < errs[0]


def test_mu_bin_nearest_and_ties():
    mu_b = np.array([1.0, 0.8, 0.5])
    assert list(D.mu_bin([1.0, 0.95, 0.9, 0.85, 0.65, 0.64, 0.1], mu_b)) == [0, 0, 0, 1, 1, 2, 2]
    # exact midpoint 0.9 between 1.0 and 0.8 goes to the lower index (larger mu)
    assert D.mu_bin([0.9], np.array([1.0, 0.8]))[0] == 0


def test_region_centre_path():
    # lon 180 deg at phase 0.5 crosses the disk centre (section 4.3.3 bump at phase 0.5)
    c = D.region_centre(0.0, 180.0, 0.5, 90.0)
    assert np.allclose(c, [0, 0, 1], atol=1e-12)
    # a quarter turn earlier it sits on the approaching (x < 0) limb
    c = D.region_centre(0.0, 180.0, 0.25, 90.0)
    assert np.allclose(c, [-1, 0, 0], atol=1e-12)
    # pole-on: the north pole points at the observer
    c = D.region_centre(90.0, 0.0, 0.3, 0.0)
    assert np.allclose(c, [0, 0, 1], atol=1e-12)
    # unit vectors
    for lat, lon, ph, inc in [(20, 33, 0.1, 60), (-50, 300, 0.7, 30)]:
        assert abs(np.linalg.norm(D.region_centre(lat, lon, ph, inc)) - 1) < 1e-14


def test_rotation_direction_consistent_with_velocity_field():
    # A surface point's x increases with phase on the visible side; the
    # velocity field v = vsini * x must then be the line-of-sight recession of
    # that rigid rotation: d(z)/dt < 0 where x > 0.
    lat, lon, inc = 10.0, 170.0, 70.0
    ph, dph = 0.45, 1e-6
    a = D.region_centre(lat, lon, ph, inc)
    b = D.region_centre(lat, lon, ph + dph, inc)
    vel = (b - a) / dph  # radians per phase * R
    # line-of-sight recession = -dz/dt, proportional to x with slope 2 pi sin i
    assert np.isclose(-vel[2], 2 * np.pi * np.sin(np.deg2rad(inc)) * a[0], rtol=1e-5)


def test_spot_box_matches_paper(golden):
    g = golden["spot_box"]
    n = g["n_grid"]
    rho = np.sqrt(g["area_fraction"])
    _, _, x, y, mu = D.disk_cells(n)
    reg = W.Region(W.SPOT, 0.0, 180.0, rho, 0.5)
    own = D.owner_map(x, y, mu, [reg], 0.5, 90.0)
    xs, ys = x[own == 0], y[own == 0]
    cols = int(round((xs.max() - xs.min()) * n / 2)) + 1
    rows = int(round((ys.max() - ys.min()) * n / 2)) + 1
    assert cols <= g["box_cells_max"] and rows <= g["box_cells_max"]
    # and the cap really is 1% of the disk: 2 rho N/2 cells across
    assert abs(cols - 2 * rho * n / 2) <= 2


def test_spot_area_closed_form():
    # Disk-centre cap of radius rho: projected region r < rho, so the covered
    # intensity is 2 pi int_{sqrt(1-rho^2)}^1 I(mu) mu dmu (exact polynomial).
    u1, u2, rho = 0.4, 0.25, 0.2
    m0 = np.sqrt(1 - rho * rho)

    def prim(m):  # antiderivative of I(mu) mu
        a = 1 - u1 - u2
        b = u1 + 2 * u2
        c = -u2
        return a * m**2 / 2 + b * m**3 / 3 + c * m**4 / 4

    exact = 2 * np.pi * (prim(1.0) - prim(m0))
    n = 400
    _, _, x, y, mu = D.disk_cells(n)
    own = D.owner_map(x, y, mu, [W.Region(W.SPOT, 0.0, 0.0, rho)], 0.0, 90.0)
    got = D.cell_area(n) * D.limb_darkening(mu[own == 0], u1, u2).sum()
    assert abs(got - exact) / exact < 1e-2


def test_owner_last_region_wins_and_same_type_counts_once():
    n = 40
    _, _, x, y, mu = D.disk_cells(n)
    fac = W.Region(W.FACULA, 10.0, 0.0, 0.4, 1.2)
    spot = W.Region(W.SPOT, 10.0, 0.0, 0.15, 0.5)
    own = D.owner_map(x, y, mu, [fac, spot], 0.0, 80.0)
    own_spot_only = D.owner_map(x, y, mu, [spot], 0.0, 80.0)
    assert np.all(own[own_spot_only == 0] == 1)
    assert np.any(own == 0)
    # reversed order: the facula overwrites the spot entirely
    own_rev = D.owner_map(x, y, mu, [spot, fac], 0.0, 80.0)
    assert not np.any(own_rev == 0) or np.all(own_rev[own_spot_only == 0] == 1)
    # duplicate identical spot: same integrated spectrum as a single one
    st = W.make_tiny(5, n_grid=14, n_pix=200, n_mu=3)
    a = S.integrated(st, 0.3, S.TOT, regions=[spot])
    b = S.integrated(st, 0.3, S.TOT, regions=[spot, spot])
    assert np.array_equal(a, b)


# ------------------------------------------------------- interpolation


def test_doppler_factor_is_rapidity():
    # ln(1 + f) = atanh(beta) for the relativistic factor of Eq. 6
    v = np.array([-3e4, -5.0, -1e-3, 0.0, 2.0, 1e4])
    assert np.allclose(np.log(S.doppler_factor(v)), np.arctanh(v / S.C_KMS), rtol=1e-12, atol=1e-15)
    assert np.all(S.doppler_factor(np.array([0.0])) == 1.0)


def test_zero_velocity_is_identity():
    rng = np.random.default_rng(0)
    lam = S.wavelengths(np.log(5000.0), 3e-6, 300)
    s = rng.uniform(0.2, 1.0, 300)
    assert np.array_equal(S.shift_spectrum(s, lam, 0.0), s)


@pytest.mark.parametrize("k", [1, 3, -2])
def test_integer_pixel_shift_is_translation(k):
    # on a log grid a velocity with atanh(beta) = k dln maps lambda_n onto
    # lambda_{n+k}: the shifted spectrum is the input moved by k pixels, to
    # larger wavelength for a receding (v > 0) source
    dln = 3e-6
    lam = S.wavelengths(np.log(5000.0), dln, 200)
    rng = np.random.default_rng(1)
    s = rng.uniform(0.2, 1.0, 200)
    v = S.C_KMS * np.tanh(k * dln)
    out = S.shift_spectrum(s, lam, v)
    if k > 0:
        assert np.allclose(out[k:], s[:-k], rtol=0, atol=1e-9)
        assert np.allclose(out[:k], s[0])
    else:
        assert np.allclose(out[:k], s[-k:], rtol=0, atol=1e-9)
        assert np.allclose(out[k:], s[-1])


def test_interpolation_exact_for_lambda_linear_spectrum():
    # Eq. 11 interpolates linearly in lambda, so a spectrum linear in lambda is
    # reproduced exactly: S'(lambda_m) = a + b lambda_m / (1 + f)
    lam = S.wavelengths(np.log(5000.0), 3e-6, 400)
    a, b = 0.3, 1.7e-4
    s = a + b * lam
    for v in (-4.1, 0.37, 2.9):
        out = S.shift_spectrum(s, lam, v)
        want = a + b * lam / S.doppler_factor(v)
        inner = slice(5, -5)
        assert np.allclose(out[inner], want[inner], rtol=1e-13, atol=0)


def test_interpolation_conserves_pixel_sum():
    # weights of each output pixel sum to one and every input pixel is used
    # with total weight one, so a line away from the ends keeps its pixel sum
    lam = S.wavelengths(np.log(5000.0), 3e-6, 500)
    q = np.arange(500)
    s = 1.0 - 0.7 * np.exp(-0.5 * ((q - 250.3) / 6.0) ** 2)
    for v in (-5.0, 1.3, 7.7):
        out = S.shift_spectrum(s, lam, v)
        assert abs((1 - out).sum() - (1 - s).sum()) < 1e-10 * (1 - s).sum()


# ---------------------------------------------------------- integration


def test_flat_spectra_give_weight_sum_everywhere():
    st = _flat_star(30)
    f = S.quiet(st)
    _, _, x, y, mu = D.disk_cells(30)
    want = D.cell_area(30) * D.limb_darkening(mu, st.ld_u1, st.ld_u2).sum()
    assert np.allclose(f, want, rtol=1e-14)


def test_no_rotation_reduces_to_weighted_bin_sum():
    st = W.make_tiny(11, n_grid=12, n_pix=150, n_mu=3, vsini_kms=0.0)
    f = S.quiet(st)
    want = np.zeros(st.n_pix)
    n = st.n_grid
    for i in range(n):
        for k in range(n):
            x = -1 + (2 * i + 1) / n
            y = -1 + (2 * k + 1) / n
            if x * x + y * y < 1:
                mu = np.sqrt(1 - x * x - y * y)
                om = 1 - mu
                inten = 1 - st.ld_u1 * om - st.ld_u2 * om * om
                b = int(np.argmin(np.abs(mu - st.mu_bins)))
                want += (2 / n) ** 2 * inten * st.spectra[0][b]
    assert np.allclose(f, want, rtol=1e-13)


@pytest.mark.parametrize("seed", [3, 4, 7])
@pytest.mark.parametrize("mode", [0, 1])
def test_bruteforce_equals_grouped(seed, mode):
    st = W.make_tiny(seed, n_grid=10, n_pix=180, n_mu=3, contrast_mode=mode)
    for eff in (S.TOT, S.FLUX, S.BCONV):
        for ph in st.phases[:2]:
            a = S.integrated_bruteforce(st, ph, eff)
            b = S.integrated(st, ph, eff)
            assert np.max(np.abs(a - b) / np.abs(a)) < 1e-13


def test_effects_identity_scalar_contrast():
    # Eqs. 1-3 with one scalar contrast C:
    # (F_tot - Q) = (F_flux - Q) + C (F_bconv - Q)
    st = W.make_tiny(21, n_grid=16, n_pix=220, n_mu=3)
    c = 0.55
    regs = [W.Region(W.SPOT, 15.0, 40.0, 0.35, c), W.Region(W.FACULA, -20.0, 10.0, 0.3, c)]
    q = S.quiet(st)
    for ph in (0.0, 0.1, 0.9):
        ft = S.integrated(st, ph, S.TOT, regs)
        ff = S.integrated(st, ph, S.FLUX, regs)
        fb = S.integrated(st, ph, S.BCONV, regs)
        assert np.allclose(ft - q, (ff - q) + c * (fb - q), rtol=0, atol=1e-13 * q.max())


def test_hidden_region_leaves_quiet_spectrum():
    st = W.make_tiny(8, n_grid=14, n_pix=160, n_mu=3)
    reg = [W.Region(W.SPOT, 0.0, 180.0, 0.2, 0.4)]
    # lon 180 at phase 0 sits at the back of an equator-on star
    st.incl_deg = 90.0
    f = S.integrated(st, 0.0, S.TOT, reg)
    assert np.array_equal(f, S.quiet(st))


def test_chromatic_contrast_in_planck_mode():
    st = W.make_tiny(9, n_grid=12, n_pix=200, n_mu=3, contrast_mode=1)
    lam = S.wavelengths(st.ln_lambda0, st.dln_lambda, st.n_pix)
    c_spot = S.contrast_array(st, W.SPOT, 0, lam)
    assert np.all(c_spot < 1) and np.all(np.diff(c_spot) > 0)  # cool spot: darker in the blue
    c_fac = S.contrast_array(st, W.FACULA, 0, lam)
    assert np.all(c_fac > 1)


# ----------------------------------------- closed-form rotational broadening


def _broadened_gaussian(q, q0, sig, depth, kpx, u1, u2, n_nodes=600):
    """1 - d (g * G)(q) / int G with G(x) the quadratic limb-darkened disk's
    strip weight 2(1-u1-u2)a + (u1+2u2)(pi/2)a^2 - u2(4/3)a^3, a = sqrt(1-x^2),
    and the line shift k x pixels for strip x.  The a and a^3 terms use
    Gauss-Chebyshev (second kind) quadrature; the a^2 term is done with erf."""
    from scipy.special import erf

    i = np.arange(1, n_nodes + 1)
    th = i * np.pi / (n_nodes + 1)
    xn = np.cos(th)
    wn = np.pi / (n_nodes + 1) * np.sin(th) ** 2  # int sqrt(1-x^2) h(x) dx
    qq = np.asarray(q, dtype=np.float64)[:, None]
    g = np.exp(-0.5 * ((qq - kpx * xn[None, :] - q0) / sig) ** 2)
    term_a = (g * wn).sum(1)
    term_a3 = (g * (1 - xn**2) * wn).sum(1)
    # int_{-1}^{1} (1 - x^2) exp(-(D - k x)^2 / 2 s^2) dx, D = q - q0
    D_ = np.asarray(q, dtype=np.float64) - q0
    lo = -kpx - D_
    hi = kpx - D_
    r2 = np.sqrt(2.0) * sig
    i0 = sig * np.sqrt(np.pi / 2) * (erf(hi / r2) - erf(lo / r2))
    i1 = sig**2 * (np.exp(-(lo**2) / (2 * sig**2)) - np.exp(-(hi**2) / (2 * sig**2)))
    i2 = sig**2 * i0 - sig**2 * (hi * np.exp(-(hi**2) / (2 * sig**2)) - lo * np.exp(-(lo**2) / (2 * sig**2)))
    term_a2 = (i0 - (i2 + 2 * D_ * i1 + D_**2 * i0) / kpx**2) / kpx
    conv = 2 * (1 - u1 - u2) * term_a + (u1 + 2 * u2) * (np.pi / 2) * term_a2 - u2 * (4 / 3) * term_a3
    norm = np.pi * (1 - u1 / 3 - u2 / 6)
    return 1 - depth * conv / norm


@pytest.mark.parametrize("u1,u2", [(0.6, 0.0), (0.4, 0.25)])
def test_rotational_broadening_closed_form(u1, u2):
    dln = 1e-7  # oversampled: 1 px = 0.03 km/s
    n_pix = 1200
    vsini = 1.5
    kpx = np.arctanh(vsini / S.C_KMS) / dln
    q = np.arange(n_pix, dtype=np.float64)
    q0, sig, depth = 600.0, 30.0, 0.6
    line = 1.0 - depth * np.exp(-0.5 * ((q - q0) / sig) ** 2)
    want = _broadened_gaussian(q, q0, sig, depth, kpx, u1, u2)
    errs = []
    for n in (100, 200, 400):
        st = W.StarInputs(
            n_grid=n, vsini_kms=vsini, incl_deg=90.0, ld_u1=u1, ld_u2=u2,
            ln_lambda0=np.log(5000.0), dln_lambda=dln, n_pix=n_pix,
            mu_bins=np.array([1.0]), spectra=[line[None, :], None, None],
        )
        f = S.quiet(st)
        f = f / f[0]  # continuum normalise (line wings are 1e-30 at the ends)
        errs.append(np.max(np.abs(f - want)) / depth)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-3
    # sign / width check: the broadened line is shallower and wider than the input
    assert want.min() > line.min()


def test_linear_limb_darkening_kernel_is_textbook_profile():
    # u2 = 0 strip weight reduces to the classical rotation profile
    # G(x) = [2(1-e) sqrt(1-x^2) + (pi e / 2)(1-x^2)] / (pi (1 - e/3))
    e = 0.6
    x = np.linspace(-0.99, 0.99, 101)
    n = 4000
    xs = D.cell_centres(n)
    ys = D.cell_centres(n)
    yy2 = ys[None, :] ** 2
    for xi in x[::10]:
        col = np.argmin(np.abs(xs - xi))
        r2 = xs[col] ** 2 + yy2[0]
        vis = r2 < 1
        strip = (2.0 / n) * D.limb_darkening(np.sqrt(1 - r2[vis]), e, 0.0).sum()
        a = np.sqrt(1 - xs[col] ** 2)
        g = (2 * (1 - e) * a + np.pi * e / 2 * a * a)
        assert abs(strip - g) < 2e-3
