"""Seeded synthetic stars, active regions and CCF masks.

Everything here is input preparation: line lists rendered into local spectra
on a log-uniform wavelength grid (one spectrum per surface type and mu bin),
plus region lists, phase lists and a binary line mask.  The recipe follows the
paper's workloads in shape (full visible range at R = 115000, a 300 x 300 disk,
spot / facula / quiet spectra with a convective-blueshift law that varies with
mu) but every value is drawn from ``numpy.random.default_rng(seed)`` in a fixed
order, so the same seed always gives the same arrays.

The local spectra are *inputs* of the method (the paper injects observed or
PHOENIX spectra per mu bin, section 4.3.2); the Doppler shift that places a
line centre at its convective-blueshift velocity here is a first-order
generator detail, not the method's relativistic shift of section 3.2.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

C_KMS = 299792.458
C_MS = C_KMS * 1e3

QUIET, SPOT, FACULA = 0, 1, 2
CONTRAST_SCALAR, CONTRAST_PLANCK, CONTRAST_ARRAY = 0, 1, 2
EFFECT_TOT, EFFECT_FLUX, EFFECT_BCONV = 0, 1, 2
PREC_FP64, PREC_FP32 = 0, 1

# Facula temperature excess law of the Sun, dT_f(mu) = a0 + a1*mu + a2*mu^2
# (section 4.3.3, quoted from Meunier et al. 2010).
FACULA_DT_SUN = (250.9, -407.7, 190.9)


@dataclass
class Region:
    """One circular active region.

    type     SPOT or FACULA
    lat_deg, lon_deg  centre latitude / longitude on the star (degrees)
    radius   sin(alpha) of the cap's angular radius, in stellar radii
    contrast scalar intensity ratio I_active / I_quiet (scalar-contrast mode)
    """

    type: int
    lat_deg: float
    lon_deg: float
    radius: float
    contrast: float = 1.0


@dataclass
class Mask:
    """Binary (or weighted) CCF line mask and the velocity grid it is run on."""

    ln_lambda: np.ndarray  # (L,) ln(lambda / Angstrom) of the line centres
    weight: np.ndarray  # (L,)
    half_width_kms: float
    v0_kms: float
    dv_kms: float
    n_v: int


@dataclass
class StarInputs:
    n_grid: int
    vsini_kms: float
    incl_deg: float
    ld_u1: float
    ld_u2: float
    ln_lambda0: float
    dln_lambda: float
    n_pix: int
    mu_bins: np.ndarray  # (B,) strictly decreasing in (0, 1]
    spectra: List[Optional[np.ndarray]]  # [QUIET, SPOT, FACULA], each (B, P) or None
    precision: int = PREC_FP64
    contrast_mode: int = CONTRAST_SCALAR
    teff_k: float = 5778.0
    dt_spot_k: float = 663.0
    dt_fac_coef: tuple = FACULA_DT_SUN
    regions: List[Region] = field(default_factory=list)
    phases: np.ndarray = field(default_factory=lambda: np.zeros(0))
    mask: Optional[Mask] = None
    name: str = ""
    # CONTRAST_ARRAY mode: per active type a (B, P) array of contrasts applied
    # after the shift (index QUIET stays None)
    contrast: List[Optional[np.ndarray]] = field(default_factory=lambda: [None, None, None])
    # differential rotation (section 3.4): omega = omega_0 (1 + diff_rot sin^2 latitude)
    diff_rot: float = 0.0

    @property
    def n_mu(self) -> int:
        return int(len(self.mu_bins))

    @property
    def dtype(self):
        return np.float64 if self.precision == PREC_FP64 else np.float32


def cb_velocity_ms(teff_k):
    """Convective-blueshift amplitude vs effective temperature (section 4.3.3).

    The paper fits a cubic to the Liebing et al. data, valid 4800-6300 K; the
    temperature is clamped to that range before evaluating it.
    """
    t = np.clip(np.asarray(teff_k, dtype=np.float64), 4800.0, 6300.0)
    return 95.2388 * ((t - 4400.0) / 1000.0) ** 3 + 91.2791


def cb_law_ms(mu_b, amplitude_ms=350.0):
    """Blueshift per mu bin: -amplitude at mu = 1, falling linearly to 0 at mu = 0.1."""
    return -amplitude_ms * (np.asarray(mu_b, dtype=np.float64) - 0.1) / 0.9


def make_velocity_grid(v0_kms, dv_kms, n_v):
    return v0_kms + dv_kms * np.arange(n_v, dtype=np.float64)


# ---------------------------------------------------------------------------
# line rendering
# ---------------------------------------------------------------------------


def _render(ln0, dln, n_pix, centre_a, depth, sigma_a, gamma_a, v_ms, nsig=8.0, nsig_voigt=40.0):
    """prod_l (1 - d_l * phi_l(lambda)) on the grid, phi normalised to peak 1.

    Gaussian lines use exp(-x^2/2); lines with gamma > 0 use the Voigt profile
    (scipy) normalised at its centre.  Each profile is truncated at nsig (or
    nsig_voigt) Gaussian sigmas, which is part of this synthetic recipe.
    """
    from scipy.special import voigt_profile

    lam = np.exp(ln0 + dln * np.arange(n_pix, dtype=np.float64))
    lam_c = centre_a * (1.0 + v_ms / C_MS)
    pc = (np.log(lam_c) - ln0) / dln
    sig_px = sigma_a / (lam_c * dln)
    log_s = np.zeros(n_pix, dtype=np.float64)
    order = np.argsort(sig_px * np.where(gamma_a > 0, nsig_voigt, nsig))
    chunk = 1024
    for s in range(0, len(order), chunk):
        sel = order[s : s + chunk]
        is_v = gamma_a[sel] > 0
        hw = np.ceil(sig_px[sel] * np.where(is_v, nsig_voigt, nsig)).astype(np.int64) + 1
        w = int(hw.max())
        offs = np.arange(-w, w + 1, dtype=np.int64)
        idx = np.rint(pc[sel]).astype(np.int64)[:, None] + offs[None, :]
        ok = (idx >= 0) & (idx < n_pix) & (np.abs(offs)[None, :] <= hw[:, None])
        idc = np.clip(idx, 0, n_pix - 1)
        x = lam[idc] - lam_c[sel][:, None]
        sg = sigma_a[sel][:, None]
        prof = np.exp(-0.5 * (x / sg) ** 2)
        if is_v.any():
            vi = np.nonzero(is_v)[0]
            g = gamma_a[sel][vi][:, None]
            sv = sg[vi]
            prof[vi] = voigt_profile(x[vi], sv, g) / voigt_profile(0.0, sv, g)
        contrib = np.log1p(-depth[sel][:, None] * prof)
        log_s += np.bincount(idx[ok], weights=contrib[ok], minlength=n_pix)
    return np.exp(log_s)


def _select_mask_lines(centre_a, depth, sigma_a, n_max):
    """Deepest lines with no neighbour deeper than 0.1*d within +-2 sigma."""
    order = np.argsort(centre_a)
    c = centre_a[order]
    d = depth[order]
    sg = sigma_a[order]
    keep = np.ones(len(c), dtype=bool)
    lo = np.searchsorted(c, c - 2 * sg, side="left")
    hi = np.searchsorted(c, c + 2 * sg, side="right")
    for i in range(len(c)):
        for j in range(lo[i], hi[i]):
            if j != i and d[j] > 0.1 * d[i]:
                keep[i] = False
                break
    cand = np.nonzero(keep)[0]
    cand = cand[np.argsort(-d[cand], kind="stable")][:n_max]
    cand = np.sort(cand)
    return c[cand], d[cand]


def input_digest(star: StarInputs) -> str:
    h = hashlib.sha256()
    for arr in star.spectra:
        if arr is not None:
            h.update(np.ascontiguousarray(arr).tobytes())
    h.update(np.ascontiguousarray(star.mu_bins).tobytes())
    h.update(np.ascontiguousarray(star.phases).tobytes())
    for r in star.regions:
        h.update(np.array([r.type, r.lat_deg, r.lon_deg, r.radius, r.contrast]).tobytes())
    if star.mask is not None:
        h.update(star.mask.ln_lambda.tobytes())
        h.update(star.mask.weight.tobytes())
    for arr in star.contrast:
        if arr is not None:
            h.update(np.ascontiguousarray(arr).tobytes())
    if star.diff_rot:
        h.update(np.float64(star.diff_rot).tobytes())
    return h.hexdigest()


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------


def make_cfg1(seed: int = 1) -> StarInputs:
    """Plain method in FP64: 100 x 100 disk, 5000-5050 A in 4096 px, 20 lines.

    5 mu bins with blueshift -350 m/s at mu = 1 to 0 at mu = 0.1; quadratic
    limb darkening (0.4, 0.25); v sin i = 2 km/s, i = 90 deg; one spot of 5%
    disk area at latitude 20 deg, contrast 0.6, lines 30% deeper; 25 phases.
    """
    rng = np.random.default_rng(seed)
    n_pix = 4096
    ln0 = np.log(5000.0)
    dln = np.log(5050.0 / 5000.0) / (n_pix - 1)
    n_lines = 20
    centre = rng.uniform(5001.0, 5049.0, n_lines)
    depth = rng.uniform(0.1, 0.8, n_lines)
    sigma = rng.uniform(0.03, 0.08, n_lines)
    gamma = np.zeros(n_lines)
    mu_b = 1.0 - 0.225 * np.arange(5)
    cb = cb_law_ms(mu_b)
    quiet = np.stack([_render(ln0, dln, n_pix, centre, depth, sigma, gamma, v) for v in cb])
    spot_depth = np.minimum(depth * 1.3, 0.99)
    spot_one = _render(ln0, dln, n_pix, centre, spot_depth, sigma, gamma, 0.0)
    spot = np.stack([spot_one] * len(mu_b))
    mlam, _ = _select_mask_lines(centre, depth, sigma, 4000)
    mask = Mask(np.log(mlam), np.ones(len(mlam)), 0.41, -20.0, 0.25, 161)
    return StarInputs(
        n_grid=100,
        vsini_kms=2.0,
        incl_deg=90.0,
        ld_u1=0.4,
        ld_u2=0.25,
        ln_lambda0=ln0,
        dln_lambda=dln,
        n_pix=n_pix,
        mu_bins=mu_b,
        spectra=[quiet, spot, None],
        precision=PREC_FP64,
        contrast_mode=CONTRAST_SCALAR,
        regions=[Region(SPOT, 20.0, 180.0, float(np.sqrt(0.05)), 0.6)],
        phases=np.arange(25, dtype=np.float64) / 25.0,
        mask=mask,
        name="cfg1: 100^2 disk, 4096 px, 5 mu bins, 1 spot, 25 phases, FP64",
    )


def make_cfg2(seed: int = 2, precision: int = PREC_FP32, n_phases: int = 100) -> StarInputs:
    """Full visible range at R = 115000 on a 300 x 300 disk (headline workload).

    3800-6900 A at dln = 1/(3*115000) (205800 px); 30k lines (deepest 10%
    Voigt); 20 mu bins; spot spectrum at T_eff - 600 K with 30% deeper lines
    plus 5k weak molecular-band lines; facula spectrum = quiet lines with no
    blueshift; chromatic Planck contrast; a facula with a spot inside it and a
    second spot; 100 phases; 4000-line binary mask.
    """
    rng = np.random.default_rng(seed)
    dln = 1.0 / (3.0 * 115000.0)
    ln0 = np.log(3800.0)
    n_pix = int(np.floor(np.log(6900.0 / 3800.0) / dln)) + 1
    n_lines = 30000
    centre, u, sigma = _headline_lines(rng)
    depth = 0.05 + 0.85 * u * u
    gamma = np.zeros(n_lines)
    deep = np.argsort(-depth)[: n_lines // 10]
    gamma[deep] = 0.1 * sigma[deep]
    n_mu = 20
    mu_b = 1.0 - 0.9 * np.arange(n_mu) / (n_mu - 1)
    cb = cb_law_ms(mu_b)
    quiet = np.stack([_render(ln0, dln, n_pix, centre, depth, sigma, gamma, v) for v in cb])
    # spot: deeper lines, no blueshift, plus weak molecular-band lines in the red
    n_weak = 5000
    band_c = 5800.0 + (np.arange(10) + 0.5) * 110.0
    wc = band_c[rng.integers(0, 10, n_weak)] + rng.uniform(-15.0, 15.0, n_weak)
    wd = rng.uniform(0.01, 0.05, n_weak)
    ws = wc * rng.uniform(1.5, 3.0, n_weak) / C_KMS
    sc = np.concatenate([centre, wc])
    sd = np.concatenate([np.minimum(depth * 1.3, 0.99), wd])
    ss = np.concatenate([sigma, ws])
    sgm = np.concatenate([gamma, np.zeros(n_weak)])
    spot_one = _render(ln0, dln, n_pix, sc, sd, ss, sgm, 0.0)
    fac_one = _render(ln0, dln, n_pix, centre, depth, sigma, gamma, 0.0)
    dt = np.float64 if precision == PREC_FP64 else np.float32
    spot = np.broadcast_to(spot_one, (n_mu, n_pix)).astype(dt)
    fac = np.broadcast_to(fac_one, (n_mu, n_pix)).astype(dt)
    mlam, _ = _select_mask_lines(centre, depth, sigma, 4000)
    mask = Mask(np.log(mlam), np.ones(len(mlam)), 0.41, -20.0, 0.25, 161)
    return StarInputs(
        n_grid=300,
        vsini_kms=2.0,
        incl_deg=90.0,
        ld_u1=0.4,
        ld_u2=0.25,
        ln_lambda0=ln0,
        dln_lambda=dln,
        n_pix=n_pix,
        mu_bins=mu_b,
        spectra=[quiet.astype(dt), spot, fac],
        precision=precision,
        contrast_mode=CONTRAST_PLANCK,
        teff_k=5778.0,
        dt_spot_k=600.0,
        dt_fac_coef=FACULA_DT_SUN,
        regions=[
            Region(FACULA, 30.0, 180.0, 0.3, 1.0),
            Region(SPOT, 30.0, 180.0, 0.1, 1.0),
            Region(SPOT, -15.0, 60.0, 0.1414, 1.0),
        ],
        phases=np.arange(n_phases, dtype=np.float64) / n_phases,
        mask=mask,
        name="cfg2: 300^2 disk, 205800 px, 20 mu bins, facula+2 spots, 100 phases",
    )


def make_tiny(
    seed: int,
    n_grid: int = 16,
    n_pix: int = 700,
    n_mu: int = 4,
    precision: int = PREC_FP64,
    contrast_mode: int = CONTRAST_SCALAR,
    n_regions: Optional[int] = None,
    n_phases: int = 5,
    vsini_kms: Optional[float] = None,
    incl_deg: Optional[float] = None,
    with_facula: bool = True,
) -> StarInputs:
    """Small random star for parity tests: every bin and type gets its own
    spectrum (random per-bin velocities for all types) so that an indexing
    mistake on any axis changes the result."""
    rng = np.random.default_rng(seed)
    dln = rng.uniform(2.0e-6, 6.0e-6)
    ln0 = np.log(rng.uniform(4000.0, 6000.0))
    lam_hi = np.exp(ln0 + dln * (n_pix - 1))
    lam_lo = np.exp(ln0)
    n_lines = max(4, n_pix // 40)
    centre = rng.uniform(lam_lo, lam_hi, n_lines)
    depth = rng.uniform(0.1, 0.9, n_lines)
    sigma = centre * rng.uniform(1.5, 4.0, n_lines) / C_KMS
    gamma = np.zeros(n_lines)
    mu_b = np.sort(rng.uniform(0.05, 1.0, n_mu))[::-1].copy()
    mu_b[0] = 1.0
    types = [QUIET, SPOT, FACULA] if with_facula else [QUIET, SPOT]
    spectra: List[Optional[np.ndarray]] = [None, None, None]
    dt = np.float64 if precision == PREC_FP64 else np.float32
    for t in types:
        scale = {QUIET: 1.0, SPOT: 1.3, FACULA: 0.9}[t]
        vb = rng.uniform(-600.0, 300.0, n_mu)
        spectra[t] = np.stack(
            [
                _render(ln0, dln, n_pix, centre, np.minimum(depth * scale, 0.99), sigma, gamma, v)
                for v in vb
            ]
        ).astype(dt)
    if vsini_kms is None:
        vsini_kms = float(rng.uniform(1.0, 8.0))
    if incl_deg is None:
        incl_deg = float(rng.uniform(20.0, 90.0))
    if n_regions is None:
        n_regions = int(rng.integers(1, 5))
    regs = []
    for _ in range(n_regions):
        t = int(rng.integers(1, 3)) if with_facula else SPOT
        regs.append(
            Region(
                t,
                float(rng.uniform(-60.0, 60.0)),
                float(rng.uniform(0.0, 360.0)),
                float(rng.uniform(0.1, 0.45)),
                float(rng.uniform(0.3, 1.4)),
            )
        )
    phases = np.sort(rng.uniform(0.0, 1.0, n_phases))
    # a short mask of the deepest lines, velocity grid wide enough for v sin i
    order = np.argsort(-depth)[: max(2, n_lines // 2)]
    mlam = np.sort(centre[order])
    mask = Mask(np.log(mlam), rng.uniform(0.5, 1.0, len(mlam)), 0.41, -15.0, 0.5, 61)
    contrast: List[Optional[np.ndarray]] = [None, None, None]
    if contrast_mode == CONTRAST_ARRAY:
        # per (type, bin): a limb-brightening factor times a smooth SED ratio
        # with a tilt and a ripple, different in every row and pixel (drawn
        # after everything else, so the other inputs do not depend on the mode)
        xm = np.arange(n_pix, dtype=np.float64)
        for t in types[1:]:
            lb = rng.uniform(0.5, 1.3, n_mu)
            tilt = rng.uniform(-0.3, 0.3, n_mu)
            amp = rng.uniform(0.0, 0.05, n_mu)
            per = rng.uniform(20.0, 200.0, n_mu)
            ph0 = rng.uniform(0.0, 2.0 * np.pi, n_mu)
            contrast[t] = (
                lb[:, None]
                * (1.0 + tilt[:, None] * (xm / n_pix - 0.5)[None, :]
                   + amp[:, None] * np.sin(2.0 * np.pi * xm[None, :] / per[:, None] + ph0[:, None]))
            ).astype(dt)
    return StarInputs(
        n_grid=n_grid,
        vsini_kms=vsini_kms,
        incl_deg=incl_deg,
        ld_u1=float(rng.uniform(0.1, 0.6)),
        ld_u2=float(rng.uniform(0.0, 0.3)),
        ln_lambda0=ln0,
        dln_lambda=dln,
        n_pix=n_pix,
        mu_bins=mu_b,
        spectra=spectra,
        precision=precision,
        contrast_mode=contrast_mode,
        teff_k=float(rng.uniform(4800.0, 6300.0)),
        dt_spot_k=float(rng.uniform(300.0, 900.0)),
        dt_fac_coef=FACULA_DT_SUN,
        regions=regs,
        phases=phases,
        mask=mask,
        name=f"tiny seed={seed} N={n_grid} P={n_pix} B={n_mu}",
        contrast=contrast,
    )


def make_cfg5(seed: int = 5, precision: int = PREC_FP32, n_grid: int = 300) -> StarInputs:
    """Star of the surrogate data set: a 20000-pixel window from 5000 A at
    R = 115000 (about 298 A), a 300 x 300 disk, 20 mu bins, solar limb
    darkening, v sin i = 2 km/s, i = 90 deg, scalar contrast.  Line density
    follows the full-range star (about 10 lines per A, the deepest 10% Voigt);
    the spot spectrum has 30% deeper lines and no blueshift.  Regions and
    phases come per sample from ``cfg5_samples``; the mask holds the window's
    deepest lines (up to 400)."""
    rng = np.random.default_rng(seed)
    dln = 1.0 / (3.0 * 115000.0)
    ln0 = np.log(5000.0)
    n_pix = 20000
    lam_hi = float(np.exp(ln0 + dln * (n_pix - 1)))
    n_lines = int(round((lam_hi - 5000.0) * 30000 / 3100.0))
    centre = rng.uniform(5002.0, lam_hi - 2.0, n_lines)
    u = rng.uniform(0.0, 1.0, n_lines)
    depth = 0.05 + 0.85 * u * u
    sigma = centre * rng.uniform(1.5, 3.0, n_lines) / C_KMS
    gamma = np.zeros(n_lines)
    deep = np.argsort(-depth)[: n_lines // 10]
    gamma[deep] = 0.1 * sigma[deep]
    n_mu = 20
    mu_b = 1.0 - 0.9 * np.arange(n_mu) / (n_mu - 1)
    cb = cb_law_ms(mu_b)
    dt = np.float64 if precision == PREC_FP64 else np.float32
    quiet = np.stack([_render(ln0, dln, n_pix, centre, depth, sigma, gamma, v) for v in cb]).astype(dt)
    spot_one = _render(ln0, dln, n_pix, centre, np.minimum(depth * 1.3, 0.99), sigma, gamma, 0.0)
    spot = np.broadcast_to(spot_one, (n_mu, n_pix)).astype(dt)
    mlam, _ = _select_mask_lines(centre, depth, sigma, 400)
    mask = Mask(np.log(mlam), np.ones(len(mlam)), 0.41, -20.0, 0.25, 161)
    return StarInputs(
        n_grid=n_grid,
        vsini_kms=2.0,
        incl_deg=90.0,
        ld_u1=0.4,
        ld_u2=0.25,
        ln_lambda0=ln0,
        dln_lambda=dln,
        n_pix=n_pix,
        mu_bins=mu_b,
        spectra=[quiet, spot, None],
        precision=precision,
        contrast_mode=CONTRAST_SCALAR,
        regions=[],
        phases=np.zeros(0),
        mask=mask,
        name=f"cfg5: {n_grid}^2 disk, 20000 px window at 5000 A, 20 mu bins, one spot per sample",
    )


@dataclass
class SpotSamples:
    """Single-spot configurations of the surrogate data set: spot k has
    (lat_deg, lon_deg, radius, contrast) and is seen at phases[k] (n_per
    phases each).  Sample i = spot i // n_per at phase phases.flat[i]."""

    lat_deg: np.ndarray
    lon_deg: np.ndarray
    radius: np.ndarray
    contrast: np.ndarray
    phases: np.ndarray  # (n_spots, n_per)

    @property
    def n(self) -> int:
        return int(self.phases.size)

    @property
    def n_per(self) -> int:
        return int(self.phases.shape[1])


def cfg5_samples(n_spots: int, n_per: int = 8, seed: int = 5) -> SpotSamples:
    """lat U[-60, 60] deg, lon U[0, 360) deg, radius U[0.01, 0.10], contrast
    U[0.3, 0.9], phases U[0, 1) (n_per per spot)."""
    rng = np.random.default_rng([seed, n_spots, n_per])
    return SpotSamples(
        lat_deg=rng.uniform(-60.0, 60.0, n_spots),
        lon_deg=rng.uniform(0.0, 360.0, n_spots),
        radius=rng.uniform(0.01, 0.10, n_spots),
        contrast=rng.uniform(0.3, 0.9, n_spots),
        phases=rng.uniform(0.0, 1.0, (n_spots, n_per)),
    )


def _headline_lines(rng):
    """The headline star's 30000 lines (centre_A, u, sigma_A), the first
    draws of its generator."""
    centre = rng.uniform(3805.0, 6895.0, 30000)
    u = rng.uniform(0.0, 1.0, 30000)
    sigma = centre * rng.uniform(1.5, 3.0, 30000) / C_KMS
    return centre, u, sigma


def full_range_lines(n_lines: int, seed: int = 2, extra_seed: int = 3):
    """Master line list of the full range (3800-6900 A): (centre_A, u,
    sigma_A) of n_lines lines, depth (0.05 + 0.85 u^2) before any T_eff
    scaling.  The first 30000 are the headline star's lines (make_cfg2 draws
    them first from the same seed, in the same order), so its mask marks
    lines of every star built on this list, as a real line mask marks the
    same atomic lines in stars of any T_eff; further lines (denser lists of
    cooler stars) come from a second stream."""
    n0 = 30000
    centre, u, sigma = _headline_lines(np.random.default_rng(seed))
    if n_lines > n0:
        r2 = np.random.default_rng([extra_seed, 77])
        m = n_lines - n0
        c2 = r2.uniform(3805.0, 6895.0, m)
        centre = np.concatenate([centre, c2])
        u = np.concatenate([u, r2.uniform(0.0, 1.0, m)])
        sigma = np.concatenate([sigma, c2 * r2.uniform(1.5, 3.0, m) / C_KMS])
    return centre[:n_lines], u[:n_lines], sigma[:n_lines]


def make_bank(teff_k: float, seed: int = 3, n_mu: int = 20):
    """Full-range local spectra (3800-6900 A at R = 115000, 205800 px) of a
    star of effective temperature teff_k, for windows of the batched
    workload: the first 30k (5778/T)^3 lines of the master list
    (full_range_lines: hotter stars keep a subset of the headline star's
    lines, cooler ones add weaker-list lines), depths scaled by (5778/T)^1.5
    (capped at 0.95), convective blueshift from the cubic in T_eff (clamped
    to its 4800-6300 K range), spot spectrum with 30% deeper lines and no
    blueshift, facula spectrum = quiet lines without blueshift.  Returns
    (ln_lambda0, dln_lambda, mu_bins, [quiet, spot, facula]) with float32
    arrays [n_mu][205800]."""
    dln = 1.0 / (3.0 * 115000.0)
    ln0 = np.log(3800.0)
    n_pix = int(np.floor(np.log(6900.0 / 3800.0) / dln)) + 1
    scale = 5778.0 / teff_k
    n_lines = int(round(30000 * scale**3))
    centre, u, sigma = full_range_lines(n_lines, extra_seed=seed)
    depth = np.minimum((0.05 + 0.85 * u * u) * scale**1.5, 0.95)
    gamma = np.zeros(n_lines)
    deep = np.argsort(-depth)[: n_lines // 10]
    gamma[deep] = 0.1 * sigma[deep]
    mu_b = 1.0 - 0.9 * np.arange(n_mu) / (n_mu - 1)
    amp = cb_velocity_ms(float(np.clip(teff_k, 4800.0, 6300.0)))
    cb = cb_law_ms(mu_b, amplitude_ms=amp)
    quiet = np.stack([_render(ln0, dln, n_pix, centre, depth, sigma, gamma, v) for v in cb]).astype(np.float32)
    spot_one = _render(ln0, dln, n_pix, centre, np.minimum(depth * 1.3, 0.99), sigma, gamma, 0.0)
    fac_one = _render(ln0, dln, n_pix, centre, depth, sigma, gamma, 0.0)
    spot = np.ascontiguousarray(np.broadcast_to(spot_one, (n_mu, n_pix)), dtype=np.float32)
    fac = np.ascontiguousarray(np.broadcast_to(fac_one, (n_mu, n_pix)), dtype=np.float32)
    return ln0, dln, mu_b, [quiet, spot, fac]


def batch_configs(n_cfg: int, seed: int = 3, n_pix_total: int = 205800):
    """Ragged configurations of the batched workload: grid U{100..400},
    pixels U[8000, 206000) in a window starting uniformly over the full
    range, phases U{25..200}, T_eff U[4500, 6500] K, v sin i U[1, 5] km/s,
    i U[30, 90] deg, 1-4 regions (spot or facula with probability 0.5,
    radius U[0.01, 0.10], lat U[-60, 60], lon U[0, 360))."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_cfg):
        n_pix = int(min(rng.integers(8000, 206000), n_pix_total))
        start = int(rng.integers(0, n_pix_total - n_pix + 1))
        nr = int(rng.integers(1, 5))
        regs = [
            Region(SPOT if rng.uniform() < 0.5 else FACULA, float(rng.uniform(-60.0, 60.0)),
                   float(rng.uniform(0.0, 360.0)), float(rng.uniform(0.01, 0.10)), 1.0)
            for _ in range(nr)
        ]
        out.append(
            dict(
                n_grid=int(rng.integers(100, 401)),
                n_pix=n_pix,
                start=start,
                n_phases=int(rng.integers(25, 201)),
                teff_k=float(rng.uniform(4500.0, 6500.0)),
                vsini_kms=float(rng.uniform(1.0, 5.0)),
                incl_deg=float(rng.uniform(30.0, 90.0)),
                regions=regs,
            )
        )
    return out


def make_bisector_star(seed: int = 9, n_grid: int = 60, n_pix: int = 3000, n_mu: int = 6,
                       precision: int = PREC_FP32, n_phases: int = 12) -> StarInputs:
    """A star whose local spectra carry depth-dependent bisectors per mu bin
    (section 4.3.2, synthetic shapes of workloads.bisectors): symmetric
    Gaussian lines rendered without a shift, then the quiet rows injected
    with a C-shaped bisector scaled by the bin's convective blueshift and the
    spot and facula rows with the inhibited (straight) active bisector.
    Planck contrast, a facula with a spot inside and a second spot."""
    from . import bisectors as BI

    rng = np.random.default_rng(seed)
    dln = 1.0 / (3.0 * 115000.0)
    ln0 = np.log(5000.0)
    lam_hi = np.exp(ln0 + dln * (n_pix - 1))
    n_lines = max(4, n_pix // 60)
    centre = rng.uniform(5000.0 + 1.0, lam_hi - 1.0, n_lines)
    depth = rng.uniform(0.2, 0.85, n_lines)
    sigma = centre * rng.uniform(2.0, 3.5, n_lines) / C_KMS
    gamma = np.zeros(n_lines)
    mu_b = 1.0 - 0.9 * np.arange(n_mu) / (n_mu - 1)
    cb = cb_law_ms(mu_b)
    dt = np.float64 if precision == PREC_FP64 else np.float32
    base = {
        QUIET: _render(ln0, dln, n_pix, centre, depth, sigma, gamma, 0.0),
        SPOT: _render(ln0, dln, n_pix, centre, np.minimum(depth * 1.3, 0.99), sigma, gamma, 0.0),
        FACULA: _render(ln0, dln, n_pix, centre, depth, sigma, gamma, 0.0),
    }
    spectra = [np.stack([base[t]] * n_mu) for t in (QUIET, SPOT, FACULA)]
    regs = [Region(FACULA, 25.0, 180.0, 0.3, 1.0), Region(SPOT, 25.0, 180.0, 0.12, 1.0),
            Region(SPOT, -10.0, 40.0, 0.15, 1.0)]
    order = np.argsort(-depth)[: max(2, n_lines // 2)]
    mlam = np.sort(centre[order])
    star = StarInputs(
        n_grid=n_grid, vsini_kms=2.0, incl_deg=90.0, ld_u1=0.4, ld_u2=0.25, ln_lambda0=ln0, dln_lambda=dln,
        n_pix=n_pix, mu_bins=mu_b, spectra=spectra, precision=precision, contrast_mode=CONTRAST_PLANCK,
        teff_k=5778.0, dt_spot_k=663.0, dt_fac_coef=FACULA_DT_SUN, regions=regs,
        phases=np.linspace(0.0, 1.0, n_phases, endpoint=False),
        mask=Mask(np.log(mlam), np.ones(len(mlam)), 0.41, -20.0, 0.25, 161),
        name=f"bisector star seed={seed} N={n_grid} P={n_pix} B={n_mu}",
    )
    star.spectra = [a.astype(dt) for a in BI.inject_star(star, cb)]
    return star


BANK_TEFF = (4750.0, 5250.0, 5750.0, 6250.0)


def batch_star(cfg, bank, precision: int = PREC_FP32) -> StarInputs:
    """The star of one batched configuration: its pixel window of the
    nearest spectral bank (ln_lambda0, dln, mu_bins, [quiet, spot, facula]),
    its grid, rotation and regions, limb darkening (0.4, 0.25), Planck
    contrast at its T_eff.  Spectra stay whatever array type the bank holds
    (sliced, not copied, for numpy banks)."""
    ln0, dln, mu_b, sp = bank
    a, n = cfg["start"], cfg["n_pix"]
    return StarInputs(
        n_grid=cfg["n_grid"], vsini_kms=cfg["vsini_kms"], incl_deg=cfg["incl_deg"], ld_u1=0.4, ld_u2=0.25,
        ln_lambda0=ln0 + a * dln, dln_lambda=dln, n_pix=n, mu_bins=np.asarray(mu_b),
        spectra=[x[:, a:a + n] for x in sp], precision=precision, contrast_mode=CONTRAST_PLANCK,
        teff_k=cfg["teff_k"], dt_spot_k=663.0, dt_fac_coef=FACULA_DT_SUN, regions=list(cfg["regions"]),
        name=f"batch N={cfg['n_grid']} P={n} T={cfg['teff_k']:.0f}",
    )


def bank_for(teff_k: float) -> float:
    """T_eff of the spectral bank that serves a configuration."""
    return min(BANK_TEFF, key=lambda t: abs(t - teff_k))


# Star grid of the multi-star surrogate data set: T_eff on a 41-point grid
# (50 K steps, so local spectra are shared), inclination and v sin i on
# coarse grids (one context per star).
CFG5_TEFF = np.arange(4500.0, 6500.0 + 1.0, 50.0)
CFG5_INCL = np.arange(30.0, 90.0 + 1.0, 10.0)
CFG5_VSINI = np.arange(1.0, 5.0 + 1.0, 1.0)


def _cfg5_lines(seed: int = 5):
    """Master line list of the 20000-pixel window: lines are taken in list
    order up to the count for a given T_eff, so cooler stars keep every line
    of hotter ones and add more."""
    rng = np.random.default_rng([seed, 55])
    dln = 1.0 / (3.0 * 115000.0)
    ln0 = np.log(5000.0)
    n_pix = 20000
    lam_hi = float(np.exp(ln0 + dln * (n_pix - 1)))
    n_sun = (lam_hi - 5000.0) * 30000 / 3100.0
    n_max = int(round(n_sun * (5778.0 / 4500.0) ** 3))
    centre = rng.uniform(5002.0, lam_hi - 2.0, n_max)
    u = rng.uniform(0.0, 1.0, n_max)
    sigma = centre * rng.uniform(1.5, 3.0, n_max) / C_KMS
    return ln0, dln, n_pix, n_sun, centre, u, sigma


def _render_row(args):
    return _render(*args)


def cfg5_window_spectra(teff_k: float, seed: int = 5, n_mu: int = 10, pool=None):
    """Quiet (n_mu rows) and spot (one row, every bin) local spectra of the
    surrogate window for T_eff: 30k (5778/T)^3-per-full-range line density,
    depths (0.05 + 0.85 u^2) (5778/T)^1.5 capped at 0.95, blueshift from the
    cubic in T_eff; spot lines 30% deeper, no blueshift.  Gaussian lines.
    float32 arrays."""
    ln0, dln, n_pix, n_sun, centre, u, sigma = _cfg5_lines(seed)
    scale = 5778.0 / teff_k
    n = int(round(n_sun * scale**3))
    c, s = centre[:n], sigma[:n]
    depth = np.minimum((0.05 + 0.85 * u[:n] ** 2) * scale**1.5, 0.95)
    g = np.zeros(n)
    mu_b = 1.0 - 0.9 * np.arange(n_mu) / (n_mu - 1)
    cb = cb_law_ms(mu_b, amplitude_ms=float(cb_velocity_ms(teff_k)))
    jobs = [(ln0, dln, n_pix, c, depth, s, g, v) for v in cb]
    jobs.append((ln0, dln, n_pix, c, np.minimum(depth * 1.3, 0.99), s, g, 0.0))
    rows = list(pool.map(_render_row, jobs)) if pool is not None else [_render_row(j) for j in jobs]
    quiet = np.stack(rows[:n_mu]).astype(np.float32)
    spot = np.ascontiguousarray(np.broadcast_to(rows[n_mu], (n_mu, n_pix)), dtype=np.float32)
    return ln0, dln, mu_b, quiet, spot


def cfg5_mask(seed: int = 5):
    """CCF mask of the surrogate window: the deepest lines of the solar-T_eff
    list (up to 400), binary weights, 161 velocities from -20 km/s."""
    ln0, dln, n_pix, n_sun, centre, u, sigma = _cfg5_lines(seed)
    n = int(round(n_sun))
    mlam, _ = _select_mask_lines(centre[:n], 0.05 + 0.85 * u[:n] ** 2, sigma[:n], 400)
    return Mask(np.log(mlam), np.ones(len(mlam)), 0.41, -20.0, 0.25, 161)


def cfg5_star(teff_k, incl_deg, vsini_kms, spectra, n_grid: int = 300) -> StarInputs:
    """StarInputs of one grid star from cfg5_window_spectra's output."""
    ln0, dln, mu_b, quiet, spot = spectra
    return StarInputs(
        n_grid=n_grid, vsini_kms=float(vsini_kms), incl_deg=float(incl_deg), ld_u1=0.4, ld_u2=0.25,
        ln_lambda0=ln0, dln_lambda=dln, n_pix=quiet.shape[1], mu_bins=mu_b, spectra=[quiet, spot, None],
        precision=PREC_FP32, contrast_mode=CONTRAST_SCALAR, teff_k=float(teff_k), regions=[],
        phases=np.zeros(0), mask=None,
        name=f"cfg5 star T={teff_k:.0f} i={incl_deg:.0f} vsini={vsini_kms:.0f}",
    )


@dataclass
class MultiSpotSamples(SpotSamples):
    """SpotSamples whose spots each belong to a star of the grid: star[k]
    indexes (teff, incl, vsini) = (CFG5_TEFF[ti], CFG5_INCL[ii],
    CFG5_VSINI[vi]) with star = (ti * len(CFG5_INCL) + ii) * len(CFG5_VSINI) + vi."""

    star: np.ndarray = None

    def star_params(self, star):
        nv, ni = len(CFG5_VSINI), len(CFG5_INCL)
        star = np.asarray(star)
        return CFG5_TEFF[star // (ni * nv)], CFG5_INCL[(star // nv) % ni], CFG5_VSINI[star % nv]


def cfg5_multi_samples(n_spots: int, n_per: int = 8, seed: int = 5, teff_subset=None) -> MultiSpotSamples:
    """Single-spot samples as cfg5_samples, each spot on a star drawn
    uniformly from the grid (optionally only the T_eff values in
    teff_subset); spots are ordered by star."""
    base = cfg5_samples(n_spots, n_per, seed)
    rng = np.random.default_rng([seed, n_spots, n_per, 77])
    tis = np.arange(len(CFG5_TEFF)) if teff_subset is None else np.searchsorted(CFG5_TEFF, teff_subset)
    ti = tis[rng.integers(0, len(tis), n_spots)]
    ii = rng.integers(0, len(CFG5_INCL), n_spots)
    vi = rng.integers(0, len(CFG5_VSINI), n_spots)
    star = (ti * len(CFG5_INCL) + ii) * len(CFG5_VSINI) + vi
    o = np.argsort(star, kind="stable")  # spots grouped by star
    return MultiSpotSamples(base.lat_deg[o], base.lon_deg[o], base.radius[o], base.contrast[o], base.phases[o],
                            star=star[o])
