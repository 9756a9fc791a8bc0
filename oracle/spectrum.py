"""Disk-integrated spectra (oracle, test infrastructure only).

Follows, in FP64:

* Eq. 6: a cell moving at line-of-sight velocity v sees lambda' = lambda (1+f),
  1 + f = sqrt((1+beta)/(1-beta)), beta = v/c.
* Eqs. 9-11: the shifted spectrum (S_n at lambda'_n) is projected back onto
  the original grid: for output pixel m find n with
  lambda'_n <= lambda_m < lambda'_{n+1} and interpolate linearly in lambda
  (the "project back to the original wavelength grid" step of Algorithm 1,
  i.e. the gather form; the scatter of Algorithm 3 is a GPU implementation
  detail of the paper).  Outside the shifted grid the end value is held
  (reading: the paper says nothing about the ends).
* Algorithm 1: quiet integrated spectrum = sum over visible cells of
  A * I(mu) * S'_quiet,bin(cell).
* Algorithm 5 with Eqs. 1-4: per phase, cells owned by an active region use
  the differences
      flux  (Eq. 1): S'_q - C * S'_q
      bconv (Eq. 2): S'_q - S'_a
      tot   (Eq. 3): S'_q - C * S'_a
  and S_final = S_quiet - sum of the differences (Eq. 4).
* Section 4.3.1: the contrast C is either a scalar per region or, in the
  chromatic mode, the ratio of two Planck functions B_lambda(T_act) /
  B_lambda(T_eff) per pixel, with T_act = T_eff - dT_spot for spots and
  T_eff + dT_f(mu_b) for faculae (dT_f the facula law of section 4.3.3,
  evaluated at the bin's mu), or, in the array mode, a per-pixel array per
  (type, mu bin) given with the star (section 4.3.3, Eqs. 12-14: the limb
  brightening times the active-to-quiet SED ratio).  It multiplies the
  spectrum after the shift, on the common grid (Eqs. 3, 13 and 14 apply it to
  shifted spectra).

* Section 3.4 (differential rotation, DIFF_ROT = star.diff_rot, 0 when
  absent): each cell's velocity is scaled by omega(theta) / omega_0 and
  regions advance at their latitude's rate (see disk.py).

Three formulations are provided and pinned against each other:
``integrated_bruteforce`` walks the cells one by one exactly as Algorithms 1
and 5 do (for small grids); ``integrated`` sums the final spectrum directly
(no quiet-minus-difference step) with cells of equal velocity grouped (one
disk column under solid-body rotation, because the velocity depends on x
only; the cells of one exact velocity value under differential rotation);
``integrated_pixels`` evaluates the same per-cell sum at chosen pixels only,
for workloads too large for the full spectrum.
"""
from __future__ import annotations

import numpy as np

from . import disk

C_KMS = 299792.458
# second radiation constant h c / k_B in m K, from the exact SI 2019 values of
# h, c and k_B
C2_MK = 6.62607015e-34 * 299792458.0 / 1.380649e-23

TOT, FLUX, BCONV = 0, 1, 2
QUIET, SPOT, FACULA = 0, 1, 2


def wavelengths(ln_lambda0: float, dln: float, n_pix: int) -> np.ndarray:
    """lambda_m = exp(ln lambda0 + m dln) (log-uniform grid)."""
    return np.exp(ln_lambda0 + dln * np.arange(n_pix, dtype=np.float64))


def doppler_factor(v_kms):
    """1 + f(beta) = sqrt((1 + beta) / (1 - beta)), Eq. 6."""
    b = np.asarray(v_kms, dtype=np.float64) / C_KMS
    return np.sqrt((1.0 + b) / (1.0 - b))


class Shift:
    """Bracketing indices and interpolation factors of Eqs. 9-11 for one velocity."""

    def __init__(self, lam: np.ndarray, v_kms: float):
        self.lam = lam
        lam_s = lam * doppler_factor(v_kms)  # lambda'_n
        p = len(lam)
        n = np.searchsorted(lam_s, lam, side="right") - 1  # lambda'_n <= lambda_m
        self.lo = n < 0
        self.hi = n >= p - 1
        self.mid = ~(self.lo | self.hi)
        nm = n[self.mid]
        self.n = nm
        # Eq. 11: (lambda_m - lambda'_n) / (lambda'_{n+1} - lambda'_n)
        self.frac = (lam[self.mid] - lam_s[nm]) / (lam_s[nm + 1] - lam_s[nm])
        idx = np.nonzero(self.mid)[0]
        self._run = None
        if len(idx) and idx[-1] - idx[0] + 1 == len(idx) and np.all(np.diff(nm) == 1):
            self._run = (int(idx[0]), int(idx[-1]) + 1, int(nm[0]))

    def apply(self, s: np.ndarray) -> np.ndarray:
        s = np.asarray(s, dtype=np.float64)
        out = np.empty(len(self.lam), dtype=np.float64)
        nm = self.n
        if self._run is not None:
            # the bracketing indices of the interior are consecutive: same
            # arithmetic on slices instead of gathers
            a, b, n0 = self._run
            lo, hi = s[n0 : n0 + (b - a)], s[n0 + 1 : n0 + 1 + (b - a)]
            out[a:b] = (hi - lo) * self.frac + lo
        else:
            out[self.mid] = (s[nm + 1] - s[nm]) * self.frac + s[nm]
        out[self.lo] = s[0]
        out[self.hi] = s[-1]
        return out


    def accumulate(self, acc: np.ndarray, w: float, s: np.ndarray) -> None:
        """acc += w * S' (same arithmetic as apply, fewer temporaries)."""
        if self._run is None or self.lo[self._run[0]:].any() or self.hi[: self._run[1]].any():
            acc += w * self.apply(s)
            return
        a, b, n0 = self._run
        lo = s[n0 : n0 + (b - a)]
        t = s[n0 + 1 : n0 + 1 + (b - a)] - lo
        t *= self.frac
        t += lo
        t *= w
        acc[a:b] += t
        acc[:a] += w * s[0]
        acc[b:] += w * s[-1]


def shift_spectrum(s, lam, v_kms):
    """S'(lambda_m) of a spectrum S(lambda_n) Doppler shifted by v (Eqs. 6, 9-11)."""
    return Shift(lam, v_kms).apply(s)


def planck_ratio(lam_a, t_act, t_ref):
    """B_lambda(T_act) / B_lambda(T_ref) (section 4.3.1, the chromatic contrast)."""
    lam_m = np.asarray(lam_a, dtype=np.float64) * 1e-10
    return np.expm1(C2_MK / (lam_m * t_ref)) / np.expm1(C2_MK / (lam_m * t_act))


def facula_dt(mu, coef):
    """dT_f(mu) = a0 + a1 mu + a2 mu^2 (section 4.3.3)."""
    mu = np.asarray(mu, dtype=np.float64)
    return coef[0] + coef[1] * mu + coef[2] * mu * mu


def contrast_array(star, typ: int, b: int, lam):
    """Per-pixel contrast of surface type ``typ`` in mu bin ``b`` (chromatic
    or array mode), or None in scalar mode."""
    if star.contrast_mode == 0:
        return None
    if star.contrast_mode == 2:
        return np.asarray(star.contrast[typ][b], dtype=np.float64)
    if typ == SPOT:
        return planck_ratio(lam, star.teff_k - star.dt_spot_k, star.teff_k)
    return planck_ratio(lam, star.teff_k + facula_dt(star.mu_bins[b], star.dt_fac_coef), star.teff_k)


def _spec(star, typ, b):
    return np.asarray(star.spectra[typ][b], dtype=np.float64)


def _diff_rot(star) -> float:
    return float(getattr(star, "diff_rot", 0.0) or 0.0)


def _velocities(star, x, y, mu):
    """Per-cell line-of-sight velocity: solid body, or differential rotation."""
    a = _diff_rot(star)
    if a == 0.0:
        return disk.los_velocity(x, star.vsini_kms)
    return disk.cell_velocity(x, y, mu, star.vsini_kms, star.incl_deg, a)


def quiet_bruteforce(star) -> np.ndarray:
    """Algorithm 1, one cell at a time."""
    lam = wavelengths(star.ln_lambda0, star.dln_lambda, star.n_pix)
    _, _, x, y, mu = disk.disk_cells(star.n_grid)
    area = disk.cell_area(star.n_grid)
    inten = disk.limb_darkening(mu, star.ld_u1, star.ld_u2)
    bins = disk.mu_bin(mu, star.mu_bins)
    vel = _velocities(star, x, y, mu)
    out = np.zeros(star.n_pix)
    for c in range(len(x)):
        out += area * inten[c] * shift_spectrum(_spec(star, QUIET, bins[c]), lam, vel[c])
    return out


def integrated_bruteforce(star, phase: float, effect: int = TOT, regions=None) -> np.ndarray:
    """Algorithm 5 with Eqs. 1-4, one cell at a time: quiet disk minus the
    summed per-cell differences of the active cells."""
    regions = star.regions if regions is None else regions
    lam = wavelengths(star.ln_lambda0, star.dln_lambda, star.n_pix)
    _, _, x, y, mu = disk.disk_cells(star.n_grid)
    area = disk.cell_area(star.n_grid)
    inten = disk.limb_darkening(mu, star.ld_u1, star.ld_u2)
    bins = disk.mu_bin(mu, star.mu_bins)
    owner = disk.owner_map(x, y, mu, regions, phase, star.incl_deg, _diff_rot(star))
    vel = _velocities(star, x, y, mu)
    s_quiet = quiet_bruteforce(star)
    diff = np.zeros(star.n_pix)
    for c in np.nonzero(owner >= 0)[0]:
        reg = regions[owner[c]]
        b = bins[c]
        v = vel[c]
        w = area * inten[c]
        sq = w * shift_spectrum(_spec(star, QUIET, b), lam, v)
        sa = w * shift_spectrum(_spec(star, reg.type, b), lam, v)
        carr = contrast_array(star, reg.type, b, lam)
        cval = reg.contrast if carr is None else carr
        if effect == FLUX:
            d = sq - cval * sq  # Eq. 1
        elif effect == BCONV:
            d = sq - sa  # Eq. 2
        else:
            d = sq - cval * sa  # Eq. 3
        diff += d
    return s_quiet - diff  # Eq. 4


def integrated(star, phase: float, effect: int = TOT, regions=None) -> np.ndarray:
    """Final spectrum summed directly over the disk, cells grouped by column.

    Each visible cell contributes A * I * X'(cell), where X is its quiet
    spectrum or, for a cell owned by an active region, the active term that
    Eqs. 1-4 leave in place of the quiet one: C * S_a (tot), C * S_q (flux),
    S_a (bconv).  Cells of one column share one velocity, so their weights are
    summed per (source spectrum, contrast) before one shift per column.
    """
    regions = star.regions if regions is None else regions
    lam = wavelengths(star.ln_lambda0, star.dln_lambda, star.n_pix)
    ix, _, x, y, mu = disk.disk_cells(star.n_grid)
    area = disk.cell_area(star.n_grid)
    inten = disk.limb_darkening(mu, star.ld_u1, star.ld_u2)
    bins = disk.mu_bin(mu, star.mu_bins)
    owner = disk.owner_map(x, y, mu, regions, phase, star.incl_deg, _diff_rot(star))
    wcell = area * inten
    # per cell: the (source type, bin, contrast type or -1) its term uses and
    # its weight, then summed per (column, key)
    src_t = np.zeros(len(x), dtype=np.int64)
    con_t = np.full(len(x), -1, dtype=np.int64)
    w = wcell.copy()
    for r_idx, reg in enumerate(regions):
        sel = owner == r_idx
        scal = reg.contrast if star.contrast_mode == 0 else 1.0
        if effect == FLUX:
            con_t[sel] = reg.type
            w[sel] = wcell[sel] * scal
        elif effect == BCONV:
            src_t[sel] = reg.type
        else:
            src_t[sel] = reg.type
            con_t[sel] = reg.type
            w[sel] = wcell[sel] * scal
    nb = len(star.mu_bins)
    code = (src_t * nb + bins) * 4 + (con_t + 1)
    ncode = 3 * nb * 4
    if _diff_rot(star) == 0.0:
        # one velocity per disk column
        n = star.n_grid
        group = ix
        xs = disk.cell_centres(n)
        gvel = disk.los_velocity(xs, star.vsini_kms)
    else:
        # one group per distinct cell velocity
        gvel, group = np.unique(_velocities(star, x, y, mu), return_inverse=True)
        n = len(gvel)
    wsum = np.bincount(group * ncode + code, weights=w, minlength=n * ncode).reshape(n, ncode)
    acc = {}
    srcs = {}
    for col in np.nonzero(wsum.any(axis=1))[0]:
        sh = Shift(lam, gvel[col])
        for cd in np.nonzero(wsum[col])[0]:
            key = (int(cd // 4 // nb), int(cd // 4 % nb), int(cd % 4) - 1)
            if key[:2] not in srcs:
                srcs[key[:2]] = _spec(star, key[0], key[1])
            if key not in acc:
                acc[key] = np.zeros(star.n_pix)
            sh.accumulate(acc[key], wsum[col, cd], srcs[key[:2]])
    out = np.zeros(star.n_pix)
    for key, a in sorted(acc.items()):
        if key[2] >= 0 and star.contrast_mode != 0:
            out += contrast_array(star, key[2], key[1], lam) * a
        else:
            out += a
    return out


def integrated_pixels(star, phase: float, pixels, effect: int = TOT, regions=None) -> np.ndarray:
    """The final spectrum of ``integrated`` at the chosen output pixels only:
    every visible cell's term evaluated at each pixel m by Eqs. 9-11 (the
    bracketing n with lambda'_n <= lambda_m < lambda'_{n+1} found among the
    shifted wavelengths around m, end values held), times its weight and,
    for active cells, its contrast at m."""
    regions = star.regions if regions is None else regions
    pixels = np.asarray(pixels, dtype=np.int64)
    p = star.n_pix
    lam = wavelengths(star.ln_lambda0, star.dln_lambda, p)
    _, _, x, y, mu = disk.disk_cells(star.n_grid)
    area = disk.cell_area(star.n_grid)
    inten = disk.limb_darkening(mu, star.ld_u1, star.ld_u2)
    bins = disk.mu_bin(mu, star.mu_bins)
    owner = disk.owner_map(x, y, mu, regions, phase, star.incl_deg, _diff_rot(star))
    fac = doppler_factor(_velocities(star, x, y, mu))
    nb = len(star.mu_bins)
    # per cell: source row (type, bin), contrast kind and weight, as in integrated
    src_t = np.zeros(len(x), dtype=np.int64)
    con_t = np.full(len(x), -1, dtype=np.int64)
    w = area * inten
    for r_idx, reg in enumerate(regions):
        sel = owner == r_idx
        scal = reg.contrast if star.contrast_mode == 0 else 1.0
        if effect == FLUX:
            con_t[sel] = reg.type
            w[sel] = w[sel] * scal
        elif effect == BCONV:
            src_t[sel] = reg.type
        else:
            src_t[sel] = reg.type
            con_t[sel] = reg.type
            w[sel] = w[sel] * scal
    rows = np.zeros((3, nb, p))
    for t in range(3):
        if star.spectra[t] is not None:
            rows[t] = np.asarray(star.spectra[t], dtype=np.float64)
    row_of = src_t * nb + bins
    flat = rows.reshape(3 * nb, p)
    # contrast at the output pixels per (type, bin), 1 where none applies
    cons = np.ones((3, nb, len(pixels)))
    if star.contrast_mode != 0 and effect != BCONV:
        for t in (SPOT, FACULA):
            for b in range(nb):
                ca = contrast_array(star, t, b, lam)
                if ca is not None:
                    cons[t, b] = ca[pixels]
    half = int(np.ceil(np.max(np.abs(np.log(fac))) / star.dln_lambda)) + 3
    out = np.zeros(len(pixels))
    for i, m in enumerate(pixels):
        n0 = max(0, m - half)
        n1 = min(p - 1, m + half)
        cand = np.arange(n0, n1 + 1)
        lam_s = lam[cand][None, :] * fac[:, None]  # lambda'_n per cell
        k = (lam_s <= lam[m]).sum(axis=1) - 1  # index in cand of the last lambda'_n <= lambda_m
        n = n0 + k
        val = np.empty(len(x))
        lo = n < 0
        hi = n >= p - 1
        mid = ~(lo | hi)
        rm = row_of[mid]
        nm = n[mid]
        ls = lam_s[mid]
        km = k[mid]
        a = ls[np.arange(len(km)), km]
        b = ls[np.arange(len(km)), km + 1]
        frac = (lam[m] - a) / (b - a)
        s_lo = flat[rm, nm]
        s_hi = flat[rm, nm + 1]
        val[mid] = (s_hi - s_lo) * frac + s_lo
        val[lo] = flat[row_of[lo], 0]
        val[hi] = flat[row_of[hi], p - 1]
        cvec = np.where(con_t >= 0, cons[np.maximum(con_t, 0), bins, i], 1.0)
        out[i] = np.sum(w * cvec * val)
    return out


def quiet(star) -> np.ndarray:
    """Quiet integrated spectrum (Algorithm 1), column-grouped."""
    return integrated(star, 0.0, TOT, regions=[])
