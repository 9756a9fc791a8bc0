"""Stellar disk geometry (oracle, test infrastructure only).

Section 2.1 (and the caption of its disk figure): the visible disk is an
N x N grid of cells; each cell gets an intensity from a limb-darkening law and
a projected velocity from the rotation period, inclination and radius.  The
paper does not fix the law's form, the cell test or the cell weight; the
readings used here are:

* cell centres x_i = -1 + (2i+1)/N (and the same for y), in stellar radii;
* a cell is on the disk when its centre is: x^2 + y^2 < 1;
* mu = sqrt(1 - x^2 - y^2), cell weight A = (2/N)^2;
* quadratic limb darkening I(mu) = 1 - u1 (1 - mu) - u2 (1 - mu)^2;
* solid-body rotation: the line-of-sight velocity is v sin i * x, positive
  (receding) for x > 0.

Section 3.4 (differential rotation): the angular velocity depends on the
latitude theta, omega = omega_0 + omega_1 sin^2(theta).  The paper's
"omega_1 = DIFF_ROT * PROT" contradicts its own solar numbers; the
consistent reading is omega_1 = DIFF_ROT * omega_0 (-0.18 x 14.371 deg/day =
-2.587 deg/day).  A cell's velocity is then scaled by omega / omega_0:
v = v sin i * x * (1 + DIFF_ROT sin^2(theta)), with sin(theta) = y sin i +
mu cos i the cell's height along the rotation axis, and a region advances in
longitude at the rate of its own latitude: 360 deg * phase * (1 + DIFF_ROT
sin^2(lat)) per unit phase (phase counts equatorial rotations).

Section 4.3.2: each cell takes the local spectrum of the mu bin closest to
its own mu (ties go to the larger mu bin, i.e. the lower index).

Section 3.3 (Algorithm 5, the InfoMap): regions are written into the disk map
in list order, so where regions overlap the last one in the list owns the
cell (a spot listed after a facula replaces it; same-type overlaps count
once).  Region position replaces the Localize rotation matrices of
section 2.1 by the equivalent rotation of the region centre: longitude
advances by 360 deg per unit phase, the rotation axis is tilted by the
inclination, and a cell belongs to a region when the angle between the cell's
surface point and the region centre is at most the region's angular radius
alpha, with radius = sin(alpha).
"""
from __future__ import annotations

import numpy as np


def cell_centres(n: int) -> np.ndarray:
    """x_i = -1 + (2i+1)/N, i = 0..N-1."""
    i = np.arange(n, dtype=np.float64)
    return (2.0 * i + 1.0) / n - 1.0


def cell_area(n: int) -> float:
    return (2.0 / n) ** 2


def disk_cells(n: int):
    """All visible cells: (ix, iy, x, y, mu) arrays, row-major over (ix, iy)."""
    c = cell_centres(n)
    ix, iy = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = c[ix]
    y = c[iy]
    r2 = x * x + y * y
    vis = r2 < 1.0
    mu = np.sqrt(1.0 - r2[vis])
    return ix[vis], iy[vis], x[vis], y[vis], mu


def limb_darkening(mu, u1: float, u2: float):
    """I(mu) = 1 - u1 (1 - mu) - u2 (1 - mu)^2."""
    om = 1.0 - np.asarray(mu, dtype=np.float64)
    return 1.0 - u1 * om - u2 * om * om


def los_velocity(x, vsini_kms: float):
    """Solid-body rotation: v = v sin i * x (km/s), receding for x > 0."""
    return vsini_kms * np.asarray(x, dtype=np.float64)


def sin_latitude(y, mu, incl_deg: float):
    """Height of a surface point (x, y, mu) along the rotation axis, whose
    direction in the observer frame is (0, sin i, cos i)."""
    inc = np.deg2rad(incl_deg)
    return np.asarray(y, dtype=np.float64) * np.sin(inc) + np.asarray(mu, dtype=np.float64) * np.cos(inc)


def cell_velocity(x, y, mu, vsini_kms: float, incl_deg: float, diff_rot: float = 0.0):
    """Differential rotation (section 3.4): v = v sin i * x * (1 + DIFF_ROT
    sin^2(theta)); DIFF_ROT = 0 is solid-body rotation."""
    st = sin_latitude(y, mu, incl_deg)
    return vsini_kms * np.asarray(x, dtype=np.float64) * (1.0 + diff_rot * st * st)


def mu_bin(mu, mu_bins) -> np.ndarray:
    """Index of the closest mu bin; ties to the lower index."""
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    d = np.abs(mu[:, None] - np.asarray(mu_bins, dtype=np.float64)[None, :])
    return np.argmin(d, axis=1)


def region_centre(lat_deg: float, lon_deg: float, phase: float, incl_deg: float,
                  diff_rot: float = 0.0) -> np.ndarray:
    """Unit vector of a region centre in the observer frame (x right, y up,
    z towards the observer) at a rotation phase.

    Star frame: longitude psi = lon + 360 deg * phase * (1 + DIFF_ROT
    sin^2(lat)) (the region turns at its latitude's rate), latitude theta,
    (X, Y, Z) = (cos th sin psi, sin th, cos th cos psi), rotation axis +Y.
    Observer frame: the axis is tilted towards the observer by 90 deg - i:
    x = X, y = Y sin i - Z cos i, z = Y cos i + Z sin i.
    """
    th = np.deg2rad(lat_deg)
    sl = np.sin(th)
    psi = np.deg2rad(lon_deg + 360.0 * phase * (1.0 + diff_rot * sl * sl))
    inc = np.deg2rad(incl_deg)
    X = np.cos(th) * np.sin(psi)
    Y = np.sin(th)
    Z = np.cos(th) * np.cos(psi)
    return np.array([X, Y * np.sin(inc) - Z * np.cos(inc), Y * np.cos(inc) + Z * np.sin(inc)])


def owner_map(x, y, mu, regions, phase: float, incl_deg: float, diff_rot: float = 0.0) -> np.ndarray:
    """InfoMap: index of the last listed region covering each cell, else -1."""
    x = np.asarray(x, dtype=np.float64)
    owner = np.full(x.shape, -1, dtype=np.int64)
    for r_idx, reg in enumerate(regions):
        c = region_centre(reg.lat_deg, reg.lon_deg, phase, incl_deg, diff_rot)
        cos_a = np.sqrt(1.0 - reg.radius * reg.radius)
        dot = x * c[0] + y * c[1] + mu * c[2]
        owner[dot >= cos_a] = r_idx
    return owner
