"""Cross-correlation function against a line mask (oracle, test infrastructure only).

Section 4.1: RVs are measured by cross-correlating each spectrum with a line
mask and fitting a Gaussian to the CCF.  The paper does not spell out the
CCF; the reading used here is the usual box-hole mask correlation:

* pixel m is a constant-flux bin spanning ln(lambda) in
  [ln lambda0 + (m - 1/2) dln, ln lambda0 + (m + 1/2) dln);
* mask line l (rest wavelength lambda_l, weight w_l) has, at trial velocity
  v_k, a hole spanning the wavelengths lambda_l (1 + f(v_k - h)) to
  lambda_l (1 + f(v_k + h)), with 1 + f the Doppler factor of Eq. 6 and h the
  hole half-width in velocity;
* CCF_k = sum_l w_l sum_m F_m * |bin_m intersect hole_l(v_k)| / dln, where
  only pixels that exist (0 <= m < P) contribute.
"""
from __future__ import annotations

import numpy as np

from .spectrum import doppler_factor


def velocity_grid(v0_kms: float, dv_kms: float, n_v: int) -> np.ndarray:
    return v0_kms + dv_kms * np.arange(n_v, dtype=np.float64)


def ccf(flux, ln_lambda0, dln, mask_ln_lambda, mask_weight, half_width_kms, v_kms) -> np.ndarray:
    flux = np.asarray(flux, dtype=np.float64)
    p = flux.shape[-1]
    v = np.asarray(v_kms, dtype=np.float64)
    lo = np.asarray(mask_ln_lambda)[:, None] + np.log(doppler_factor(v - half_width_kms))[None, :]
    hi = np.asarray(mask_ln_lambda)[:, None] + np.log(doppler_factor(v + half_width_kms))[None, :]
    # pixel coordinate in which bin m spans [m, m + 1)
    qlo = (lo - ln_lambda0) / dln + 0.5
    qhi = (hi - ln_lambda0) / dln + 0.5
    m0 = np.floor(qlo).astype(np.int64)
    span = int(np.max(np.ceil(qhi).astype(np.int64) - m0))
    w = np.asarray(mask_weight, dtype=np.float64)[:, None]
    out = np.zeros(flux.shape[:-1] + (len(v),), dtype=np.float64)
    for s in range(span + 1):
        m = m0 + s
        ov = np.minimum(qhi, m + 1.0) - np.maximum(qlo, m)
        ok = (ov > 0.0) & (m >= 0) & (m < p)
        ovw = np.where(ok, ov, 0.0) * w
        mc = np.clip(m, 0, p - 1)
        # sum over lines of F[..., m] * overlap * weight
        out += np.einsum("...lk,lk->...k", flux[..., mc], ovw)
    return out
