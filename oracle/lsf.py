"""Resolution lowering to the instrument's line-spread function (oracle, test
infrastructure only).

Algorithm 2 and Algorithm 5 end by lowering the resolution of each final
spectrum to that of the spectrograph (HARPS-N, R = 115000).  The paper does
not spell the operation out; the reading here:

* the line-spread function is a Gaussian whose full width at half maximum is
  lambda / R, i.e. 1/R in ln(lambda), so on the log-uniform grid its width is
  the same at every pixel: sigma = 1 / (R dln 2 sqrt(2 ln 2)) pixels;
* the kernel is that Gaussian sampled at whole-pixel offsets k, |k| <= K with
  K = ceil(4 sigma), and normalised to sum 1;
* out[m] = sum_k w_k F[m - k], with source indices held inside [0, P - 1]
  (end values held, as for the Doppler shift).

This is written as the plain sum over offsets, one shifted copy at a time.
"""
from __future__ import annotations

import math

import numpy as np


def sigma_pixels(resolution: float, dln: float) -> float:
    """Standard deviation of the line-spread function in pixels."""
    return 1.0 / (resolution * dln * 2.0 * math.sqrt(2.0 * math.log(2.0)))


def kernel(resolution: float, dln: float) -> np.ndarray:
    """w_k for k = -K .. K, K = ceil(4 sigma), normalised to sum 1."""
    s = sigma_pixels(resolution, dln)
    k_max = int(math.ceil(4.0 * s))
    k = np.arange(-k_max, k_max + 1, dtype=np.float64)
    w = np.exp(-0.5 * (k / s) ** 2)
    return w / w.sum()


def lower_resolution(flux, resolution: float, dln: float) -> np.ndarray:
    """out[..., m] = sum_k w_k flux[..., clamp(m - k)] over the last axis."""
    f = np.asarray(flux, dtype=np.float64)
    w = kernel(resolution, dln)
    k_max = (len(w) - 1) // 2
    p = f.shape[-1]
    out = np.zeros_like(f)
    m = np.arange(p)
    for i, wk in enumerate(w):
        k = i - k_max
        src = np.clip(m - k, 0, p - 1)
        out += wk * f[..., src]
    return out
