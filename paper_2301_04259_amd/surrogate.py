"""Surrogate driver: data set from the full synthesis, PCA basis, training,
and gated inference (argument marshalling and host bookkeeping around the
library's kernels).

Pipeline (the synthesis it stands in for: Algorithm 5, Eqs. 1-4; its RV:
section 4.1):

  synthesize      runs soap_active_spectra_jobs over the single-spot samples and
                  keeps the spectra F (device, float32)
  fit_basis       offline: mean and the first k principal axes of the
                  differences F - Q from an FP64 SVD of a subset (host), then
                  per-component normalisation of the projected coefficients
  train           Adam steps of every ensemble member on shuffled batches
                  (soap_surrogate_train_step)
  calibrate       on held-out samples with known full-synthesis RVs, the
                  factor that turns the members' RV spread into a predicted
                  error bound (a quantile of |error| / spread)
  rv              surrogate RVs of a batch: soap_surrogate_predict ->
                  soap_ccf_linear_rv (CCF of the quiet-plus-basis expansion,
                  by linearity) -> soap_surrogate_gate; samples whose
                  predicted error is not below the threshold go through the
                  full synthesis (soap_active_spectra_jobs + soap_ccf_rv)

The input features of a sample are its spot latitude, the sine and cosine of
its longitude at the observed phase (longitude + 360 deg x phase: the star
looks the same for equal values of that sum), the same two scaled by the
cosine of the latitude (for an equator-on star, the spot centre's position
across the disk and its mu), its radius and its contrast, each scaled to
about unit range.
"""
from __future__ import annotations

import math
from collections import namedtuple
from dataclasses import dataclass

import numpy as np

from . import (
    EFFECT_TOT,
    PREC_FP32,
    RV_DTYPE,
    SPOT,
    soap_active_spectra_jobs,
    soap_ccf_linear_rv,
    soap_ccf_rv,
    soap_quiet_spectrum,
    soap_surrogate_create,
    soap_surrogate_gate,
    soap_surrogate_predict,
    soap_surrogate_train_step,
)

N_FEATURES = 7

Region = namedtuple("Region", "type lat_deg lon_deg radius contrast")


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the surrogate driver needs a GPU")
    return torch


def features(lat_deg, lon_deg, radius, contrast, phase):
    """float32 [n][7] inputs of the network (see the module docstring)."""
    lat = np.deg2rad(np.asarray(lat_deg, np.float64))
    th = np.deg2rad(np.asarray(lon_deg, np.float64) + 360.0 * np.asarray(phase, np.float64))
    x = np.stack(
        [
            lat / np.deg2rad(60.0),
            np.sin(th),
            np.cos(th),
            np.cos(lat) * np.sin(th),
            np.cos(lat) * np.cos(th),
            (np.asarray(radius, np.float64) - 0.055) / 0.045,
            (np.asarray(contrast, np.float64) - 0.6) / 0.3,
        ],
        axis=-1,
    )
    return np.ascontiguousarray(x, dtype=np.float32)


def sample_features(samples, idx=None):
    """Features of samples (a SpotSamples), optionally of the indices idx."""
    n_per = samples.n_per
    i = np.arange(samples.n) if idx is None else np.asarray(idx)
    k = i // n_per
    return features(samples.lat_deg[k], samples.lon_deg[k], samples.radius[k], samples.contrast[k],
                    samples.phases.reshape(-1)[i])


def _region(samples, k):
    return Region(SPOT, float(samples.lat_deg[k]), float(samples.lon_deg[k]), float(samples.radius[k]),
                  float(samples.contrast[k]))


def synthesize(ctx, samples, out, idx=None):
    """Full synthesis of samples (all, or the sorted indices idx) into out
    [n][n_pix] (device): one soap_active_spectra_jobs call, one job per spot
    with the phases of its selected samples."""
    n_per = samples.n_per
    idx = np.arange(samples.n) if idx is None else np.asarray(idx)
    if len(idx) == 0:
        return out
    spots = idx // n_per
    starts = np.flatnonzero(np.r_[True, spots[1:] != spots[:-1]])
    ends = np.r_[starts[1:], len(idx)]
    ph = samples.phases.reshape(-1)
    regions = [[_region(samples, int(spots[a]))] for a in starts]
    phases = [ph[idx[a:b]] for a, b in zip(starts, ends)]
    soap_active_spectra_jobs(ctx, regions, phases, EFFECT_TOT, out[: len(idx)])
    return out


def plain_rv(ctx, samples, mask, idx=None, chunk=4096):
    """RVs of samples (or of the sorted indices idx) by the full synthesis:
    host RV_DTYPE records."""
    torch = _torch()
    idx = np.arange(samples.n) if idx is None else np.asarray(idx)
    rv = np.zeros(len(idx), dtype=RV_DTYPE)
    if len(idx) == 0:
        return rv
    dt = torch.float32 if ctx.precision == PREC_FP32 else torch.float64
    buf = torch.empty((min(chunk, len(idx)), ctx.n_pix), dtype=dt, device="cuda")
    for a in range(0, len(idx), chunk):
        b = min(len(idx), a + chunk)
        synthesize(ctx, samples, buf[: b - a], idx[a:b])
        part = np.zeros(b - a, dtype=RV_DTYPE)
        soap_ccf_rv(ctx, buf[: b - a], mask, rv_out=part, n_spec=b - a)
        rv[a:b] = part
    return rv


@dataclass
class Basis:
    """PCA basis of F - Q: mean [P] and V [P][k] (float64 host copies), and
    the coefficient normalisation mu, sigma [k]."""

    mean: np.ndarray
    V: np.ndarray
    mu: np.ndarray
    sigma: np.ndarray


def quiet(ctx):
    """Quiet integrated spectrum (host float64)."""
    q = np.zeros(ctx.n_pix, dtype=ctx.dtype)
    soap_quiet_spectrum(ctx, q)
    return q.astype(np.float64)


def fit_basis(F_host_subset, Q, k):
    """Offline principal axes of F - Q from a host subset (FP64 SVD)."""
    D = np.asarray(F_host_subset, np.float64) - Q
    mean = D.mean(axis=0)
    _, _, vt = np.linalg.svd(D - mean, full_matrices=False)
    V = np.ascontiguousarray(vt[:k].T)
    return mean, V


class SurrogateModel:
    """Trained surrogate of one star: network, basis, linear CCF tables and
    the gate's calibration.  Device tables live on the current GPU."""

    def __init__(self, ctx, mask, n_components=64, hidden=256, n_ensemble=4, seed=0):
        self.torch = _torch()
        self.ctx, self.mask = ctx, mask
        self.k, self.hidden, self.n_ens = int(n_components), int(hidden), int(n_ensemble)
        self.net = soap_surrogate_create(N_FEATURES, self.hidden, self.k, self.n_ens, seed)
        self.Q = quiet(ctx)
        self.basis = None
        self.calib = 1.0
        self.threshold_kms = 1e-4  # 10 cm/s

    # -- data ---------------------------------------------------------------
    def project(self, F_dev):
        """Raw PCA coefficients [n][k] (device, float32) of spectra F."""
        torch = self.torch
        from . import soap_pca_project

        n = int(F_dev.shape[0])
        coef = torch.empty((n, self.k), dtype=torch.float32, device="cuda")
        soap_pca_project(F_dev, self._centre_dev, self._V_dev, coef)
        return coef

    def set_basis(self, mean, V, coef_train, norm="global"):
        """Installs the basis and the normalisation of the training
        coefficients (host [n][k]): centred, then divided by their own
        standard deviations (norm="component") or all by the largest one
        (norm="global", which keeps the loss proportional to the spectral
        error)."""
        c = np.asarray(coef_train, np.float64)
        mu = c.mean(axis=0)
        sd = c.std(axis=0)
        if norm == "global":
            sd = np.full_like(sd, sd.max())
        sd = np.where(sd > 0, sd, 1.0)
        self.basis = Basis(np.asarray(mean, np.float64), np.asarray(V, np.float64), mu, sd)
        self._build_ccf_tables()
        return mu, sd

    def install_projection(self, mean, V):
        """Device arrays used by project(): centre = Q + mean, V (float32)."""
        torch = self.torch
        self._centre_dev = torch.from_numpy((self.Q + mean).astype(np.float32)).cuda()
        self._V_dev = torch.from_numpy(np.ascontiguousarray(V, dtype=np.float32)).cuda()

    def _build_ccf_tables(self):
        """CCF of F0 = Q + mean + V mu and of B_k = sigma_k V_k, so that the
        CCF of a prediction y is base + y @ basis."""
        torch = self.torch
        b = self.basis
        f0 = self.Q + b.mean + b.V @ b.mu
        rows = np.concatenate([f0[None, :], (b.V * b.sigma[None, :]).T], axis=0)
        dt = torch.float32 if self.ctx.precision == PREC_FP32 else torch.float64
        rows_dev = torch.from_numpy(np.ascontiguousarray(rows).astype(self.ctx.dtype)).to("cuda", dt)
        n_v = int(self.mask.n_v)
        ccf = torch.empty((rows.shape[0], n_v), dtype=torch.float64, device="cuda")
        soap_ccf_rv(self.ctx, rows_dev, self.mask, ccf_out=ccf, n_spec=rows.shape[0])
        self.base_ccf = ccf[0].contiguous()
        self.basis_ccf = ccf[1:].contiguous()

    def normalise(self, coef_host):
        b = self.basis
        return ((np.asarray(coef_host, np.float64) - b.mu) / b.sigma).astype(np.float32)

    # -- training -----------------------------------------------------------
    def train(self, X, Y, epochs, batch=512, lr=2e-3, lr_final=1e-4, seed=0, log=None):
        """Adam over shuffled batches (X [n][5], Y [n][k] normalised, host
        float32).  The learning rate decays geometrically from lr to
        lr_final.  Returns the per-epoch mean losses."""
        torch = self.torch
        rng = np.random.default_rng(seed)
        n = (len(X) // batch) * batch
        steps = max(1, epochs * (n // batch))
        g = (lr_final / lr) ** (1.0 / steps)
        losses, step = [], 0
        for ep in range(epochs):
            perm = rng.permutation(len(X))[:n]
            xd = torch.from_numpy(np.ascontiguousarray(X[perm])).cuda()
            yd = torch.from_numpy(np.ascontiguousarray(Y[perm])).cuda()
            tot = 0.0
            nb = n // batch
            for j in range(nb):
                want = j == nb - 1
                l = soap_surrogate_train_step(self.net, xd[j * batch:(j + 1) * batch], yd[j * batch:(j + 1) * batch],
                                              lr * g**step, want_loss=want)
                step += 1
                if want:
                    tot = l
            losses.append(tot)
            if log:
                log(f"epoch {ep} loss {tot:.4g}")
        return losses

    # -- inference ----------------------------------------------------------
    def alloc(self, n):
        """Device buffers for surrogate_rv on n samples (n a multiple of 16)."""
        torch = self.torch
        E = self.n_ens
        return dict(
            Y=torch.empty(((1 + E) * n, self.k), dtype=torch.float32, device="cuda"),
            rv=torch.empty(((1 + E) * n * RV_DTYPE.itemsize,), dtype=torch.uint8, device="cuda"),
            rv_kms=torch.empty((n,), dtype=torch.float64, device="cuda"),
            err=torch.empty((n,), dtype=torch.float64, device="cuda"),
            fallback=torch.empty((n,), dtype=torch.int32, device="cuda"),
            n=n,
        )

    def surrogate_rv(self, x_dev, bufs, calib=None, threshold_kms=None):
        """Enqueues predict -> linear CCF fits -> gate for x_dev [n][5]."""
        n = bufs["n"]
        Y = bufs["Y"]
        soap_surrogate_predict(self.net, x_dev, Y[:n], Y[n:])
        soap_ccf_linear_rv(self.ctx, Y, self.base_ccf, self.basis_ccf, None, bufs["rv"])
        soap_surrogate_gate(bufs["rv"], n, self.n_ens, self.calib if calib is None else calib,
                            self.threshold_kms if threshold_kms is None else threshold_kms, bufs["rv_kms"],
                            bufs["fallback"], err_kms=bufs["err"])

    def rv(self, samples, idx, bufs, threshold_kms=None):
        """Gated RVs (km/s, host float64) of samples[idx]; idx sorted, its
        length a multiple of 16.  Returns (rv, fallback flags, predicted
        errors)."""
        torch = self.torch
        x = torch.from_numpy(sample_features(samples, idx)).cuda()
        self.surrogate_rv(x, bufs, threshold_kms=threshold_kms)
        fb = bufs["fallback"].cpu().numpy().astype(bool)
        out = bufs["rv_kms"].cpu().numpy().copy()
        err = bufs["err"].cpu().numpy().copy()
        sel = np.asarray(idx)[fb]
        if len(sel):
            out[fb] = plain_rv(self.ctx, samples, self.mask, sel)["rv_kms"]
        return out, fb, err

    def calibrate(self, samples, idx, rv_plain_kms, bufs, threshold_kms=None, margin=1.25):
        """Sets calib from held-out samples with known full-synthesis RVs:
        the smallest factor for which every held-out sample whose surrogate
        error reaches the threshold is predicted to reach it too (times a
        margin; the 99th percentile of |error| / spread when no sample
        reaches the threshold).  Returns (|error|, spread) in km/s."""
        torch = self.torch
        thr = self.threshold_kms if threshold_kms is None else threshold_kms
        x = torch.from_numpy(sample_features(samples, idx)).cuda()
        self.surrogate_rv(x, bufs, calib=1.0, threshold_kms=math.inf)
        spread = np.maximum(bufs["err"].cpu().numpy(), 1e-12)
        err = np.abs(bufs["rv_kms"].cpu().numpy() - rv_plain_kms)
        bad = err >= thr
        if bad.any():
            self.calib = float(margin * np.max(thr / spread[bad]))
        else:
            self.calib = float(np.quantile(err / spread, 0.99))
        return err, spread
