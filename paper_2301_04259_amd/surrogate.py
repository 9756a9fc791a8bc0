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
                  soap_surrogate_rv (CCF of the quiet-plus-basis expansion by
                  linearity, its fit, the members' first-order RV spread and
                  the gate); samples whose
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
from dataclasses import dataclass

import numpy as np

from . import (
    EFFECT_TOT,
    PREC_FP32,
    RV_DTYPE,
    SPOT,
    region_array,
    soap_active_spectra_jobs,
    soap_ccf_rv,
    soap_quiet_spectrum,
    soap_surrogate_create,
    soap_surrogate_rv,
    soap_surrogate_predict,
    soap_surrogate_train_step,
)

N_FEATURES = 7


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
    k = spots[starts]
    regions = region_array(SPOT, samples.lat_deg[k], samples.lon_deg[k], samples.radius[k], samples.contrast[k])
    roff = np.arange(len(starts) + 1, dtype=np.int32)
    poff = np.r_[starts, len(idx)].astype(np.int32)
    soap_active_spectra_jobs(ctx, regions, ph[idx], EFFECT_TOT, out[: len(idx)], region_offsets=roff,
                             phase_offsets=poff)
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

    def rv_weights(self, Yn, eps=0.05):
        """RMS over the rows of Yn (normalised coefficients, host [m][k]) of
        the RV change per unit change of each coefficient, by central
        differences through soap_ccf_linear_rv."""
        torch = self.torch
        from . import soap_ccf_linear_rv

        m, k = Yn.shape
        rows = np.repeat(np.asarray(Yn, np.float32)[:, None, :], 2 * k, axis=1)
        for j in range(k):
            rows[:, 2 * j, j] += eps
            rows[:, 2 * j + 1, j] -= eps
        rows = rows.reshape(-1, k)
        rv = torch.empty(len(rows) * RV_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        soap_ccf_linear_rv(self.ctx, torch.from_numpy(np.ascontiguousarray(rows)).cuda(), self.base_ccf,
                           self.basis_ccf, None, rv)
        r = np.frombuffer(rv.cpu().numpy().tobytes(), dtype=RV_DTYPE)["rv_kms"].reshape(m, k, 2)
        return np.sqrt(np.mean(((r[:, :, 0] - r[:, :, 1]) / (2 * eps)) ** 2, axis=0))

    def reweight(self, w):
        """Rescales the normalised coefficients by w / rms(w), so that the
        training loss weighs each coefficient by its RV sensitivity."""
        b = self.basis
        w = np.maximum(np.asarray(w, np.float64), 1e-6 * np.max(w))
        b.sigma = b.sigma * np.sqrt(np.mean(w * w)) / w
        self._build_ccf_tables()

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
        """Enqueues predict -> fused mean-CCF fit, member RV spread and gate
        for x_dev [n][features]."""
        n = bufs["n"]
        Y = bufs["Y"]
        soap_surrogate_predict(self.net, x_dev, Y[:n], Y[n:])
        soap_surrogate_rv(self.ctx, Y[:n], Y[n:], self.base_ccf, self.basis_ccf,
                          self.calib if calib is None else calib,
                          self.threshold_kms if threshold_kms is None else threshold_kms, bufs["rv_kms"],
                          bufs["fallback"], err_kms=bufs["err"], rv_out=bufs["rv"])

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


def build(ctx, mask, train, heldout, n_components=64, hidden=256, n_ensemble=4, epochs=100, batch=512,
          svd_subset=2048, seed=0, weighting="rv", log=None):
    """Data set, basis, training and gate calibration of a surrogate for the
    star of ctx (an FP32 context) from SpotSamples train / heldout.  Returns
    the model and a dict of what it took."""
    torch = _torch()
    say = log or (lambda *a: None)
    info = {}
    model = SurrogateModel(ctx, mask, n_components, hidden, n_ensemble, seed)
    F = torch.empty((train.n, ctx.n_pix), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t = __import__("time").perf_counter()
    synthesize(ctx, train, F)
    torch.cuda.synchronize()
    info["synth_s"] = __import__("time").perf_counter() - t
    say(f"synthesised {train.n} training spectra in {info['synth_s']:.2f} s")
    sub = np.sort(np.random.default_rng(seed).choice(train.n, min(svd_subset, train.n), replace=False))
    Fh = F[torch.from_numpy(sub).cuda()].cpu().numpy()
    mean, V = fit_basis(Fh, model.Q, n_components)
    del Fh
    model.install_projection(mean, V)
    coef = model.project(F).cpu().numpy()
    del F
    model.set_basis(mean, V, coef, norm="component")
    if weighting == "rv":
        sel = np.random.default_rng(seed + 1).choice(len(coef), min(512, len(coef)), replace=False)
        w = model.rv_weights(model.normalise(coef[sel]))
        model.reweight(w)
        info["rv_weights"] = [float(v) for v in w[:8]]
    X = sample_features(train)
    Y = model.normalise(coef)
    t = __import__("time").perf_counter()
    losses = model.train(X, Y, epochs, batch=batch, seed=seed)
    torch.cuda.synchronize()
    info["train_s"] = __import__("time").perf_counter() - t
    info["train_steps"] = epochs * (len(X) // batch)
    info["final_loss"] = losses[-1]
    say(f"trained {info['train_steps']} steps in {info['train_s']:.2f} s, loss {losses[-1]:.3g}")
    rvp = plain_rv(ctx, heldout, mask)["rv_kms"]
    n_ho = (heldout.n // 16) * 16
    err, spread = model.calibrate(heldout, np.arange(n_ho), rvp[:n_ho], model.alloc(n_ho))
    info["calib"] = model.calib
    info["heldout_err_cms"] = {"median": float(np.median(err) * 1e5), "p99": float(np.quantile(err, 0.99) * 1e5),
                               "max": float(err.max() * 1e5)}
    return model, info
