"""Surrogate driver: data set from the full synthesis, PCA basis, training,
and gated inference (argument marshalling and host bookkeeping around the
library's kernels).

Pipeline (the synthesis it stands in for: Algorithm 5, Eqs. 1-4; its RV:
section 4.1):

  synthesize      runs soap_active_spectra_jobs over the single-spot samples
                  of each star (one context per star) and keeps the spectra F
                  (device, float32)
  fit_basis       offline: mean and the first k principal axes of the
                  differences F - Q (Q the sample's own star's quiet
                  spectrum) from an FP64 SVD of a subset (host), then
                  per-component normalisation of the projected coefficients
  train           Adam steps of every ensemble member on shuffled batches
                  (soap_surrogate_train_step)
  calibrate       on held-out samples with known full-synthesis RVs, the
                  factor that turns the members' RV spread into a predicted
                  error bound
  rv              surrogate RVs of a batch: soap_surrogate_predict ->
                  soap_surrogate_rv (CCF of the star's quiet-plus-basis
                  expansion by linearity, its fit, the members' first-order
                  RV spread and the gate); samples whose predicted error is
                  not below the threshold go through the full synthesis
                  (soap_active_spectra_jobs + soap_ccf_rv)

Stars: a `Stars` set maps star ids to contexts that share one wavelength
window and one mask (the stars differ in T_eff, inclination and v sin i).
Samples are SpotSamples (one star, id 0) or MultiSpotSamples (a star id per
spot, spots ordered by star so that any sorted subset is grouped by star).

Input features of a sample: spot latitude; sine and cosine of its longitude
at the observed phase (longitude + 360 deg x phase: the star looks the same
for equal values of that sum); the spot centre's position across the disk,
along the projected axis and towards the observer for the star's
inclination; radius; contrast; T_eff, inclination and v sin i of the star;
each scaled to about unit range.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import (
    EFFECT_TOT,
    PREC_FP32,
    RV_DTYPE,
    SPOT,
    region_array,
    soap_active_spectra_jobs,
    soap_active_spectra_multi_arrays,
    soap_ccf_rv,
    soap_quiet_spectrum,
    soap_surrogate_create,
    soap_surrogate_features,
    soap_surrogate_predict,
    soap_surrogate_rv,
    soap_surrogate_train_step,
)

N_FEATURES = 12


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the surrogate driver needs a GPU")
    return torch


def features(lat_deg, lon_deg, radius, contrast, phase, teff_k, incl_deg, vsini_kms):
    """float32 [n][12] inputs of the network (see the module docstring)."""
    lat = np.deg2rad(np.asarray(lat_deg, np.float64))
    th = np.deg2rad(np.asarray(lon_deg, np.float64) + 360.0 * np.asarray(phase, np.float64))
    inc = np.deg2rad(np.asarray(incl_deg, np.float64))
    cl = np.cos(lat)
    x = cl * np.sin(th)
    y = np.sin(lat) * np.sin(inc) - cl * np.cos(th) * np.cos(inc)
    z = np.sin(lat) * np.cos(inc) + cl * np.cos(th) * np.sin(inc)
    f = np.stack(
        [
            lat / np.deg2rad(60.0),
            np.sin(th),
            np.cos(th),
            x,
            y,
            z,
            (np.asarray(radius, np.float64) - 0.055) / 0.045,
            (np.asarray(contrast, np.float64) - 0.6) / 0.3,
            (np.asarray(teff_k, np.float64) - 5500.0) / 1000.0,
            (np.rad2deg(inc) - 60.0) / 30.0,
            (np.asarray(vsini_kms, np.float64) - 3.0) / 2.0,
            np.ones_like(lat),
        ],
        axis=-1,
    )
    return np.ascontiguousarray(f, dtype=np.float32)


class Stars:
    """Contexts of the stars of a data set: ids -> context and
    (T_eff, inclination, v sin i).  All share the wavelength window."""

    def __init__(self):
        self.ids, self.ctxs, self.params = [], [], []
        self.row = {}
        self._lut = None  # (sorted ids, their rows), rebuilt after add

    def add(self, star_id, ctx, teff_k, incl_deg, vsini_kms):
        self.row[int(star_id)] = len(self.ids)
        self.ids.append(int(star_id))
        self.ctxs.append(ctx)
        self.params.append((float(teff_k), float(incl_deg), float(vsini_kms)))
        self._lut = None
        self._pa = None

    def handle_array(self):
        """Context handle per row, uint64."""
        if getattr(self, "_ha", None) is None or len(self._ha) != len(self.ctxs):
            self._ha = np.array([c.handle.value for c in self.ctxs], dtype=np.uint64)
        return self._ha

    def param_array(self):
        """(T_eff, inclination, v sin i) per row, float64 [rows][3]."""
        if getattr(self, "_pa", None) is None or len(self._pa) != len(self.params):
            self._pa = np.asarray(self.params, np.float64).reshape(-1, 3)
        return self._pa

    @property
    def ref(self):
        return self.ctxs[0]

    def rows(self, star_ids):
        """Row of each star id (KeyError for an id not added)."""
        if self._lut is None:
            ids = np.fromiter(self.row.keys(), dtype=np.int64, count=len(self.row))
            rows = np.fromiter(self.row.values(), dtype=np.int32, count=len(self.row))
            order = np.argsort(ids, kind="stable")
            self._lut = (ids[order], rows[order])
        ids, rows = self._lut
        s = np.asarray(star_ids, dtype=np.int64).reshape(-1)
        if len(ids) == 0:
            if len(s):
                raise KeyError(int(s[0]))
            return np.zeros(0, np.int32)
        pos = np.minimum(np.searchsorted(ids, s), len(ids) - 1)
        bad = ids[pos] != s
        if bad.any():
            raise KeyError(int(s[np.flatnonzero(bad)[0]]))
        return rows[pos]


def single_star(ctx, teff_k=5778.0):
    s = Stars()
    st = ctx.star
    s.add(0, ctx, teff_k, st.incl_deg, st.vsini_kms)
    return s


def sample_stars(samples, idx):
    """Star id of each sample (0 for one-star sample sets)."""
    star = getattr(samples, "star", None)
    k = np.asarray(idx) // samples.n_per
    return np.zeros(len(k), np.int64) if star is None else np.asarray(star)[k]


def sample_features(stars, samples, idx=None):
    i = np.arange(samples.n) if idx is None else np.asarray(idx)
    k = i // samples.n_per
    p = np.asarray(stars.params)[stars.rows(sample_stars(samples, i))]
    return features(samples.lat_deg[k], samples.lon_deg[k], samples.radius[k], samples.contrast[k],
                    samples.phases.reshape(-1)[i], p[:, 0], p[:, 1], p[:, 2])


def sample_raw(stars, samples, idx=None, rows=None):
    """Raw descriptions [n][8] (float64) of samples[idx] for
    soap_surrogate_features: spot lat, lon, radius, contrast, phase and the
    star's T_eff, inclination, v sin i (rows: the samples' star rows, if
    already known)."""
    i = np.arange(samples.n) if idx is None else np.asarray(idx)
    k = i // samples.n_per
    if rows is None:
        rows = stars.rows(sample_stars(samples, i))
    out = np.empty((len(i), 8), np.float64)
    out[:, 0] = samples.lat_deg[k]
    out[:, 1] = samples.lon_deg[k]
    out[:, 2] = samples.radius[k]
    out[:, 3] = samples.contrast[k]
    out[:, 4] = samples.phases.reshape(-1)[i]
    out[:, 5:8] = stars.param_array()[rows]
    return out


def _groups(keys):
    keys = np.asarray(keys)
    starts = np.flatnonzero(np.r_[True, keys[1:] != keys[:-1]])
    return starts, np.r_[starts[1:], len(keys)]


def synthesize(stars, samples, out, idx=None):
    """Full synthesis of samples (all, or the sorted indices idx) into out
    [n][n_pix] (device).  One star: one soap_active_spectra_jobs call, one job
    per spot with the phases of its selected samples.  Several stars: one
    soap_active_spectra_multi call, one configuration per spot (its star's
    context, its phases, its rows of out)."""
    n_per = samples.n_per
    idx = np.arange(samples.n) if idx is None else np.asarray(idx)
    if len(idx) == 0:
        return out
    sid = sample_stars(samples, idx)
    ph = samples.phases.reshape(-1)
    starts_star, _ = _groups(sid)
    if len(starts_star) > 1:
        spots = idx // n_per
        sst, _ = _groups(spots)
        k = spots[sst]
        handles = stars.handle_array()[stars.rows(sid[sst])]
        regions = region_array(SPOT, samples.lat_deg[k], samples.lon_deg[k], samples.radius[k], samples.contrast[k])
        roff = np.arange(len(sst) + 1, dtype=np.int32)
        poff = np.r_[sst, len(idx)].astype(np.int32)
        row_bytes = out.shape[1] * out.element_size()
        assert out.is_contiguous()
        ptrs = np.uint64(out.data_ptr()) + sst.astype(np.uint64) * np.uint64(row_bytes)
        for a in range(0, len(sst), 65536):  # the call takes at most 65536 configurations
            b = min(len(sst), a + 65536)
            soap_active_spectra_multi_arrays(handles[a:b], regions[a:b], roff[a:b + 1] - roff[a],
                                             ph[idx[poff[a]:poff[b]]], poff[a:b + 1] - poff[a], EFFECT_TOT,
                                             ptrs[a:b])
        return out
    for a0, b0 in zip(*_groups(sid)):
        ctx = stars.ctxs[stars.row[int(sid[a0])]]
        sub = idx[a0:b0]
        spots = sub // n_per
        starts, _ = _groups(spots)
        k = spots[starts]
        regions = region_array(SPOT, samples.lat_deg[k], samples.lon_deg[k], samples.radius[k],
                               samples.contrast[k])
        roff = np.arange(len(starts) + 1, dtype=np.int32)
        poff = np.r_[starts, len(sub)].astype(np.int32)
        soap_active_spectra_jobs(ctx, regions, ph[sub], EFFECT_TOT, out[a0:b0], region_offsets=roff,
                                 phase_offsets=poff)
    return out


def plain_rv(stars, samples, mask, idx=None, chunk=4096):
    """RVs of samples (or of the sorted indices idx) by the full synthesis:
    host RV_DTYPE records.  The CCF and fit of every chunk run on the
    reference context (the stars share the wavelength window)."""
    torch = _torch()
    if not isinstance(stars, Stars):
        stars = single_star(stars)
    idx = np.arange(samples.n) if idx is None else np.asarray(idx)
    rv = np.zeros(len(idx), dtype=RV_DTYPE)
    if len(idx) == 0:
        return rv
    ref = stars.ref
    dt = torch.float32 if ref.precision == PREC_FP32 else torch.float64
    buf = torch.empty((min(chunk, len(idx)), ref.n_pix), dtype=dt, device="cuda")
    for a in range(0, len(idx), chunk):
        b = min(len(idx), a + chunk)
        synthesize(stars, samples, buf[: b - a], idx[a:b])
        part = np.zeros(b - a, dtype=RV_DTYPE)
        soap_ccf_rv(ref, buf[: b - a], mask, rv_out=part, n_spec=b - a)
        rv[a:b] = part
    return rv


def calib_for_miss_rate(err, spread, thr, alpha):
    """The gate factor c that accepts the most samples (c * spread < thr)
    while at most a fraction alpha of the accepted ones have err >= thr.
    Sample i is accepted iff c < t_i = thr / spread_i, so the candidate
    accepted sets are the m samples of largest t; c is then the (m+1)-th
    largest t, moved to the geometric midpoint between the m-th and the
    (m+1)-th so that rounding of c * spread cannot move the boundary (half
    the smallest t when every sample is accepted, twice the largest when none
    can be)."""
    err = np.asarray(err, np.float64)
    t = thr / np.maximum(np.asarray(spread, np.float64), 1e-300)
    order = np.argsort(-t, kind="stable")
    bad = np.cumsum(err[order] >= thr)
    m = np.arange(1, len(t) + 1)
    ok = np.flatnonzero(bad <= alpha * m)
    if len(ok) == 0:
        return float(t[order[0]]) * 2.0
    mm = int(ok[-1]) + 1
    if mm == len(t):
        return float(0.5 * t[order[-1]])
    return float(np.sqrt(t[order[mm - 1]] * t[order[mm]]))


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


def fit_basis(D_host_subset, k):
    """Offline principal axes of differences D = F - Q (FP64 SVD).  LAPACK's
    divide-and-conquer SVD can fail to converge on some inputs; the QR-based
    one is tried then."""
    D = np.asarray(D_host_subset, np.float64)
    if not np.all(np.isfinite(D)):
        raise ValueError("fit_basis: differences are not finite")
    mean = D.mean(axis=0)
    try:
        _, _, vt = np.linalg.svd(D - mean, full_matrices=False)
    except np.linalg.LinAlgError:
        import scipy.linalg

        _, _, vt = scipy.linalg.svd(D - mean, full_matrices=False, lapack_driver="gesvd")
    return mean, np.ascontiguousarray(vt[:k].T)


class SurrogateModel:
    """Trained surrogate of a set of stars: network, basis, linear CCF
    tables and the gate's calibration.  Device tables live on the current
    GPU."""

    def __init__(self, stars, mask, n_components=64, hidden=256, n_ensemble=4, seed=0):
        self.torch = _torch()
        if not isinstance(stars, Stars):
            stars = single_star(stars)
        self.stars, self.mask = stars, mask
        self.ctx = stars.ref
        self.k, self.hidden, self.n_ens = int(n_components), int(hidden), int(n_ensemble)
        self.net = soap_surrogate_create(N_FEATURES, self.hidden, self.k, self.n_ens, seed)
        self.Q = np.stack([quiet(c) for c in stars.ctxs])  # [rows][P]
        self.basis = None
        self.calib = 1.0
        self.threshold_kms = 1e-4  # 10 cm/s

    # -- data ---------------------------------------------------------------
    def differences_host(self, F_dev, star_ids):
        """F - Q of device spectra (host float64), for the offline SVD."""
        return F_dev.cpu().numpy().astype(np.float64) - self.Q[self.stars.rows(star_ids)]

    def install_projection(self, mean, V):
        """Device arrays of project(): per-star centres Q_s + mean and V
        (float32)."""
        torch = self.torch
        self._centre_dev = torch.from_numpy((self.Q + np.asarray(mean)[None, :]).astype(np.float32)).cuda()
        self._V_dev = torch.from_numpy(np.ascontiguousarray(V, dtype=np.float32)).cuda()

    def project(self, F_dev, star_ids):
        """Raw PCA coefficients (host float64 [n][k]) of spectra F of the
        given stars: (F - (Q_s + mean)) V, each row centred on its own
        star."""
        torch = self.torch
        from . import soap_pca_project

        n = int(F_dev.shape[0])
        coef = torch.empty((n, self.k), dtype=torch.float32, device="cuda")
        rows = torch.from_numpy(self.stars.rows(star_ids)).cuda()
        soap_pca_project(F_dev, self._centre_dev, self._V_dev, coef, mean_index=rows)
        return coef.cpu().numpy().astype(np.float64)

    def rv_weights(self, Yn, rows, eps=0.05):
        """RMS over the rows of Yn (normalised coefficients, host [m][k], of
        star rows `rows`) of the RV change per unit change of each
        coefficient, by central differences through the fused RV kernel's
        mean fit."""
        torch = self.torch
        m, k = Yn.shape
        X = np.repeat(np.asarray(Yn, np.float32)[:, None, :], 2 * k, axis=1)
        for j in range(k):
            X[:, 2 * j, j] += eps
            X[:, 2 * j + 1, j] -= eps
        X = X.reshape(-1, k)
        r = self._fit_rows(torch.from_numpy(np.ascontiguousarray(X)).cuda(),
                           torch.from_numpy(np.repeat(np.asarray(rows, np.int32), 2 * k)).cuda(), len(X))
        r = r.reshape(m, k, 2)
        return np.sqrt(np.mean(((r[:, :, 0] - r[:, :, 1]) / (2 * eps)) ** 2, axis=0))

    def _fit_rows(self, coef_dev, rows_dev, n):
        """RVs (host) of normalised coefficient rows, through
        soap_surrogate_rv with two identical members (only its mean fit
        matters here)."""
        torch = self.torch
        mem = torch.stack([coef_dev, coef_dev]).contiguous()
        rv_kms = torch.empty(n, dtype=torch.float64, device="cuda")
        fb = torch.empty(n, dtype=torch.int32, device="cuda")
        soap_surrogate_rv(self.ctx, coef_dev, mem, self.base_ccf, self.basis_ccf, 1.0, math.inf, rv_kms, fb,
                          base_index=rows_dev)
        return rv_kms.cpu().numpy()

    def reweight(self, w):
        """Rescales the normalised coefficients by w / rms(w), so that the
        training loss weighs each coefficient by its RV sensitivity."""
        b = self.basis
        w = np.maximum(np.asarray(w, np.float64), 1e-6 * np.max(w))
        b.sigma = b.sigma * np.sqrt(np.mean(w * w)) / w
        self._build_ccf_tables()

    def set_basis(self, mean, V, coef_train):
        """Installs the basis and the per-coefficient normalisation of the
        training coefficients (host [n][k]): centred, divided by their
        standard deviations."""
        c = np.asarray(coef_train, np.float64)
        mu = c.mean(axis=0)
        sd = c.std(axis=0)
        sd = np.where(sd > 0, sd, 1.0)
        self.basis = Basis(np.asarray(mean, np.float64), np.asarray(V, np.float64), mu, sd)
        self._build_ccf_tables()
        return mu, sd

    def _build_ccf_tables(self):
        """CCF of F0_s = Q_s + mean + V mu for every star and of
        B_k = sigma_k V_k, so that the CCF of a prediction y of star s is
        base[s] + y @ basis."""
        torch = self.torch
        b = self.basis
        f0 = self.Q + (b.mean + b.V @ b.mu)[None, :]
        rows = np.concatenate([f0, (b.V * b.sigma[None, :]).T], axis=0)
        dt = torch.float32 if self.ctx.precision == PREC_FP32 else torch.float64
        rows_dev = torch.from_numpy(np.ascontiguousarray(rows).astype(self.ctx.dtype)).to("cuda", dt)
        n_v = int(self.mask.n_v)
        ccf = torch.empty((rows.shape[0], n_v), dtype=torch.float64, device="cuda")
        soap_ccf_rv(self.ctx, rows_dev, self.mask, ccf_out=ccf, n_spec=rows.shape[0])
        ns = len(self.Q)
        self.base_ccf = ccf[:ns].contiguous()
        self.basis_ccf = ccf[ns:].contiguous()

    def normalise(self, coef_host):
        b = self.basis
        return ((np.asarray(coef_host, np.float64) - b.mu) / b.sigma).astype(np.float32)

    # -- training -----------------------------------------------------------
    def train(self, X, Y, epochs, batch=512, lr=2e-3, lr_final=1e-4, seed=0, log=None, log_every=1):
        """Adam over shuffled batches (X [n][features], Y [n][k] normalised,
        host float32).  The learning rate decays geometrically from lr to
        lr_final.  Returns the last batch's loss of every epoch; log (if
        given) gets a line every log_every epochs."""
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
            if log and ((ep + 1) % log_every == 0 or ep + 1 == epochs):
                log(f"epoch {ep + 1} of {epochs}, loss {tot:.4g}")
        return losses

    # -- inference ----------------------------------------------------------
    def alloc(self, n):
        """Device buffers for surrogate_rv on n samples (n a multiple of 16)."""
        torch = self.torch
        E = self.n_ens
        return dict(
            Y=torch.empty(((1 + E) * n, self.k), dtype=torch.float32, device="cuda"),
            rv=torch.empty((n * RV_DTYPE.itemsize,), dtype=torch.uint8, device="cuda"),
            rv_kms=torch.empty((n,), dtype=torch.float64, device="cuda"),
            err=torch.empty((n,), dtype=torch.float64, device="cuda"),
            fallback=torch.empty((n,), dtype=torch.int32, device="cuda"),
            n=n,
        )

    def surrogate_rv(self, x_dev, rows_dev, bufs, calib=None, threshold_kms=None):
        """Enqueues predict -> fused mean-CCF fit, member RV spread and gate
        for x_dev [n][features] of star rows rows_dev (int32 [n], device)."""
        n = bufs["n"]
        Y = bufs["Y"]
        soap_surrogate_predict(self.net, x_dev, Y[:n], Y[n:])
        soap_surrogate_rv(self.ctx, Y[:n], Y[n:], self.base_ccf, self.basis_ccf,
                          self.calib if calib is None else calib,
                          self.threshold_kms if threshold_kms is None else threshold_kms, bufs["rv_kms"],
                          bufs["fallback"], err_kms=bufs["err"], rv_out=bufs["rv"], base_index=rows_dev)

    def inputs(self, samples, idx):
        """Device features (computed on the device from the samples' raw
        descriptions) and star rows of samples[idx]."""
        torch = self.torch
        rows = self.stars.rows(sample_stars(samples, idx))
        raw = torch.from_numpy(sample_raw(self.stars, samples, idx, rows)).cuda()
        x = torch.empty((len(rows), N_FEATURES), dtype=torch.float32, device="cuda")
        soap_surrogate_features(raw, x)
        return x, torch.from_numpy(rows).cuda()

    def rv(self, samples, idx, bufs, threshold_kms=None, calib=None):
        """Gated RVs (km/s, host float64) of samples[idx]; idx sorted, its
        length a multiple of 16.  Returns (rv, fallback flags, predicted
        errors).  One device-to-host read brings back the flags, RVs and
        errors together."""
        torch = self.torch
        x, r = self.inputs(samples, idx)
        self.surrogate_rv(x, r, bufs, calib=calib, threshold_kms=threshold_kms)
        n = bufs["n"]
        host = torch.stack([bufs["rv_kms"][:n], bufs["err"][:n], bufs["fallback"][:n].to(torch.float64)]).cpu().numpy()
        out = host[0].copy()
        err = host[1].copy()
        fb = host[2] != 0.0
        sel = np.asarray(idx)[fb]
        if len(sel):
            out[fb] = plain_rv(self.stars, samples, self.mask, sel)["rv_kms"]
        return out, fb, err

    def calibrate(self, samples, idx, rv_plain_kms, bufs, threshold_kms=None, alpha=1e-3):
        """Sets calib from held-out samples with known full-synthesis RVs:
        the factor that accepts the most held-out samples (predicted error
        calib x spread below the threshold) while at most a fraction alpha
        of the accepted ones miss the full synthesis by the threshold or
        more (alpha = 0: none may).  Returns (|error|, spread) in km/s."""
        thr = self.threshold_kms if threshold_kms is None else threshold_kms
        x, r = self.inputs(samples, idx)
        self.surrogate_rv(x, r, bufs, calib=1.0, threshold_kms=math.inf)
        spread = np.maximum(bufs["err"].cpu().numpy(), 1e-300)
        err = np.abs(bufs["rv_kms"].cpu().numpy() - rv_plain_kms)
        self.calib = calib_for_miss_rate(err, spread, thr, alpha)
        return err, spread

def build(stars, mask, train, heldout, n_components=64, hidden=256, n_ensemble=4, epochs=100, batch=512,
          svd_subset=2048, seed=0, weighting="rv", alpha=1e-3, log=None):
    """Data set, basis, training and gate calibration of a surrogate for a
    Stars set (FP32 contexts; or one context) from SpotSamples or
    MultiSpotSamples train / heldout.  Returns the model and a dict of what
    it took."""
    torch = _torch()
    say = log or (lambda *a: None)
    info = {}
    model = SurrogateModel(stars, mask, n_components, hidden, n_ensemble, seed)
    stars = model.stars
    F = torch.empty((train.n, model.ctx.n_pix), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    synthesize(stars, train, F)
    torch.cuda.synchronize()
    info["synth_s"] = time.perf_counter() - t
    say(f"synthesised {train.n} training spectra in {info['synth_s']:.2f} s")
    sid = sample_stars(train, np.arange(train.n))
    sub = np.sort(np.random.default_rng(seed).choice(train.n, min(svd_subset, train.n), replace=False))
    D = model.differences_host(F[torch.from_numpy(sub).cuda()], sid[sub])
    mean, V = fit_basis(D, n_components)
    del D
    model.install_projection(mean, V)
    coef = np.concatenate([model.project(F[a:a + 8192], sid[a:a + 8192]) for a in range(0, train.n, 8192)])
    del F
    model.set_basis(mean, V, coef)
    rows = stars.rows(sid)
    if weighting == "rv":
        sel = np.random.default_rng(seed + 1).choice(len(coef), min(512, len(coef)), replace=False)
        w = model.rv_weights(model.normalise(coef[sel]), rows[sel])
        model.reweight(w)
        info["rv_weights"] = [float(v) for v in w[:8]]
    X = model.inputs(train, np.arange(train.n))[0].cpu().numpy()
    Y = model.normalise(coef)
    t = time.perf_counter()
    losses = model.train(X, Y, epochs, batch=batch, seed=seed, log=log, log_every=max(1, epochs // 10))
    torch.cuda.synchronize()
    info["train_s"] = time.perf_counter() - t
    info["train_steps"] = epochs * (len(X) // batch)
    info["final_loss"] = losses[-1]
    say(f"trained {info['train_steps']} steps in {info['train_s']:.2f} s, loss {losses[-1]:.3g}")
    n_ho = (heldout.n // 16) * 16
    rvp = plain_rv(stars, heldout, mask, np.arange(n_ho))["rv_kms"]
    err, spread = model.calibrate(heldout, np.arange(n_ho), rvp, model.alloc(n_ho), alpha=alpha)
    info["calib"] = model.calib
    # the factor for no tolerated miss on the held-out set, for reporting
    # the gate at alpha = 0 beside the chosen alpha
    info["calib_alpha0"] = calib_for_miss_rate(err, spread, model.threshold_kms, 0.0)
    acc = model.calib * spread < model.threshold_kms
    info["heldout_accepted_frac"] = float(acc.mean())
    info["heldout_accepted_over_thr_frac"] = float(np.mean(err[acc] >= model.threshold_kms)) if acc.any() else 0.0
    info["heldout_err_cms"] = {"median": float(np.median(err) * 1e5), "p99": float(np.quantile(err, 0.99) * 1e5),
                               "max": float(err.max() * 1e5)}
    return model, info
