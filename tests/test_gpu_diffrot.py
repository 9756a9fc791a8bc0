"""Differential rotation (section 3.4) on the GPU against the oracle: every
cell with its own shift, regions drifting at their latitude's rate.  Small
stars are compared over the whole spectrum (and RV); the headline workload
with the solar DIFF_ROT = -0.18 at sampled pixels of sampled phases, the
oracle evaluating the per-cell sum pixel by pixel."""
import dataclasses
import multiprocessing
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

import workloads as W
from oracle import ccf as OC
from oracle import fit as OF
from oracle import spectrum as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2301_04259_amd", reason="libsoap.so not built")

_JOBS = []


def _say(*a):
    print("[gpu-diffrot]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _err(got, want):
    got = np.asarray(got, np.float64)
    return float(np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-3 * np.abs(want).max())))


CASES = [
    # seed, N, P, B, precision, contrast, incl, diff_rot
    (71, 24, 1500, 4, W.PREC_FP64, W.CONTRAST_SCALAR, 90.0, -0.18),
    (72, 37, 2222, 5, W.PREC_FP32, W.CONTRAST_PLANCK, 60.0, -0.3),
    (73, 30, 1801, 3, W.PREC_FP32, W.CONTRAST_ARRAY, 40.0, 0.25),
    (74, 45, 3000, 6, W.PREC_FP64, W.CONTRAST_PLANCK, 85.0, -0.6),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"seed{c[0]}-i{c[6]}-a{c[7]}")
@pytest.mark.parametrize("effect", [W.EFFECT_TOT, W.EFFECT_FLUX, W.EFFECT_BCONV])
def test_small_stars_match_oracle(case, effect):
    seed, n, p, b, prec, cmode, incl, a = case
    st = W.make_tiny(seed, n_grid=n, n_pix=p, n_mu=b, precision=prec, contrast_mode=cmode, incl_deg=incl,
                     n_phases=6)
    st.diff_rot = a
    _say(case, effect)
    ctx = L.soap_grid_init(st)
    dt = torch.float32 if prec == W.PREC_FP32 else torch.float64
    out = torch.empty((len(st.phases), st.n_pix), dtype=dt, device="cuda")
    L.soap_active_spectra(ctx, st.regions, st.phases, effect, out)
    q = torch.empty(st.n_pix, dtype=dt, device="cuda")
    L.soap_quiet_spectrum(ctx, q)
    torch.cuda.synchronize()
    bar = 1e-6 if prec == W.PREC_FP32 else 1e-9
    assert _err(q.cpu().numpy(), OS.quiet(st)) <= bar
    want = np.stack([OS.integrated(st, ph, effect) for ph in st.phases])
    assert _err(out.cpu().numpy(), want) <= bar


def test_rv_with_differential_rotation():
    st = W.make_tiny(75, n_grid=64, n_pix=4000, n_mu=4, precision=W.PREC_FP32, contrast_mode=W.CONTRAST_PLANCK,
                     incl_deg=70.0, n_phases=8, vsini_kms=4.0)
    st.diff_rot = -0.18
    ctx = L.soap_grid_init(st)
    out = torch.empty((8, st.n_pix), dtype=torch.float32, device="cuda")
    L.soap_active_spectra(ctx, st.regions, st.phases, W.EFFECT_TOT, out)
    rv = L.rv_records(8)
    L.soap_ccf_rv(ctx, out, st.mask, rv_out=rv)
    torch.cuda.synchronize()
    want = np.stack([OS.integrated(st, ph, OS.TOT) for ph in st.phases])
    assert _err(out.cpu().numpy(), want) <= 1e-6
    m = st.mask
    v = W.make_velocity_grid(m.v0_kms, m.dv_kms, m.n_v)
    c = OC.ccf(want, st.ln_lambda0, st.dln_lambda, m.ln_lambda, m.weight, m.half_width_kms, v)
    rv_or = np.array([OF.gauss_fit(v, ci)["mu"] for ci in c])
    assert np.max(np.abs(rv["rv_kms"] - rv_or)) * 1e5 < 1.0
    # the solar rate changes the RVs: a solid-body star differs
    solid = dataclasses.replace(st, diff_rot=0.0)
    ctx2 = L.soap_grid_init(solid)
    out2 = torch.empty_like(out)
    L.soap_active_spectra(ctx2, st.regions, st.phases, W.EFFECT_TOT, out2)
    rv2 = L.rv_records(8)
    L.soap_ccf_rv(ctx2, out2, st.mask, rv_out=rv2)
    assert np.max(np.abs(rv2["rv_kms"] - rv["rv_kms"])) * 1e5 > 10.0


def _oracle_pixels(i):
    st, ph, pix = _JOBS[i]
    return OS.integrated_pixels(st, ph, pix, OS.TOT)


@pytest.mark.timeout(900)
def test_headline_with_solar_differential_rotation_sampled():
    st = W.make_cfg2()
    st.diff_rot = -0.18
    ctx = L.soap_grid_init(st)
    out = torch.empty((len(st.phases), st.n_pix), dtype=torch.float32, device="cuda")
    _say("headline, diff_rot -0.18")
    L.soap_active_spectra(ctx, st.regions, st.phases, W.EFFECT_TOT, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.isfinite(got).all()
    rng = np.random.default_rng(5)
    # pixels: both ends, the deepest points and a random spread
    q = np.zeros(st.n_pix, dtype=np.float32)
    L.soap_quiet_spectrum(ctx, q)
    deep = np.argsort(q)[:40]
    pix = np.unique(np.concatenate([[0, 1, 2, st.n_pix - 3, st.n_pix - 2, st.n_pix - 1], deep,
                                    rng.integers(0, st.n_pix, 120)]))
    idx = [0, 30, 55, 62, 70, 95]
    global _JOBS
    _JOBS = [(st, st.phases[i], pix) for i in idx]
    with ProcessPoolExecutor(max_workers=len(idx), mp_context=multiprocessing.get_context("fork")) as ex:
        want = list(ex.map(_oracle_pixels, range(len(idx))))
    err = 0.0
    scale = np.abs(q.astype(np.float64)).max()
    for i, w in zip(idx, want):
        g = got[i][pix].astype(np.float64)
        err = max(err, float(np.max(np.abs(g - w) / np.maximum(np.abs(w), 1e-3 * scale))))
    _say("max relative flux error at", len(pix), "pixels x", len(idx), "phases:", err)
    assert err <= 1e-6
