"""GPU checks of the boundary's error behaviour: caller-supplied contrast
arrays on the device, non-finite device inputs, the fixed-point range guard,
and the fit status of CCFs that cannot be fitted (section 4.1: the RV is the
mean of a fitted Gaussian, so a failed fit must say so)."""
import numpy as np
import pytest

import workloads as W
from oracle import spectrum as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2301_04259_amd", reason="libsoap.so not built")


def _say(*a):
    print("[gpu-boundary]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _flux_err(got, want):
    scale = np.maximum(np.abs(want), 1e-3 * np.abs(want).max())
    return float(np.max(np.abs(np.asarray(got, dtype=np.float64) - want) / scale))


def test_device_contrast_arrays_equal_host_ones():
    mk = lambda: W.make_tiny(25, n_grid=26, n_pix=1300, n_mu=3, precision=W.PREC_FP32,
                             contrast_mode=W.CONTRAST_ARRAY, n_phases=5)
    star = mk()
    _say("array contrast, host vs device inputs")
    ctx = L.soap_grid_init(star)
    ref = torch.empty((5, star.n_pix), dtype=torch.float32, device="cuda")
    L.soap_active_spectra(ctx, star.regions, star.phases, W.EFFECT_TOT, ref)
    dev = mk()
    dev.spectra = [None if s is None else torch.from_numpy(np.ascontiguousarray(s)).cuda() for s in star.spectra]
    dev.contrast = [None if c is None else torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in star.contrast]
    ctx2 = L.soap_grid_init(dev)
    out = torch.empty_like(ref)
    L.soap_active_spectra(ctx2, star.regions, star.phases, W.EFFECT_TOT, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    want = np.stack([OS.integrated(star, p, OS.TOT) for p in star.phases])
    assert _flux_err(out.cpu().numpy(), want) <= 1e-6


def test_array_mode_requires_contrast_rows():
    star = W.make_tiny(26, n_grid=12, n_pix=400, n_mu=2, precision=W.PREC_FP64, contrast_mode=W.CONTRAST_ARRAY)
    star.contrast = [None, star.contrast[1], None]
    with pytest.raises(L.SoapError, match="contrast"):
        L.soap_grid_init(star)


def test_non_finite_device_spectrum_is_an_argument_error():
    star = W.make_tiny(27, n_grid=12, n_pix=500, n_mu=2, precision=W.PREC_FP32)
    spec = [None if s is None else torch.from_numpy(np.ascontiguousarray(s)).cuda() for s in star.spectra]
    spec[W.SPOT][1, 321] = float("nan")
    star.spectra = spec
    _say("nan device spectrum")
    with pytest.raises(L.SoapError, match="non-finite") as e:
        L.soap_grid_init(star)
    assert e.value.status == L.SOAP_ERR_ARG


def test_contrast_beyond_fixed_point_range_is_rejected():
    # disk weight ~3.0 (limb darkening u1 = 0.1) x contrast 6 reaches the
    # |x| < 16 range of the fixed-point tap sums in split tables
    star = W.make_tiny(28, n_grid=40, n_pix=600, n_mu=3, precision=W.PREC_FP64, n_phases=3)
    star.ld_u1, star.ld_u2 = 0.1, 0.0
    ctx = L.soap_grid_init(star)
    out = torch.empty((3, star.n_pix), dtype=torch.float64, device="cuda")
    big = [W.Region(W.FACULA, 0.0, 0.0, 0.9, 6.0)]
    with pytest.raises(L.SoapError) as e:
        L.soap_active_spectra(ctx, big, star.phases, W.EFFECT_TOT, out)
    assert e.value.status == L.SOAP_ERR_UNSUPPORTED
    ok = [W.Region(W.FACULA, 0.0, 0.0, 0.9, 4.5)]
    L.soap_active_spectra(ctx, ok, star.phases, W.EFFECT_TOT, out)
    torch.cuda.synchronize()
    want = np.stack([OS.integrated(star, p, OS.TOT, ok) for p in star.phases])
    assert _flux_err(out.cpu().numpy(), want) <= 1e-9


def test_fit_status_of_nan_and_flat_ccfs():
    star = W.make_tiny(29, n_grid=24, n_pix=2000, n_mu=2, precision=W.PREC_FP64, n_phases=1)
    ctx = L.soap_grid_init(star)
    q = np.zeros(star.n_pix)
    L.soap_quiet_spectrum(ctx, q)
    m = star.mask
    # a NaN inside a mask line's holes, a flat spectrum, and the quiet
    # spectrum.  The flat spectrum's CCF is not flat to rounding: each hole
    # spans atanh((v + h)/c) - atanh((v - h)/c) in ln(lambda), which grows
    # with |v| relatively by about (v/c)^2 (4e-9 at 20 km/s), so its fit has
    # nothing to converge to and must not report success (status 1 or 2).
    lnl = star.ln_lambda0 + star.dln_lambda * np.arange(star.n_pix)
    k = int(np.argmin(np.abs(lnl - m.ln_lambda[len(m.ln_lambda) // 2])))
    rows = np.stack([q.copy(), np.full(star.n_pix, 2.5), q.copy()])
    rows[0, k] = np.nan
    _say("fit status")
    rv = L.rv_records(3)
    ccf = np.zeros((3, m.n_v))
    L.soap_ccf_rv(ctx, rows, m, ccf_out=ccf, rv_out=rv)
    assert not np.all(np.isfinite(ccf[0]))
    assert rv["status"][0] == 2, rv
    c1 = ccf[1]
    assert np.all(np.isfinite(c1)) and (c1.max() - c1.min()) <= 1e-7 * c1.max()
    assert rv["status"][1] in (1, 2), rv
    assert rv["status"][2] == 0, rv


def test_device_byte_cap_refuses_cleanly_and_leaks_nothing(monkeypatch):
    import gc

    gc.collect()
    torch.cuda.synchronize()
    base = L.device_bytes()
    star = W.make_tiny(31, n_grid=20, n_pix=900, n_mu=3, precision=W.PREC_FP32, n_phases=6)
    _say("device byte cap: init refused under a 4 KiB allowance")
    monkeypatch.setenv("SOAP_MAX_DEVICE_BYTES", str(base + 4096))
    with pytest.raises(L.SoapError) as ei:
        L.soap_grid_init(star)
    assert ei.value.status == L.SOAP_ERR_OOM and "SOAP_MAX_DEVICE_BYTES" in str(ei.value)
    assert L.device_bytes() == base
    monkeypatch.setenv("SOAP_MAX_DEVICE_BYTES", "12x")
    with pytest.raises(L.SoapError) as ei:
        L.soap_grid_init(star)
    assert ei.value.status == L.SOAP_ERR_OOM and "not a byte count" in str(ei.value)
    assert L.device_bytes() == base

    monkeypatch.delenv("SOAP_MAX_DEVICE_BYTES")
    ctx = L.soap_grid_init(star)
    held = L.device_bytes()
    assert held > base
    n_ph = len(star.phases)
    out = torch.empty((n_ph, star.n_pix), dtype=torch.float32, device="cuda")
    _say("device byte cap: first synthesis refused, context usable after the cap is lifted")
    monkeypatch.setenv("SOAP_MAX_DEVICE_BYTES", str(held))
    with pytest.raises(L.SoapError) as ei:
        L.soap_active_spectra(ctx, star.regions, star.phases, W.EFFECT_TOT, out)
    assert ei.value.status == L.SOAP_ERR_OOM
    monkeypatch.delenv("SOAP_MAX_DEVICE_BYTES")
    L.soap_active_spectra(ctx, star.regions, star.phases, W.EFFECT_TOT, out)
    torch.cuda.synchronize()
    fresh = L.soap_grid_init(star)
    ref = torch.empty_like(out)
    L.soap_active_spectra(fresh, star.regions, star.phases, W.EFFECT_TOT, ref)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    L.soap_destroy(fresh)
    L.soap_destroy(ctx)
    assert L.device_bytes() == base
