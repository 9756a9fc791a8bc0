"""Resolution lowering on the GPU (the last step of Algorithms 2 and 5)
against the oracle's plain sum over offsets: seeded rows of ragged lengths
and both precisions, the lowering inside the synthesis call, and the
headline workload lowered to R = 115000 on sampled phases."""
import multiprocessing
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

import workloads as W
from oracle import lsf as OL
from oracle import spectrum as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2301_04259_amd", reason="libsoap.so not built")

_STAR = None


def _say(*a):
    print("[gpu-lsf]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _err(got, want):
    return float(np.max(np.abs(np.asarray(got, np.float64) - want) / np.maximum(np.abs(want), 1e-3 * np.abs(want).max())))


@pytest.mark.parametrize("prec,n_pix,res", [(W.PREC_FP32, 5003, 115000.0), (W.PREC_FP32, 4096, 60000.0),
                                            (W.PREC_FP64, 2051, 115000.0), (W.PREC_FP64, 1200, 30000.0)])
def test_lsf_rows_match_oracle(prec, n_pix, res):
    st = W.make_tiny(51, n_grid=8, n_pix=n_pix, n_mu=2, precision=prec)
    st.dln_lambda = 1.0 / (3.0 * 115000.0)
    ctx = L.soap_grid_init(st)
    rng = np.random.default_rng(n_pix)
    dt = np.float32 if prec == W.PREC_FP32 else np.float64
    rows = (1.0 - 0.6 * rng.uniform(0, 1, (7, n_pix)) ** 8).astype(dt)
    _say("rows", prec, n_pix, res)
    dev_in = torch.from_numpy(rows).cuda()
    dev_out = torch.empty_like(dev_in)
    L.soap_instrument_lsf(ctx, dev_in, dev_out, res)
    host_out = np.zeros_like(rows)
    L.soap_instrument_lsf(ctx, rows, host_out, res)
    torch.cuda.synchronize()
    got = dev_out.cpu().numpy()
    assert np.array_equal(got, host_out)
    want = OL.lower_resolution(rows.astype(np.float64), res, st.dln_lambda)
    bar = 1e-6 if prec == W.PREC_FP32 else 1e-12
    assert _err(got, want) <= bar
    # an unaligned output view gives the same values
    big = torch.zeros(7 * n_pix + 1, dtype=dev_in.dtype, device="cuda")
    L.soap_instrument_lsf(ctx, dev_in, big[1:].view(7, n_pix), res)
    torch.cuda.synchronize()
    assert np.array_equal(big[1:].view(7, n_pix).cpu().numpy(), got)


def test_lsf_argument_checks():
    st = W.make_tiny(52, n_grid=8, n_pix=800, n_mu=2, precision=W.PREC_FP32)
    ctx = L.soap_grid_init(st)
    x = torch.ones((2, 800), dtype=torch.float32, device="cuda")
    with pytest.raises(L.SoapError, match="overlap"):
        L.soap_instrument_lsf(ctx, x, x, 50000.0)
    with pytest.raises(L.SoapError) as e:
        L.soap_instrument_lsf(ctx, x, torch.empty_like(x), 100.0)  # kernel far wider than 32 pixels
    assert e.value.status == L.SOAP_ERR_UNSUPPORTED
    with pytest.raises(L.SoapError):
        L.soap_set_instrument(ctx, -1.0)


def test_synthesis_with_lowering_equals_two_calls_and_oracle():
    st = W.make_tiny(53, n_grid=40, n_pix=3333, n_mu=4, precision=W.PREC_FP32, contrast_mode=W.CONTRAST_PLANCK,
                     n_phases=9)
    ctx = L.soap_grid_init(st)
    raw = torch.empty((9, st.n_pix), dtype=torch.float32, device="cuda")
    L.soap_active_spectra(ctx, st.regions, st.phases, W.EFFECT_TOT, raw)
    two = torch.empty_like(raw)
    L.soap_instrument_lsf(ctx, raw, two, 80000.0)
    L.soap_set_instrument(ctx, 80000.0)
    one = torch.empty_like(raw)
    L.soap_active_spectra(ctx, st.regions, st.phases, W.EFFECT_TOT, one)
    L.soap_set_instrument(ctx, 0.0)
    again = torch.empty_like(raw)
    L.soap_active_spectra(ctx, st.regions, st.phases, W.EFFECT_TOT, again)
    torch.cuda.synchronize()
    assert torch.equal(one, two)
    assert torch.equal(again, raw)
    want = np.stack([OL.lower_resolution(OS.integrated(st, p, OS.TOT), 80000.0, st.dln_lambda) for p in st.phases])
    assert _err(one.cpu().numpy(), want) <= 1e-6


def _oracle(i):
    st = _STAR
    return OL.lower_resolution(OS.integrated(st, st.phases[i], OS.TOT), 115000.0, st.dln_lambda)


@pytest.mark.timeout(600)
def test_headline_lowered_to_r115000_sampled_phases():
    st = W.make_cfg2()
    ctx = L.soap_grid_init(st)
    L.soap_set_instrument(ctx, 115000.0)
    out = torch.empty((len(st.phases), st.n_pix), dtype=torch.float32, device="cuda")
    _say("headline lowered")
    L.soap_active_spectra(ctx, st.regions, st.phases, W.EFFECT_TOT, out)
    torch.cuda.synchronize()
    idx = [0, 55, 70]
    global _STAR
    _STAR = st
    with ProcessPoolExecutor(max_workers=3, mp_context=multiprocessing.get_context("fork")) as ex:
        want = list(ex.map(_oracle, idx))
    got = out.cpu().numpy()
    err = max(_err(got[i], w) for i, w in zip(idx, want))
    _say("max relative flux error", err)
    assert err <= 1e-6
