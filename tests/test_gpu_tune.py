"""Shift-and-sum shapes and their tuner: every shape gives the same spectra
bit for bit (and the oracle's), the tuner picks one of them and its file
cache returns the same choice."""
import json
import os
import tempfile

import numpy as np
import pytest

import workloads as W
from oracle import spectrum as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2301_04259_amd", reason="libsoap.so not built")

SHAPES = [(t, w, False) for t in (64, 128, 256, 512) for w in (1, 16, 48)] + [(256, w, True) for w in (1, 16, 48)]


def _say(*a):
    print("[tune]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.mark.parametrize(
    "precision,contrast,n_pix,seed",
    [
        (W.PREC_FP32, W.CONTRAST_PLANCK, 5000, 1),  # paired tables, several tiles, ragged tail
        (W.PREC_FP32, W.CONTRAST_SCALAR, 2100, 2),  # split tables
        (W.PREC_FP64, W.CONTRAST_SCALAR, 3001, 3),
    ],
)
def test_every_shape_gives_identical_spectra(precision, contrast, n_pix, seed):
    star = W.make_tiny(seed, n_grid=32, n_pix=n_pix, precision=precision, contrast_mode=contrast, n_phases=21)
    ctx = L.soap_grid_init(star)
    dt = torch.float32 if precision == W.PREC_FP32 else torch.float64
    ref = None
    for t, w, sg in SHAPES:
        L.soap_set_apply_shape(ctx, t, w, sg)
        out = torch.empty((len(star.phases), star.n_pix), dtype=dt, device="cuda")
        L.soap_active_spectra(ctx, star.regions, star.phases, W.EFFECT_TOT, out)
        got = out.cpu().numpy()
        if ref is None:
            ref = got
            f = OS.integrated(star, star.phases[3], OS.TOT)
            e = np.max(np.abs(got[3] - f) / np.maximum(np.abs(f), 1e-3 * np.abs(f).max()))
            _say(f"P={n_pix} shape {t}x{w}: rel err vs oracle {e:.2e}")
            assert e <= (1e-6 if precision == W.PREC_FP32 else 1e-9)
        else:
            np.testing.assert_array_equal(got, ref, err_msg=f"shape {t} x {w} staged {sg}")
    with pytest.raises(L.SoapError):
        L.soap_set_apply_shape(ctx, 96, 16)
    with pytest.raises(L.SoapError):
        L.soap_set_apply_shape(ctx, 128, 16, True)
    L.soap_destroy(ctx)


def test_autotune_and_cache_round_trip():
    star = W.make_tiny(5, n_grid=48, n_pix=9000, precision=W.PREC_FP32, n_phases=40)
    ctx = L.soap_grid_init(star)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        a = L.soap_autotune(ctx, star.regions, star.phases, W.EFFECT_TOT, cache_path=path)
        _say("tuned", a)
        assert (a["threads"], a["lds_win"]) in [(t, w) for t in (64, 128, 256, 512) for w in (16, 32, 48)]
        assert not a["staged"] or a["threads"] == 256
        assert not a["from_cache"] and a["n_tried"] >= 4 and a["apply_us"] > 0
        cache = json.load(open(path))
        assert cache[a["key"]][:3] == [a["threads"], a["lds_win"], int(a["staged"])]
        L.soap_set_apply_shape(ctx, 64, 1)
        b = L.soap_autotune(ctx, star.regions, star.phases, W.EFFECT_TOT, cache_path=path)
        assert b["from_cache"] and (b["threads"], b["lds_win"], b["staged"]) == (a["threads"], a["lds_win"], a["staged"])
        # the tuned context still gives the oracle's spectra
        out = torch.empty((len(star.phases), star.n_pix), dtype=torch.float32, device="cuda")
        L.soap_active_spectra(ctx, star.regions, star.phases, W.EFFECT_TOT, out)
        f = OS.integrated(star, star.phases[7], OS.TOT)
        e = np.max(np.abs(out[7].cpu().numpy() - f) / np.maximum(np.abs(f), 1e-3 * np.abs(f).max()))
        assert e <= 1e-6
    L.soap_destroy(ctx)
