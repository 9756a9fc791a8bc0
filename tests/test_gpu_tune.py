"""Shift-and-sum shapes and their tuner: every shape (phases per chunk, which
is the tap tables' layout, windows in flight, item order) gives the same
spectra bit for bit (and the oracle's), the tuner picks one of them and its
file cache returns the same choice."""
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

SHAPES = [(d, o) for d in (2, 3) for o in (0, 1)]
PCS = {W.PREC_FP32: (8, 16), W.PREC_FP64: (4, 8)}


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
    for pc in PCS[precision]:
        for d, o in SHAPES:
            L.soap_set_apply_shape(ctx, d, o, pc)
            out = torch.empty((len(star.phases), star.n_pix), dtype=dt, device="cuda")
            L.soap_active_spectra(ctx, star.regions, star.phases, W.EFFECT_TOT, out)
            got = out.cpu().numpy()
            if ref is None:
                ref = got
                f = OS.integrated(star, star.phases[3], OS.TOT)
                e = np.max(np.abs(got[3] - f) / np.maximum(np.abs(f), 1e-3 * np.abs(f).max()))
                _say(f"P={n_pix} shape pc {pc}, depth {d}, order {o}: rel err vs oracle {e:.2e}")
                assert e <= (1e-6 if precision == W.PREC_FP32 else 1e-9)
            else:
                np.testing.assert_array_equal(got, ref, err_msg=f"shape pc {pc}, depth {d}, order {o}")
    with pytest.raises(L.SoapError):
        L.soap_set_apply_shape(ctx, 4, 0)
    with pytest.raises(L.SoapError):
        L.soap_set_apply_shape(ctx, 2, 2)
    with pytest.raises(L.SoapError):
        L.soap_set_apply_shape(ctx, 2, 0, 12)
    other = PCS[W.PREC_FP64 if precision == W.PREC_FP32 else W.PREC_FP32]
    with pytest.raises(L.SoapError):
        L.soap_set_apply_shape(ctx, 2, 0, [p for p in other if p not in PCS[precision]][0])
    L.soap_destroy(ctx)


def test_autotune_and_cache_round_trip():
    star = W.make_tiny(5, n_grid=48, n_pix=9000, precision=W.PREC_FP32, n_phases=40)
    ctx = L.soap_grid_init(star)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        a = L.soap_autotune(ctx, star.regions, star.phases, W.EFFECT_TOT, cache_path=path)
        _say("tuned", a)
        assert (a["depth"], a["order"]) in SHAPES and a["phases_per_chunk"] in PCS[W.PREC_FP32]
        assert not a["from_cache"] and a["n_tried"] == 2 * len(SHAPES) and a["apply_us"] > 0
        cache = json.load(open(path))
        assert cache[a["key"]][:3] == [a["phases_per_chunk"], a["depth"], a["order"]]
        L.soap_set_apply_shape(ctx, 3, 1, 16 if a["phases_per_chunk"] == 8 else 8)
        b = L.soap_autotune(ctx, star.regions, star.phases, W.EFFECT_TOT, cache_path=path)
        assert b["from_cache"]
        assert (b["phases_per_chunk"], b["depth"], b["order"]) == (a["phases_per_chunk"], a["depth"], a["order"])
        # the tuned context still gives the oracle's spectra
        out = torch.empty((len(star.phases), star.n_pix), dtype=torch.float32, device="cuda")
        L.soap_active_spectra(ctx, star.regions, star.phases, W.EFFECT_TOT, out)
        f = OS.integrated(star, star.phases[7], OS.TOT)
        e = np.max(np.abs(out[7].cpu().numpy() - f) / np.maximum(np.abs(f), 1e-3 * np.abs(f).max()))
        assert e <= 1e-6
    L.soap_destroy(ctx)
