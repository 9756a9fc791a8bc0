"""Host-side checks of the C ABI: the library loads, exports every function the
header declares, and rejects invalid star descriptions before touching the
GPU (validation runs before any HIP call, so these need no device)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

L = pytest.importorskip("paper_2301_04259_amd", reason="libsoap.so not built")
import workloads as W  # noqa: E402


def _declared():
    with open(os.path.join(ROOT, "include", "soap.h")) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(soap_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    import ctypes

    lib = ctypes.CDLL(L.LIB_PATH)
    names = _declared()
    assert "soap_grid_init" in names and "soap_active_spectra" in names and "soap_ccf_rv" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.SYMBOLS) == names


def test_exports_nothing_else():
    import subprocess

    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    funcs = sorted(ln.split()[-1] for ln in out.splitlines() if " T " in ln)
    assert funcs == _declared()


def test_abi_version_and_status_strings():
    assert L.abi_version() == 4
    assert L._lib.soap_status_string(0) == b"SOAP_OK"
    assert L._lib.soap_status_string(-1) == b"SOAP_ERR_ARG"


def test_struct_sizes_match_header():
    import ctypes

    assert ctypes.sizeof(L.RegionC) == 40
    assert ctypes.sizeof(L.MaskC) == 56
    assert L.RV_DTYPE.itemsize == 56
    assert ctypes.sizeof(L.StarDesc) == 8 * 2 + 8 * 6 + 8 + 24 + 16 + 16 + 24 + 24 + 8
    assert ctypes.sizeof(L.TuneC) == 4 * 4 + 8 + 4 * 2 + 128


def _bad(**kw):
    st = W.make_tiny(1, n_grid=8, n_pix=256, n_mu=3)
    for k, v in kw.items():
        setattr(st, k, v)
    return st


@pytest.mark.parametrize(
    "kw,msg",
    [
        (dict(n_grid=1), "n_grid"),
        (dict(n_grid=100000), "n_grid"),
        (dict(mu_bins=np.array([1.0, 0.5, 0.7])), "decreasing"),
        (dict(mu_bins=np.array([1.2, 0.5, 0.2])), "mu_bins"),
        (dict(vsini_kms=float("nan")), "vsini"),
        (dict(incl_deg=200.0), "incl"),
        (dict(dln_lambda=-1e-6), "dln_lambda"),
        (dict(precision=7), "precision"),
        (dict(contrast_mode=5), "contrast_mode"),
        (dict(contrast_mode=1, teff_k=50.0), "teff"),
        (dict(vsini_kms=400.0), "shift"),
    ],
)
def test_grid_init_rejects_invalid_star(kw, msg):
    with pytest.raises(L.SoapError) as e:
        L.soap_grid_init(_bad(**kw))
    assert e.value.status == -1
    assert msg in str(e.value)
    assert msg in L.soap_last_error(None)


def test_grid_init_rejects_missing_quiet_spectrum():
    st = _bad()
    st.spectra = [None, st.spectra[1], st.spectra[2]]
    with pytest.raises(L.SoapError, match="SOAP_QUIET"):
        L.soap_grid_init(st)


def test_grid_init_rejects_nan_spectrum():
    st = _bad()
    q = st.spectra[0].copy()
    q[1, 17] = np.nan
    st.spectra = [q, st.spectra[1], st.spectra[2]]
    with pytest.raises(L.SoapError, match="non-finite"):
        L.soap_grid_init(st)


def test_grid_init_rejects_disk_weight_beyond_fixed_point_range():
    # I(mu) = 1 + 15 (1 - mu) gives a disk weight near 6 pi: beyond the
    # |x| < 16 range of the fixed-point tap sums (checked before any device call)
    st = _bad(ld_u1=-15.0, ld_u2=0.0)
    with pytest.raises(L.SoapError, match="fixed-point") as e:
        L.soap_grid_init(st)
    assert e.value.status == L.SOAP_ERR_UNSUPPORTED


def test_grid_init_rejects_array_mode_without_rows_and_rows_outside_it():
    st = W.make_tiny(2, n_grid=8, n_pix=256, n_mu=3, contrast_mode=W.CONTRAST_ARRAY)
    st.contrast = [None, None, st.contrast[2]]
    with pytest.raises(L.SoapError, match=r"contrast\[1\]"):
        L.soap_grid_init(st)
    st = W.make_tiny(2, n_grid=8, n_pix=256, n_mu=3, contrast_mode=W.CONTRAST_ARRAY)
    st.contrast[2] = st.contrast[2].copy()
    st.contrast[2][0, 5] = np.inf
    with pytest.raises(L.SoapError, match="non-finite"):
        L.soap_grid_init(st)
