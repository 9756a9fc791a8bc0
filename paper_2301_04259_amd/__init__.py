"""Python binding of libsoap (include/soap.h): argument marshalling only.

Every computation runs in the HIP kernels of ``libsoap.so``; this module
converts Python objects into the C structs of the ABI and passes pointers.
Device buffers are torch tensors on the GPU (torch is used for device memory
and streams only); host buffers are numpy arrays.  Importing this module
fails loudly when the built library is missing: there is no fallback.

Functions carry the ABI names:

    ctx = soap_grid_init(star, stream=None)
    soap_quiet_spectrum(ctx, out)
    soap_active_spectra(ctx, regions, phases, effect, out)
    soap_ccf_rv(ctx, flux, mask, ccf_out=None, rv_out=None)
    soap_sync(ctx); soap_destroy(ctx); soap_last_error(ctx)

``star`` is any object with the fields of ``soap_star_desc`` (n_grid,
vsini_kms, incl_deg, ld_u1, ld_u2, ln_lambda0, dln_lambda, n_pix, mu_bins,
spectra[3], precision, contrast_mode, teff_k, dt_spot_k, dt_fac_coef);
regions carry type / lat_deg / lon_deg / radius / contrast; a mask carries
ln_lambda / weight / half_width_kms / v0_kms / dv_kms / n_v.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SOAP_LIB names another build of the same library (the host-sanitizer
# build); by default the in-tree libsoap.so is loaded
LIB_PATH = os.environ.get("SOAP_LIB") or os.path.join(_HERE, "libsoap.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python paper_2301_04259_amd/build.py` "
        "(hipcc, gfx950) before importing the binding"
    )

# torch ships its own HIP runtime under the same soname as the system one.
# Loading torch first makes libsoap bind to that single runtime, so device
# pointers and streams from torch's allocator are valid in this library's
# calls; loading libsoap first would bring a second runtime into the process.
try:
    import torch  # noqa: F401
except ImportError:  # host-only use (argument checks, symbol tests)
    torch = None

_lib = C.CDLL(LIB_PATH)

SOAP_OK = 0
SOAP_ERR_ARG, SOAP_ERR_OOM, SOAP_ERR_HIP, SOAP_ERR_STATE, SOAP_ERR_NOCONV, SOAP_ERR_UNSUPPORTED = -1, -2, -3, -4, -5, -6
QUIET, SPOT, FACULA = 0, 1, 2
EFFECT_TOT, EFFECT_FLUX, EFFECT_BCONV = 0, 1, 2
PREC_FP64, PREC_FP32 = 0, 1
CONTRAST_SCALAR, CONTRAST_PLANCK, CONTRAST_ARRAY = 0, 1, 2

SYMBOLS = (
    "soap_grid_init",
    "soap_quiet_spectrum",
    "soap_active_spectra",
    "soap_ccf_rv",
    "soap_sync",
    "soap_destroy",
    "soap_last_error",
    "soap_status_string",
    "soap_abi_version",
    "soap_device_bytes",
    "soap_profile_enable",
    "soap_profile_read",
    "soap_ccf_linear_rv",
    "soap_active_spectra_jobs",
    "soap_surrogate_rv",
    "soap_set_apply_shape",
    "soap_autotune",
    "soap_batch_create",
    "soap_batch_create_rv",
    "soap_active_spectra_multi",
    "soap_batch_run",
    "soap_batch_n_spectra",
    "soap_batch_last_error",
    "soap_batch_destroy",
    "soap_surrogate_create",
    "soap_surrogate_n_params",
    "soap_surrogate_train_step",
    "soap_surrogate_predict",
    "soap_surrogate_get_params",
    "soap_surrogate_set_params",
    "soap_surrogate_get_grads",
    "soap_surrogate_save",
    "soap_surrogate_load",
    "soap_surrogate_last_error",
    "soap_surrogate_destroy",
    "soap_pca_project",
    "soap_surrogate_gate",
    "soap_surrogate_features",
    "soap_evolution_size",
    "soap_active_spectra_evolving",
    "soap_instrument_lsf",
    "soap_set_instrument",
    "soap_ccf_rv_noalloc",
)


class StarDesc(C.Structure):
    _fields_ = [
        ("n_grid", C.c_int32),
        ("n_mu", C.c_int32),
        ("n_pix", C.c_int64),
        ("vsini_kms", C.c_double),
        ("incl_deg", C.c_double),
        ("ld_u1", C.c_double),
        ("ld_u2", C.c_double),
        ("ln_lambda0", C.c_double),
        ("dln_lambda", C.c_double),
        ("mu_bins", C.POINTER(C.c_double)),
        ("spectra", C.c_void_p * 3),
        ("spectra_on_device", C.c_int32),
        ("precision", C.c_int32),
        ("contrast_mode", C.c_int32),
        ("reserved0", C.c_int32),
        ("teff_k", C.c_double),
        ("dt_spot_k", C.c_double),
        ("dt_fac_coef", C.c_double * 3),
        ("contrast", C.c_void_p * 3),
        ("diff_rot", C.c_double),
    ]


class RegionC(C.Structure):
    _fields_ = [
        ("type", C.c_int32),
        ("reserved0", C.c_int32),
        ("lat_deg", C.c_double),
        ("lon_deg", C.c_double),
        ("radius", C.c_double),
        ("contrast", C.c_double),
    ]


class MaskC(C.Structure):
    _fields_ = [
        ("n_lines", C.c_int64),
        ("ln_lambda", C.POINTER(C.c_double)),
        ("weight", C.POINTER(C.c_double)),
        ("half_width_kms", C.c_double),
        ("v0_kms", C.c_double),
        ("dv_kms", C.c_double),
        ("n_v", C.c_int32),
        ("reserved0", C.c_int32),
    ]


class ProfileC(C.Structure):
    _fields_ = [
        ("weights_ms", C.c_double),
        ("compact_ms", C.c_double),
        ("apply_ms", C.c_double),
        ("ccf_ms", C.c_double),
        ("gfit_ms", C.c_double),
        ("lsf_ms", C.c_double),
        ("active_calls", C.c_int64),
        ("ccf_calls", C.c_int64),
        ("src_arrays", C.c_int64),
        ("con_arrays", C.c_int64),
        ("last_phases", C.c_int64),
        ("taps_nonzero", C.c_int64),
        ("taps_offsets", C.c_int64),
        ("fma_issued", C.c_int64),
    ]


RV_DTYPE = np.dtype(
    [
        ("rv_kms", "<f8"),
        ("fwhm_kms", "<f8"),
        ("c0", "<f8"),
        ("amp", "<f8"),
        ("sigma_kms", "<f8"),
        ("chi2", "<f8"),
        ("iters", "<i4"),
        ("status", "<i4"),
    ]
)

_ctx_p = C.c_void_p
_lib.soap_grid_init.argtypes = [C.POINTER(StarDesc), C.c_void_p, C.POINTER(_ctx_p)]
_lib.soap_grid_init.restype = C.c_int
_lib.soap_quiet_spectrum.argtypes = [_ctx_p, C.c_void_p, C.c_int32]
_lib.soap_quiet_spectrum.restype = C.c_int
_lib.soap_active_spectra.argtypes = [
    _ctx_p, C.POINTER(RegionC), C.c_int32, C.POINTER(C.c_double), C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
]
_lib.soap_active_spectra.restype = C.c_int
_lib.soap_ccf_rv.argtypes = [
    _ctx_p, C.c_void_p, C.c_int32, C.c_int64, C.POINTER(MaskC), C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
]
_lib.soap_ccf_rv.restype = C.c_int
_lib.soap_sync.argtypes = [_ctx_p]
_lib.soap_sync.restype = C.c_int
_lib.soap_destroy.argtypes = [_ctx_p]
_lib.soap_destroy.restype = None
_lib.soap_last_error.argtypes = [_ctx_p]
_lib.soap_last_error.restype = C.c_char_p
_lib.soap_status_string.argtypes = [C.c_int]
_lib.soap_status_string.restype = C.c_char_p
_lib.soap_profile_enable.argtypes = [_ctx_p, C.c_int32]
_lib.soap_profile_enable.restype = C.c_int
_lib.soap_profile_read.argtypes = [_ctx_p, C.POINTER(ProfileC)]
_lib.soap_profile_read.restype = C.c_int
_lib.soap_abi_version.argtypes = []
_lib.soap_abi_version.restype = C.c_int32
_lib.soap_device_bytes.argtypes = []
_lib.soap_device_bytes.restype = C.c_uint64
_lib.soap_ccf_linear_rv.argtypes = [_ctx_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p]
_lib.soap_ccf_linear_rv.restype = C.c_int
_lib.soap_surrogate_rv.argtypes = [_ctx_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p,
                                   C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_double, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p]
_lib.soap_surrogate_rv.restype = C.c_int
class TuneC(C.Structure):
    _fields_ = [
        ("depth", C.c_int32),
        ("order", C.c_int32),
        ("phases_per_chunk", C.c_int32),
        ("from_cache", C.c_int32),
        ("apply_us", C.c_double),
        ("n_tried", C.c_int32),
        ("reserved", C.c_int32),
        ("key", C.c_char * 128),
    ]


_lib.soap_set_apply_shape.argtypes = [_ctx_p, C.c_int32, C.c_int32, C.c_int32]
_lib.soap_set_apply_shape.restype = C.c_int
_lib.soap_autotune.argtypes = [_ctx_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_char_p,
                               C.POINTER(TuneC)]
_lib.soap_autotune.restype = C.c_int
_lib.soap_batch_create.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                   C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]
_lib.soap_batch_create.restype = C.c_int
_lib.soap_batch_create_rv.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_int32, C.c_void_p, C.POINTER(MaskC), C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(C.c_void_p)]
_lib.soap_batch_create_rv.restype = C.c_int
_lib.soap_active_spectra_multi.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_int32, C.c_void_p, C.c_void_p]
_lib.soap_active_spectra_multi.restype = C.c_int
_lib.soap_batch_run.argtypes = [C.c_void_p]
_lib.soap_batch_run.restype = C.c_int
_lib.soap_batch_n_spectra.argtypes = [C.c_void_p]
_lib.soap_batch_n_spectra.restype = C.c_int64
_lib.soap_batch_last_error.argtypes = [C.c_void_p]
_lib.soap_batch_last_error.restype = C.c_char_p
_lib.soap_batch_destroy.argtypes = [C.c_void_p]
_lib.soap_batch_destroy.restype = None
_lib.soap_active_spectra_jobs.argtypes = [_ctx_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                          C.c_int32, C.c_void_p, C.c_int32]
_lib.soap_active_spectra_jobs.restype = C.c_int
_sg_p = C.c_void_p
_lib.soap_surrogate_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_void_p,
                                       C.POINTER(_sg_p)]
_lib.soap_surrogate_create.restype = C.c_int
_lib.soap_surrogate_n_params.argtypes = [_sg_p]
_lib.soap_surrogate_n_params.restype = C.c_int64
_lib.soap_surrogate_train_step.argtypes = [_sg_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                           C.POINTER(C.c_float)]
_lib.soap_surrogate_train_step.restype = C.c_int
_lib.soap_surrogate_predict.argtypes = [_sg_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
_lib.soap_surrogate_predict.restype = C.c_int
for _n in ("soap_surrogate_get_params", "soap_surrogate_set_params", "soap_surrogate_get_grads"):
    getattr(_lib, _n).argtypes = [_sg_p, C.c_int32, C.c_void_p]
    getattr(_lib, _n).restype = C.c_int
for _n in ("soap_surrogate_save", "soap_surrogate_load"):
    getattr(_lib, _n).argtypes = [_sg_p, C.c_char_p]
    getattr(_lib, _n).restype = C.c_int
_lib.soap_surrogate_last_error.argtypes = [_sg_p]
_lib.soap_surrogate_last_error.restype = C.c_char_p
_lib.soap_surrogate_destroy.argtypes = [_sg_p]
_lib.soap_surrogate_destroy.restype = None
_lib.soap_pca_project.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_int32,
                                  C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
_lib.soap_pca_project.restype = C.c_int
_lib.soap_surrogate_features.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
_lib.soap_surrogate_features.restype = C.c_int
_lib.soap_surrogate_gate.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_double, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p]
_lib.soap_surrogate_gate.restype = C.c_int


class SoapError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        super().__init__(f"{_lib.soap_status_string(status).decode()}: {message}")


def _is_tensor(x):
    return type(x).__module__.startswith("torch")


def _ptr(x):
    """(pointer, on_device) of a torch tensor or a numpy array."""
    if _is_tensor(x):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr(), 1 if x.is_cuda else 0
    if not x.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return x.ctypes.data, 0


def _stream_handle(stream):
    if stream is None:
        try:
            import torch

            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except ImportError:
            pass
        return None
    return getattr(stream, "cuda_stream", stream)


class Context:
    """Owns a soap_ctx* and the host objects its pointers were made from."""

    def __init__(self, handle, star, keep):
        self._pid = os.getpid()
        self.handle = handle
        self.star = star
        self._keep = keep
        self.precision = int(star.precision)
        self.n_pix = int(star.n_pix)
        self.dtype = np.float32 if self.precision == PREC_FP32 else np.float64

    def __del__(self, _destroy=_lib.soap_destroy):
        if getattr(self, "_pid", None) != os.getpid():
            return  # a forked child must not touch its parent's device state
        h = getattr(self, "handle", None)
        if h:
            _destroy(h)
            self.handle = None


def _check(st, ctx_handle):
    if st != SOAP_OK:
        raise SoapError(st, _lib.soap_last_error(ctx_handle).decode())


def abi_version():
    return int(_lib.soap_abi_version())


def device_bytes():
    """Bytes of device memory the library holds in this process."""
    return int(_lib.soap_device_bytes())


def soap_grid_init(star, stream=None):
    d = StarDesc()
    d.n_grid = int(star.n_grid)
    mu = np.ascontiguousarray(star.mu_bins, dtype=np.float64)
    d.n_mu = len(mu)
    d.n_pix = int(star.n_pix)
    d.vsini_kms = float(star.vsini_kms)
    d.incl_deg = float(star.incl_deg)
    d.ld_u1 = float(star.ld_u1)
    d.ld_u2 = float(star.ld_u2)
    d.ln_lambda0 = float(star.ln_lambda0)
    d.dln_lambda = float(star.dln_lambda)
    d.mu_bins = mu.ctypes.data_as(C.POINTER(C.c_double))
    keep = [mu]
    on_dev = None
    want = np.float32 if int(star.precision) == PREC_FP32 else np.float64
    for t in range(3):
        s = star.spectra[t]
        if s is None:
            d.spectra[t] = None
            continue
        if not _is_tensor(s):
            s = np.ascontiguousarray(s, dtype=want)
        keep.append(s)
        p, dev = _ptr(s)
        if on_dev is None:
            on_dev = dev
        elif on_dev != dev:
            raise ValueError("spectra must all be host arrays or all device tensors")
        d.spectra[t] = p
    d.spectra_on_device = int(on_dev or 0)
    d.precision = int(star.precision)
    d.contrast_mode = int(getattr(star, "contrast_mode", CONTRAST_SCALAR))
    con = getattr(star, "contrast", None) or [None, None, None]
    for t in range(3):
        a = con[t] if d.contrast_mode == CONTRAST_ARRAY else None
        if a is None:
            d.contrast[t] = None
            continue
        if not _is_tensor(a):
            a = np.ascontiguousarray(a, dtype=want)
        keep.append(a)
        p, dev = _ptr(a)
        if dev != d.spectra_on_device:
            raise ValueError("contrast arrays must sit where the spectra are (host or device)")
        d.contrast[t] = p
    d.teff_k = float(getattr(star, "teff_k", 5778.0))
    d.dt_spot_k = float(getattr(star, "dt_spot_k", 0.0))
    coef = tuple(getattr(star, "dt_fac_coef", (0.0, 0.0, 0.0)))
    for i in range(3):
        d.dt_fac_coef[i] = float(coef[i])
    d.diff_rot = float(getattr(star, "diff_rot", 0.0) or 0.0)
    h = _ctx_p()
    st = _lib.soap_grid_init(C.byref(d), _stream_handle(stream), C.byref(h))
    _check(st, None)
    return Context(h, star, keep)


def soap_quiet_spectrum(ctx, out):
    p, dev = _ptr(out)
    _check(_lib.soap_quiet_spectrum(ctx.handle, p, dev), ctx.handle)
    return out


def _regions(regions):
    arr = (RegionC * max(1, len(regions)))()
    for i, r in enumerate(regions):
        arr[i].type = int(r.type)
        arr[i].lat_deg = float(r.lat_deg)
        arr[i].lon_deg = float(r.lon_deg)
        arr[i].radius = float(r.radius)
        arr[i].contrast = float(r.contrast)
    return arr


def soap_active_spectra(ctx, regions, phases, effect, out):
    ph = np.ascontiguousarray(phases, dtype=np.float64)
    regs = _regions(regions)
    p, dev = _ptr(out)
    st = _lib.soap_active_spectra(
        ctx.handle, regs, len(regions), ph.ctypes.data_as(C.POINTER(C.c_double)), len(ph), int(effect), p, dev
    )
    _check(st, ctx.handle)
    return out


REGION_DTYPE = np.dtype(
    [("type", "<i4"), ("reserved0", "<i4"), ("lat_deg", "<f8"), ("lon_deg", "<f8"), ("radius", "<f8"),
     ("contrast", "<f8")]
)


def region_array(type_, lat_deg, lon_deg, radius, contrast):
    """Host soap_region array from per-region columns (numpy)."""
    a = np.zeros(len(np.atleast_1d(lat_deg)), dtype=REGION_DTYPE)
    a["type"], a["lat_deg"], a["lon_deg"], a["radius"], a["contrast"] = type_, lat_deg, lon_deg, radius, contrast
    return a


def soap_active_spectra_jobs(ctx, job_regions, job_phases, effect, out, region_offsets=None, phase_offsets=None):
    """Many (region list, phases) jobs of one star in one call; out rows
    follow the jobs' phases in order.  Either lists of region lists and of
    phase arrays, or (fast path) a REGION_DTYPE array, a flat phase array and
    the two offset arrays."""
    if region_offsets is None:
        regs = [r for rl in job_regions for r in rl]
        arr = np.zeros(len(regs), dtype=REGION_DTYPE)
        for i, r in enumerate(regs):
            arr[i] = (int(r.type), 0, float(r.lat_deg), float(r.lon_deg), float(r.radius), float(r.contrast))
        roff = np.zeros(len(job_regions) + 1, np.int32)
        roff[1:] = np.cumsum([len(rl) for rl in job_regions])
        ph = np.concatenate([np.asarray(p, np.float64).reshape(-1) for p in job_phases])
        poff = np.zeros(len(job_phases) + 1, np.int32)
        poff[1:] = np.cumsum([np.asarray(p).size for p in job_phases])
    else:
        arr = np.ascontiguousarray(job_regions, dtype=REGION_DTYPE)
        ph = job_phases
        roff = np.ascontiguousarray(region_offsets, dtype=np.int32)
        poff = np.ascontiguousarray(phase_offsets, dtype=np.int32)
    ph = np.ascontiguousarray(ph, dtype=np.float64)
    if len(arr) == 0:
        arr = np.zeros(1, dtype=REGION_DTYPE)
    p, dev = _ptr(out)
    st = _lib.soap_active_spectra_jobs(ctx.handle, arr.ctypes.data, roff.ctypes.data, ph.ctypes.data,
                                       poff.ctypes.data, len(roff) - 1, int(effect), p, dev)
    _check(st, ctx.handle)
    return out


EVOLVE_NONE, EVOLVE_LINEAR_GROWTH, EVOLVE_LINEAR_DECAY, EVOLVE_ASYM_GAUSS = 0, 1, 2, 3


class EvolutionC(C.Structure):
    _fields_ = [
        ("mode", C.c_int32),
        ("reserved0", C.c_int32),
        ("t0_days", C.c_double),
        ("size0_msh", C.c_double),
        ("rate_msh_day", C.c_double),
        ("fwhm_days", C.c_double),
        ("asym_per_day", C.c_double),
    ]


_lib.soap_evolution_size.argtypes = [C.POINTER(EvolutionC), C.c_double]
_lib.soap_evolution_size.restype = C.c_double
_lib.soap_active_spectra_evolving.argtypes = [_ctx_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                              C.c_double, C.c_int32, C.c_void_p, C.c_int32]
_lib.soap_active_spectra_evolving.restype = C.c_int


def _law(law):
    e = EvolutionC()
    e.mode = int(law["mode"])
    e.t0_days = float(law["t0_days"])
    e.size0_msh = float(law["size0_msh"])
    e.rate_msh_day = float(law.get("rate_msh_day", 0.0))
    e.fwhm_days = float(law.get("fwhm_days", 1.0))
    e.asym_per_day = float(law.get("asym_per_day", 0.0))
    return e


def soap_evolution_size(law, t_days):
    """Size in MSH of a region following ``law`` (a dict of soap_evolution's
    fields) at time t_days."""
    e = _law(law)
    return float(_lib.soap_evolution_size(C.byref(e), float(t_days)))


def soap_active_spectra_evolving(ctx, regions, laws, phases, prot_days, effect, out):
    """Spectra of regions whose sizes follow ``laws`` (one dict per region)."""
    ph = np.ascontiguousarray(phases, dtype=np.float64)
    regs = _regions(regions)
    arr = (EvolutionC * max(1, len(laws)))()
    for i, law in enumerate(laws):
        arr[i] = _law(law)
    p, dev = _ptr(out)
    st = _lib.soap_active_spectra_evolving(ctx.handle, regs, arr, len(regions), ph.ctypes.data, len(ph),
                                           float(prot_days), int(effect), p, dev)
    _check(st, ctx.handle)
    return out


_lib.soap_instrument_lsf.argtypes = [_ctx_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_int32]
_lib.soap_instrument_lsf.restype = C.c_int
_lib.soap_set_instrument.argtypes = [_ctx_p, C.c_double]
_lib.soap_set_instrument.restype = C.c_int


def soap_instrument_lsf(ctx, flux, out, resolution):
    """Lowers the rows of flux ([n_spec][n_pix]) to ``resolution`` into out."""
    pi, di = _ptr(flux)
    po, do = _ptr(out)
    if di != do:
        raise ValueError("flux and out must both be host arrays or both device tensors")
    n = int(flux.shape[0]) if len(flux.shape) == 2 else 1
    _check(_lib.soap_instrument_lsf(ctx.handle, pi, po, n, float(resolution), di), ctx.handle)
    return out


def soap_set_instrument(ctx, resolution):
    """Later active-spectra calls return spectra lowered to ``resolution``
    (0 = off)."""
    _check(_lib.soap_set_instrument(ctx.handle, float(resolution)), ctx.handle)


_lib.soap_ccf_rv_noalloc.argtypes = [_ctx_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.soap_ccf_rv_noalloc.restype = C.c_int


def soap_ccf_rv_noalloc(ctx, flux, mask, ccf_out=None, rv_out=None):
    """soap_ccf_rv without allocation: device flux, device outputs (or None),
    the context's current mask."""
    pf, df = _ptr(flux)
    if not df:
        raise ValueError("flux must be a device tensor")
    n = int(flux.shape[0]) if len(flux.shape) == 2 else 1
    m, keep = _mask(mask)
    pc = 0
    if ccf_out is not None:
        pc, dc = _ptr(ccf_out)
        if not dc:
            raise ValueError("ccf_out must be a device tensor")
    pr = 0
    if rv_out is not None:
        pr, dr = _ptr(rv_out)
        if not dr:
            raise ValueError("rv_out must be a device tensor")
    st = _lib.soap_ccf_rv_noalloc(ctx.handle, pf, n, C.byref(m), pc or None, pr or None)
    _check(st, ctx.handle)
    return ccf_out, rv_out


def _mask(mask):
    m = MaskC()
    lnl = np.ascontiguousarray(mask.ln_lambda, dtype=np.float64)
    w = np.ascontiguousarray(mask.weight, dtype=np.float64)
    m.n_lines = len(lnl)
    m.ln_lambda = lnl.ctypes.data_as(C.POINTER(C.c_double))
    m.weight = w.ctypes.data_as(C.POINTER(C.c_double))
    m.half_width_kms = float(mask.half_width_kms)
    m.v0_kms = float(mask.v0_kms)
    m.dv_kms = float(mask.dv_kms)
    m.n_v = int(mask.n_v)
    return m, (lnl, w)


def soap_ccf_rv(ctx, flux, mask, ccf_out=None, rv_out=None, n_spec=None):
    """CCF (double, [n_spec][n_v]) and Gaussian-fit RVs (RV_DTYPE records)."""
    fp, fdev = _ptr(flux)
    if n_spec is None:
        n_spec = int(np.prod(flux.shape[:-1])) if len(flux.shape) > 1 else 1
    m, keep = _mask(mask)
    cp, cdev = (None, 0) if ccf_out is None else _ptr(ccf_out)
    rp, rdev = (None, 0) if rv_out is None else _ptr(rv_out)
    st = _lib.soap_ccf_rv(ctx.handle, fp, fdev, int(n_spec), C.byref(m), cp, cdev, rp, rdev)
    del keep
    _check(st, ctx.handle)
    return ccf_out, rv_out


def soap_profile_enable(ctx, on=True):
    _check(_lib.soap_profile_enable(ctx.handle, 1 if on else 0), ctx.handle)


def soap_profile_read(ctx):
    p = ProfileC()
    _check(_lib.soap_profile_read(ctx.handle, C.byref(p)), ctx.handle)
    return {k: getattr(p, k) for k, _ in ProfileC._fields_}


def soap_sync(ctx):
    _check(_lib.soap_sync(ctx.handle), ctx.handle)


def soap_destroy(ctx):
    if ctx.handle:
        _lib.soap_destroy(ctx.handle)
        ctx.handle = None


def soap_last_error(ctx=None):
    return _lib.soap_last_error(ctx.handle if ctx is not None else None).decode()


def rv_records(n):
    """Host array for soap_ccf_rv's rv_out."""
    return np.zeros(n, dtype=RV_DTYPE)


# ---- linear CCF, surrogate network, PCA projection, gate --------------------


def _dptr(x, what):
    """Device pointer of a contiguous GPU tensor (None passes through)."""
    if x is None:
        return None
    if not (_is_tensor(x) and x.is_cuda and x.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous GPU tensor")
    return x.data_ptr()


def soap_ccf_linear_rv(ctx, coef, base, basis, ccf_out=None, rv_out=None):
    """Fits CCF rows base + coef @ basis (device tensors; see soap.h)."""
    n, k = int(coef.shape[0]), int(coef.shape[1])
    st = _lib.soap_ccf_linear_rv(ctx.handle, _dptr(coef, "coef"), n, k, _dptr(base, "base"), _dptr(basis, "basis"),
                                 _dptr(ccf_out, "ccf_out"), _dptr(rv_out, "rv_out"))
    _check(st, ctx.handle)
    return ccf_out, rv_out


class Surrogate:
    """Owns a soap_surrogate*."""

    def __init__(self, handle, n_in, hidden, n_out, n_ens):
        self._pid = os.getpid()
        self.handle = handle
        self.n_in, self.hidden, self.n_out, self.n_ens = n_in, hidden, n_out, n_ens

    def __del__(self, _destroy=_lib.soap_surrogate_destroy):
        if getattr(self, "_pid", None) != os.getpid():
            return  # a forked child must not touch its parent's device state
        h = getattr(self, "handle", None)
        if h:
            _destroy(h)
            self.handle = None


def _sg_check(st, s):
    if st != SOAP_OK:
        msg = _lib.soap_surrogate_last_error(s.handle).decode() if s is not None and s.handle else ""
        raise SoapError(st, msg)


def soap_surrogate_create(n_in, hidden, n_out, n_ensemble=1, seed=0, stream=None):
    h = _sg_p()
    st = _lib.soap_surrogate_create(int(n_in), int(hidden), int(n_out), int(n_ensemble), int(seed) & (2**64 - 1),
                                    _stream_handle(stream), C.byref(h))
    _sg_check(st, None)
    return Surrogate(h, int(n_in), int(hidden), int(n_out), int(n_ensemble))


def soap_surrogate_n_params(s):
    return int(_lib.soap_surrogate_n_params(s.handle))


def soap_surrogate_train_step(s, x, y, lr, want_loss=True):
    loss = C.c_float(0.0)
    st = _lib.soap_surrogate_train_step(s.handle, _dptr(x, "x"), _dptr(y, "y"), int(x.shape[0]), float(lr),
                                        C.byref(loss) if want_loss else None)
    _sg_check(st, s)
    return float(loss.value) if want_loss else None


def soap_surrogate_predict(s, x, coef, members=None):
    st = _lib.soap_surrogate_predict(s.handle, _dptr(x, "x"), int(x.shape[0]), _dptr(coef, "coef"),
                                     _dptr(members, "members"))
    _sg_check(st, s)
    return coef, members


def _host_f32(a, n):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.size != n:
        raise ValueError(f"expected {n} floats, got {a.size}")
    return a


def soap_surrogate_get_params(s, member=0):
    out = np.empty(soap_surrogate_n_params(s), np.float32)
    _sg_check(_lib.soap_surrogate_get_params(s.handle, int(member), out.ctypes.data), s)
    return out


def soap_surrogate_get_grads(s, member=0):
    out = np.empty(soap_surrogate_n_params(s), np.float32)
    _sg_check(_lib.soap_surrogate_get_grads(s.handle, int(member), out.ctypes.data), s)
    return out


def soap_surrogate_set_params(s, member, params):
    a = _host_f32(params, soap_surrogate_n_params(s))
    _sg_check(_lib.soap_surrogate_set_params(s.handle, int(member), a.ctypes.data), s)


def soap_surrogate_save(s, path):
    _sg_check(_lib.soap_surrogate_save(s.handle, os.fsencode(path)), s)


def soap_surrogate_load(s, path):
    _sg_check(_lib.soap_surrogate_load(s.handle, os.fsencode(path)), s)


def soap_surrogate_destroy(s):
    if s.handle:
        _lib.soap_surrogate_destroy(s.handle)
        s.handle = None


def soap_pca_project(d, mean, V, coef, n_pix=None, stream=None, mean_index=None):
    """coef[n][k] = (d[:, :n_pix] - mean) @ V, FP32 on the GPU (mean row
    mean_index[i] of a [rows][n_pix] mean when mean_index is given)."""
    n, ld = int(d.shape[0]), int(d.shape[1])
    n_pix = ld if n_pix is None else int(n_pix)
    n_mean = int(mean.shape[0]) if (mean_index is not None and mean.dim() == 2) else 1
    st = _lib.soap_pca_project(_dptr(d, "d"), n, n_pix, ld, _dptr(mean, "mean"), _dptr(mean_index, "mean_index"),
                               n_mean, _dptr(V, "V"), int(V.shape[1]), _dptr(coef, "coef"), _stream_handle(stream))
    _sg_check(st, None)
    return coef


def soap_surrogate_features(raw, x, stream=None):
    """Network inputs x [n][12] (float32, device) of raw sample descriptions
    raw [n][8] (float64, device; see soap.h)."""
    n = int(raw.shape[0])
    if tuple(raw.shape) != (n, 8) or tuple(x.shape) != (n, 12):
        raise ValueError("raw must be [n][8] and x [n][12]")
    st = _lib.soap_surrogate_features(_dptr(raw, "raw"), n, _dptr(x, "x"), _stream_handle(stream))
    _sg_check(st, None)
    return x


def soap_surrogate_gate(rv, n, n_ens, calib, threshold_kms, rv_kms, fallback, err_kms=None, stream=None):
    st = _lib.soap_surrogate_gate(_dptr(rv, "rv"), int(n), int(n_ens), float(calib), float(threshold_kms),
                                  _dptr(rv_kms, "rv_kms"), _dptr(err_kms, "err_kms"), _dptr(fallback, "fallback"),
                                  _stream_handle(stream))
    _sg_check(st, None)


def soap_surrogate_rv(ctx, coef, members, base, basis, calib, threshold_kms, rv_kms, fallback, err_kms=None,
                      rv_out=None, base_index=None):
    """Fused surrogate RV + gate (see soap.h); members [n_ens][n][k]; with
    base_index (int32 [n]) base is [rows][n_v], one row per star."""
    n, k = int(coef.shape[0]), int(coef.shape[1])
    n_ens = int(members.shape[0]) if members.dim() == 3 else int(members.shape[0]) // n
    st = _lib.soap_surrogate_rv(ctx.handle, _dptr(coef, "coef"), _dptr(members, "members"), n, n_ens, k,
                                _dptr(base, "base"), _dptr(base_index, "base_index"),
                                int(base.shape[0]) if base_index is not None else 1, _dptr(basis, "basis"),
                                float(calib), float(threshold_kms),
                                _dptr(rv_out, "rv_out"), _dptr(rv_kms, "rv_kms"), _dptr(err_kms, "err_kms"),
                                _dptr(fallback, "fallback"))
    _check(st, ctx.handle)


def soap_set_apply_shape(ctx, depth=2, order=0, phases_per_chunk=0):
    """Shape of later shift-and-sum calls; phases_per_chunk 0 = the default."""
    _check(_lib.soap_set_apply_shape(ctx.handle, int(depth), int(order), int(phases_per_chunk)), ctx.handle)


def soap_autotune(ctx, regions, phases, effect, cache_path=None):
    """Times the shift-and-sum shapes on this workload; returns the choice."""
    ph = np.ascontiguousarray(phases, dtype=np.float64)
    regs = _regions(regions)
    t = TuneC()
    st = _lib.soap_autotune(ctx.handle, C.cast(regs, C.c_void_p), len(regions), ph.ctypes.data, len(ph), int(effect),
                            None if cache_path is None else os.fsencode(cache_path), C.byref(t))
    _check(st, ctx.handle)
    return {"depth": t.depth, "order": t.order, "phases_per_chunk": t.phases_per_chunk, "apply_us": t.apply_us,
            "from_cache": bool(t.from_cache),
            "n_tried": t.n_tried, "key": t.key.decode()}


class Batch:
    """Owns a soap_batch* and keeps its contexts and outputs alive."""

    def __init__(self, handle, ctxs, outs):
        self._pid = os.getpid()
        self.handle = handle
        self._ctxs = ctxs
        self.outs = outs

    def __del__(self, _destroy=_lib.soap_batch_destroy):
        if getattr(self, "_pid", None) != os.getpid():
            return  # a forked child must not touch its parent's device state
        h = getattr(self, "handle", None)
        if h:
            _destroy(h)
            self.handle = None


def soap_batch_create(ctxs, cfg_regions, cfg_phases, effect, outs, stream=None, mask=None, ccf_outs=None,
                      rv_outs=None):
    """One configuration per (ctx, region list, phases, output tensor).
    With mask, each run also computes every configuration's CCF (ccf_outs:
    device [phases][n_v] float64 tensors, or None) and Gaussian-fit RVs
    (rv_outs: device RV_DTYPE buffers, or None)."""
    n = len(ctxs)
    handles = (C.c_void_p * n)(*[C.cast(c.handle, C.c_void_p) for c in ctxs])
    regs = [r for rl in cfg_regions for r in rl]
    arr = np.zeros(max(1, len(regs)), dtype=REGION_DTYPE)
    for i, r in enumerate(regs):
        arr[i] = (int(r.type), 0, float(r.lat_deg), float(r.lon_deg), float(r.radius), float(r.contrast))
    roff = np.zeros(n + 1, np.int32)
    roff[1:] = np.cumsum([len(rl) for rl in cfg_regions])
    ph = np.ascontiguousarray(np.concatenate([np.asarray(p, np.float64).reshape(-1) for p in cfg_phases]))
    poff = np.zeros(n + 1, np.int32)
    poff[1:] = np.cumsum([np.asarray(p).size for p in cfg_phases])
    fl = (C.c_void_p * n)(*[_dptr(o, "flux") for o in outs])
    h = C.c_void_p()
    if mask is None:
        st = _lib.soap_batch_create(handles, n, arr.ctypes.data, roff.ctypes.data, ph.ctypes.data, poff.ctypes.data,
                                    int(effect), fl, _stream_handle(stream), C.byref(h))
        keep = []
    else:
        m, mkeep = _mask(mask)
        cc = (C.c_void_p * n)(*[None if ccf_outs is None or ccf_outs[i] is None else _dptr(ccf_outs[i], "ccf")
                                for i in range(n)])
        rr = (C.c_void_p * n)(*[None if rv_outs is None or rv_outs[i] is None else _dptr(rv_outs[i], "rv")
                                for i in range(n)])
        st = _lib.soap_batch_create_rv(handles, n, arr.ctypes.data, roff.ctypes.data, ph.ctypes.data,
                                       poff.ctypes.data, int(effect), fl, C.byref(m), cc, rr, _stream_handle(stream),
                                       C.byref(h))
        keep = [mkeep, ccf_outs, rv_outs]
    if st != SOAP_OK:
        raise SoapError(st, _lib.soap_batch_last_error(None).decode())
    b = Batch(h, list(ctxs), list(outs))
    b._keep = keep
    return b


def _batch_arrays(ctxs, cfg_regions, cfg_phases, outs):
    n = len(ctxs)
    handles = (C.c_void_p * n)(*[C.cast(c.handle, C.c_void_p) for c in ctxs])
    regs = [r for rl in cfg_regions for r in rl]
    arr = np.zeros(max(1, len(regs)), dtype=REGION_DTYPE)
    for i, r in enumerate(regs):
        arr[i] = (int(r.type), 0, float(r.lat_deg), float(r.lon_deg), float(r.radius), float(r.contrast))
    roff = np.zeros(n + 1, np.int32)
    roff[1:] = np.cumsum([len(rl) for rl in cfg_regions])
    ph = np.ascontiguousarray(np.concatenate([np.asarray(p, np.float64).reshape(-1) for p in cfg_phases]))
    poff = np.zeros(n + 1, np.int32)
    poff[1:] = np.cumsum([np.asarray(p).size for p in cfg_phases])
    fl = (C.c_void_p * n)(*[_dptr(o, "flux") for o in outs])
    return handles, arr, roff, ph, poff, fl


def soap_active_spectra_multi(ctxs, cfg_regions, cfg_phases, effect, outs, stream=None):
    """One synthesis call over many configurations of many stars (ctx, region
    list, phases, device output each); waits for the stream."""
    n = len(ctxs)
    handles, arr, roff, ph, poff, fl = _batch_arrays(ctxs, cfg_regions, cfg_phases, outs)
    st = _lib.soap_active_spectra_multi(handles, n, arr.ctypes.data, roff.ctypes.data, ph.ctypes.data,
                                        poff.ctypes.data, int(effect), fl, _stream_handle(stream))
    if st != SOAP_OK:
        raise SoapError(st, _lib.soap_batch_last_error(None).decode())


def soap_active_spectra_multi_arrays(handles, regions, region_offsets, phases, phase_offsets, effect, flux_ptrs,
                                     stream=None):
    """The same call from prepared arrays: context handles and flux row
    pointers as uint64 arrays, REGION_DTYPE regions with int32 offsets,
    float64 phases with int32 offsets (no per-configuration Python work)."""
    h = np.ascontiguousarray(handles, dtype=np.uint64)
    regs = np.ascontiguousarray(regions)
    roff = np.ascontiguousarray(region_offsets, dtype=np.int32)
    ph = np.ascontiguousarray(phases, dtype=np.float64)
    poff = np.ascontiguousarray(phase_offsets, dtype=np.int32)
    fl = np.ascontiguousarray(flux_ptrs, dtype=np.uint64)
    n = len(h)
    if len(fl) != n or len(roff) != n + 1 or len(poff) != n + 1:
        raise ValueError("one handle, flux pointer and region / phase range per configuration")
    st = _lib.soap_active_spectra_multi(h.ctypes.data, n, regs.ctypes.data, roff.ctypes.data, ph.ctypes.data,
                                        poff.ctypes.data, int(effect), fl.ctypes.data, _stream_handle(stream))
    if st != SOAP_OK:
        raise SoapError(st, _lib.soap_batch_last_error(None).decode())


def soap_batch_run(batch):
    st = _lib.soap_batch_run(batch.handle)
    if st != SOAP_OK:
        raise SoapError(st, _lib.soap_batch_last_error(batch.handle).decode())


def soap_batch_n_spectra(batch):
    return int(_lib.soap_batch_n_spectra(batch.handle))


def soap_batch_destroy(batch):
    if batch.handle:
        _lib.soap_batch_destroy(batch.handle)
        batch.handle = None
