"""CCF (section 4.1, holes Doppler-shifted by Eq. 6) against the oracle over
the kernel's shape variants: holes one to eight pixels wide, velocity grids
wider than one thread per velocity and than the narrow stage, FP64 flux,
mask lines near, past and far past the spectrum ends, an unsorted mask and
a spectrum count that is not a multiple of the spectra per block.  The flux
rows are seeded uniform values, so every pixel's contribution counts."""
import numpy as np
import pytest
import torch

import paper_2301_04259_amd as L
import workloads as W
from oracle import ccf as OC

pytestmark = pytest.mark.gpu

C_KMS = 299792.458

# (seed, precision, hole width in pixels, n_v, velocity span in pixels,
#  lines past the ends, shuffled mask)
CASES = [
    (31, W.PREC_FP32, 1.5, 61, 40.0, False, False),
    (32, W.PREC_FP32, 3.0, 61, 60.0, False, False),
    (33, W.PREC_FP32, 6.0, 41, 80.0, False, False),
    (34, W.PREC_FP32, 0.9, 300, 200.0, False, False),
    (35, W.PREC_FP32, 0.9, 500, 300.0, False, False),
    (36, W.PREC_FP64, 0.9, 161, 46.0, False, False),
    (37, W.PREC_FP64, 2.5, 250, 400.0, False, False),
    (38, W.PREC_FP32, 0.9, 161, 46.0, True, True),
]


@pytest.mark.parametrize("seed,prec,hole_px,n_v,span_px,edge,shuffle", CASES)
def test_ccf_shapes_match_oracle(seed, prec, hole_px, n_v, span_px, edge, shuffle):
    n_pix, n_spec, n_lines = 3000, 13, 70
    star = W.make_tiny(seed, n_grid=8, n_pix=n_pix, n_mu=2, precision=prec, n_phases=1)
    print(f"[ccf-shapes] seed {seed} prec {prec} hole {hole_px} px n_v {n_v} span {span_px} px", flush=True)
    ctx = L.soap_grid_init(star)
    rng = np.random.default_rng(seed)
    px_kms = C_KMS * star.dln_lambda
    h = 0.5 * hole_px * px_kms
    dv = span_px * px_kms / (n_v - 1)
    v0 = -0.5 * dv * (n_v - 1)
    q = np.sort(rng.uniform(0.0, n_pix, n_lines))
    if edge:
        q[:3] = [-0.3 * span_px, -2.0, -1.0e5]
        q[-3:] = [n_pix + 1.5, n_pix + 0.4 * span_px, n_pix + 1.0e5]
    if shuffle:
        q = q[rng.permutation(n_lines)]
    ln_l = star.ln_lambda0 + (q - 0.5) * star.dln_lambda
    mask = W.Mask(ln_l, rng.uniform(0.5, 1.5, n_lines), h, v0, dv, n_v)
    dt = np.float64 if prec == W.PREC_FP64 else np.float32
    flux_h = rng.uniform(0.2, 1.0, (n_spec, n_pix)).astype(dt)
    flux = torch.from_numpy(flux_h).cuda()
    ccf = torch.empty((n_spec, n_v), dtype=torch.float64, device="cuda")
    L.soap_ccf_rv(ctx, flux, mask, ccf_out=ccf)
    torch.cuda.synchronize()
    v = W.make_velocity_grid(v0, dv, n_v)
    c_or = OC.ccf(flux_h.astype(np.float64), star.ln_lambda0, star.dln_lambda, ln_l, mask.weight, h, v)
    got = ccf.cpu().numpy()
    # FP64: hole edges ~1e-16 in ln(lambda) on either side, ~1e-10 pixel.
    # FP32 spectra are accumulated in FP32 per block of 32 lines: at most
    # 32 lines x 10 pixels of FMAs into one partial, each rounding by 2^-24
    # of the running (positive) sum, bounds the error by 2e-5 relative
    rel = np.max(np.abs(got - c_or) / np.abs(c_or))
    assert rel < (1e-9 if prec == W.PREC_FP64 else 2e-5), rel


def test_fit_wave_per_spectrum_equals_block_per_spectrum():
    """Calls of more than 512 spectra fit with one wave per spectrum, smaller
    ones with a block of four waves per spectrum; both add the partial CCFs
    in the same order, so the CCF and RV records are the same bit for bit."""
    star = W.make_tiny(39, n_grid=8, n_pix=3000, n_mu=2, precision=W.PREC_FP32, n_phases=1)
    print("[ccf-shapes] wave-per-spectrum fit vs block-per-spectrum fit, 700 spectra", flush=True)
    ctx = L.soap_grid_init(star)
    rng = np.random.default_rng(39)
    base = np.asarray(star.spectra[0][0], dtype=np.float64)
    flux_h = (base[None, :] * (1.0 + 1e-3 * rng.standard_normal((700, star.n_pix)))).astype(np.float32)
    flux = torch.from_numpy(flux_h).cuda()
    m = star.mask
    out = []
    for parts in ([700], [350, 350]):
        ccf = torch.empty((700, m.n_v), dtype=torch.float64, device="cuda")
        rv = torch.zeros(700 * L.RV_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        a = 0
        for n in parts:
            L.soap_ccf_rv(ctx, flux[a:a + n], m, ccf_out=ccf[a:a + n],
                          rv_out=rv[a * L.RV_DTYPE.itemsize:(a + n) * L.RV_DTYPE.itemsize])
            a += n
        torch.cuda.synchronize()
        out.append((ccf.cpu().numpy(), rv.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    rec = np.frombuffer(out[0][1].tobytes(), dtype=L.RV_DTYPE)
    assert np.mean(rec["status"] == 0) > 0.9
    L.soap_destroy(ctx)
