"""Batches over many stars as one HIP graph (soap_batch_*): every
configuration's spectra equal the single call's bit for bit, on every
replay, and match the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import spectrum as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2301_04259_amd", reason="libsoap.so not built")


def _say(*a):
    print("[batch]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _stars():
    import dataclasses

    return [
        W.make_tiny(11, n_grid=16, n_pix=700, precision=W.PREC_FP64),
        W.make_tiny(12, n_grid=40, n_pix=3300, n_mu=6, precision=W.PREC_FP32, contrast_mode=W.CONTRAST_PLANCK),
        W.make_tiny(13, n_grid=24, n_pix=1500, n_mu=3, precision=W.PREC_FP32),
        W.make_tiny(14, n_grid=64, n_pix=5000, n_mu=8, precision=W.PREC_FP32, with_facula=False),
        # differential rotation: its table kernels stay one launch per configuration
        dataclasses.replace(W.make_tiny(15, n_grid=30, n_pix=2000, n_mu=4, precision=W.PREC_FP32), diff_rot=-0.18),
    ]


def test_batch_equals_single_calls_on_every_replay():
    stars = _stars()
    ctxs = [L.soap_grid_init(s) for s in stars]
    # stars on different apply shapes: one launch per group of equal shape
    L.soap_set_apply_shape(ctxs[0], 2, 0, 8)
    L.soap_set_apply_shape(ctxs[2], 3, 0, 16)
    L.soap_set_apply_shape(ctxs[3], 2, 1, 16)
    rng = np.random.default_rng(7)
    cfg_ctx, cfg_star, cfg_regs, cfg_ph, outs = [], [], [], [], []
    for i in range(16):  # stars repeat; region lists and phase counts vary
        k = i % len(stars)
        s = stars[k]
        nr = int(rng.integers(0, 4))
        types = [W.SPOT, W.FACULA] if s.spectra[W.FACULA] is not None else [W.SPOT]
        regs = [W.Region(int(rng.choice(types)), float(rng.uniform(-60, 60)), float(rng.uniform(0, 360)),
                         float(rng.uniform(0.05, 0.4)), float(rng.choice([1.0, rng.uniform(0.3, 1.4)])))
                for _ in range(nr)]
        ph = rng.uniform(0, 1, int(rng.integers(1, 40)))
        dt = torch.float32 if s.precision == W.PREC_FP32 else torch.float64
        cfg_ctx.append(ctxs[k])
        cfg_star.append(s)
        cfg_regs.append(regs)
        cfg_ph.append(ph)
        outs.append(torch.full((len(ph), s.n_pix), -1.0, dtype=dt, device="cuda"))
    b = L.soap_batch_create(cfg_ctx, cfg_regs, cfg_ph, W.EFFECT_TOT, outs)
    assert L.soap_batch_n_spectra(b) == sum(len(p) for p in cfg_ph)
    want = []
    for c, s, regs, ph, o in zip(cfg_ctx, cfg_star, cfg_regs, cfg_ph, outs):
        one = torch.empty_like(o)
        L.soap_active_spectra(c, regs, ph, W.EFFECT_TOT, one)
        want.append(one.cpu().numpy())
    for rep in range(3):
        for o in outs:
            o.fill_(-1.0)
        torch.cuda.synchronize()
        L.soap_batch_run(b)
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            np.testing.assert_array_equal(o.cpu().numpy(), want[i], err_msg=f"replay {rep} configuration {i}")
        # eager work on the same contexts between replays
        L.soap_active_spectra(cfg_ctx[1], cfg_regs[1], cfg_ph[1], W.EFFECT_TOT, torch.empty_like(outs[1]))
        torch.cuda.synchronize()
    worst = 0.0
    for i in (0, 1, 2, 4, 7):
        s = cfg_star[i]
        f = OS.integrated(s, cfg_ph[i][0], OS.TOT, regions=cfg_regs[i])
        e = np.max(np.abs(want[i][0] - f) / np.maximum(np.abs(f), 1e-3 * np.abs(f).max()))
        worst = max(worst, e)
    _say(f"16 configurations over 5 stars, worst relative error vs oracle {worst:.2e}")
    assert worst <= 1e-6
    L.soap_batch_destroy(b)
    for c in ctxs:
        L.soap_destroy(c)


def test_batch_argument_checks():
    s = _stars()[2]
    c = L.soap_grid_init(s)
    o = torch.empty((2, s.n_pix), dtype=torch.float32, device="cuda")
    r = W.Region(W.FACULA, 10.0, 20.0, 0.2, 0.5)  # this star has no facula spectra
    with pytest.raises(L.SoapError):
        L.soap_batch_create([c], [[W.Region(W.SPOT, 10.0, 20.0, 1.5, 0.5)]], [np.array([0.1, 0.2])],
                            W.EFFECT_TOT, [o])
    s4 = _stars()[3]
    c4 = L.soap_grid_init(s4)
    o4 = torch.empty((1, s4.n_pix), dtype=torch.float32, device="cuda")
    with pytest.raises(L.SoapError):
        L.soap_batch_create([c4], [[r]], [np.array([0.1])], W.EFFECT_TOT, [o4])
    L.soap_destroy(c)
    L.soap_destroy(c4)


def test_batch_ccf_and_fit_equal_single_calls():
    """The CCF + fit stage of a batch graph gives, on every replay, what
    soap_ccf_rv gives on the same spectra, bit for bit (section 4.1)."""
    stars = [W.make_tiny(21, n_grid=30, n_pix=2600, n_mu=4, precision=W.PREC_FP32, contrast_mode=W.CONTRAST_PLANCK),
             W.make_tiny(21, n_grid=44, n_pix=2600, n_mu=4, precision=W.PREC_FP32),
             # FP64: a second CCF layout, so a second pair of work-list launches
             W.make_tiny(21, n_grid=36, n_pix=2600, n_mu=4, precision=W.PREC_FP64)]
    mask = stars[0].mask
    ctxs = [L.soap_grid_init(s) for s in stars]
    L.soap_set_apply_shape(ctxs[1], 2, 0, 16)
    rng = np.random.default_rng(9)
    cfg_ctx, cfg_regs, cfg_ph, outs, ccfs, rvs = [], [], [], [], [], []
    for i in range(7):
        k = i % 3
        regs = [W.Region(W.SPOT, float(rng.uniform(-50, 50)), float(rng.uniform(0, 360)), float(rng.uniform(0.1, 0.3)),
                         0.6)]
        ph = np.sort(rng.uniform(0, 1, int(rng.integers(3, 30))))
        cfg_ctx.append(ctxs[k])
        cfg_regs.append(regs)
        cfg_ph.append(ph)
        dt = torch.float32 if stars[k].precision == W.PREC_FP32 else torch.float64
        outs.append(torch.empty((len(ph), stars[k].n_pix), dtype=dt, device="cuda"))
        ccfs.append(torch.full((len(ph), mask.n_v), -1.0, dtype=torch.float64, device="cuda") if i != 3 else None)
        rvs.append(torch.zeros(len(ph) * L.RV_DTYPE.itemsize, dtype=torch.uint8, device="cuda") if i != 5 else None)
    _say("batch with CCF + fit: 7 configurations over 3 stars, two precisions")
    b = L.soap_batch_create(cfg_ctx, cfg_regs, cfg_ph, W.EFFECT_TOT, outs, mask=mask, ccf_outs=ccfs, rv_outs=rvs)
    for rep in range(2):
        for o in outs:
            o.fill_(-1.0)
        torch.cuda.synchronize()
        L.soap_batch_run(b)
        torch.cuda.synchronize()
        for i in range(7):
            c1 = torch.empty((len(cfg_ph[i]), mask.n_v), dtype=torch.float64, device="cuda")
            r1 = torch.zeros(len(cfg_ph[i]) * L.RV_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
            L.soap_ccf_rv(cfg_ctx[i], outs[i], mask, ccf_out=c1, rv_out=r1)
            torch.cuda.synchronize()
            if ccfs[i] is not None:
                np.testing.assert_array_equal(ccfs[i].cpu().numpy(), c1.cpu().numpy(), err_msg=f"replay {rep} ccf {i}")
            if rvs[i] is not None:
                got = np.frombuffer(rvs[i].cpu().numpy().tobytes(), dtype=L.RV_DTYPE)
                want = np.frombuffer(r1.cpu().numpy().tobytes(), dtype=L.RV_DTYPE)
                np.testing.assert_array_equal(got["rv_kms"], want["rv_kms"], err_msg=f"replay {rep} rv {i}")
                assert np.array_equal(got["status"], want["status"])
    L.soap_batch_destroy(b)
    for c in ctxs:
        L.soap_destroy(c)


def test_multi_context_call_equals_single_calls():
    """soap_active_spectra_multi: one call over configurations of several
    stars gives every configuration's single-call spectra bit for bit; a
    second, larger call reuses and grows the library's arena."""
    stars = _stars()
    ctxs = [L.soap_grid_init(s) for s in stars]
    rng = np.random.default_rng(17)
    for n_cfg in (6, 23):
        cfg_ctx, cfg_star, cfg_regs, cfg_ph, outs = [], [], [], [], []
        for i in range(n_cfg):
            k = int(rng.integers(0, len(stars)))
            s = stars[k]
            types = [W.SPOT, W.FACULA] if s.spectra[W.FACULA] is not None else [W.SPOT]
            regs = [W.Region(int(rng.choice(types)), float(rng.uniform(-60, 60)), float(rng.uniform(0, 360)),
                             float(rng.uniform(0.05, 0.3)), 1.0) for _ in range(int(rng.integers(0, 3)))]
            ph = rng.uniform(0, 1, int(rng.integers(1, 20)))
            dt = torch.float32 if s.precision == W.PREC_FP32 else torch.float64
            cfg_ctx.append(ctxs[k])
            cfg_star.append(s)
            cfg_regs.append(regs)
            cfg_ph.append(ph)
            outs.append(torch.full((len(ph), s.n_pix), -1.0, dtype=dt, device="cuda"))
        _say(f"multi-context call: {n_cfg} configurations")
        L.soap_active_spectra_multi(cfg_ctx, cfg_regs, cfg_ph, W.EFFECT_TOT, outs)
        for i in range(n_cfg):
            one = torch.empty_like(outs[i])
            L.soap_active_spectra(cfg_ctx[i], cfg_regs[i], cfg_ph[i], W.EFFECT_TOT, one)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(outs[i].cpu().numpy(), one.cpu().numpy(), err_msg=f"{n_cfg}: cfg {i}")
    for c in ctxs:
        L.soap_destroy(c)
