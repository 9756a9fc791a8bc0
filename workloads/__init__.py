"""Seeded synthetic inputs shaped like the paper's workloads.

This module only *makes inputs*: local spectra per (surface type, mu bin),
active-region lists, phase lists and CCF masks.  It holds none of the disk
integration, interpolation, CCF or fitting arithmetic; the HIP library and the
CPU oracle each implement those on their own and both consume what is made
here.  The paper's own inputs (Kitt Peak atlases, PHOENIX spectra, the SOAP 2.0
CCF mask) are not available, so line-list spectra of the same shape stand in
for them.
"""
from . import bisectors  # noqa: F401
from .stars import (  # noqa: F401
    C_KMS,
    StarInputs,
    Region,
    Mask,
    QUIET,
    SPOT,
    FACULA,
    CONTRAST_SCALAR,
    CONTRAST_PLANCK,
    CONTRAST_ARRAY,
    EFFECT_TOT,
    EFFECT_FLUX,
    EFFECT_BCONV,
    PREC_FP64,
    PREC_FP32,
    cb_velocity_ms,
    make_cfg1,
    make_cfg2,
    make_cfg5,
    cfg5_window_spectra,
    cfg5_mask,
    cfg5_star,
    cfg5_multi_samples,
    MultiSpotSamples,
    CFG5_TEFF,
    CFG5_INCL,
    CFG5_VSINI,
    make_bank,
    full_range_lines,
    batch_configs,
    batch_star,
    bank_for,
    BANK_TEFF,
    cfg5_samples,
    SpotSamples,
    make_tiny,
    make_bisector_star,
    make_velocity_grid,
    input_digest,
)
