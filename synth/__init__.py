"""Seeded synthetic speckle bursts.

This package simulates the *inputs* of the speckle-masking reconstruction:
a granulation-like object, short-exposure frames blurred by independent
Kolmogorov turbulence, photon noise and 12-bit digitisation, plus a Monte
Carlo speckle transfer function table.  It holds none of the reconstruction
arithmetic and is shared by the oracle tests and the GPU tests/benchmarks as
the single source of inputs.
"""
from .burst import (  # noqa: F401
    CONFIGS,
    BurstConfig,
    make_object,
    phase_screen,
    pupil_psf,
    make_burst,
    stf_table,
    config_by_name,
    burst_seed,
)
