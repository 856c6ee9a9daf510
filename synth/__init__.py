"""Seeded synthetic sampler data for the spectrometer path.

This package emulates the digital sampler that feeds the spectrometer
(Gaussian noise, tones and weak spectral lines, quantised to 2/4/8-bit codes
and packed into the wire layout).  It holds none of the spectrometer's own
arithmetic and is shared by the tests, the benchmark and the oracle harness.
"""
from .gen import (  # noqa: F401
    SEED_BASE,
    rng_for,
    quantize,
    pack_codes,
    make_tiny,
    make_paper,
    make_precision,
    make_batching,
    batching_params,
    make_differentiation,
    make_tone_f32,
    make_identical_streams,
    make_fully_polarized_f32,
    make_correlated_noise,
    MODES,
    make_mode,
)
