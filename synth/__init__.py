"""Seeded synthetic signal generators shared by the tests, the CPU oracle's
callers and the benchmark.

This package holds no codec arithmetic: it only draws random numbers and
builds float32 time series shaped like the four signal domains the codec is
evaluated on (biomedical, seismic, power-grid, meteorological).
"""
from .signals import (  # noqa: F401
    DOMAINS,
    ROOT_SEED,
    eeg_like,
    seismic_like,
    power_like,
    meteo_like,
    multichannel_eeg,
    domain_signal,
    stream_rng,
    training_rng,
    batch_lengths,
)
