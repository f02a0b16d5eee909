"""Seeded synthetic scans shared by the tests, the bench and the oracle checks.

This package only *draws inputs*: pointing (pixel index per sample), polariser
weights, stationary-interval boundaries, per-interval noise-PSD parameters, a
sky map and a noise realisation.  It contains none of the map-making solver's
arithmetic (no noise weighting, no pointing or de-pointing of maps, no
preconditioner, no Krylov solver): each consumer builds the time-ordered data
d = P m + n from these pieces with its own code.
"""

from .scans import (  # noqa: F401
    Scan,
    cfg1_raster_i,
    cfg2_raster_iqu,
    cfg3_ring_iqu,
    cfg4_batched_iqu,
    cfg5_raster_iqu,
    raster_i,
    raster_iqu,
    ring_iqu,
    noise_realisation,
    subset_intervals,
)
