"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds input generators only (fields, block cuts, initial parameter
draws, explicit coordinate sets).  It contains none of the representation's
arithmetic: no resolution tables, no hashing, no interpolation of the method's
own, no network.  Both sides of every parity test import it; neither side is
imported by it.
"""
from .fields import (  # noqa: F401
    gaussian_sum_field,
    kolmogorov_field,
    kolmogorov_field_torch,
    advected_blobs_field,
    advected_blob_trajectories,
    advected_blobs_series_torch,
    cut_blocks,
    uneven_block_sizes,
    init_param_draws,
    uniform_coords,
    adversarial_coords,
)
