"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only draws random numbers and assembles test matrices from planted
spectra; it holds none of the arithmetic of the partial-spectrum method itself.
"""
from .generators import (  # noqa: F401
    rng, haar, planted_sym, planted_general,
    eig_uniform, eig_clustered, svd_geometric, svd_loguniform,
    haar_complex, planted_herm, heig_uniform, heig_clustered,
    request_trace, CONFIG_SEEDS,
)
