"""Seeded synthetic inputs shared by the HIP path, the oracle tests and the benchmark.

This package only draws random numbers and builds input arrays (Hamiltonian block
bands, lead self-energies, energy grids).  It holds none of the selected-inversion
arithmetic: both the GPU library and the CPU oracle consume the arrays it returns.
"""
from .generators import (  # noqa: F401
    make_random,
    CONFIGS,
    Workload,
    band_block,
    lead_sigma,
    make_config,
    make_dominant,
    make_uniform_chain,
    midpoint_grid,
    random_hermitian_band,
    surface_sigma,
)
