"""Seeded synthetic inputs shared by the CPU oracle tests and the HIP path.

This package only *generates* inputs: sparse matrices in CSR form, start
blocks, intervals and request streams.  It contains none of the filtering
method's arithmetic (no coefficients, no recurrence, no projections), so the
oracle and the GPU path can both draw from it without sharing method code.
"""
from .matrices import (
    CSR,
    laplacian_2d_dirichlet,
    laplacian_3d_dirichlet,
    tight_binding_3d_periodic,
    random_banded_symmetric,
    random_dense_symmetric_csr,
    gershgorin_bounds,
)
from .blocks import probe_block, start_block
from .configs import CONFIGS, WorkloadConfig, build_config

__all__ = [
    "CSR",
    "laplacian_2d_dirichlet",
    "laplacian_3d_dirichlet",
    "tight_binding_3d_periodic",
    "random_banded_symmetric",
    "random_dense_symmetric_csr",
    "gershgorin_bounds",
    "probe_block",
    "start_block",
    "CONFIGS",
    "WorkloadConfig",
    "build_config",
]
