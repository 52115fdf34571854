"""The synthetic workloads: matrix recipe, spectral bounds, interval, block width, degree.

Sizes follow the five workloads the build is measured on:

1. 2D 5-point Dirichlet Laplacian 64x64 (n = 4096), window holding exactly 40
   eigenvalues (#38..#77 of the closed-form spectrum), p = 64, degree 60, Jackson, FP64.
2. 3D 7-point Dirichlet Laplacian 100^3 (n = 1e6) + 2*U(0,1) diagonal potential,
   mid-spectrum window, p = 256, degree 120, Jackson, FP64 and FP32 filter.
3. Complex tight-binding 64^3 periodic lattice (n = 262144), window around 0,
   p = 192, degree 150, Jackson, complex FP64 and complex FP32 filter.
4. Random irregular symmetric n = 2e6, ~24 nnz/row, central window,
   p = 640, degree 200, Jackson, FP32 filter with FP64 projections.
5. Serving stream (see :mod:`workloads.stream`).

plus a degree-consistent reduction of workload 2 that converges at its degree:
27^3 grid (n = 19683), the same recipe, a mid-spectrum window sized for ~200
eigenvalues at the measured density of states (0.1435 per site per unit energy),
p = 360 (1.8 x 200), degree 120, Jackson.

Spectral bounds are the closed form for config 1 and Gershgorin discs otherwise.
``scale`` shrinks a workload for tests (grid edge or n); the recipe stays the same.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable

import numpy as np

from .matrices import (
    CSR,
    gershgorin_bounds,
    laplacian_2d_dirichlet,
    laplacian_3d_dirichlet,
    random_banded_symmetric,
    tight_binding_3d_periodic,
)


@dataclass
class WorkloadConfig:
    name: str
    description: str
    make_matrix: Callable[[int, int], CSR]  # (size, seed) -> CSR
    size: int                               # grid edge or n at full scale
    p: int
    degree: int
    damping: str
    complex_: bool
    filter_dtypes: tuple
    interval: Callable[[float, float], tuple]  # (lo, hi) -> (a, b)
    exact_bounds: Callable[[int], tuple] | None = None
    extra: dict = field(default_factory=dict)


def _centred(width: float):
    def f(lo, hi):
        c = 0.5 * (lo + hi)
        return (c - 0.5 * width, c + 0.5 * width)

    return f


def _lap2d_bounds(N):
    c = np.cos(np.pi / (N + 1))
    return (4.0 - 4.0 * c, 4.0 + 4.0 * c)


CONFIGS = {
    "lap2d_64": WorkloadConfig(
        name="lap2d_64",
        description="2D 5-point Dirichlet Laplacian 64x64, n=4096, 40-eigenvalue window",
        make_matrix=lambda size, seed: laplacian_2d_dirichlet(size),
        size=64,
        p=64,
        degree=60,
        damping="jackson",
        complex_=False,
        filter_dtypes=("f64",),
        interval=lambda lo, hi: (0.128538339316, 0.255551112680),
        exact_bounds=_lap2d_bounds,
    ),
    "lap3d_pot_100": WorkloadConfig(
        name="lap3d_pot_100",
        description="3D 7-point Dirichlet Laplacian 100^3 + 2*U(0,1) potential, n=1e6",
        make_matrix=lambda size, seed: laplacian_3d_dirichlet(size, potential_scale=2.0, seed=seed),
        size=100,
        p=256,
        degree=120,
        damping="jackson",
        complex_=False,
        filter_dtypes=("f64", "f32"),
        interval=_centred(1.39e-3),
        extra={"grid": 3},  # a cube grid of size^3 points, natural row index (x N + y) N + z
    ),
    "lap3d_pot_27": WorkloadConfig(
        name="lap3d_pot_27",
        description="3D 7-point Dirichlet Laplacian 27^3 + 2*U(0,1) potential, n=19683, ~200-eigenvalue window",
        make_matrix=lambda size, seed: laplacian_3d_dirichlet(size, potential_scale=2.0, seed=seed),
        size=27,
        p=360,
        degree=120,
        damping="jackson",
        complex_=False,
        filter_dtypes=("f64", "f32"),
        interval=_centred(200.0 / (0.1435 * 27 ** 3)),
        extra={"grid": 3},  # a cube grid of size^3 points, natural row index (x N + y) N + z
    ),
    "tb3d_64": WorkloadConfig(
        name="tb3d_64",
        description="complex tight-binding 64^3 periodic, random bond phases, n=262144",
        make_matrix=lambda size, seed: tight_binding_3d_periodic(size, seed=seed),
        size=64,
        p=192,
        degree=150,
        damping="jackson",
        complex_=True,
        filter_dtypes=("c128", "c64"),
        interval=_centred(4.85e-3),
    ),
    "rand_2m": WorkloadConfig(
        name="rand_2m",
        description="random irregular symmetric n=2e6, half banded (+-64) half random columns",
        make_matrix=lambda size, seed: random_banded_symmetric(size, seed=seed),
        size=2_000_000,
        p=640,
        degree=200,
        damping="jackson",
        complex_=False,
        filter_dtypes=("f32", "f64"),
        interval=_centred(4.0e-3),
    ),
}


# The spurious-Ritz-value scenario (Section 3.3.2) on a synthetic matrix: the 1D
# Dirichlet chain of N = 400 points with diagonal 4 (the 2D recipe on an N x 1 grid;
# eigenvalues 4 - 2cos(j pi / 401), symmetric about 4) and exact bounds symmetric about
# 4, so the filter of a window centred at 4 takes equal values at 4 - x and 4 + x.  The
# window holds the 10 eigenvalues nearest 4 (ends mid-gap); with p = 15 the block holds
# them, two outside pairs and one vector of the third pair, which no filter of this
# window can separate: its Ritz value sits at 4, inside, with a residual near 0.11.
CONFIGS["chain_400"] = WorkloadConfig(
    name="chain_400",
    description="1D Dirichlet chain N=400, diagonal 4, window of 10 eigenvalues centred at 4",
    make_matrix=lambda size, seed: laplacian_2d_dirichlet(size, 1),
    size=400,
    p=15,
    degree=120,
    damping="jackson",
    complex_=False,
    filter_dtypes=("f64",),
    interval=lambda lo, hi: (3.921676678665852, 4.078323321334147),
    exact_bounds=lambda N: (4.0 - 2.0 * np.cos(np.pi / (N + 1)), 4.0 + 2.0 * np.cos(np.pi / (N + 1))),
)


def build_config(name: str, size: int | None = None, seed: int = 0):
    """Return (A, (lo, hi), (a, b), cfg) for a named workload, optionally resized."""
    cfg = CONFIGS[name]
    size = cfg.size if size is None else size
    A = cfg.make_matrix(size, seed)
    if cfg.exact_bounds is not None:
        lo, hi = cfg.exact_bounds(size)
    else:
        lo, hi = gershgorin_bounds(A)
    a, b = cfg.interval(lo, hi)
    return A, (lo, hi), (a, b), cfg
