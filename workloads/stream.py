"""Seeded request streams for the serving workload.

A stream is a list of requests with Poisson arrival times.  Each request is
either a spectrum slice of one shared matrix (the 3D Laplacian + potential of
n = 100^3, cut into contiguous slices around the spectrum's centre) or an
independent 3D Laplacian + potential matrix with n log-uniform in [1e4, 1e6],
block width p in {32, 64, 128, 256} and degree uniform in [40, 200], whose
interval is sized to hold about p / 1.8 eigenvalues.

Interval widths come from a density-of-states estimate of this matrix family
(about 0.1435 eigenvalues per unit energy per grid point near the centre of the
spectrum, measured on small grids); they are workload definitions, not part of
the method.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

DOS_CENTRE = 0.1435


@dataclass
class Request:
    kind: str            # "slice" or "matrix"
    arrival: float       # seconds after the stream starts
    grid: int            # N of the N^3 grid
    seed: int            # matrix seed (matrix requests) and start-block seed
    a: float
    b: float
    p: int
    degree: int
    slice_index: int = -1


def slice_intervals(n: int, centre: float, count: int, per_slice: int):
    """`count` contiguous intervals around `centre`, each holding ~`per_slice` eigenvalues."""
    w = per_slice / (DOS_CENTRE * n)
    lo = centre - 0.5 * count * w
    return [(lo + i * w, lo + (i + 1) * w) for i in range(count)]


def serving_stream(num: int, rate_hz: float, seed: int = 0, slice_frac: float = 0.5,
                   slice_grid: int = 100, n_range=(1e4, 1e6), slices: int = 16,
                   slice_p: int = 96, slice_degree: int = 120, slice_eigs: int = 50,
                   p_choices=(32, 64, 128, 256), degree_range=(40, 200)):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    n_slice = slice_grid ** 3
    centre = 7.0  # centre of the Gershgorin interval [0, 14] of this family
    ivs = slice_intervals(n_slice, centre, slices, slice_eigs)
    for i in range(num):
        t += rng.exponential(1.0 / rate_hz)
        if rng.uniform() < slice_frac:
            k = int(rng.integers(0, slices))
            a, b = ivs[k]
            out.append(Request("slice", t, slice_grid, 1000 + i, a, b, slice_p, slice_degree, k))
        else:
            n = float(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))))
            N = max(4, int(round(n ** (1.0 / 3.0))))
            p = int(rng.choice(p_choices))
            deg = int(rng.integers(degree_range[0], degree_range[1] + 1))
            w = (p / 1.8) / (DOS_CENTRE * N ** 3)
            out.append(Request("matrix", t, N, 2000 + i, centre - w / 2, centre + w / 2, p, deg))
    return out
