"""Seeded start blocks X0 (n x p, row-major) for the filter and the solver."""
from __future__ import annotations

import numpy as np


def start_block(n: int, p: int, seed: int = 0, complex_: bool = False) -> np.ndarray:
    """N(0,1) entries from ``default_rng(seed)``; complex blocks use (N + iN)/sqrt(2).

    The block is C-contiguous (row-major), float64 or complex128.
    """
    rng = np.random.default_rng(seed)
    if not complex_:
        return rng.standard_normal((n, p))
    re = rng.standard_normal((n, p))
    im = rng.standard_normal((n, p))
    return (re + 1j * im) / np.sqrt(2.0)


def probe_block(n: int, m: int, seed: int = 0, complex_: bool = False) -> np.ndarray:
    """m probe vectors for trace estimation: independent +-1 entries from ``default_rng(seed)``
    (complex: (+-1 +- i)/sqrt(2)), so that E[z z^H] = I.  C-contiguous n x m."""
    rng = np.random.default_rng(seed)
    re = rng.integers(0, 2, size=(n, m)) * 2.0 - 1.0
    if not complex_:
        return re
    im = rng.integers(0, 2, size=(n, m)) * 2.0 - 1.0
    return (re + 1j * im) / np.sqrt(2.0)
