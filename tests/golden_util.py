"""Readers for the stored expected values under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def lap2d_window() -> np.ndarray:
    """The 40 closed-form eigenvalues of the 64x64 Dirichlet Laplacian in the config-1 window."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "lap2d_64_window.txt")) if not l.startswith("#")]
    return np.array([float(r[1]) for r in rows])
