"""Readers for the stored expected values under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def lap2d_window() -> np.ndarray:
    """The 40 closed-form eigenvalues of the 64x64 Dirichlet Laplacian in the config-1 window."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "lap2d_64_window.txt")) if not l.startswith("#")]
    return np.array([float(r[1]) for r in rows])


def lap3d27_window() -> np.ndarray:
    """The eigenvalues of the 27^3 Laplacian + potential (seed 0) inside its window,
    written by make_golden.py from the oracle's banded eigensolver."""
    rows = [l for l in open(os.path.join(GOLDEN, "lap3d_pot_27_window.txt")) if not l.startswith("#")]
    return np.array([float(r) for r in rows if r.strip()])


def lap3d27_header() -> dict:
    """Window, bounds and nearest outside eigenvalues recorded in the 27^3 fixture header."""
    import re

    head = "".join(l for l in open(os.path.join(GOLDEN, "lap3d_pot_27_window.txt")) if l.startswith("#"))
    num = r"([-+0-9.eE]+)"
    lo, hi = map(float, re.search(r"bounds \[" + num + ", " + num + r"\]", head).groups())
    a, b = map(float, re.search(r"\[a, b\] = \[" + num + ", " + num + r"\]", head).groups())
    below, above = map(float, re.search(r"below " + num + ", above " + num, head).groups())
    return {"lo": lo, "hi": hi, "a": a, "b": b, "below": below, "above": above}
