"""Write the stored expected values under tests/golden/ from the oracle alone.

Run from the repository root:  python tests/golden/make_golden.py [--lap3d27]
(--lap3d27 also writes the 27^3 window: about 15 minutes of banded eigensolver time)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import closed_form, spectra  # noqa: E402
from workloads import build_config  # noqa: E402


def lap3d27_window():
    """Eigenvalues of the 27^3 Laplacian + potential inside its window (banded solver)."""
    A, (lo, hi), (a, b), cfg = build_config("lap3d_pot_27", seed=0)
    pad = 0.01
    w = [float(x) for x in spectra.eigenvalues_in_interval(A, a - pad, b + pad)]
    lo, hi, a, b = float(lo), float(hi), float(a), float(b)
    inside = [x for x in w if a <= x <= b]
    below = max(x for x in w if x < a)
    above = min(x for x in w if x > b)
    with open(os.path.join(HERE, "lap3d_pot_27_window.txt"), "w") as f:
        f.write(f"# {cfg.description}; seed 0\n")
        f.write(f"# Gershgorin bounds [{lo!r}, {hi!r}]; window [a, b] = [{a!r}, {b!r}]\n")
        f.write("# eigenvalues in the window from the banded symmetric eigensolver (oracle.spectra)\n")
        f.write(f"# nearest outside: below {below!r}, above {above!r}\n")
        for x in inside:
            f.write(f"{x!r}\n")


def main():
    w = closed_form.lap2d_eigs(64)
    a, b = 0.128538339316, 0.255551112680
    inside = [(i + 1, float(x)) for i, x in enumerate(w) if a <= x <= b]
    with open(os.path.join(HERE, "lap2d_64_window.txt"), "w") as f:
        f.write("# 64x64 Dirichlet 5-point Laplacian, eigenvalues 4-2cos(i pi/65)-2cos(j pi/65)\n")
        f.write(f"# sorted ascending; those inside [a, b] = [{a!r}, {b!r}]\n")
        f.write("# columns: 1-based index in the sorted spectrum, eigenvalue (repr)\n")
        for idx, x in inside:
            f.write(f"{idx} {x!r}\n")


if __name__ == "__main__":
    main()
    if "--lap3d27" in sys.argv:
        lap3d27_window()
