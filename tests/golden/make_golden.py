"""Write the stored expected values under tests/golden/ from the oracle alone.

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import closed_form  # noqa: E402


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
