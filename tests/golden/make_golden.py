"""Write the stored expected values under tests/golden/ from the oracle alone.

Run from the repository root:  python tests/golden/make_golden.py [--lap3d27] [--pot27-tau6 SEED]
(--lap3d27 also writes the 27^3 window: about 15 minutes of banded eigensolver time;
--pot27-tau6 SEED writes the oracle's Algorithm 4 result on that workload at the fixed
Jackson degree 120 and tau_c = 1e-6 from start block SEED: about an hour of host time)
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


def pot27_tau6(seed: int):
    """The oracle's subspace iteration (Algorithm 4, fixed Jackson degree 120, p = 360,
    tau_c = 1e-6) on the 27^3 Laplacian + potential from start block `seed`: the count,
    the iteration count and the locked eigenvalues."""
    from oracle import solver
    from workloads import start_block

    A, (lo, hi), (a, b), cfg = build_config("lap3d_pot_27", seed=0)
    X0 = start_block(A.n, cfg.p, seed=seed)
    o = solver.Options(kmax=cfg.degree, damping="jackson", tau_c=1e-6, max_iter=1500)
    r = solver.solve(A, a, b, lo, hi, X0, o)
    with open(os.path.join(HERE, f"lap3d_pot_27_tau1e-6_seed{seed}.txt"), "w") as f:
        f.write(f"# {cfg.description}; matrix seed 0, start block seed {seed}\n")
        f.write(f"# oracle Algorithm 4: fixed Jackson degree {cfg.degree}, p = {cfg.p}, tau_c = 1e-6\n")
        f.write(f"# count {r.eigenvalues.size} iterations {r.iterations} converged {int(r.converged)}\n")
        for x in r.eigenvalues:
            f.write(f"{float(x)!r}\n")


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
    if "--pot27-tau6" in sys.argv:
        pot27_tau6(int(sys.argv[sys.argv.index("--pot27-tau6") + 1]))
        sys.exit(0)
    main()
    if "--lap3d27" in sys.argv:
        lap3d27_window()
