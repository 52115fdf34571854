"""Stored values: the paper's printed parameters and Table 2, and a closed-form fixture."""
import csv
import json
import os

import numpy as np

from oracle import closed_form
from oracle import solver
from workloads import laplacian_2d_dirichlet

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_window_fixture_matches_dense_eigvalsh():
    # tests/golden/lap2d_64_window.txt was written from the closed form; pin it to LAPACK
    rows = [l.split() for l in open(os.path.join(GOLDEN, "lap2d_64_window.txt")) if not l.startswith("#")]
    idx = np.array([int(r[0]) for r in rows])
    vals = np.array([float(r[1]) for r in rows])
    assert vals.size == 40 and idx[0] == 38 and idx[-1] == 77
    w = np.linalg.eigvalsh(laplacian_2d_dirichlet(64).to_dense())
    assert np.max(np.abs(w[idx - 1] - vals)) < 1e-12
    assert np.max(np.abs(closed_form.lap2d_eigs(64) - w)) < 1e-12


def test_oracle_defaults_are_the_papers_parameters():
    p = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))
    o = solver.Options()
    assert o.tau_a == p["tau_a"] and o.tau_c == p["tau_c"] and o.C == p["C"] and o.m_exp == p["m"]


def test_table2_speedups_match_the_text():
    rows = [r for r in csv.DictReader(l for l in open(os.path.join(GOLDEN, "paper_table2.csv")) if not l.startswith("#"))]
    t = {(r["matrix"], r["method"]): float(r["runtime_s"]) for r in rows}
    mats = sorted({r["matrix"] for r in rows})
    evsl = [t[(m, "EVSL-PSI")] / t[(m, "AdaPolySI")] for m in mats]
    cj = [t[(m, "CJ-FEAST")] / t[(m, "AdaPolySI")] for m in mats]
    # abstract / Section 4.1: 14.5x mean and 25.9x peak over EVSL, 2.14x mean and 2.39x peak over CJ-FEAST
    assert round(np.mean(evsl), 1) == 14.5 and round(max(evsl), 1) == 25.9
    assert round(np.mean(cj), 2) == 2.14 and round(max(cj), 2) == 2.39
