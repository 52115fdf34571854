"""Pins of the benchmark's byte model (no GPU): the algorithmic bytes per steady Clenshaw
launch that the reported roofline fraction divides by, against the workload's sizes
worked out by hand."""
import numpy as np

import bench
from workloads import CONFIGS


def test_steady_launch_bytes_of_the_100_cubed_workload():
    # n = 100^3 rows, nnz = 7 n - 6 N^2 (the Dirichlet faces drop one neighbour each),
    # p = 256 columns.  Steady launch: the CSR matrix once (value + int32 column per
    # entry, int32 row pointers) plus four passes over an n x p block (gathered source,
    # b_{j+2} in place, X, write).
    n, N, p = 10 ** 6, 100, 256
    nnz = 7 * n - 6 * N * N
    assert nnz == 6_940_000
    zeros = np.zeros(121)
    _, fp64 = bench.filter_bytes(nnz, n, p, 8, 8, zeros, 120)
    assert fp64 == 6_940_000 * 12 + 4 * 1_000_001 + 4 * 1_000_000 * 256 * 8 == 8_279_280_004
    _, fp32 = bench.filter_bytes(nnz, n, p, 4, 4, zeros, 120)
    assert fp32 == 6_940_000 * 8 + 4 * 1_000_001 + 4 * 1_000_000 * 256 * 4 == 4_155_520_004
    assert CONFIGS["lap3d_pot_100"].p == p and CONFIGS["lap3d_pot_100"].size == N


def test_filter_bytes_counts_x_only_for_nonzero_coefficients():
    # degree 4: product s = 0 reads X and writes; s = 1 (j = 2) adds X when a_2 - a_4 is
    # nonzero; s = 2, 3 (j = 1, 0) read the source and V in place, write, and read X when
    # a_j is nonzero.  Toy sizes: 96 entries with 0-byte values, n = 10 rows, one 1-byte
    # column, so A costs 96 * 4 + 4 * 11 bytes and a block pass 10 bytes.
    c = np.array([1.0, 0.0, 2.0, 0.0, 3.0])
    total, steady = bench.filter_bytes(96, 10, 1, 1, 0, c, 4)
    a_bytes, pb = 96 * 4 + 4 * 11, 10
    # passes: 2 (s = 0), 3 (a_2 - a_4 = -1), 3 (a_1 = 0), 4 (a_0 = 1)
    assert total == 4 * a_bytes + (2 + 3 + 3 + 4) * pb
    assert steady == a_bytes + 4 * pb
