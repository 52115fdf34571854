"""GPU parity of the Clenshaw filter (Algorithm 2) against the oracle, through the C ABI.

Tolerances (floating point, derived in the design notes): FP64 blocks agree with
the FP64 oracle to 1e-12 relative (Frobenius and max-element); FP32 blocks to
(k+1) * 2^-21 relative, the FP32 rounding of k three-term steps with |sigma A| <= 2.
"""
import numpy as np
import pytest

from oracle import closed_form
from oracle import coefficients as co
from oracle.filter import clenshaw_filter
from paper_2604_00914_amd import afsi
from tests.gpu_util import DEV, max_rel, rel_fro, to_dev, torch
from workloads import (
    build_config,
    gershgorin_bounds,
    laplacian_3d_dirichlet,
    random_dense_symmetric_csr,
    start_block,
    tight_binding_3d_periodic,
)

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


def f32_tol(k):
    return (k + 1) * 2.0 ** -21


def _tdt(cplx, single):
    t = torch()
    if cplx:
        return t.complex64 if single else t.complex128
    return t.float32 if single else t.float64


def gpu_filter(A, X0, lmin, lmax, coeffs, degree, single=False, pad=0, offset=0):
    t = torch()
    M = afsi.Matrix(A, bounds=(lmin, lmax))
    n, p = X0.shape
    dt = _tdt(np.iscomplexobj(X0) or np.iscomplexobj(A.val), single)
    bufs = [t.zeros((n, p + pad), dtype=dt, device=DEV) for _ in range(3)]
    X, Y, W = (b[:, offset: offset + p] for b in bufs)
    X.copy_(t.from_numpy(X0).to(DEV).to(dt))
    afsi.afsi_filter_block(M.handle, coeffs, degree, X, Y, W)
    t.cuda.synchronize()
    out = Y.cpu().numpy().astype(np.complex128 if np.iscomplexobj(X0) else np.float64)
    M.close()
    return out


def oracle_filter(A, X0, lmin, lmax, a, b, degree, damping="jackson"):
    c = co.filter_coefficients(lmin, lmax, a, b, degree, damping)
    l1, l2 = co.affine_map(lmin, lmax)
    return clenshaw_filter(A, X0, c, l1, l2)


def _check(got, ref, tol):
    assert rel_fro(got, ref) <= tol, rel_fro(got, ref)
    assert max_rel(got, ref) <= 10 * tol, max_rel(got, ref)


def test_config1_full_size_parity():
    A, (lmin, lmax), (a, b), cfg = build_config("lap2d_64")
    X0 = start_block(A.n, cfg.p, seed=0)
    c = afsi.afsi_filter_coefficients(lmin, lmax, a, b, cfg.degree, "jackson")
    got = gpu_filter(A, X0, lmin, lmax, c, cfg.degree)
    _check(got, oracle_filter(A, X0, lmin, lmax, a, b, cfg.degree), F64_TOL)


_SMALL = random_dense_symmetric_csr(1001, 0.01, seed=9)
_SMALL_W = (-30.0, 30.0)


@pytest.mark.parametrize("p", [1, 2, 3, 7, 16, 24, 32, 64, 96, 100, 128, 192, 256, 320, 640])
def test_widths_fp64(p):
    X0 = start_block(_SMALL.n, p, seed=p)
    lmin, lmax = _SMALL_W
    c = afsi.afsi_filter_coefficients(lmin, lmax, -2.0, 3.0, 9, "jackson")
    got = gpu_filter(_SMALL, X0, lmin, lmax, c, 9)
    _check(got, oracle_filter(_SMALL, X0, lmin, lmax, -2.0, 3.0, 9), F64_TOL)


@pytest.mark.parametrize("p", [1, 3, 4, 8, 64, 160, 256, 640])
def test_widths_fp32(p):
    X0 = start_block(_SMALL.n, p, seed=p)
    lmin, lmax = _SMALL_W
    k = 9
    c = afsi.afsi_filter_coefficients(lmin, lmax, -2.0, 3.0, k, "jackson")
    got = gpu_filter(_SMALL, X0, lmin, lmax, c, k, single=True)
    ref = oracle_filter(_SMALL, X0, lmin, lmax, -2.0, 3.0, k)
    assert rel_fro(got, ref) <= f32_tol(k)


@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("p", [1, 3, 8, 64, 192])
def test_complex_widths(p, single):
    A = tight_binding_3d_periodic(6, seed=3)
    X0 = start_block(A.n, p, seed=p, complex_=True)
    lmin, lmax = -7.0, 7.0
    k = 31  # odd degree with a symmetric interval: every odd coefficient is zero
    c = afsi.afsi_filter_coefficients(lmin, lmax, -0.4, 0.4, k, "jackson")
    got = gpu_filter(A, X0, lmin, lmax, c, k, single=single)
    ref = oracle_filter(A, X0, lmin, lmax, -0.4, 0.4, k)
    if single:
        assert rel_fro(got, ref) <= f32_tol(k)
    else:
        _check(got, ref, F64_TOL)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("symmetric", [False, True])
def test_low_degrees(k, symmetric):
    A = laplacian_3d_dirichlet(7, 2.0, seed=1)
    lmin, lmax = 0.0, 14.0
    a, b = (6.5, 7.5) if symmetric else (2.0, 3.1)
    X0 = start_block(A.n, 16, seed=k)
    c = afsi.afsi_filter_coefficients(lmin, lmax, a, b, k, "lanczos", 0.5)
    got = gpu_filter(A, X0, lmin, lmax, c, k)
    _check(got, oracle_filter(A, X0, lmin, lmax, a, b, k, "lanczos"), F64_TOL)


@pytest.mark.parametrize("pad,offset", [(8, 0), (5, 3), (1, 1), (64, 32)])
@pytest.mark.parametrize("p", [2, 64, 100])
def test_strided_and_unaligned_views(p, pad, offset):
    A = laplacian_3d_dirichlet(8, 2.0, seed=2)
    X0 = start_block(A.n, p, seed=1)
    c = afsi.afsi_filter_coefficients(0.0, 14.0, 4.0, 5.0, 12, "jackson")
    got = gpu_filter(A, X0, 0.0, 14.0, c, 12, pad=pad, offset=offset)
    _check(got, oracle_filter(A, X0, 0.0, 14.0, 4.0, 5.0, 12), F64_TOL)


def test_untouched_neighbour_columns():
    # columns outside a view must keep their contents (no vector over-write)
    t = torch()
    A = laplacian_3d_dirichlet(5, 0.0)
    M = afsi.Matrix(A, bounds=(0.0, 12.0))
    c = afsi.afsi_filter_coefficients(0.0, 12.0, 2.0, 3.0, 6, "jackson")
    bufs = [t.full((A.n, 9), 7.0, dtype=t.float64, device=DEV) for _ in range(3)]
    X, Y, W = (bb[:, 1:4] for bb in bufs)
    X.copy_(to_dev(start_block(A.n, 3, 0)))
    afsi.afsi_filter_block(M.handle, c, 6, X, Y, W)
    t.cuda.synchronize()
    for bb in bufs[1:]:
        assert bool((bb[:, 0] == 7.0).all()) and bool((bb[:, 4:] == 7.0).all())
    M.close()


def test_ragged_and_degenerate_matrices():
    # n = 1, rows without entries, an all-zero matrix
    from workloads import CSR

    for A in [
        CSR(1, np.array([0, 1]), np.array([0], np.int32), np.array([2.0])),
        CSR(5, np.array([0, 0, 2, 2, 3, 3]), np.array([1, 3, 3], np.int32), np.array([1.0, 2.0, 3.0])),
        CSR(6, np.zeros(7, np.int64), np.zeros(0, np.int32), np.zeros(0)),
    ]:
        X0 = start_block(A.n, 6, seed=2)
        c = afsi.afsi_filter_coefficients(-4.0, 4.0, -1.0, 1.5, 5, "jackson")
        got = gpu_filter(A, X0, -4.0, 4.0, c, 5)
        _check(got, oracle_filter(A, X0, -4.0, 4.0, -1.0, 1.5, 5), F64_TOL)


def _ragged_symmetric(n=1001, seed=5, complex_=False):
    """Symmetric (Hermitian) matrix whose row lengths run from 0 to ~34: every residue
    mod 8 (the Clenshaw kernels fetch eight nonzeros at a time), exact multiples of 8,
    rows longer than one and two fetch chunks, and empty rows and columns."""
    from workloads import CSR

    rng = np.random.default_rng(seed)
    mask = np.triu(rng.uniform(size=(n, n)) < 0.0035, 1)
    long_rows = np.zeros(n, bool)
    long_rows[3::53] = True
    mask |= np.triu(long_rows[:, None] & (rng.uniform(size=(n, n)) < 0.02), 1)
    M = rng.standard_normal((n, n))
    if complex_:
        M = M + 1j * rng.standard_normal((n, n))
    H = np.where(mask, M, 0)
    H = H + H.conj().T + np.diag(rng.standard_normal(n))
    H[::37, :] = 0
    H[:, ::37] = 0
    rows, cols = np.nonzero(H)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return CSR(n, row_ptr, cols.astype(np.int32), H[rows, cols])


@pytest.mark.parametrize(
    "p,single,cplx,pad,offset",
    [
        (256, False, False, 0, 0),   # 2 vectors x 64 lanes: one row per wave
        (512, False, False, 0, 0),   # 4 x 64
        (96, False, False, 0, 0),    # 3 x 16: four rows per wave
        (64, False, False, 0, 0),    # 1 x 32
        (128, False, False, 0, 0),   # 2 x 32
        (192, False, False, 0, 0),   # 3 x 32
        (100, False, False, 0, 0),   # no exact lane mapping: masked kernel
        (64, False, False, 1, 1),    # 8-byte offset view: scalar kernel
        (256, True, False, 0, 0),    # FP32, 2 x 32
        (512, True, False, 0, 0),    # FP32, 2 x 64
        (192, False, True, 0, 0),    # complex FP64, 3 x 64
        (192, True, True, 0, 0),     # complex FP32, 3 x 32
    ],
)
def test_ragged_row_lengths_every_lane_mapping(p, single, cplx, pad, offset):
    A = _ragged_symmetric(complex_=cplx)
    lengths = np.diff(A.row_ptr)
    assert lengths.min() == 0 and lengths.max() >= 32
    assert set(np.unique(lengths % 8)) == set(range(8))
    lmin, lmax = gershgorin_bounds(A)
    k = 12
    c = afsi.afsi_filter_coefficients(lmin, lmax, -0.5, 0.7, k, "jackson")
    X0 = start_block(A.n, p, seed=p + pad, complex_=cplx)
    got = gpu_filter(A, X0, lmin, lmax, c, k, single=single, pad=pad, offset=offset)
    ref = oracle_filter(A, X0, lmin, lmax, -0.5, 0.7, k)
    if single:
        assert rel_fro(got, ref) <= f32_tol(k), rel_fro(got, ref)
    else:
        _check(got, ref, F64_TOL)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 9])
@pytest.mark.parametrize("p,single,cplx", [(256, False, False), (256, True, False), (192, False, True)])
def test_staged_step_small_n(n, p, single, cplx):
    # one row per wave with the source rows staged in LDS: workgroups whose rows run past
    # n and staging windows clipped at row 0 and row n - 1 (tridiagonal plus a corner entry)
    from workloads import CSR

    rng = np.random.default_rng(n)
    H = np.diag(rng.standard_normal(n) + 2.0).astype(np.complex128 if cplx else np.float64)
    for i in range(n - 1):
        z = rng.standard_normal() + (1j * rng.standard_normal() if cplx else 0.0)
        H[i, i + 1], H[i + 1, i] = z, np.conj(z)
    if n > 2:
        H[0, n - 1] = H[n - 1, 0] = 0.5
    rows, cols = np.nonzero(H)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    A = CSR(n, row_ptr, cols.astype(np.int32), H[rows, cols])
    lmin, lmax = gershgorin_bounds(A)
    lmin, lmax = lmin - 1.0, lmax + 1.0  # n = 1: Gershgorin's interval is a point
    X0 = start_block(n, p, seed=n, complex_=cplx)
    k = 7
    c = afsi.afsi_filter_coefficients(lmin, lmax, lmin + 0.3 * (lmax - lmin), lmin + 0.6 * (lmax - lmin), k, "jackson")
    got = gpu_filter(A, X0, lmin, lmax, c, k, single=single)
    ref = oracle_filter(A, X0, lmin, lmax, lmin + 0.3 * (lmax - lmin), lmin + 0.6 * (lmax - lmin), k)
    if single:
        assert rel_fro(got, ref) <= f32_tol(k), rel_fro(got, ref)
    else:
        _check(got, ref, F64_TOL)


def test_repeatable_bitwise():
    A, (lmin, lmax), (a, b), cfg = build_config("lap2d_64")
    X0 = start_block(A.n, cfg.p, seed=3)
    c = afsi.afsi_filter_coefficients(lmin, lmax, a, b, cfg.degree, "jackson")
    y1 = gpu_filter(A, X0, lmin, lmax, c, cfg.degree)
    y2 = gpu_filter(A, X0, lmin, lmax, c, cfg.degree)
    assert np.array_equal(y1, y2)


BATCH_LAYOUTS = {
    # narrow: 52 vectors per row (2 per lane), groups cover every column
    "narrow": (104, [(0, 32, 7, (3.0, 3.5), 0), (32, 64, 12, (5.0, 5.3), 2), (96, 8, 5, (9.0, 11.0), 4)]),
    # wide: 300 vectors per row (4 per lane, ragged second chunk), columns 200..209 and
    # 546..599 in no group
    "wide": (600, [(0, 200, 7, (3.0, 3.5), 0), (210, 328, 12, (5.0, 5.3), 2), (538, 8, 5, (9.0, 11.0), 4)]),
    # groups one step apart read different source blocks in the same launch (the general
    # kernel); launches where every active group reads one block take the same-source kernel
    "parity": (256, [(0, 64, 9, (3.0, 3.5), 0), (64, 96, 10, (5.0, 5.3), 1), (160, 96, 6, (9.0, 11.0), 3)]),
}


@pytest.mark.parametrize("matrix", ["laplacian", "ragged"])
@pytest.mark.parametrize("layout", sorted(BATCH_LAYOUTS))
def test_batched_groups_bitwise_equal_to_single_filters(layout, matrix):
    t = torch()
    if matrix == "ragged":
        A = _ragged_symmetric()
        lmin, lmax = gershgorin_bounds(A)
    else:
        A = laplacian_3d_dirichlet(10, 2.0, seed=4)
        lmin, lmax = 0.0, 14.0
    l1, l2 = co.affine_map(lmin, lmax)
    ptot, groups = BATCH_LAYOUTS[layout]
    X0 = start_block(A.n, ptot, seed=5)
    M = afsi.Matrix(A, bounds=(lmin, lmax))
    X = to_dev(X0)
    P0 = t.zeros_like(X)
    P1 = t.zeros_like(X)
    coeffs = {g: afsi.afsi_filter_coefficients(lmin, lmax, iv[0], iv[1], k, "jackson") for g, (c0, nc, k, iv, st) in enumerate(groups)}
    total = max(st + k for (c0, nc, k, iv, st) in groups)
    for step in range(total):
        gs = []
        for g, (c0, nc, k, iv, st) in enumerate(groups):
            s = step - st
            if 0 <= s < k:
                gs.append(afsi.afsi_clenshaw_step_params(coeffs[g], k, s, l1, l2, col0=c0, ncols=nc))
        afsi.afsi_clenshaw_step_batched(M.handle, gs, X, P0, P1)
    t.cuda.synchronize()
    for g, (c0, nc, k, iv, st) in enumerate(groups):
        Yb = (P0 if (k - 1) % 2 == 0 else P1)[:, c0:c0 + nc].cpu().numpy()
        Xs = to_dev(X0[:, c0:c0 + nc])
        Ys, Ws = t.empty_like(Xs), t.empty_like(Xs)
        afsi.afsi_filter_block(M.handle, coeffs[g], k, Xs, Ys, Ws)
        t.cuda.synchronize()
        assert np.array_equal(Yb, Ys.cpu().numpy()), g
        ref = oracle_filter(A, X0[:, c0:c0 + nc], lmin, lmax, iv[0], iv[1], k)
        _check(Yb, ref, F64_TOL)
    # columns outside every group are never written
    covered = np.zeros(ptot, bool)
    for (c0, nc, k, iv, st) in groups:
        covered[c0:c0 + nc] = True
    for P in (P0, P1):
        assert not P.cpu().numpy()[:, ~covered].any()
    M.close()


def test_full_size_config2_closed_form_modes():
    # 100^3 Dirichlet Laplacian (no potential): 256 closed-form eigenvectors map to rho(lambda) v
    t = torch()
    N = 100
    A = laplacian_3d_dirichlet(N, 0.0)
    lmin, lmax = 0.0, 12.0
    k, p = 120, 256
    rng = np.random.default_rng(0)
    idx = rng.integers(1, N + 1, size=(p, 3))
    lams = np.array([closed_form.lap3d_mode(N, *m)[0] for m in idx])
    mid = float(np.median(lams))
    a, b = mid - 0.3, mid + 0.3
    c = afsi.afsi_filter_coefficients(lmin, lmax, a, b, k, "jackson")
    X = t.empty((A.n, p), dtype=t.float64, device=DEV)
    for j, m in enumerate(idx):
        X[:, j] = to_dev(closed_form.lap3d_mode(N, *m)[1])
    M = afsi.Matrix(A, bounds=(lmin, lmax))
    Y, W = t.empty_like(X), t.empty_like(X)
    afsi.afsi_filter_block(M.handle, c, k, X, Y, W)
    rho = t.from_numpy(co.filter_value(lams, co.filter_coefficients(lmin, lmax, a, b, k, "jackson"), lmin, lmax)).to(DEV)
    err = (Y - X * rho[None, :]).abs().max().item()
    assert err < 1e-12, err
    M.close()


def test_full_size_config2_low_degree_vs_oracle():
    # the production shape (n = 1e6, p = 256, FP64) at degree 3 against the full oracle
    A, (lmin, lmax), (a, b), cfg = build_config("lap3d_pot_100")
    X0 = start_block(A.n, cfg.p, seed=0)
    c = afsi.afsi_filter_coefficients(lmin, lmax, a, b, 3, "jackson")
    got = gpu_filter(A, X0, lmin, lmax, c, 3)
    ref = oracle_filter(A, X0, lmin, lmax, a, b, 3)
    _check(got, ref, F64_TOL)


def _gpu_filter_columns(M, X0, coeffs, degree, single, cols):
    """Filter the whole block on the GPU (the launch configuration the benchmark times)
    and return only the requested columns."""
    t = torch()
    dt = _tdt(np.iscomplexobj(X0), single)
    X = t.from_numpy(X0).to(DEV).to(dt)
    Y, W = t.empty_like(X), t.empty_like(X)
    afsi.afsi_filter_block(M.handle, coeffs, degree, X, Y, W)
    t.cuda.synchronize()
    out = Y[:, cols].cpu().numpy().astype(np.complex128 if np.iscomplexobj(X0) else np.float64)
    del X, Y, W
    t.cuda.empty_cache()
    return out


@pytest.mark.parametrize("name,cols", [("lap3d_pot_100", [0, 101, 255]), ("tb3d_64", [0, 77, 191]),
                                       ("rand_2m", [0, 639])])
def test_full_size_sampled_columns(name, cols):
    # full n, p and degree of the workload, both precisions: the filter acts on every
    # column separately, so sampled columns of the GPU's block equal the oracle's filter
    # of those columns of the start block
    A, (lmin, lmax), (a, b), cfg = build_config(name)
    X0 = start_block(A.n, cfg.p, seed=0, complex_=A.is_complex)
    c = afsi.afsi_filter_coefficients(lmin, lmax, a, b, cfg.degree, cfg.damping)
    ref = oracle_filter(A, np.ascontiguousarray(X0[:, cols]), lmin, lmax, a, b, cfg.degree, cfg.damping)
    M = afsi.Matrix(A, bounds=(lmin, lmax))
    for single in (False, True):
        got = _gpu_filter_columns(M, X0, c, cfg.degree, single, cols)
        _check(got, ref, f32_tol(cfg.degree) if single else F64_TOL)
    M.close()


@pytest.mark.parametrize("stagger", [0, 1])
def test_full_size_batched_slices_sampled_columns(stagger):
    # the batched step at full size (16 slices x 96 columns of the 100^3 matrix, degree
    # 120, each slice with its own coefficients); stagger 0: every launch reads one source
    # block; stagger 1: odd slices one step behind, so launches mix source blocks; one
    # sampled column per slice against the oracle's filter of that column
    from workloads.stream import slice_intervals

    t = torch()
    A, (lo, hi), _, cfg = build_config("lap3d_pot_100")
    k, G, cols = cfg.degree, 16, 96
    l1, l2 = co.affine_map(lo, hi)
    ivs = slice_intervals(A.n, 0.5 * (lo + hi), G, 50)
    coeffs = [afsi.afsi_filter_coefficients(lo, hi, a, b, k, "jackson") for a, b in ivs]
    ref_coeffs = [co.filter_coefficients(lo, hi, a, b, k, "jackson") for a, b in ivs]
    X0 = start_block(A.n, G * cols, seed=0)
    M = afsi.Matrix(A, bounds=(lo, hi))
    X = to_dev(X0)
    P0, P1 = t.zeros_like(X), t.zeros_like(X)
    for step in range(k + stagger):
        gs = [afsi.afsi_clenshaw_step_params(coeffs[g], k, step - stagger * (g % 2), l1, l2, col0=g * cols,
                                             ncols=cols)
              for g in range(G) if 0 <= step - stagger * (g % 2) < k]
        afsi.afsi_clenshaw_step_batched(M.handle, gs, X, P0, P1)
    t.cuda.synchronize()
    out = P0 if (k - 1) % 2 == 0 else P1
    pick = [g * cols + (7 * g) % cols for g in range(G)]
    got = out[:, pick].cpu().numpy()
    del X, P0, P1
    t.cuda.empty_cache()
    M.close()
    for j, g in enumerate(range(G)):
        ref = clenshaw_filter(A, np.ascontiguousarray(X0[:, pick[j]:pick[j] + 1]), ref_coeffs[g], l1, l2)
        _check(got[:, j:j + 1], ref, F64_TOL)


@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("stagger", [0, 1])
def test_full_size_grouped_slices_sampled_columns(stagger, single):
    # the server's slice step (the grouped kernel) at full size: 16 slices x 96 columns of
    # the 100^3 matrix, degree 120, every slice in its own n x 96 blocks with its own
    # coefficients; stagger 1 puts odd slices one step behind, so one launch mixes source
    # blocks and V / X flags; one sampled column per slice against the oracle's filter
    from workloads.stream import slice_intervals

    t = torch()
    A, (lo, hi), _, cfg = build_config("lap3d_pot_100")
    k, G, cols = cfg.degree, 16, 96
    l1, l2 = co.affine_map(lo, hi)
    ivs = slice_intervals(A.n, 0.5 * (lo + hi), G, 50)
    coeffs = [afsi.afsi_filter_coefficients(lo, hi, a, b, k, "jackson") for a, b in ivs]
    ref_coeffs = [co.filter_coefficients(lo, hi, a, b, k, "jackson") for a, b in ivs]
    dt = t.float32 if single else t.float64
    M = afsi.Matrix(A, bounds=(lo, hi))
    pick, cols0, blocks = [], [], []
    for g in range(G):
        X0 = start_block(A.n, cols, seed=100 + g)
        c = (7 * g) % cols
        pick.append(c)
        cols0.append(np.ascontiguousarray(X0[:, c:c + 1]))
        X = t.from_numpy(X0).to(DEV).to(dt)
        blocks.append((X, t.zeros_like(X), t.zeros_like(X)))
        del X0
    for step in range(k + stagger):
        sl = []
        for g in range(G):
            s_g = step - stagger * (g % 2)
            if 0 <= s_g < k:
                sl.append((afsi.afsi_clenshaw_step_params(coeffs[g], k, s_g, l1, l2, ncols=cols), *blocks[g]))
        afsi.afsi_clenshaw_step_grouped(M.handle, sl)
    t.cuda.synchronize()
    got = [blocks[g][1 + (k - 1) % 2][:, pick[g]].cpu().numpy().astype(np.float64) for g in range(G)]
    del blocks
    t.cuda.empty_cache()
    M.close()
    for g in range(G):
        ref = clenshaw_filter(A, cols0[g], ref_coeffs[g], l1, l2)
        _check(got[g][:, None], ref, f32_tol(k) if single else F64_TOL)


@pytest.mark.parametrize("cplx,single", [(False, False), (False, True), (True, False), (True, True)])
def test_filter_batched_equals_single_filters(cplx, single):
    # the whole-filter slice call: slices of different widths (grouped-kernel widths and
    # widths that fall back to one product each), degrees and intervals; every slice's Y
    # bit-identical to afsi_filter_block on that slice alone and within tolerance of the
    # oracle's filter
    t = torch()
    if cplx:
        A = tight_binding_3d_periodic(8, seed=3)
        lmin, lmax = -7.5, 7.5
        shift = -5.0
    else:
        A = laplacian_3d_dirichlet(10, 2.0, seed=4)
        lmin, lmax = 0.0, 14.0
        shift = 0.0
    dt = _tdt(cplx, single)
    M = afsi.Matrix(A, bounds=(lmin, lmax))
    spec = [(64, 72, 9, (5.0, 5.3)), (64, 64, 4, (7.0, 7.4)), (96, 96, 11, (2.0, 2.4)),
            (10, 12, 6, (4.0, 4.6)), (128, 128, 1, (8.0, 9.0))]
    slices, X0s, cs = [], [], []
    for g, (nc, ld, k, (a, b)) in enumerate(spec):
        X0 = start_block(A.n, nc, seed=40 + g, complex_=cplx)
        X0s.append(X0)
        c = afsi.afsi_filter_coefficients(lmin, lmax, a + shift, b + shift, k, "jackson")
        cs.append(c)
        bufs = [t.zeros((A.n, ld), dtype=dt, device=DEV) for _ in range(3)]
        bufs[0][:, :nc] = t.from_numpy(X0).to(DEV).to(dt)
        slices.append((c, k, *(b_[:, :nc] for b_ in bufs)))
    afsi.afsi_filter_batched(M.handle, slices)
    t.cuda.synchronize()
    for g, (nc, ld, k, (a, b)) in enumerate(spec):
        Y = slices[g][3].cpu().numpy()
        Xs = t.from_numpy(X0s[g]).to(DEV).to(dt)
        Ys, Ws = t.empty_like(Xs), t.empty_like(Xs)
        afsi.afsi_filter_block(M.handle, cs[g], k, Xs, Ys, Ws)
        t.cuda.synchronize()
        assert np.array_equal(Y, Ys.cpu().numpy()), g
        ref = oracle_filter(A, X0s[g], lmin, lmax, a + shift, b + shift, k)
        _check(Y.astype(np.complex128 if cplx else np.float64), ref, f32_tol(k) if single else F64_TOL)
    M.close()


def test_filter_batched_errors():
    t = torch()
    A = laplacian_3d_dirichlet(6, 1.0, seed=2)
    M = afsi.Matrix(A, bounds=(0.0, 14.0))
    c = afsi.afsi_filter_coefficients(0.0, 14.0, 3.0, 4.0, 5)
    X = to_dev(start_block(A.n, 32, seed=1))
    Y, W = t.zeros_like(X), t.zeros_like(X)
    with pytest.raises(afsi.AfsiError):  # degree 0
        afsi.afsi_filter_batched(M.handle, [(c, 0, X, Y, W)])
    with pytest.raises(afsi.AfsiError):  # two slices write one block
        afsi.afsi_filter_batched(M.handle, [(c, 5, X, Y, W), (c, 5, to_dev(start_block(A.n, 32, seed=2)), Y,
                                                             t.zeros_like(X))])
    afsi.afsi_filter_batched(M.handle, [])  # nothing to do
    M.close()


# (ncols, ld, degree, interval, first step): widths with an exact lane mapping (the
# grouped kernel, two slices share a launch), a padded leading dimension, and widths
# that fall back to one product per slice (10 columns: no exact mapping; 3 columns: not
# whole 16-byte vectors)
GROUPED = [(32, 32, 7, (3.0, 3.5), 0), (96, 104, 12, (5.0, 5.3), 1), (32, 32, 5, (9.0, 11.0), 2),
           (64, 64, 8, (7.0, 7.4), 1), (128, 136, 9, (2.0, 2.4), 2), (10, 10, 6, (4.0, 4.6), 0),
           (3, 4, 4, (6.0, 6.2), 1)]


@pytest.mark.parametrize("matrix", ["stencil", "ragged"])
@pytest.mark.parametrize("cplx,single", [(False, False), (False, True), (True, False), (True, True)])
def test_grouped_slices_bitwise_equal_to_single_filters(cplx, single, matrix):
    t = torch()
    if cplx:
        A = tight_binding_3d_periodic(8, seed=3) if matrix == "stencil" else _ragged_symmetric(complex_=True)
        lmin, lmax = (-7.5, 7.5) if matrix == "stencil" else gershgorin_bounds(A)
        groups = [(nc, ld, k, (iv[0] - 5.0, iv[1] - 5.0), st) for nc, ld, k, iv, st in GROUPED]
    else:
        A = laplacian_3d_dirichlet(10, 2.0, seed=4) if matrix == "stencil" else _ragged_symmetric()
        lmin, lmax = (0.0, 14.0) if matrix == "stencil" else gershgorin_bounds(A)
        groups = GROUPED
    l1, l2 = co.affine_map(lmin, lmax)
    dt = _tdt(cplx, single)
    M = afsi.Matrix(A, bounds=(lmin, lmax))
    blocks, storage, X0s, coeffs = [], [], [], []
    for g, (nc, ld, k, iv, st) in enumerate(groups):
        X0 = start_block(A.n, nc, seed=20 + g, complex_=cplx)
        X0s.append(X0)
        coeffs.append(afsi.afsi_filter_coefficients(lmin, lmax, iv[0], iv[1], k, "jackson"))
        bufs = [t.zeros((A.n, ld), dtype=dt, device=DEV) for _ in range(3)]
        bufs[0][:, :nc] = t.from_numpy(X0).to(DEV).to(dt)
        storage.append(bufs)
        blocks.append([b[:, :nc] for b in bufs])
    total = max(st + k for (nc, ld, k, iv, st) in groups)
    for step in range(total):
        sl = []
        for g, (nc, ld, k, iv, st) in enumerate(groups):
            s = step - st
            if 0 <= s < k:
                sl.append((afsi.afsi_clenshaw_step_params(coeffs[g], k, s, l1, l2, ncols=nc), *blocks[g]))
        afsi.afsi_clenshaw_step_grouped(M.handle, sl)
    t.cuda.synchronize()
    for g, (nc, ld, k, iv, st) in enumerate(groups):
        X, P0, P1 = blocks[g]
        Yg = (P0 if (k - 1) % 2 == 0 else P1).cpu().numpy()
        Xs = t.from_numpy(X0s[g]).to(DEV).to(dt)
        Ys, Ws = t.empty_like(Xs), t.empty_like(Xs)
        afsi.afsi_filter_block(M.handle, coeffs[g], k, Xs, Ys, Ws)
        t.cuda.synchronize()
        assert np.array_equal(Yg, Ys.cpu().numpy()), g
        ref = oracle_filter(A, X0s[g], lmin, lmax, iv[0], iv[1], k)
        _check(Yg.astype(np.complex128 if cplx else np.float64), ref, f32_tol(k) if single else F64_TOL)
        # the padding columns of the slice's storage are never written
        for b in storage[g][1:]:
            assert not b[:, nc:].cpu().numpy().any()
    M.close()


def test_grouped_rejects_overlapping_slices():
    t = torch()
    A = laplacian_3d_dirichlet(6, 1.0, seed=2)
    M = afsi.Matrix(A, bounds=(0.0, 14.0))
    c = afsi.afsi_filter_coefficients(0.0, 14.0, 3.0, 4.0, 5)
    l1, l2 = co.affine_map(0.0, 14.0)
    X = to_dev(start_block(A.n, 32, seed=1))
    P = t.zeros((A.n, 64), dtype=t.float64, device=DEV)
    g = afsi.afsi_clenshaw_step_params(c, 5, 2, l1, l2, ncols=32)
    with pytest.raises(afsi.AfsiError):  # P0 and P1 of one slice overlap
        afsi.afsi_clenshaw_step_grouped(M.handle, [(g, X, P[:, :32], P[:, 16:48])])
    Q0, Q1 = t.zeros_like(X), t.zeros_like(X)
    with pytest.raises(afsi.AfsiError):  # two slices share a block
        afsi.afsi_clenshaw_step_grouped(M.handle, [(g, X, Q0, Q1), (g, X, t.zeros_like(X), t.zeros_like(X))])
    M.close()


@pytest.mark.parametrize("cplx,single", [(False, False), (False, True), (True, False)])
def test_column_blocks_give_the_same_bits(cplx, single):
    # products in column blocks of the dense operand (afsi_matrix_set_column_block, the
    # MaSpMM loop over column blocks) against whole-row passes: identical bits for every
    # block width, and the oracle's filter on sampled columns
    from workloads import random_banded_symmetric

    t = torch()
    A = random_banded_symmetric(6000, seed=5)
    if cplx:
        A = _ragged_symmetric(complex_=True)
    lmin, lmax = gershgorin_bounds(A)
    mid = 0.5 * (lmin + lmax)
    a, b = mid - 0.05 * (lmax - lmin), mid + 0.05 * (lmax - lmin)
    p, k = 160, 9
    X0 = start_block(A.n, p, seed=3, complex_=cplx)
    c = afsi.afsi_filter_coefficients(lmin, lmax, a, b, k, "jackson")
    M = afsi.Matrix(A, bounds=(lmin, lmax))
    assert afsi.afsi_matrix_get_column_block(M.handle) == 0
    dt = _tdt(cplx, single)
    X = t.from_numpy(X0).to(DEV).to(dt)
    outs = {}
    for seg in (0, 64, 128, 256):
        afsi.afsi_matrix_set_column_block(M.handle, seg)
        Y, W = t.zeros_like(X), t.zeros_like(X)
        afsi.afsi_filter_block(M.handle, c, k, X, Y, W)
        t.cuda.synchronize()
        outs[seg] = Y.cpu().numpy()
    for seg in (64, 128, 256):
        assert np.array_equal(outs[seg], outs[0]), seg
    for bad in (24, 48, -16):
        with pytest.raises(afsi.AfsiError):
            afsi.afsi_matrix_set_column_block(M.handle, bad)
    M.close()
    cols = [0, 77, p - 1]
    ref = oracle_filter(A, np.ascontiguousarray(X0[:, cols]), lmin, lmax, a, b, k)
    _check(outs[64][:, cols].astype(np.complex128 if cplx else np.float64), ref,
           f32_tol(k) if single else F64_TOL)


@pytest.mark.parametrize("name", ["lap3d_pot_100", "tb3d_64"])
@pytest.mark.parametrize("p,pad", [(1, 0), (2, 0), (3, 0), (1, 40), (3, 5), (8, 0), (16, 0)])
def test_narrow_products_full_size(name, p, pad):
    # the one-lane-per-row kernel at full size (the bounds estimate's single vectors,
    # narrow Krylov blocks): A X on p <= 16 columns, inside a wider block (ld = p + pad)
    # and contiguous, against the oracle's CSR product; the bits equal a column-by-column
    # run (every column takes the same entry order)
    from oracle import native

    t = torch()
    A, (lo, hi), _, cfg = build_config(name)
    cplx = A.is_complex
    X0 = start_block(A.n, p, seed=p + pad, complex_=cplx)
    M = afsi.Matrix(A, bounds=(lo, hi))
    dt = t.complex128 if cplx else t.float64
    Xs = t.zeros((A.n, p + pad), dtype=dt, device=DEV)
    Ys = t.zeros_like(Xs)
    Xs[:, :p] = t.from_numpy(X0).to(DEV)
    X, Y = Xs[:, :p], Ys[:, :p]
    afsi.afsi_spmm(M.handle, X, Y)
    t.cuda.synchronize()
    got = Y.cpu().numpy()
    ref = native.spmm(A, X0)
    assert rel_fro(got, ref) <= 1e-14 and max_rel(got, ref) <= 1e-13
    if pad:
        assert not Ys[:, p:].cpu().numpy().any()  # the rest of the wide block untouched
    one = t.zeros((A.n, 1), dtype=dt, device=DEV)
    out = t.zeros_like(one)
    for j in range(p):
        one.copy_(X[:, j:j + 1])
        afsi.afsi_spmm(M.handle, one, out)
        t.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy()[:, 0], got[:, j]), j
    M.close()
