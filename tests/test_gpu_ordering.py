"""GPU tests of the locality ordering (afsi_permute_rows, products and solves on P A P^T).

* afsi_permute_rows moves rows bit for bit (gather and inverse scatter, every element
  type, aligned and unaligned views) as numpy's indexing does;
* the filter of the reordered matrix applied to the reordered start block, moved back
  to the natural order, equals the oracle's filter of the natural matrix (FP64 to
  1e-12, FP32 to (k + 1) 2^-21 relative): at a size the whole oracle runs, and at the
  100^3 workload's full size in the 25 x 25 pencil ordering that the benchmark times
  (sampled columns, full degree);
* a whole solve on the reordered 27^3 window finds the 196 eigenvalues of the banded
  fixture, and its eigenvectors, moved back, are eigenvectors of the natural matrix.
"""
import numpy as np
import pytest

from oracle import coefficients as co
from oracle.filter import clenshaw_filter
from paper_2604_00914_amd import afsi
from tests.gpu_util import DEV, max_rel, rel_fro, to_dev, torch
from workloads import build_config, laplacian_3d_dirichlet, start_block

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


def f32_tol(k):
    return (k + 1) * 2.0 ** -21


def _check(got, ref, tol):
    assert rel_fro(got, ref) <= tol, rel_fro(got, ref)
    assert max_rel(got, ref) <= 10 * tol, max_rel(got, ref)


@pytest.mark.parametrize("dtype", ["f64", "f32", "c128", "c64"])
@pytest.mark.parametrize("p,pad,offset", [(1, 0, 0), (3, 2, 1), (64, 0, 0), (100, 7, 3), (256, 0, 0)])
def test_permute_rows_bitwise(dtype, p, pad, offset):
    t = torch()
    tdt = {"f64": t.float64, "f32": t.float32, "c128": t.complex128, "c64": t.complex64}[dtype]
    n = 1037
    rng = np.random.default_rng(p + pad)
    perm = rng.permutation(n)
    src_np = rng.standard_normal((n, p + pad)) + (1j * rng.standard_normal((n, p + pad)) if dtype[0] == "c" else 0)
    S = t.from_numpy(src_np).to(tdt).to(DEV)
    D = t.zeros_like(S)
    src, dst = S[:, offset: offset + p], D[:, offset: offset + p]
    afsi.afsi_permute_rows(src, perm, dst)
    ref = src.cpu().numpy()[perm]
    assert np.array_equal(dst.cpu().numpy(), ref)
    # the columns outside the view stay untouched
    if pad:
        assert not D[:, :offset].abs().sum().item() and not D[:, offset + p:].abs().sum().item()
    back = t.zeros_like(dst)
    afsi.afsi_permute_rows(dst, perm, back, inverse=True)
    assert np.array_equal(back.cpu().numpy(), src.cpu().numpy())


def test_permute_rows_rejects_bad_permutations():
    t = torch()
    X = t.zeros((10, 4), dtype=t.float64, device=DEV)
    Y = t.zeros_like(X)
    for bad in (np.zeros(10, dtype=np.int64), np.arange(1, 11), np.arange(9)):
        with pytest.raises(afsi.AfsiError) as e:
            afsi.afsi_permute_rows(X, bad, Y)
        assert e.value.status == -1
    with pytest.raises(afsi.AfsiError):
        afsi.afsi_permute_rows(X, np.arange(10), X)


def _ordered_filter(B, perm, X0, lmin, lmax, coeffs, degree, single, cols=None):
    """Filter P X0 with P A P^T on the GPU, move the result back with P^T."""
    t = torch()
    M = afsi.Matrix(B, bounds=(lmin, lmax))
    dt = t.float32 if single else t.float64
    Xn = t.from_numpy(X0).to(DEV).to(dt)
    X = t.empty_like(Xn)
    afsi.afsi_permute_rows(Xn, perm, X)
    Y, W = t.empty_like(X), t.empty_like(X)
    afsi.afsi_filter_block(M.handle, coeffs, degree, X, Y, W)
    afsi.afsi_permute_rows(Y, perm, Xn, inverse=True)
    t.cuda.synchronize()
    out = (Xn if cols is None else Xn[:, cols]).cpu().numpy().astype(np.float64)
    del X, Y, W, Xn
    t.cuda.empty_cache()
    M.close()
    return out


@pytest.mark.parametrize("tiles", [(8, 8), (5, 7), (30, 30)])
def test_ordered_filter_matches_oracle(tiles):
    N = 30
    A = laplacian_3d_dirichlet(N, 2.0, seed=7)
    lmin, lmax = 0.0, 14.0
    a, b, k = 6.9, 7.3, 40
    perm = afsi.afsi_grid_order(N, N, N, *tiles)
    B = afsi.afsi_csr_permute(A, perm)
    X0 = start_block(A.n, 64, seed=2)
    c = co.filter_coefficients(lmin, lmax, a, b, k, "jackson")
    l1, l2 = co.affine_map(lmin, lmax)
    ref = clenshaw_filter(A, X0, c, l1, l2)
    for single in (False, True):
        got = _ordered_filter(B, perm, X0, lmin, lmax, c, k, single)
        _check(got, ref, f32_tol(k) if single else F64_TOL)


@pytest.mark.parametrize("single", [False, True])
def test_folded_order_filter_on_periodic_lattice(single):
    # the complex periodic lattice in folded pencils (C128 and C64): the filter of P A P^T
    # on P X, moved back, against the oracle's filter of the natural matrix
    from workloads import tight_binding_3d_periodic

    t = torch()
    L = 16
    A = tight_binding_3d_periodic(L, seed=3)
    lmin, lmax, a, b, k = -7.0, 7.0, -0.4, 0.3, 60
    perm = afsi.afsi_grid_order(L, L, L, 8, 8, fold_x=True)
    B = afsi.afsi_csr_permute(A, perm)
    X0 = start_block(A.n, 32, seed=4, complex_=True)
    c = co.filter_coefficients(lmin, lmax, a, b, k, "jackson")
    l1, l2 = co.affine_map(lmin, lmax)
    ref = clenshaw_filter(A, X0, c, l1, l2)
    M = afsi.Matrix(B, bounds=(lmin, lmax))
    dt = t.complex64 if single else t.complex128
    Xn = t.from_numpy(X0).to(DEV).to(dt)
    X = t.empty_like(Xn)
    afsi.afsi_permute_rows(Xn, perm, X)
    Y, W = t.empty_like(X), t.empty_like(X)
    afsi.afsi_filter_block(M.handle, c, k, X, Y, W)
    afsi.afsi_permute_rows(Y, perm, Xn, inverse=True)
    got = Xn.cpu().numpy().astype(np.complex128)
    M.close()
    _check(got, ref, f32_tol(k) if single else F64_TOL)


def test_full_size_pencil_order_sampled_columns():
    # the benchmark's launch configuration: lap3d_pot_100 in 25 x 25 pencils, n = 1e6,
    # p = 256, the workload's degree, FP64 and FP32; columns act independently, so
    # sampled columns equal the oracle's filter of those start columns
    A, (lmin, lmax), (a, b), cfg = build_config("lap3d_pot_100")
    perm = afsi.afsi_grid_order(100, 100, 100, 25, 25)
    B = afsi.afsi_csr_permute(A, perm)
    cols = [0, 129, 255]
    X0 = start_block(A.n, cfg.p, seed=0)
    c = co.filter_coefficients(lmin, lmax, a, b, cfg.degree, cfg.damping)
    l1, l2 = co.affine_map(lmin, lmax)
    ref = clenshaw_filter(A, np.ascontiguousarray(X0[:, cols]), c, l1, l2)
    for single in (False, True):
        got = _ordered_filter(B, perm, X0, lmin, lmax, c, cfg.degree, single, cols)
        _check(got, ref, f32_tol(cfg.degree) if single else F64_TOL)


def test_solve_on_pencil_ordered_window():
    # the 27^3 window (196 eigenvalues) in 9 x 9 pencils, the paper's adaptive mode:
    # the eigenvalues of the fixture, exact count; eigenvectors moved back to the
    # natural order are eigenvectors of the natural matrix
    from tests.golden_util import lap3d27_window

    t = torch()
    A, (lmin, lmax), (a, b), cfg = build_config("lap3d_pot_27")
    perm = afsi.afsi_grid_order(27, 27, 27, 9, 9)
    B = afsi.afsi_csr_permute(A, perm)
    ref = lap3d27_window()
    normA = max(abs(lmin), abs(lmax))
    M = afsi.Matrix(B, bounds=(lmin, lmax))
    o = afsi.afsi_options_default(cfg.degree)
    o.adaptive, o.damping, o.max_iter = 1, afsi.DAMP_LANCZOS, 600
    Xn = to_dev(start_block(A.n, cfg.p, 0))
    X = t.empty_like(Xn)
    afsi.afsi_permute_rows(Xn, perm, X)
    E = t.zeros_like(X)
    st, lam, res, r = afsi.afsi_solve(M.handle, a, b, o, X, E, cfg.p)
    assert st == 0 and r.converged and r.count == ref.size == 196
    assert np.max(np.abs(lam - ref)) <= 1e-10 * normA
    En = t.zeros_like(E)
    afsi.afsi_permute_rows(E, perm, En, inverse=True)
    V = En[:, : r.count].cpu().numpy()
    R = A.to_scipy() @ V - V * lam
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-9 * normA
    M.close()


@pytest.mark.parametrize("single", [False, True])
def test_full_size_grouped_slices_pencil_order(single):
    # the serving path's grouped step on the 50 x 50 pencil ordering the slice benchmark
    # uses: 16 slices x 96 columns of the 100^3 matrix, degree 120, odd slices one step
    # behind; one sampled column per slice, moved back to the natural order, against the
    # oracle's filter of the natural matrix
    from workloads.stream import slice_intervals

    t = torch()
    A, (lo, hi), _, cfg = build_config("lap3d_pot_100")
    perm = afsi.afsi_grid_order(100, 100, 100, 50, 50)
    B = afsi.afsi_csr_permute(A, perm)
    k, G, cols = cfg.degree, 16, 96
    l1, l2 = co.affine_map(lo, hi)
    ivs = slice_intervals(A.n, 0.5 * (lo + hi), G, 50)
    coeffs = [co.filter_coefficients(lo, hi, a, b, k, "jackson") for a, b in ivs]
    dt = t.float32 if single else t.float64
    M = afsi.Matrix(B, bounds=(lo, hi))
    pick, cols0, blocks = [], [], []
    for g in range(G):
        X0 = start_block(A.n, cols, seed=200 + g)
        c = (5 * g + 3) % cols
        pick.append(c)
        cols0.append(np.ascontiguousarray(X0[:, c:c + 1]))
        X = t.from_numpy(np.ascontiguousarray(X0[perm])).to(DEV).to(dt)
        blocks.append((X, t.zeros_like(X), t.zeros_like(X)))
        del X0
    for step in range(k + 1):
        sl = []
        for g in range(G):
            s_g = step - (g % 2)
            if 0 <= s_g < k:
                sl.append((afsi.afsi_clenshaw_step_params(coeffs[g], k, s_g, l1, l2, ncols=cols), *blocks[g]))
        afsi.afsi_clenshaw_step_grouped(M.handle, sl)
    t.cuda.synchronize()
    got = []
    for g in range(G):
        y = blocks[g][1 + (k - 1) % 2][:, pick[g]].cpu().numpy().astype(np.float64)
        nat = np.empty_like(y)
        nat[perm] = y
        got.append(nat)
    del blocks
    t.cuda.empty_cache()
    M.close()
    for g in range(G):
        ref = clenshaw_filter(A, cols0[g], coeffs[g], l1, l2)
        _check(got[g][:, None], ref, f32_tol(k) if single else F64_TOL)
