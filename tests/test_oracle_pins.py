"""The CPU oracle pinned to things other than itself.

Every check compares the oracle with a closed form, an invariant the
mathematics fixes, a textbook/library routine on a special case, or brute
force on a tiny input.  None re-types the oracle's own formulas.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from paper_2410_02408_amd import workloads as w


def mu(j, n):
    """Eigenvalues of tridiag(-1, 2, -1) of order n: 2 - 2 cos(j pi / (n + 1))."""
    return 2.0 - 2.0 * np.cos(j * np.pi / (n + 1))


def sine(j, n):
    return np.sin(j * np.pi * np.arange(1, n + 1) / (n + 1))


def blockdiag_dense(D, off):
    M = np.zeros_like(D)
    for s, e in zip(off[:-1], off[1:]):
        M[s:e, s:e] = D[s:e, s:e]
    return M


def csr_from_rows(n, rows):
    """CSR from explicit per-row (col, val) lists (keeps order and duplicates)."""
    rp = np.zeros(n + 1, np.int32)
    ci, vv = [], []
    for i, row in enumerate(rows):
        for c, v in row:
            ci.append(c)
            vv.append(v)
        rp[i + 1] = len(ci)
    return w.CsrMatrix(n, rp, np.array(ci, np.int32), np.array(vv, float))


# ---------------------------------------------------------------- SpMV

@pytest.mark.parametrize("shape,modes", [((17,), [(1,), (5,), (17,)]),
                                         ((9, 7), [(1, 1), (3, 6), (9, 7)]),
                                         ((5, 4, 6), [(1, 1, 1), (2, 4, 5)])])
def test_spmv_laplacian_sine_modes(orc, shape, modes):
    """Dirichlet Laplacian: A s = (sum_a mu_{j_a}) s for separable sine modes."""
    A = w.dirichlet_laplacian(shape)
    for js in modes:
        s = np.ones(1)
        lam = 0.0
        for a, j in enumerate(js):          # x fastest -> kron(z, y, x)
            s = np.kron(sine(j, shape[a]), s)
            lam += mu(j, shape[a])
        np.testing.assert_allclose(orc.spmv(A, s), lam * s, atol=1e-13 * np.abs(s).max() * 8)


def test_spmv_dense_bruteforce_duplicates_unsorted(orc):
    rng = np.random.default_rng(5)
    n = 7
    rows = []
    for i in range(n):
        cols = rng.integers(0, n, size=5)   # repeats and arbitrary order
        rows.append([(int(c), float(v)) for c, v in zip(cols, rng.standard_normal(5))])
    A = csr_from_rows(n, rows)
    x = rng.standard_normal(n)
    np.testing.assert_allclose(orc.spmv(A, x), A.to_dense() @ x, rtol=0, atol=1e-13)


def test_spmv_row_sum_shift(orc):
    """Diagonally dominant generators: A 1 = shift 1 exactly (graph Laplacian + shift)."""
    A = w.random_spd(3000, np.random.default_rng(1))
    np.testing.assert_allclose(orc.spmv(A, np.ones(A.n)), 0.01, atol=1e-12)
    P = w.powerlaw_spd(1 << 12, seed=9)
    np.testing.assert_allclose(orc.spmv(P, np.ones(P.n)), 0.1, atol=1e-11)


def test_dot_exact_small(orc):
    a = np.array([1.0, 2.0, 3.0, 0.5])
    assert orc.dot(a, a) == 14.25


def test_validate(orc):
    A = w.poisson2d(4)
    assert orc.validate(A) == "OK"
    bad = w.CsrMatrix(A.n, A.row_ptr.copy(), A.col_idx.copy(), A.val.copy())
    bad.col_idx[3] = A.n
    assert orc.validate(bad) == "EINVAL"
    bad = w.CsrMatrix(A.n, A.row_ptr.copy(), A.col_idx.copy(), A.val.copy())
    bad.row_ptr[5], bad.row_ptr[6] = bad.row_ptr[6], bad.row_ptr[5]
    assert orc.validate(bad) == "EINVAL"
    bad = w.CsrMatrix(A.n, A.row_ptr.copy(), A.col_idx.copy(), A.val.copy())
    bad.val[0] = np.nan
    assert orc.validate(bad) == "ENONFINITE"


# ---------------------------------------------------------------- blocks

@pytest.mark.parametrize("n,nb", [(100, 10), (100, 16), (5, 8), (64, 64), (1, 1), (33, 32)])
def test_uniform_offsets_match_partition_slicing(orc, n, nb):
    """Section 4.2 slices A[i:i+bs] for i in range(0, n, bs): last block ragged."""
    expected = [min(i, n) for i in range(0, n, nb)] + [n]
    assert orc.uniform_offsets(n, nb).tolist() == expected


def test_extract_single_block_is_dense_matrix(orc):
    A = w.random_spd(40, np.random.default_rng(2))
    np.testing.assert_array_equal(orc.extract_block(A, 0, A.n), A.to_dense())


def test_extract_block_size_one_is_diagonal(orc):
    """Block size 1: the tile is A_ii (the paper's point-Jacobi operand)."""
    A = w.diffusion3d(5)
    D = A.to_dense()
    for i in [0, 7, 124]:
        assert orc.extract_block(A, i, i + 1)[0, 0] == D[i, i]


def test_extract_sums_duplicates_and_ignores_outside(orc):
    A = csr_from_rows(4, [[(0, 1.0), (3, 9.0), (1, 2.0), (0, 0.5)],
                          [(1, 4.0), (2, 7.0), (0, 2.0)],
                          [(2, 1.0)], [(3, 1.0)]])
    np.testing.assert_array_equal(orc.extract_block(A, 0, 2), [[1.5, 2.0], [2.0, 4.0]])


def test_extract_stencil_tiles_are_tridiagonal(orc):
    """Blocks inside one grid line of a 2D stencil see only the x-couplings."""
    A = w.poisson2d(32)
    T = orc.extract_block(A, 16, 32)
    expected = 4 * np.eye(16) - np.eye(16, k=1) - np.eye(16, k=-1)
    np.testing.assert_array_equal(T, expected)


def test_extract_partition_conserves_nnz(orc):
    """Sum of block-tile entries + entries outside the blocks = all entries."""
    A = w.random_spd(200, np.random.default_rng(3))
    off = orc.uniform_offsets(A.n, 16)
    D = A.to_dense()
    inside = sum(orc.extract_block(A, s, e).sum() for s, e in zip(off[:-1], off[1:]))
    assert np.isclose(inside + (D - blockdiag_dense(D, off)).sum(), D.sum(), atol=1e-10)


# ---------------------------------------------------------------- Cholesky / apply

def test_cholesky_matches_lapack(orc):
    rng = np.random.default_rng(4)
    for m in [1, 2, 5, 16, 33, 64]:
        G = rng.standard_normal((m, m))
        S = G @ G.T + m * np.eye(m)
        np.testing.assert_allclose(orc.cholesky(S), np.linalg.cholesky(S), rtol=1e-12, atol=1e-12)


def test_cholesky_rejects_indefinite(orc):
    S = np.array([[1.0, 2.0], [2.0, 1.0]])
    with pytest.raises(orc.OracleError) as e:
        orc.cholesky(S)
    assert e.value.status == "ENOTSPD"


def test_apply_is_block_solve(orc):
    A = w.random_spd(150, np.random.default_rng(6))
    off = orc.uniform_offsets(A.n, 32)        # ragged last block of 22
    M = orc.Precond(A, off)
    D = A.to_dense()
    r = np.random.default_rng(7).standard_normal(A.n)
    z = M.apply(r)
    for s, e in zip(off[:-1], off[1:]):
        np.testing.assert_allclose(z[s:e], np.linalg.solve(D[s:e, s:e], r[s:e]), rtol=1e-11)


def test_apply_block_size_one_is_point_jacobi(orc):
    """n_b = 1 is the paper's M_i = 1 / A_ii (Section 3.3, CUDA kernel of 4.3)."""
    A = w.diffusion3d(6)
    M = orc.Precond.uniform(A, 1)
    r = np.random.default_rng(8).standard_normal(A.n)
    np.testing.assert_allclose(M.apply(r), r / np.diag(A.to_dense()), rtol=1e-15)


def test_precondition_reports_first_failing_block(orc):
    A = w.random_spd(100, np.random.default_rng(9))
    D = A.to_dense()
    i = 3 * 16 + 5
    A.val[np.nonzero((np.repeat(np.arange(A.n), np.diff(A.row_ptr)) == i) & (A.col_idx == i))[0]] = -1.0
    with pytest.raises(orc.OracleError) as e:
        orc.Precond.uniform(A, 16)
    assert e.value.status == "ENOTSPD" and e.value.failed_block == 3
    assert D[i, i] > 0


def test_factor_reconstructs_block(orc):
    A = w.diffusion3d(6)
    M = orc.Precond.uniform(A, 64)
    D = A.to_dense()
    for t in [0, 1, 3]:
        L = M.factor(t)
        s, e = M.offsets[t], M.offsets[t + 1]
        np.testing.assert_allclose(L @ L.T, D[s:e, s:e], rtol=1e-13, atol=1e-13)
        assert np.all(np.triu(L, 1) == 0)


# ---------------------------------------------------------------- PCG

def test_pcg_single_block_one_iteration(orc):
    """One block spanning A: M^-1 A = I, PCG finishes in one step with x = A^-1 b."""
    A = w.poisson2d(8)                        # N = 64, the largest tile
    b = w.rhs(64, 11)
    r = orc.pcg(A, b, orc.Precond.uniform(A, 64))
    assert r.status == "OK" and r.iterations == 1
    np.testing.assert_allclose(r.x, np.linalg.solve(A.to_dense(), b), rtol=1e-12)


def test_pcg_block_diagonal_is_aggregate(orc):
    """Block-diagonal A aligned with the partition: x is the concatenation of
    the block solutions (Section 3.6) after one iteration."""
    rng = np.random.default_rng(12)
    blocks = []
    rows, cols, vals = [], [], []
    s = 0
    for m in [16, 16, 16, 7]:
        G = rng.standard_normal((m, m))
        S = G @ G.T + m * np.eye(m)
        blocks.append((s, S))
        r, c = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        rows.append((r + s).ravel()); cols.append((c + s).ravel()); vals.append(S.ravel())
        s += m
    A = w.from_coo(s, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))
    b = rng.standard_normal(s)
    res = orc.pcg(A, b, orc.Precond.uniform(A, 16))
    assert res.status == "OK" and res.iterations == 1
    for s0, S in blocks:
        np.testing.assert_allclose(res.x[s0:s0 + len(S)], np.linalg.solve(S, b[s0:s0 + len(S)]), rtol=1e-11)


def test_pcg_diagonal_matrix_point_jacobi(orc):
    d = np.linspace(1.0, 1e4, 300)
    A = w.from_coo(300, np.arange(300), np.arange(300), d)
    b = w.rhs(300, 13)
    r = orc.pcg(A, b, orc.Precond.uniform(A, 1))
    assert r.iterations == 1 and r.status == "OK"
    np.testing.assert_allclose(r.x, b / d, rtol=1e-15)


def test_cg_finite_termination_on_few_eigenvectors(orc):
    """b in the span of k eigenvectors: exact CG needs at most k steps."""
    n = 40
    A = w.laplacian1d(n)
    b = sine(2, n) + 0.5 * sine(9, n) - 2 * sine(31, n)
    r = orc.pcg(A, b, None, tol=1e-12)
    assert r.status == "OK" and r.iterations <= 3
    x_exact = sine(2, n) / mu(2, n) + 0.5 * sine(9, n) / mu(9, n) - 2 * sine(31, n) / mu(31, n)
    np.testing.assert_allclose(r.x, x_exact, rtol=1e-10, atol=1e-12)


def test_pcg_manufactured_solution(orc):
    n = 24
    A = w.poisson2d(n)
    xs = np.kron(sine(3, n), sine(2, n))
    b = (mu(3, n) + mu(2, n)) * xs
    for nb in [1, 8, 24, 64]:
        r = orc.pcg(A, b, orc.Precond.uniform(A, nb), tol=1e-12)
        assert r.status == "OK"
        assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < 1e-10


def test_pcg_solution_vs_sparse_direct(orc):
    import scipy.sparse.linalg as spl

    W = w.workload("diffusion3d_12")
    M = orc.Precond.uniform(W.A, 64)
    r = orc.pcg(W.A, W.b, M, tol=1e-10)
    xd = spl.spsolve(W.A.to_scipy().tocsc(), W.b)
    assert r.status == "OK" and r.rel_res_true <= 1e-10
    kap = np.linalg.cond(W.A.to_dense())
    assert np.linalg.norm(r.x - xd) / np.linalg.norm(xd) <= 1e-10 * kap
    resid = np.linalg.norm(W.A.to_scipy() @ r.x - W.b) / np.linalg.norm(W.b)
    assert resid <= 1e-10 and abs(resid - r.rel_res_true) < 1e-12


def test_pcg_energy_error_monotone_and_bounded(orc):
    """CG minimises the A-norm error over growing Krylov spaces: it decreases
    monotonically and obeys 2((sqrt(k)-1)/(sqrt(k)+1))^j (k = kappa(M^-1 A))."""
    A = w.poisson2d(20)
    D = A.to_dense()
    b = w.rhs(A.n, 14)
    xs = np.linalg.solve(D, b)
    M = orc.Precond.uniform(A, 10)
    ev = sl.eigh(D, blockdiag_dense(D, orc.uniform_offsets(A.n, 10)), eigvals_only=True)
    q = (np.sqrt(ev[-1] / ev[0]) - 1) / (np.sqrt(ev[-1] / ev[0]) + 1)
    e0 = np.sqrt(xs @ D @ xs)
    prev = e0
    for k in range(1, 25):
        r = orc.pcg(A, b, M, max_iter=k, max_replacements=0, tol=1e-14)
        e = r.x - xs
        en = np.sqrt(e @ D @ e)
        assert en < prev
        assert en <= 2 * q ** k * e0 * (1 + 1e-9)
        prev = en


def test_pcg_b_zero(orc):
    A = w.poisson2d(6)
    r = orc.pcg(A, np.zeros(36), orc.Precond.uniform(A, 4), x0=np.ones(36))
    assert r.status == "OK" and r.iterations == 0 and np.all(r.x == 0)


def test_pcg_max_iter_returns_noconv(orc):
    A = w.poisson2d(16)
    r = orc.pcg(A, w.rhs(256, 15), orc.Precond.uniform(A, 8), max_iter=1)
    assert r.status == "ENOCONV" and r.iterations == 1 and 0 < r.rel_res_true < 1


def test_pcg_nonfinite_rhs(orc):
    A = w.poisson2d(4)
    b = np.ones(16)
    b[3] = np.nan
    assert orc.pcg(A, b).status == "ENONFINITE"


def test_pcg_indefinite_breaks_down(orc):
    """SPD diagonal blocks but an indefinite A: p^T A p <= 0 is detected."""
    n = 32
    rows, cols, vals = list(range(n)), list(range(n)), [1.0] * n
    for i in range(0, n, 2):              # couple rows across block boundaries
        j = (i + 17) % n
        rows += [i, j]; cols += [j, i]; vals += [3.0, 3.0]
    A = w.from_coo(n, np.array(rows), np.array(cols), np.array(vals))
    ev, vec = np.linalg.eigh(A.to_dense())
    assert ev[0] < 0
    # the diagonal blocks are identities (M = I), so p_1 = b and p^T A p < 0
    r = orc.pcg(A, vec[:, 0], orc.Precond.uniform(A, 8))
    assert r.status == "EBREAKDOWN" and r.iterations == 0


def test_pcg_warm_start_from_solution(orc):
    A = w.poisson2d(10)
    b = w.rhs(100, 16)
    xs = np.linalg.solve(A.to_dense(), b)
    r = orc.pcg(A, b, orc.Precond.uniform(A, 5), x0=xs)
    assert r.status == "OK" and r.iterations == 0


# ---------------------------------------------------------------- kappa

@pytest.mark.parametrize("shape", [(32,), (32, 32), (10, 10, 10)])
def test_kappa_laplacian_closed_form(orc, shape):
    """kappa(A) = cot^2(pi / (2(n+1))) for the Dirichlet Laplacian on an n^d grid."""
    A = w.dirichlet_laplacian(shape)
    n = shape[0]
    exact = 1.0 / np.tan(np.pi / (2 * (n + 1))) ** 2
    k = orc.kappa(A, w.rhs(A.n, 17), 100)
    assert abs(k.kappa - exact) / exact < 1e-9


def test_kappa_cfg_small_closed_form_and_dense(orc):
    """2D 32x32, blocks of 16: kappa(A) = cot^2(pi/66); kappa(M^-1 A) against a
    dense generalised eigensolve; 2-cyclic block graph gives l_min + l_max = 2."""
    W = w.workload("poisson2d_32")
    kA = orc.kappa(W.A, W.b, 100)
    assert abs(kA.kappa - 1 / np.tan(np.pi / 66) ** 2) / kA.kappa < 1e-9
    M = orc.Precond.uniform(W.A, 16)
    kM = orc.kappa(W.A, W.b, 100, M)
    D = W.A.to_dense()
    ev = sl.eigh(D, blockdiag_dense(D, M.offsets), eigvals_only=True)
    assert abs(kM.kappa - ev[-1] / ev[0]) / kM.kappa < 1e-9
    assert abs(kM.theta_min + kM.theta_max - 2.0) < 1e-10


def test_kappa_line_block_closed_form(orc):
    """Blocks = whole x-lines of the 2D Laplacian: kappa = 1 / (1 - cos(pi/(n+1)))."""
    n = 32
    A = w.poisson2d(n)
    M = orc.Precond.uniform(A, n)
    k = orc.kappa(A, w.rhs(A.n, 18), 100, M)
    exact = 1.0 / (1.0 - np.cos(np.pi / (n + 1)))
    assert abs(k.kappa - exact) / exact < 1e-9


def test_kappa_3d_line_block_closed_form(orc):
    """3D Laplacian with x-line blocks: kappa = (8 - mu_1) / (3 mu_1)."""
    n = 12
    A = w.poisson3d(n)
    M = orc.Precond.uniform(A, n)
    k = orc.kappa(A, w.rhs(A.n, 19), 150, M)
    m1 = mu(1, n)
    exact = (8 - m1) / (3 * m1)
    assert abs(k.kappa - exact) / exact < 1e-8


def test_kappa_single_block_is_one(orc):
    A = w.poisson2d(8)
    k = orc.kappa(A, w.rhs(64, 20), 30, orc.Precond.uniform(A, 64))
    assert k.steps == 1 and abs(k.kappa - 1) < 1e-12


def test_kappa_diagonal_point_jacobi_is_one(orc):
    d = np.linspace(1, 50, 100)
    A = w.from_coo(100, np.arange(100), np.arange(100), d)
    k = orc.kappa(A, np.ones(100), 20, orc.Precond.uniform(A, 1))
    assert k.steps == 1 and abs(k.kappa - 1) < 1e-12
    kA = orc.kappa(A, np.ones(100), 100)
    assert abs(kA.kappa - 50.0) < 1e-9


def test_lanczos_full_run_reproduces_spectrum(orc):
    """N steps of reorthogonalised Lanczos: T has the spectrum of M^-1 A."""
    A = w.random_spd(60, np.random.default_rng(21), shift=0.5)
    D = A.to_dense()
    v0 = w.rhs(60, 22)
    lz = orc.lanczos(A, v0, 60)
    T = np.diag(lz.alpha) + np.diag(lz.beta, 1) + np.diag(lz.beta, -1)
    np.testing.assert_allclose(np.linalg.eigvalsh(T), np.linalg.eigvalsh(D), rtol=1e-10)
    M = orc.Precond.uniform(A, 8)
    lz = orc.lanczos(A, v0, 60, M)
    T = np.diag(lz.alpha) + np.diag(lz.beta, 1) + np.diag(lz.beta, -1)
    ev = sl.eigh(D, blockdiag_dense(D, M.offsets), eigvals_only=True)
    np.testing.assert_allclose(np.linalg.eigvalsh(T), ev, rtol=1e-10)


def test_lanczos_estimate_bounds_and_monotone(orc):
    """Ritz values interlace: theta_min >= lambda_min, theta_max <= lambda_max,
    and the estimate grows with the step count."""
    W = w.workload("diffusion3d_8")
    D = W.A.to_dense()
    M = orc.Precond.uniform(W.A, 64)
    ev = sl.eigh(D, blockdiag_dense(D, M.offsets), eigvals_only=True)
    prev = 0
    for m in [5, 10, 20, 40]:
        k = orc.kappa(W.A, W.b, m, M)
        assert k.theta_min >= ev[0] * (1 - 1e-12) and k.theta_max <= ev[-1] * (1 + 1e-12)
        assert k.kappa >= prev
        prev = k.kappa
    assert prev <= ev[-1] / ev[0] * (1 + 1e-10)


def test_lanczos_zero_start_breaks_down(orc):
    A = w.poisson2d(4)
    assert orc.lanczos(A, np.zeros(16), 5).status == "EBREAKDOWN"


# ---------------------------------------------------------------- tridiagonal

def test_tridiag_extremes_closed_form(orc):
    for m in [1, 2, 7, 50, 200]:
        lo, hi = orc.tridiag_extremes(np.full(m, 2.0), np.full(m - 1, -1.0))
        assert abs(lo - mu(1, m)) <= 4e-16 * 4 + 1e-15 and abs(hi - mu(m, m)) <= 1e-15 * 4


def test_tridiag_extremes_vs_lapack(orc):
    rng = np.random.default_rng(23)
    for m in [3, 17, 100, 200]:
        a = rng.standard_normal(m) * 10
        b = rng.standard_normal(m - 1)
        ev = sl.eigh_tridiagonal(a, b, eigvals_only=True)
        lo, hi = orc.tridiag_extremes(a, b)
        assert abs(lo - ev[0]) <= 1e-13 * np.abs(ev).max()
        assert abs(hi - ev[-1]) <= 1e-13 * np.abs(ev).max()


def test_sturm_count_vs_eigenvalues(orc):
    rng = np.random.default_rng(24)
    a = rng.standard_normal(30)
    b = rng.standard_normal(29)
    ev = sl.eigh_tridiagonal(a, b, eigvals_only=True)
    for x in rng.uniform(ev[0] - 1, ev[-1] + 1, size=40):
        assert orc.sturm_count(a, b, x) == int(np.sum(ev < x))


# ---------------------------------------------------------------- adjoint

def _loss_dense(A, b, xt):
    x = np.linalg.solve(A.to_dense(), b)
    return np.sum((x - xt) ** 2)


def test_edge_grad_vs_finite_differences(orc):
    g = w.edge_graph2d(6)
    c = w.edge_conductivities(g, seed=3)
    A = w.edge_poisson2d(g, c)
    b, xt = w.rhs(g.n_rows, 3), w.target(g.n_rows, 3)
    D = A.to_dense()
    x = np.linalg.solve(D, b)
    lam = np.linalg.solve(D, 2 * (x - xt))
    grad = orc.edge_grad(g, lam, x)
    h = 1e-6
    for e in list(range(0, len(c), 7)) + [len(c) - 1]:
        cp, cm = c.copy(), c.copy()
        cp[e] += h
        cm[e] -= h
        fd = (_loss_dense(w.edge_poisson2d(g, cp), b, xt) - _loss_dense(w.edge_poisson2d(g, cm), b, xt)) / (2 * h)
        assert abs(fd - grad[e]) <= 1e-6 * max(1.0, abs(fd))


def test_value_grad_vs_finite_differences(orc):
    A = w.random_spd(30, np.random.default_rng(25), shift=1.0)
    b, xt = w.rhs(30, 26), w.target(30, 26)
    D = A.to_dense()
    x = np.linalg.solve(D, b)
    lam = np.linalg.solve(D, 2 * (x - xt))
    grad = orc.value_grad(A, lam, x)
    h = 1e-6
    for k in range(0, A.nnz, 11):
        vp = A.val.copy(); vp[k] += h
        vm = A.val.copy(); vm[k] -= h
        Lp = _loss_dense(w.CsrMatrix(30, A.row_ptr, A.col_idx, vp), b, xt)
        Lm = _loss_dense(w.CsrMatrix(30, A.row_ptr, A.col_idx, vm), b, xt)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(fd))


# ---------------------------------------------------------------- residual replacement

def _true_residual_ld(A, x, b):
    """||b - A x|| / ||b|| evaluated in extended precision (x86 long double,
    64-bit mantissa): independent of the oracle's FP64 evaluation and far
    more accurate than its ~4e-16 rounding floor."""
    D = A.to_dense().astype(np.longdouble)
    r = b.astype(np.longdouble) - D @ np.asarray(x).astype(np.longdouble)
    return float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(b.astype(np.longdouble) ** 2)))


def test_pcg_residual_replacement_converges(orc):
    """2D 32x32, blocks of 16, tol 1e-14: the recursive residual drifts from
    b - A x, so when the recursion first meets tol the true residual does not
    (Section 3.7's check).  A solve may only report OK with a true residual
    <= tol; that needs a replacement here, and the reported true residual is
    the real one (an extended-precision evaluation agrees to the FP64 floor).
    x equals a dense LAPACK solve."""
    W = w.workload("poisson2d_32")
    M = orc.Precond.uniform(W.A, 16)
    r = orc.pcg(W.A, W.b, M, tol=1e-14, max_replacements=3)
    assert r.status == "OK" and r.rel_res_true <= 1e-14 and r.replacements >= 1
    assert abs(_true_residual_ld(W.A, r.x, W.b) - r.rel_res_true) <= 1e-15
    xs = sl.solve(W.A.to_dense(), W.b, assume_a="pos")
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) <= 1e-12
    # without the replacement budget the same recursion ends unconverged
    r0 = orc.pcg(W.A, W.b, M, tol=1e-14, max_replacements=0)
    assert r0.status == "ENOCONV" and r0.replacements == 0 and r0.rel_res_true > 1e-14
    assert abs(_true_residual_ld(W.A, r0.x, W.b) - r0.rel_res_true) <= 1e-15


@pytest.mark.parametrize("nb", [16, 0])
def test_pcg_replacement_budget_below_rounding_floor(orc, nb):
    """tol 1e-16 lies below the rounding floor of an FP64 evaluation of
    b - A x (~4e-16 here), so every true-residual check fails: the solve
    ends ENOCONV after exactly max_replacements restarts, each followed by
    at least one iteration, and every reported true residual is the real one
    and above tol."""
    W = w.workload("poisson2d_32")
    M = orc.Precond.uniform(W.A, nb) if nb else None
    prev = 0
    for m in range(4):
        r = orc.pcg(W.A, W.b, M, tol=1e-16, max_replacements=m)
        assert r.status == "ENOCONV" and r.replacements == m and r.iterations < W.A.n
        assert r.iterations > prev
        prev = r.iterations
        t = _true_residual_ld(W.A, r.x, W.b)
        assert t > 1e-16 and abs(t - r.rel_res_true) <= 1e-15


def test_pcg_no_replacement_without_iterations_left(orc):
    """When the recursion meets tol at exactly max_iter and the true residual
    does not, no iteration is left for a restart: ENOCONV, the replacement
    count unchanged and x the last iterate; one more allowed iteration is
    enough to converge after the replacement."""
    W = w.workload("poisson2d_32")
    M = orc.Precond.uniform(W.A, 16)
    k1 = orc.pcg(W.A, W.b, M, tol=1e-14, max_replacements=0).iterations
    full = orc.pcg(W.A, W.b, M, tol=1e-14, max_replacements=3)
    assert full.replacements == 1 and full.iterations == k1 + 1
    r = orc.pcg(W.A, W.b, M, tol=1e-14, max_iter=k1, max_replacements=3)
    assert r.status == "ENOCONV" and r.iterations == k1 and r.replacements == 0
    assert r.rel_res_true > 1e-14
    r = orc.pcg(W.A, W.b, M, tol=1e-14, max_iter=k1 + 1, max_replacements=3)
    assert r.status == "OK" and r.iterations == k1 + 1 and r.replacements == 1
