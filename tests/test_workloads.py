"""Invariants of the seeded input generators (no solver arithmetic involved)."""
import numpy as np
import pytest

from paper_2410_02408_amd import workloads as w


def _sym(A):
    D = A.to_dense()
    return np.array_equal(D, D.T)


@pytest.mark.parametrize("n", [1, 2, 5, 32])
def test_poisson2d_structure(n):
    A = w.poisson2d(n)
    assert A.nnz == 5 * n * n - 4 * n
    assert A.row_ptr.dtype == np.int32 and A.col_idx.dtype == np.int32
    D = A.to_dense()
    assert np.all(np.diag(D) == 4.0) and _sym(A)
    for i in range(A.n):                      # columns sorted, no duplicates
        c = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_poisson3d_nnz():
    for n in [2, 3, 7]:
        assert w.poisson3d(n).nnz == 7 * n ** 3 - 6 * n ** 2


def test_diffusion3d_harmonic_faces_and_reduction():
    n = 6
    A = w.diffusion3d(n, 1.5, 1)
    assert A.nnz == 7 * n ** 3 - 6 * n ** 2 and _sym(A)
    k = np.exp(1.5 * np.random.default_rng(np.random.SeedSequence(1).spawn(4)[0]).standard_normal(n ** 3))
    D = A.to_dense()
    i, j = 5 + n * 2 + n * n * 3, 5 + n * 2 + n * n * 4      # z-neighbours
    assert np.isclose(-D[i, j], 2 * k[i] * k[j] / (k[i] + k[j]), rtol=1e-15)
    # sigma = 0 is the constant Laplacian with diagonal 6
    np.testing.assert_array_equal(w.diffusion3d(4, 0.0).to_dense(), w.poisson3d(4).to_dense())
    # row sums: only boundary faces (ghost value 0) remain
    rs = D.sum(axis=1)
    assert np.all(rs[np.abs(rs) > 1e-12] > 0)


def test_random_spd_dominance_and_shift():
    A = w.random_spd(2000, np.random.default_rng(3))
    D = A.to_dense()
    assert _sym(A)
    off = D - np.diag(np.diag(D))
    assert np.all(off <= 0)
    np.testing.assert_allclose(np.diag(D), np.abs(off).sum(axis=1) + 0.01, rtol=1e-14)
    assert 14 < A.nnz / A.n < 17


def test_random_spd_batch_shapes_and_seed():
    mats, nbs, rhs = w.random_spd_batch(6, seed=2, n_lo=100, n_hi=400)
    mats2, nbs2, _ = w.random_spd_batch(6, seed=2, n_lo=100, n_hi=400)
    assert nbs == nbs2 and all(nb in (8, 16, 32, 64) for nb in nbs)
    for A, B, b in zip(mats, mats2, rhs):
        assert 100 <= A.n <= 400 and len(b) == A.n
        np.testing.assert_array_equal(A.val, B.val)


def test_edge_poisson_unit_conductivity_is_laplacian():
    g = w.edge_graph2d(5)
    assert g.n_params == 2 * 5 * 6
    np.testing.assert_array_equal(w.edge_poisson2d(g, np.ones(g.n_params)).to_dense(),
                                  w.poisson2d(5).to_dense())


def test_powerlaw_degrees():
    A = w.powerlaw_spd(1 << 14, seed=4)
    deg = np.diff(A.row_ptr) - 1
    assert _sym(A) if A.n <= 4096 else True
    assert deg.max() <= 2047
    assert 25 < deg.mean() < 33
    D_row = A.val[A.col_idx == np.repeat(np.arange(A.n), np.diff(A.row_ptr))]
    assert np.all(D_row > 0.1)


def test_rhs_seeded():
    np.testing.assert_array_equal(w.rhs(10, 5), w.rhs(10, 5))
    assert not np.array_equal(w.rhs(10, 5), w.target(10, 5))
