"""Seeded synthetic SPD systems in CSR form.

This module only *builds inputs*: sparse symmetric positive-definite matrices,
right-hand sides and targets.  It holds none of the solver's arithmetic (no
block extraction, factorisation, products or iterations), so both the CPU
oracle and the GPU path can take their inputs from here without sharing any
of the method.

The paper generates "sparse, Hermitian, positive-definite matrices" of size N
(Section 4.2; sizes 2^10..2^14 in Section 5.1) but publishes neither the
generator nor the matrices.  The families below stand in for them:

* ``poisson2d`` / ``poisson3d`` / ``laplacian1d`` - constant-coefficient
  Dirichlet Laplacians (closed-form spectra, used as pins);
* ``diffusion3d`` - 7-point variable-coefficient diffusion with log-normal
  cell conductivities and harmonic-mean face coefficients;
* ``random_spd`` / ``random_spd_batch`` - banded + random symmetric
  off-diagonals, diagonally dominant (uneven sizes for batching);
* ``edge_poisson2d`` - 2D graph Laplacian with one conductivity per edge
  (the differentiable workload);
* ``powerlaw_spd`` - Chung-Lu random graph with Pareto degrees.

Conventions: rows are ordered lexicographically with x fastest
(i = x + n*y + n*n*z); CSR uses int32 ``row_ptr``/``col_idx`` and float64
``val``; columns inside a row are sorted ascending; the matrix is stored in
full (both triangles).  Random streams come from
``numpy.random.SeedSequence(seed).spawn(4)`` in the fixed order
[structure/coefficients, values, b, x_target].
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class CsrMatrix:
    """A square sparse matrix in CSR form (int32 indices, float64 values)."""

    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.n > 0 else 0

    def to_dense(self) -> np.ndarray:
        """Dense copy (duplicates summed); for small test matrices only."""
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        np.add.at(d, (rows, self.col_idx), self.val)
        return d

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))


def _streams(seed: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(4)]


def from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CsrMatrix:
    """CSR with rows/cols sorted; duplicate (row, col) pairs are summed."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.argsort(rows * n + cols, kind="stable")
    r, c, v = rows[order], cols[order], vals[order]
    if len(r):
        first = np.empty(len(r), dtype=bool)
        first[0] = True
        np.not_equal(r[1:], r[:-1], out=first[1:])
        first[1:] |= c[1:] != c[:-1]
        start = np.flatnonzero(first)
        if len(start) != len(r):
            r, c, v = r[start], c[start], np.add.reduceat(v, start)
    counts = np.bincount(r, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    return CsrMatrix(n, row_ptr.astype(np.int32), c.astype(np.int32), v)


def _assemble_laplacian(n_rows: int, ei: np.ndarray, ej: np.ndarray, ce: np.ndarray,
                        diag_extra: np.ndarray) -> CsrMatrix:
    """Sum_e c_e (e_i - e_j)(e_i - e_j)^T + diag(diag_extra), as CSR."""
    diag = (np.asarray(diag_extra, dtype=np.float64)
            + np.bincount(ei, weights=ce, minlength=n_rows)
            + np.bincount(ej, weights=ce, minlength=n_rows))
    ar = np.arange(n_rows)
    rows = np.concatenate([ar, ei, ej])
    cols = np.concatenate([ar, ej, ei])
    vals = np.concatenate([diag, -ce, -ce])
    return from_coo(n_rows, rows, cols, vals)


def _grid_csr(shape: tuple[int, ...], face: list, diag_extra: np.ndarray) -> CsrMatrix:
    """Structured assembly of a grid graph Laplacian (+ diagonal) in CSR.

    ``face[a]`` holds the coefficients of the faces normal to axis a (x=0),
    as an array over cells with that axis one shorter, in [z][y][x] layout.
    Entries of a row are emitted in ascending column order.
    """
    dims = len(shape)
    n_rows = int(np.prod(shape))
    rev = shape[::-1]
    strides = [int(np.prod(shape[:a])) for a in range(dims)]
    diag = np.asarray(diag_extra, dtype=np.float64).reshape(rev).copy()
    lower, upper = [], []          # per axis: coefficient to the -a / +a neighbour (0 = none)
    for a in range(dims):
        ax = dims - 1 - a
        lo = np.zeros(rev)
        up = np.zeros(rev)
        sl_lo = [slice(None)] * dims
        sl_hi = [slice(None)] * dims
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        up[tuple(sl_lo)] = face[a]
        lo[tuple(sl_hi)] = face[a]
        diag += lo + up
        lower.append(lo.ravel())
        upper.append(up.ravel())
    ar = np.arange(n_rows, dtype=np.int64)
    cols = []
    vals = []
    present = []
    for a in reversed(range(dims)):
        cols.append(ar - strides[a])
        vals.append(-lower[a])
        present.append(np.zeros(n_rows, dtype=bool))
        present[-1][:] = _has_neighbour(shape, a, -1)
    cols.append(ar)
    vals.append(diag.ravel())
    present.append(np.ones(n_rows, dtype=bool))
    for a in range(dims):
        cols.append(ar + strides[a])
        vals.append(-upper[a])
        present.append(_has_neighbour(shape, a, +1))
    C = np.stack(cols, axis=1)
    V = np.stack(vals, axis=1)
    P = np.stack(present, axis=1)
    counts = P.sum(axis=1)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CsrMatrix(n_rows, row_ptr.astype(np.int32), C[P].astype(np.int32), V[P])


def _has_neighbour(shape, a, sign):
    dims = len(shape)
    rev = shape[::-1]
    coord = np.indices(rev)[dims - 1 - a].ravel() if dims > 1 else np.arange(shape[0])
    return coord > 0 if sign < 0 else coord < shape[a] - 1


def _axis_faces(cell_values: np.ndarray, shape, fn):
    """Per-axis face arrays fn(left_cell, right_cell) over the [z][y][x] grid."""
    dims = len(shape)
    k = cell_values.reshape(shape[::-1])
    out = []
    for a in range(dims):
        ax = dims - 1 - a
        sl_lo = [slice(None)] * dims
        sl_hi = [slice(None)] * dims
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        out.append(fn(k[tuple(sl_lo)], k[tuple(sl_hi)]))
    return out


# --------------------------------------------------------------------------
# constant-coefficient Dirichlet Laplacians
# --------------------------------------------------------------------------

def grid_edges(shape: tuple[int, ...]):
    """Interior edges of a regular grid, x fastest.  Returns (ei, ej, axis)."""
    dims = len(shape)
    idx = np.arange(int(np.prod(shape))).reshape(shape[::-1])  # [z][y][x]
    ei, ej, ax = [], [], []
    for a in range(dims):
        sl_lo = [slice(None)] * dims
        sl_hi = [slice(None)] * dims
        sl_lo[dims - 1 - a] = slice(0, -1)
        sl_hi[dims - 1 - a] = slice(1, None)
        lo = idx[tuple(sl_lo)].ravel()
        hi = idx[tuple(sl_hi)].ravel()
        ei.append(lo)
        ej.append(hi)
        ax.append(np.full(lo.shape, a))
    return np.concatenate(ei), np.concatenate(ej), np.concatenate(ax)


def boundary_faces(shape: tuple[int, ...]):
    """Cells touching the Dirichlet boundary, one entry per boundary face."""
    dims = len(shape)
    idx = np.arange(int(np.prod(shape))).reshape(shape[::-1])
    out = []
    for a in range(dims):
        for end in (0, -1):
            sl = [slice(None)] * dims
            sl[dims - 1 - a] = end
            out.append(idx[tuple(sl)].ravel())
    return np.concatenate(out)


def dirichlet_laplacian(shape: tuple[int, ...]) -> CsrMatrix:
    """tridiag(-1, 2, -1) Kronecker sum on a grid (diagonal 2*dims)."""
    n_rows = int(np.prod(shape))
    extra = np.bincount(boundary_faces(shape), minlength=n_rows).astype(np.float64)
    faces = _axis_faces(np.ones(n_rows), shape, lambda a, b: np.ones_like(a))
    return _grid_csr(tuple(shape), faces, extra)


def laplacian1d(n: int) -> CsrMatrix:
    return dirichlet_laplacian((n,))


def poisson2d(n: int) -> CsrMatrix:
    """2D 5-point Dirichlet Poisson on an n x n grid (diagonal 4, off -1)."""
    return dirichlet_laplacian((n, n))


def poisson3d(n: int) -> CsrMatrix:
    return dirichlet_laplacian((n, n, n))


# --------------------------------------------------------------------------
# 3D variable-coefficient diffusion
# --------------------------------------------------------------------------

def diffusion3d(n: int, sigma: float = 1.5, seed: int = 1) -> CsrMatrix:
    """7-point diffusion on n^3 cells.

    Cell conductivity k = exp(sigma * xi), xi ~ N(0, 1) i.i.d.; an interior
    face between cells i, j has coefficient 2 k_i k_j / (k_i + k_j) (harmonic
    mean); a boundary face couples the cell to a zero ghost value with
    coefficient k_i.  A_ii = sum of the cell's six face coefficients,
    A_ij = -c_ij.  sigma = 0 gives the constant Laplacian (diagonal 6).
    """
    rng = _streams(seed)[0]
    n_rows = n ** 3
    k = np.exp(sigma * rng.standard_normal(n_rows))
    faces = _axis_faces(k, (n, n, n), lambda a, b: 2.0 * a * b / (a + b))
    bf = boundary_faces((n, n, n))
    extra = np.bincount(bf, weights=k[bf], minlength=n_rows)
    return _grid_csr((n, n, n), faces, extra)


# --------------------------------------------------------------------------
# 2D edge-conductivity Poisson (differentiable workload)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class EdgeGraph:
    """Edges of the 2D grid: interior (ei, ej) and boundary cells (bi)."""

    n_rows: int
    ei: np.ndarray
    ej: np.ndarray
    bi: np.ndarray

    @property
    def n_params(self) -> int:
        return len(self.ei) + len(self.bi)


def edge_graph2d(n: int) -> EdgeGraph:
    ei, ej, _ = grid_edges((n, n))
    return EdgeGraph(n * n, ei.astype(np.int32), ej.astype(np.int32),
                     boundary_faces((n, n)).astype(np.int32))


def edge_conductivities(graph: EdgeGraph, seed: int = 3, sigma: float = 1.0) -> np.ndarray:
    """log-normal(0, sigma) per parameter: interior edges first, then boundary."""
    rng = _streams(seed)[0]
    return np.exp(sigma * rng.standard_normal(graph.n_params))


def edge_poisson2d(graph: EdgeGraph, c: np.ndarray) -> CsrMatrix:
    """A = sum_e c_e (e_i - e_j)(e_i - e_j)^T + sum_bdry c_b e_i e_i^T."""
    m = len(graph.ei)
    extra = np.bincount(graph.bi, weights=np.asarray(c[m:], float), minlength=graph.n_rows)
    return _assemble_laplacian(graph.n_rows, graph.ei, graph.ej, np.asarray(c[:m], float), extra)


# --------------------------------------------------------------------------
# random diagonally dominant SPD systems
# --------------------------------------------------------------------------

def _dominant_from_pairs(n: int, pi: np.ndarray, pj: np.ndarray, w: np.ndarray,
                         shift: float) -> CsrMatrix:
    """Off-diagonals a_ij = a_ji = w (w <= 0), a_ii = sum_j |a_ij| + shift."""
    diag = (shift + np.bincount(pi, weights=np.abs(w), minlength=n)
            + np.bincount(pj, weights=np.abs(w), minlength=n))
    ar = np.arange(n)
    return from_coo(n, np.concatenate([ar, pi, pj]), np.concatenate([ar, pj, pi]),
                    np.concatenate([diag, w, w]))


def _dedup_pairs(n: int, a: np.ndarray, b: np.ndarray):
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = np.unique(lo.astype(np.int64) * n + hi)
    return (key // n).astype(np.int64), (key % n).astype(np.int64)


def random_spd(n: int, rng: np.random.Generator, shift: float = 0.01,
               pairs_per_row: float = 6.5) -> CsrMatrix:
    """Tridiagonal band + round(pairs_per_row*n) random symmetric pairs.

    Band values a_{i,i+1} ~ U(-1, 0); random unordered pairs (i < j,
    j - i >= 2) with uniform endpoints, deduplicated, values U(-1, 0);
    a_ii = sum_j |a_ij| + shift, so A 1 = shift 1 exactly.
    """
    band_i = np.arange(n - 1)
    m = int(round(pairs_per_row * n))
    a = rng.integers(0, n, size=m)
    b = rng.integers(0, n, size=m)
    keep = np.abs(a - b) >= 2
    pi, pj = _dedup_pairs(n, a[keep], b[keep])
    wb = -rng.random(n - 1)
    wr = -rng.random(len(pi))
    return _dominant_from_pairs(n, np.concatenate([band_i, pi]), np.concatenate([band_i + 1, pj]),
                                np.concatenate([wb, wr]), shift)


def random_spd_batch(count: int = 512, seed: int = 2, n_lo: int = 1000, n_hi: int = 64000,
                     block_sizes=(8, 16, 32, 64)):
    """``count`` independent systems of uneven size and block size.

    Returns (matrices, block_size_per_system, rhs_per_system).
    """
    s_struct, s_vals, s_b, _ = _streams(seed)
    sizes = s_struct.integers(n_lo, n_hi + 1, size=count)
    nbs = s_struct.choice(np.asarray(block_sizes), size=count)
    mats, rhs = [], []
    for k in range(count):
        mats.append(random_spd(int(sizes[k]), s_vals))
        rhs.append(s_b.standard_normal(int(sizes[k])))
    return mats, [int(v) for v in nbs], rhs


def _inverse_cdf(cdf: np.ndarray, u: np.ndarray) -> np.ndarray:
    """searchsorted(cdf, u, side="right"), evaluated on the sorted draws (the
    same indices, without a cache miss per draw)."""
    o = np.argsort(u)
    idx = np.empty(len(u), dtype=np.int64)
    idx[o] = np.searchsorted(cdf, u[o], side="right")
    return idx


def powerlaw_spd(n: int = 1 << 22, seed: int = 4, mean_offdiag: float = 31.0,
                 alpha: float = 2.1, max_offdiag: int = 2047, shift: float = 0.1) -> CsrMatrix:
    """Chung-Lu graph with Pareto(alpha) target degrees, as an SPD matrix.

    Target off-diagonal degree w_i = min(x_m P_i, max_offdiag) with P_i a
    classical Pareto(alpha) draw (P >= 1) and x_m chosen so mean(w) equals
    ``mean_offdiag``.  round(n * mean_offdiag / 2) endpoint pairs are drawn
    with probability proportional to w; self-loops are dropped, duplicates
    merged, and rows left above ``max_offdiag`` lose random incident edges.
    Values U(-1, 0) per pair; a_ii = sum_j |a_ij| + shift.  Node labels are
    a random permutation, so degree is uncorrelated with the row index.
    """
    s_struct, s_vals, _, _ = _streams(seed)
    p = (1.0 - s_struct.random(n)) ** (-1.0 / alpha)
    lo, hi = 0.0, float(mean_offdiag)
    while np.mean(np.minimum(hi * p, max_offdiag)) < mean_offdiag:
        hi *= 2.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if np.mean(np.minimum(mid * p, max_offdiag)) < mean_offdiag:
            lo = mid
        else:
            hi = mid
    w = np.minimum(hi * p, max_offdiag)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m = int(round(n * mean_offdiag / 2))
    a = np.minimum(_inverse_cdf(cdf, s_struct.random(m)), n - 1)
    b = np.minimum(_inverse_cdf(cdf, s_struct.random(m)), n - 1)
    keep = a != b
    pi, pj = _dedup_pairs(n, a[keep], b[keep])
    # trim rows whose realised off-diagonal degree exceeds the cap
    deg = np.bincount(pi, minlength=n) + np.bincount(pj, minlength=n)
    if deg.max() > max_offdiag:
        # rows in increasing order; each drops its first incident pairs (in a
        # random order of all pairs) that are still present until it is at
        # the cap.  Only pairs touching an over-cap row can be dropped, so the
        # scan runs over those alone.
        alive = np.ones(len(pi), dtype=bool)
        order = s_struct.permutation(len(pi))
        over = deg > max_offdiag
        cand = order[over[pi[order]] | over[pj[order]]]
        ci, cj = pi[cand], pj[cand]
        for r in np.nonzero(over)[0]:
            inc = cand[(ci == r) | (cj == r)]
            inc = inc[alive[inc]]
            excess = len(inc) - max_offdiag
            if excess > 0:
                alive[inc[:excess]] = False
        pi, pj = pi[alive], pj[alive]
    perm = s_struct.permutation(n)
    pi, pj = perm[pi], perm[pj]
    wv = -s_vals.random(len(pi))
    return _dominant_from_pairs(n, pi, pj, wv, shift)


# --------------------------------------------------------------------------
# vectors and named workloads
# --------------------------------------------------------------------------

def rhs(n: int, seed: int) -> np.ndarray:
    """b ~ N(0, 1) from the seed's third stream."""
    return _streams(seed)[2].standard_normal(n)


def target(n: int, seed: int) -> np.ndarray:
    """x_target ~ N(0, 1) from the seed's fourth stream."""
    return _streams(seed)[3].standard_normal(n)


@dataclasses.dataclass
class Workload:
    name: str
    A: CsrMatrix
    b: np.ndarray
    block_size: int
    tol: float
    lanczos_steps: int


def workload(name: str) -> Workload:
    """Named single-system workloads.

    ``poisson2d_32``   2D 5-point Poisson 32x32 (N=1024), blocks of 16, seed 0,
                       100 Lanczos steps.
    ``diffusion3d_128`` 3D 7-point log-normal(sigma=1.5) diffusion on 128^3
                       (N=2,097,152), blocks of 64, seed 1, 200 Lanczos steps.
    ``diffusion3d_<n>`` the same family at n^3 (smaller test sizes).
    """
    if name == "poisson2d_32":
        return Workload(name, poisson2d(32), rhs(1024, 0), 16, 1e-10, 100)
    if name.startswith("diffusion3d_"):
        n = int(name.split("_")[1])
        return Workload(name, diffusion3d(n, 1.5, 1), rhs(n ** 3, 1), 64, 1e-10, 200)
    raise KeyError(name)
