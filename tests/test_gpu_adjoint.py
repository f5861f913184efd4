"""Adjoint (differentiation) path on the GPU against the oracle and against
finite differences of dense solves.

Workload: 2D edge-conductivity Poisson, log-normal(0,1) conductivity per
interior edge and per Dirichlet boundary face, loss L = ||x - x_target||^2,
block size 32; finite differences on the 32x32 instance with step 1e-6 in
FP64 and dense Cholesky forward solves (a PCG forward at 1e-10 would inject
~kappa 1e-10 / h noise into the difference quotient)."""
import numpy as np
import pytest
import scipy.linalg as sl
import torch

from paper_2410_02408_amd import workloads as w

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_value_grad_matches_oracle(gpu, orc):
    A = w.random_spd(3000, np.random.default_rng(40))
    lam, x = w.rhs(A.n, 41), w.rhs(A.n, 42)
    g = gpu.value_grad(gpu.DeviceCsr.from_host(A, DEV), torch.as_tensor(lam, device=DEV),
                       torch.as_tensor(x, device=DEV)).cpu().numpy()
    np.testing.assert_array_equal(g, orc.value_grad(A, lam, x))


def _setup(n):
    g = w.edge_graph2d(n)
    c = w.edge_conductivities(g, seed=3)
    A = w.edge_poisson2d(g, c)
    return g, c, A, w.rhs(g.n_rows, 3), w.target(g.n_rows, 3)


def _fd_edge(g, c, b, xt, e, h):
    """(L(c + h e_e) - L(c - h e_e)) / 2h evaluated without cancellation:
    A(c+h) - A(c-h) = 2h dA_e exactly, so x+ - x- = -2h A(c+h)^-1 dA_e x-, and
    L+ - L- = (x+ - x-) . (x+ + x- - 2 x_target)."""
    cp, cm = c.copy(), c.copy()
    cp[e] += h
    cm[e] -= h
    Ap = w.edge_poisson2d(g, cp).to_dense()
    Am = w.edge_poisson2d(g, cm).to_dense()
    xm = sl.cho_solve(sl.cho_factor(Am), b)
    m = len(g.ei)
    dAx = np.zeros_like(xm)
    if e < m:
        i, j = g.ei[e], g.ej[e]
        dAx[i] += xm[i] - xm[j]
        dAx[j] -= xm[i] - xm[j]
    else:
        i = g.bi[e - m]
        dAx[i] += xm[i]
    dx = -2 * h * sl.cho_solve(sl.cho_factor(Ap), dAx)
    xp = xm + dx
    return dx @ (xp + xm - 2 * xt) / (2 * h)


def _fd_rhs(A, b, xt, i, h):
    D = A.to_dense()
    f = sl.cho_factor(D)
    bm = b.copy()
    bm[i] -= h
    xm = sl.cho_solve(f, bm)
    e = np.zeros_like(b)
    e[i] = 2 * h
    dx = sl.cho_solve(f, e)
    return dx @ (2 * xm + dx - 2 * xt) / (2 * h)


def test_adjoint_gradients_32x32(gpu, orc):
    """GPU forward + adjoint PCG (tol 1e-13) against the dense reference
    gradient (1e-8) and against central differences with step 1e-6 (1e-6)."""
    from paper_2410_02408_amd import autograd as ad

    g, c, A, b, xt = _setup(32)
    pat = ad.Pattern.from_host(A, DEV)
    asm = ad.EdgeAssembly(g, A, DEV)
    ct = torch.as_tensor(c, device=DEV).requires_grad_(True)
    bt = torch.as_tensor(b, device=DEV).requires_grad_(True)
    infos = []
    x = ad.pcg_solve_diff(asm.assemble(ct), bt, pat, 32, tol=1e-13, info_out=infos)
    loss = torch.sum((x - torch.as_tensor(xt, device=DEV)) ** 2)
    loss.backward()
    assert len(infos) == 2 and all(i.status == "OK" for i in infos)
    gc = ct.grad.cpu().numpy()
    gb = bt.grad.cpu().numpy()

    # dense reference gradient
    D = A.to_dense()
    xd = sl.cho_solve(sl.cho_factor(D), b)
    lam = sl.cho_solve(sl.cho_factor(D), 2 * (xd - xt))
    ref_c = orc.edge_grad(g, lam, xd)
    assert np.linalg.norm(gb - lam) / np.linalg.norm(lam) < 1e-8
    assert np.linalg.norm(gc - ref_c) / np.linalg.norm(ref_c) < 1e-8
    assert abs(loss.item() - np.sum((xd - xt) ** 2)) < 1e-9 * loss.item()

    # central finite differences of dense forward solves, step 1e-6
    h = 1e-6
    for e in list(range(0, len(c), 97)) + [len(c) - 1]:
        fd = _fd_edge(g, c, b, xt, e, h)
        assert abs(fd - gc[e]) <= 1e-6 * max(1e-3, abs(fd)), (e, fd, gc[e])
    for i in [0, 100, 1023]:
        fd = _fd_rhs(A, b, xt, i, h)
        assert abs(fd - gb[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, gb[i])


def test_adjoint_value_grad_against_fd_entries(gpu):
    """Gradient w.r.t. raw stored values (entries taken independently)."""
    from paper_2410_02408_amd import autograd as ad

    A = w.random_spd(60, np.random.default_rng(43), shift=1.0)
    b, xt = w.rhs(60, 44), w.target(60, 44)
    pat = ad.Pattern.from_host(A, DEV)
    v = torch.as_tensor(A.val, device=DEV).requires_grad_(True)
    x = ad.pcg_solve_diff(v, torch.as_tensor(b, device=DEV), pat, 8, tol=1e-13)
    torch.sum((x - torch.as_tensor(xt, device=DEV)) ** 2).backward()
    gv = v.grad.cpu().numpy()
    h = 1e-6
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    D = A.to_dense()
    for k in range(0, A.nnz, 37):
        # stored entry k perturbed alone (dA = e_i e_j^T), difference quotient
        # evaluated without cancellation as above
        i, j = rows[k], A.col_idx[k]
        Dm = D.copy()
        Dm[i, j] -= h
        Dp = D.copy()
        Dp[i, j] += h
        xm = np.linalg.solve(Dm, b)
        dAx = np.zeros(60)
        dAx[i] = xm[j]
        dx = -2 * h * np.linalg.solve(Dp, dAx)
        fd = dx @ (2 * xm + dx - 2 * xt) / (2 * h)
        assert abs(fd - gv[k]) <= 1e-6 * max(1e-3, abs(fd)), (k, fd, gv[k])
