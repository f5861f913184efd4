"""Control paths of the GPU solver against the oracle: residual replacement
(Section 3.7's true-residual check, forced by tolerances below what the
recursion alone can certify), the replacement budget, a replacement that
falls due at max_iter, partitions whose block size exceeds n, and the start
without a guess (r = b) against a start from x0 = 0."""
import numpy as np
import pytest
import torch

from paper_2410_02408_amd import workloads as w

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def dev(A):
    from paper_2410_02408_amd import bjp

    return bjp.DeviceCsr.from_host(A, DEV)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# spmv_lanes = 0: the one-workgroup solver (these systems have 1024 rows); -1: the multi-launch solver
BOTH_SOLVERS = pytest.mark.parametrize("lanes", [0, -1], ids=["one-workgroup", "multi-launch"])


@BOTH_SOLVERS
@pytest.mark.parametrize("nb", [16, 0])
def test_replacement_budget_matches_oracle(gpu, orc, nb, lanes):
    """tol 1e-16 (below the rounding floor of b - A x): every true-residual
    check fails, so both sides end ENOCONV after exactly max_replacements
    restarts.  Runs with budgets 0..3 give the length of every leg between
    restarts; each leg is within one iteration of the oracle's, and each
    iterate agrees with the oracle's at the same budget."""
    W = w.workload("poisson2d_32")
    A = dev(W.A)
    Md = gpu.precondition(A, block_size=nb) if nb else None
    Mo = orc.Precond.uniform(W.A, nb) if nb else None
    prev_g = prev_o = 0
    for m in range(4):
        print(f"case nb={nb} max_replacements={m}", flush=True)
        x, info = gpu.pcg_solve(A, Md, W.b, tol=1e-16, max_replacements=m if m else 0, spmv_lanes=lanes)
        ref = orc.pcg(W.A, W.b, Mo, tol=1e-16, max_replacements=m)
        assert ref.status == "ENOCONV" and ref.replacements == m
        assert info.status == "ENOCONV" and info.replacements == m, info
        leg_g, leg_o = info.iterations - prev_g, ref.iterations - prev_o
        print(f"  leg {m}: gpu {leg_g} oracle {leg_o}", flush=True)
        assert abs(leg_g - leg_o) <= 1
        prev_g, prev_o = info.iterations, ref.iterations
        xg = x.cpu().numpy()
        assert _rel(xg, ref.x) <= 1e-10
        assert info.rel_res_true > 1e-16


@BOTH_SOLVERS
def test_replacement_converges_matches_oracle(gpu, orc, lanes):
    """tol 1e-14: the recursion meets tol before b - A x does; one
    replacement later both sides converge, with x equal to the oracle's."""
    W = w.workload("poisson2d_32")
    A = dev(W.A)
    x, info = gpu.pcg_solve(A, gpu.precondition(A, block_size=16), W.b, tol=1e-14, spmv_lanes=lanes)
    ref = orc.pcg(W.A, W.b, orc.Precond.uniform(W.A, 16), tol=1e-14)
    assert ref.status == "OK" and ref.replacements == 1
    assert info.status == "OK" and info.replacements == ref.replacements
    assert abs(info.iterations - ref.iterations) <= 1
    xg = x.cpu().numpy()
    assert _rel(xg, ref.x) <= 1e-10
    true = np.linalg.norm(orc.spmv(W.A, xg) - W.b) / np.linalg.norm(W.b)
    assert info.rel_res_true <= 1e-14 and true <= 1.1e-14


@BOTH_SOLVERS
@pytest.mark.parametrize("nb", [16, 0])
def test_no_replacement_at_max_iter(gpu, orc, nb, lanes):
    """The recursion meets tol at exactly max_iter while b - A x does not: no
    iteration is left for a restart, so the solve ends ENOCONV at max_iter
    with no replacement, and the residual history (max_iter + 1 entries) is
    written no further than its end."""
    W = w.workload("poisson2d_32")
    A = dev(W.A)
    Md = gpu.precondition(A, block_size=nb) if nb else None
    Mo = orc.Precond.uniform(W.A, nb) if nb else None
    tol = 1e-14 if nb else 1e-15
    _, first = gpu.pcg_solve(A, Md, W.b, tol=tol, max_replacements=0, spmv_lanes=lanes)
    assert first.status == "ENOCONV" and first.replacements == 0
    k1 = first.iterations
    guard = 64
    hist = torch.full((k1 + 1 + guard,), float("nan"), dtype=torch.float64, device=DEV)
    for ce in (1, 16):
        hist.fill_(float("nan"))
        x, info = gpu.pcg_solve(A, Md, W.b, tol=tol, max_iter=k1, check_every=ce, history=hist, spmv_lanes=lanes)
        assert info.status == "ENOCONV" and info.iterations == k1 and info.replacements == 0, info
        h = hist.cpu().numpy()
        assert np.all(np.isfinite(h[: k1 + 1])) and np.all(np.isnan(h[k1 + 1:]))
        ref = orc.pcg(W.A, W.b, Mo, tol=tol, max_iter=k1)
        assert ref.status == "ENOCONV" and ref.replacements == 0
        assert _rel(x.cpu().numpy(), ref.x) <= 1e-10
    # one iteration more: the replacement happens and the solve continues
    x, info = gpu.pcg_solve(A, Md, W.b, tol=tol, max_iter=k1 + 1, spmv_lanes=lanes)
    assert info.replacements == 1 and info.iterations == k1 + 1


@pytest.mark.parametrize("n,nb", [(20, 64), (20, 40), (50, 64), (64, 64), (37, 37), (5, 8)])
def test_block_larger_than_system(gpu, orc, n, nb):
    """A block size at or above n gives one block spanning A: M^-1 A = I, so
    kappa(M^-1 A) = 1, PCG finishes in one iteration with x = A^-1 b, and
    every entry point accepts the handle."""
    A = w.random_spd(n, np.random.default_rng(n + nb), shift=0.5)
    Ad = dev(A)
    M = gpu.precondition(Ad, block_size=nb)
    assert M.num_blocks == 1
    b = w.rhs(n, 60)
    z = gpu.apply(M, torch.as_tensor(b, device=DEV)).cpu().numpy()
    xs = np.linalg.solve(A.to_dense(), b)
    assert _rel(z, xs) <= 1e-12
    x, info = gpu.pcg_solve(Ad, M, b)
    ref = orc.pcg(A, b, orc.Precond.uniform(A, nb))
    assert info.status == ref.status == "OK" and info.iterations == ref.iterations == 1
    assert _rel(x.cpu().numpy(), xs) <= 1e-12
    k = gpu.kappa_estimate(Ad, b, 10, M)
    ko = orc.kappa(A, b, 10, orc.Precond.uniform(A, nb))
    assert k.status == "OK" and k.steps == ko.steps == 1
    assert abs(k.kappa - 1.0) <= 1e-6 and abs(ko.kappa - 1.0) <= 1e-6


@pytest.mark.parametrize("lanes", [-1, 4, -2], ids=["row-blocks", "lane-groups", "column-panels"])
def test_zero_start_matches_zero_guess(gpu, orc, lanes):
    """Without a starting guess the solve begins with r = b (no product); given
    x0 = 0 it forms r = b - A x0 with the residual product of its schedule.
    The two are the same iteration up to the order of the b^T b sum: the same
    iteration count, solutions within rounding of each other and within the
    parity bar of the oracle's."""
    n = 5000
    A_h = w.random_spd(n, np.random.default_rng(21))
    b = w.rhs(n, 22)
    A = dev(A_h)
    M = gpu.precondition(A, block_size=32)
    x1, i1 = gpu.pcg_solve(A, M, b, spmv_lanes=lanes)
    x2, i2 = gpu.pcg_solve(A, M, b, x0=np.zeros(n), spmv_lanes=lanes)
    ref = orc.pcg(A_h, b, orc.Precond.uniform(A_h, 32))
    assert i1.status == i2.status == "OK"
    assert i1.iterations == i2.iterations and abs(i1.iterations - ref.iterations) <= 1
    x1, x2 = x1.cpu().numpy(), x2.cpu().numpy()
    assert _rel(x1, x2) <= 1e-12
    assert _rel(x1, ref.x) <= 1e-10
