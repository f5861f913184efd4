"""The allocation-free solve (bjp_pcg_solve_noalloc, static per-GPU scratch)
against the workspace solve (bjp_pcg_solve) through the C ABI: the same
options give the same iterates, so x must be bitwise equal and the infos
identical; both must also meet the oracle bar (x within 1e-10 of the
oracle's solution, iteration counts within one).  Two calls in a row, the
second on a smaller system, check that nothing left in the shared scratch by
the first call leaks into the second."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2410_02408_amd import workloads as w

DEV = torch.device("cuda:0")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _both(gpu, orc, A_h, b_h, nb, **kw):
    A = gpu.DeviceCsr.from_host(A_h, DEV)
    M = gpu.precondition(A, block_size=nb) if nb else None
    b = torch.as_tensor(b_h, device=DEV)
    x_ref, info_ref = gpu.pcg_solve(A, M, b, **kw)
    x = torch.full((A_h.n,), float("nan"), dtype=torch.float64, device=DEV)
    info = gpu.pcg_solve_noalloc(A, M, b, x, **kw)
    print(f"  noalloc {info.status} {info.iterations} it, workspace solve {info_ref.status} "
          f"{info_ref.iterations} it", flush=True)
    assert info.status == info_ref.status == "OK"
    assert (info.iterations, info.replacements) == (info_ref.iterations, info_ref.replacements)
    assert info.rel_res_true == info_ref.rel_res_true
    assert torch.equal(x, x_ref)
    ref = orc.pcg(A_h, b_h, orc.Precond.uniform(A_h, nb) if nb else None, tol=kw.get("tol", 1e-10))
    assert abs(info.iterations - ref.iterations) <= 1
    assert _rel(x.cpu().numpy(), ref.x) <= 1e-10
    return info


@pytest.mark.gpu
def test_noalloc_matches_workspace_solve_twice(gpu, orc):
    """A 4096-row 3D diffusion system, then the smaller 1024-row 2D Poisson
    system, each matching the workspace solve bit for bit."""
    print("case diffusion3d_16 nb=64", flush=True)
    W = w.workload("diffusion3d_16")
    _both(gpu, orc, W.A, W.b, 64)
    print("case poisson2d_32 nb=16", flush=True)
    W = w.workload("poisson2d_32")
    _both(gpu, orc, W.A, W.b, 16)


@pytest.mark.gpu
def test_noalloc_schedules_and_plain_cg(gpu, orc):
    """Lane-group and streaming schedules, plain CG (M = NULL), a ragged random
    SPD system with long rows, then a smaller one."""
    A = w.random_spd(5000, np.random.default_rng(10))
    for lanes in (0, -1, 4):
        print(f"case random_spd_5000 nb=32 lanes={lanes}", flush=True)
        _both(gpu, orc, A, w.rhs(A.n, 34), 32, spmv_lanes=lanes)
    print("case random_spd_5000 plain CG", flush=True)
    _both(gpu, orc, A, w.rhs(A.n, 35), 0)
    A2 = w.random_spd(700, np.random.default_rng(11))
    print("case random_spd_700 nb=8", flush=True)
    _both(gpu, orc, A2, w.rhs(A2.n, 36), 8)


@pytest.mark.gpu
def test_noalloc_rejects_column_panels(gpu):
    A_h = w.random_spd(5000, np.random.default_rng(10))
    A = gpu.DeviceCsr.from_host(A_h, DEV)
    b = torch.as_tensor(w.rhs(A_h.n, 1), device=DEV)
    x = torch.empty_like(b)
    with pytest.raises(gpu.BjpError) as e:
        gpu.pcg_solve_noalloc(A, None, b, x, spmv_lanes=-2)
    assert e.value.status == "EINVAL"


def test_noalloc_size_limit_without_gpu():
    """Systems beyond the static scratch are refused before any HIP call
    (dummy pointers are never touched); the 128^3 stencil fits."""
    from paper_2410_02408_amd import bjp

    L = bjp.load()
    info = bjp.PcgInfoT()
    cap = bjp.NOALLOC_SCRATCH_BYTES
    for n, nnz in [(2_600_000, 7 * 2_600_000), (3_400_000, 3_400_000), (3_400_000, 40 * 3_400_000)]:
        need = 40 * n + (2 * nnz if nnz < 12 * n else 0)
        assert need > cap
        csr = bjp.CsrT(n, nnz, 1, 1, 1)
        st = L.bjp_pcg_solve_noalloc(C.byref(csr), None, 1, 1, None, C.byref(info), None)
        assert st == -6 and info.status == -6
    assert 40 * 2097152 + 2 * 14581760 + 70000 < cap
