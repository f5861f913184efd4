"""GPU path (C-ABI via the binding) against the CPU oracle, element by element.

Tolerances (derived in the design notes):
  * z = M^-1 r: the GPU multiplies by an explicit inverse, the oracle solves
    with the Cholesky factor; both are backward stable, so the difference is
    O(kappa(A_tt) eps): relative 1e-10 for the FP64 path.
  * PCG: same algorithm and stopping rule on both sides; pass if the
    iteration counts differ by at most one, ||x_gpu - x_or|| / ||x_or|| <= 1e-10
    and the GPU's true residual (recomputed by the oracle) <= tol.
  * kappa: relative difference <= 1e-6 with equal step counts.
"""
import numpy as np
import pytest
import torch

from paper_2410_02408_amd import workloads as w

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def dev(A):
    from paper_2410_02408_amd import bjp

    return bjp.DeviceCsr.from_host(A, DEV)


def diag_pos(G, k, lane):
    """Position of d_k[lane] in a packet: full diagonals in lane-interleaved
    pairs, an unpaired last one as a row, then the half diagonal."""
    K = G // 2
    Kp = K & ~1
    if k < Kp:
        return (k >> 1) * 128 + 2 * lane + (k & 1)
    if k < K or K == 0:
        return Kp * 64 + (k - Kp) * 64 + lane
    return K * 64 + (lane // G) * K + ((lane % G) & (K - 1))


def decode_inverses(M, off):
    """Dense block inverses from the diagonal-packet layout (layout only)."""
    G = M.handle.group
    P = 64 // G
    E = M.handle.packet_elems
    D = M.tiles().double().cpu().numpy()
    out = []
    for t in range(len(off) - 1):
        n = off[t + 1] - off[t]
        pk, g = divmod(t, P)
        base = pk * E
        S = np.zeros((n, n))
        for k in range(max(G // 2, 1)):
            if 2 * k > n:
                continue
            for i in range(n):
                j = (i + k) % n
                S[i, j] = S[j, i] = D[base + diag_pos(G, k, g * G + i)]
        if G > 1 and n == G:
            for i in range(G // 2):
                S[i, i + G // 2] = S[i + G // 2, i] = D[base + diag_pos(G, G // 2, g * G + i)]
        out.append(S)
    return out


CASES = [
    ("poisson2d_32/16", lambda: w.poisson2d(32), 16),
    ("diffusion3d_16/64", lambda: w.diffusion3d(16), 64),
    ("random_spd_1000/64 ragged", lambda: w.random_spd(1000, np.random.default_rng(1)), 64),
    ("random_spd_777/32 ragged", lambda: w.random_spd(777, np.random.default_rng(2)), 32),
    ("random_spd_500/16", lambda: w.random_spd(500, np.random.default_rng(3)), 16),
    ("random_spd_300/8", lambda: w.random_spd(300, np.random.default_rng(4)), 8),
    ("random_spd_301/4", lambda: w.random_spd(301, np.random.default_rng(5)), 4),
    ("random_spd_199/2", lambda: w.random_spd(199, np.random.default_rng(6)), 2),
    ("diffusion3d_8/1", lambda: w.diffusion3d(8), 1),
    ("random_spd_150/24 (pow2 group 32)", lambda: w.random_spd(150, np.random.default_rng(7)), 24),
]


@pytest.mark.parametrize("name,make,nb", CASES, ids=[c[0] for c in CASES])
def test_apply_matches_oracle(gpu, orc, name, make, nb):
    A = make()
    print(f"case {name}", flush=True)
    M = gpu.precondition(dev(A), block_size=nb)
    Mo = orc.Precond.uniform(A, nb)
    r = w.rhs(A.n, 31)
    z = gpu.apply(M, torch.as_tensor(r, device=DEV)).cpu().numpy()
    zo = Mo.apply(r)
    assert np.linalg.norm(z - zo) / np.linalg.norm(zo) <= 1e-10
    np.testing.assert_array_equal(M.offsets(), orc.uniform_offsets(A.n, nb))


@pytest.mark.parametrize("name,make,nb", CASES[:6], ids=[c[0] for c in CASES[:6]])
def test_block_inverses(gpu, orc, name, make, nb):
    A = make()
    M = gpu.precondition(dev(A), block_size=nb)
    off = orc.uniform_offsets(A.n, nb)
    inv = decode_inverses(M, off)
    for t in sorted(set([0, 1, len(off) - 2]) & set(range(len(off) - 1))):
        s, e = off[t], off[t + 1]
        T = orc.extract_block(A, s, e)
        np.testing.assert_allclose(inv[t] @ T, np.eye(e - s), atol=1e-11 * np.linalg.cond(T))


def test_explicit_offsets(gpu, orc):
    A = w.random_spd(400, np.random.default_rng(8))
    off = np.array([0, 5, 64, 70, 100, 133, 197, 250, 251, 300, 364, 400], np.int32)
    M = gpu.precondition(dev(A), offsets=off)
    assert M.handle.group == 64
    r = w.rhs(400, 32)
    z = gpu.apply(M, torch.as_tensor(r, device=DEV)).cpu().numpy()
    zo = orc.Precond(A, off).apply(r)
    assert np.linalg.norm(z - zo) / np.linalg.norm(zo) <= 1e-10
    x, info = gpu.pcg_solve(dev(A), M, r)
    ref = orc.pcg(A, r, orc.Precond(A, off))
    assert info.status == "OK" and abs(info.iterations - ref.iterations) <= 1


def test_apply_fp32_store(gpu, orc):
    A = w.diffusion3d(16)
    M = gpu.precondition(dev(A), block_size=64, precision="fp32")
    assert M.precision == gpu.FP32_STORE
    r = w.rhs(A.n, 33)
    z = gpu.apply(M, torch.as_tensor(r, device=DEV)).cpu().numpy()
    zo = orc.Precond.uniform(A, 64).apply(r)
    assert np.linalg.norm(z - zo) / np.linalg.norm(zo) <= 1e-4


def test_not_spd_reports_block(gpu, orc):
    A = w.random_spd(100, np.random.default_rng(9))
    i = 3 * 16 + 5
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    A.val[np.nonzero((rows == i) & (A.col_idx == i))[0]] = -1.0
    with pytest.raises(gpu.BjpError) as e:
        gpu.precondition(dev(A), block_size=16)
    assert e.value.status == "ENOTSPD" and e.value.failed_block == 3


def test_malformed_csr_rejected(gpu):
    A = w.poisson2d(8)
    bad = w.CsrMatrix(A.n, A.row_ptr.copy(), A.col_idx.copy(), A.val.copy())
    bad.col_idx[7] = 1000
    with pytest.raises(gpu.BjpError) as e:
        gpu.precondition(dev(bad), block_size=8)
    assert e.value.status == "EINVAL"
    with pytest.raises(gpu.BjpError):
        gpu.pcg_solve(dev(bad), None, np.ones(A.n))
    bad = w.CsrMatrix(A.n, A.row_ptr.copy(), A.col_idx.copy(), A.val.copy())
    bad.row_ptr[10] = bad.row_ptr[12]
    with pytest.raises(gpu.BjpError):
        gpu.precondition(dev(bad), block_size=8)
    nan = w.CsrMatrix(A.n, A.row_ptr, A.col_idx, A.val.copy())
    nan.val[3] = np.inf
    with pytest.raises(gpu.BjpError) as e:
        gpu.precondition(dev(nan), block_size=8)
    assert e.value.status == "ENONFINITE"


# Cases whose iteration count may differ from the oracle's by more than one,
# with the bar and the difference observed on the GPU.  Finite-precision CG
# loses orthogonality at a rate set by rounding, so on ill-conditioned
# systems two correct implementations that round differently can take a few
# more or fewer steps (Greenbaum & Strakos 1992); x still agrees to 1e-10.
WIDE_ITERATION_BAR = {
    "diffusion3d_16/none": 8,   # plain CG, kappa(A) ~ 1e4: observed 352 (GPU) vs 359 (oracle)
}


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _pcg_parity(gpu, orc, A, b, nb, tol=1e-10, case=None, **kw):
    """Same algorithm and stopping rule on both sides.  Pass if the iteration
    counts differ by at most one (or the case's listed bar), x agrees with
    the oracle's solution to 1e-10 relative (with the oracle stopped at the
    GPU's count when the counts differ) and both true residuals are below
    tol."""
    Md = gpu.precondition(dev(A), block_size=nb) if nb else None
    Mo = orc.Precond.uniform(A, nb) if nb else None
    x, info = gpu.pcg_solve(dev(A), Md, b, tol=tol, **kw)
    ref = orc.pcg(A, b, Mo, tol=tol)
    xg = x.cpu().numpy()
    true_res = np.linalg.norm(orc.spmv(A, xg) - b) / np.linalg.norm(b)
    err = _rel(xg, ref.x)
    d = info.iterations - ref.iterations
    print(f"  it gpu {info.iterations} oracle {ref.iterations} (delta {d}) err {err:.2e} res {true_res:.2e}",
          flush=True)
    assert info.status == "OK" and ref.status == "OK"
    assert abs(d) <= WIDE_ITERATION_BAR.get(case, 1), (case, info.iterations, ref.iterations)
    if d != 0:
        ref_k = orc.pcg(A, b, Mo, tol=tol, max_iter=info.iterations)
        err_k = _rel(xg, ref_k.x)
        print(f"  oracle stopped at {ref_k.iterations}: err {err_k:.2e}", flush=True)
        assert err_k <= 1e-10
    assert true_res <= tol and info.rel_res_true <= tol
    assert abs(info.rel_res_true - true_res) <= 1e-3 * tol
    assert err <= 1e-10
    return info, ref


def test_pcg_small_workload_exact_count(gpu, orc):
    """2D Poisson 32x32, blocks of 16: iteration count within one of the oracle."""
    W = w.workload("poisson2d_32")
    _pcg_parity(gpu, orc, W.A, W.b, 16)


PCG_CASES = [
    ("poisson2d_32/16", lambda: w.workload("poisson2d_32"), 16),
    ("diffusion3d_16/64", lambda: w.workload("diffusion3d_16"), 64),
    ("diffusion3d_24/64", lambda: w.workload("diffusion3d_24"), 64),
    ("diffusion3d_16/none", lambda: w.workload("diffusion3d_16"), 0),
    ("diffusion3d_16/1", lambda: w.workload("diffusion3d_16"), 1),
    ("diffusion3d_16/8", lambda: w.workload("diffusion3d_16"), 8),
]


@pytest.mark.parametrize("name,make,nb", PCG_CASES, ids=[c[0] for c in PCG_CASES])
def test_pcg_matches_oracle(gpu, orc, name, make, nb):
    print(f"case {name}", flush=True)
    W = make()
    _pcg_parity(gpu, orc, W.A, W.b, nb, case=name)


def test_pcg_random_spd_ragged(gpu, orc):
    A = w.random_spd(5000, np.random.default_rng(10))
    _pcg_parity(gpu, orc, A, w.rhs(A.n, 34), 32, case="random_spd_5000/32")


@pytest.mark.parametrize("lanes", [-1, 1, 2, 4, 8, 16, 32, 64])
def test_pcg_schedules_agree(gpu, orc, lanes):
    """Every SpMV schedule (row-block streaming, every lane-group width)
    gives oracle-parity results."""
    W = w.workload("diffusion3d_16")
    _pcg_parity(gpu, orc, W.A, W.b, 64, case="diffusion3d_16/64", spmv_lanes=lanes)


# spmv_lanes = 0 lets systems of <= 2048 rows take the one-workgroup solver;
# -1 forces the multi-launch solver (row blocks streamed through LDS).  The
# tests run on both use systems of at most 2048 rows (3D: 12^3 = 1728).
BOTH_SOLVERS = pytest.mark.parametrize("lanes", [0, -1], ids=["one-workgroup", "multi-launch"])


@BOTH_SOLVERS
def test_pcg_single_block_one_iteration(gpu, lanes):
    A = w.poisson2d(8)
    b = w.rhs(64, 11)
    x, info = gpu.pcg_solve(dev(A), gpu.precondition(dev(A), block_size=64), b, spmv_lanes=lanes)
    assert info.status == "OK" and info.iterations == 1
    np.testing.assert_allclose(x.cpu().numpy(), np.linalg.solve(A.to_dense(), b), rtol=1e-12)


@BOTH_SOLVERS
@pytest.mark.parametrize("n,nb", [(20, 64), (5, 64), (33, 40)])
def test_block_wider_than_system(gpu, lanes, n, nb):
    """A requested block size above n gives one block spanning A (the group
    sized for n, e.g. 32 lanes for 20 rows): M^-1 = A^-1, so the application
    solves with A, PCG converges in one iteration and kappa(M^-1 A) = 1."""
    A = w.laplacian1d(n)
    Ad = dev(A)
    M = gpu.precondition(Ad, block_size=nb)
    assert M.offsets().tolist() == [0, n]
    dense = A.to_dense()
    r = w.rhs(n, 93)
    z = gpu.apply(M, torch.as_tensor(r, device=DEV))
    np.testing.assert_allclose(z.cpu().numpy(), np.linalg.solve(dense, r), rtol=1e-11, atol=1e-12)
    x, info = gpu.pcg_solve(Ad, M, r, spmv_lanes=lanes)
    assert info.status == "OK" and info.iterations == 1
    np.testing.assert_allclose(x.cpu().numpy(), np.linalg.solve(dense, r), rtol=1e-11, atol=1e-12)
    k = gpu.kappa_estimate(Ad, r, 10, M)
    assert k.status == "OK" and k.steps == 1 and abs(k.kappa - 1) < 1e-12


@BOTH_SOLVERS
@pytest.mark.parametrize("n", [1, 2, 3])
def test_tiny_systems(gpu, orc, lanes, n):
    """Systems of one to three rows (most lanes of the one-workgroup kernels
    idle, a single packet): plain CG and block-Jacobi PCG against a dense
    solve and the oracle's iteration counts, kappa against the eigenvalues."""
    A = w.laplacian1d(n) if n > 1 else w.from_coo(1, [0], [0], [4.0])
    Ad = dev(A)
    dense = A.to_dense()
    b = w.rhs(n, 97)
    xs = np.linalg.solve(dense, b)
    ev = np.linalg.eigvalsh(dense)
    for nb in (0, 1, 2):
        Md = gpu.precondition(Ad, block_size=nb) if nb else None
        Mo = orc.Precond.uniform(A, nb) if nb else None
        x, info = gpu.pcg_solve(Ad, Md, b, spmv_lanes=lanes)
        ref = orc.pcg(A, b, Mo)
        assert info.status == ref.status == "OK" and info.iterations == ref.iterations
        np.testing.assert_allclose(x.cpu().numpy(), xs, rtol=1e-12, atol=1e-14)
    k = gpu.kappa_estimate(Ad, b, 10)
    ko = orc.kappa(A, b, 10)
    assert k.status == ko.status == "OK" and k.steps == ko.steps <= n
    assert abs(k.kappa - ev[-1] / ev[0]) <= 1e-12 * ev[-1] / ev[0]


@BOTH_SOLVERS
def test_pcg_deterministic(gpu, lanes):
    W = w.workload("diffusion3d_12")
    A = dev(W.A)
    M = gpu.precondition(A, block_size=64)
    x1, i1 = gpu.pcg_solve(A, M, W.b, spmv_lanes=lanes)
    x2, i2 = gpu.pcg_solve(A, M, W.b, spmv_lanes=lanes)
    assert i1.iterations == i2.iterations
    assert torch.equal(x1, x2)


@BOTH_SOLVERS
def test_pcg_edge_cases(gpu, lanes):
    A = w.poisson2d(16)
    Ad = dev(A)
    M = gpu.precondition(Ad, block_size=8)
    x, info = gpu.pcg_solve(Ad, M, np.zeros(256), x0=np.ones(256), spmv_lanes=lanes)
    assert info.status == "OK" and info.iterations == 0 and torch.all(x == 0)
    x, info = gpu.pcg_solve(Ad, M, w.rhs(256, 15), max_iter=1, spmv_lanes=lanes)
    assert info.status == "ENOCONV" and info.iterations == 1 and 0 < info.rel_res_true < 1
    b = np.ones(256)
    b[3] = np.nan
    x, info = gpu.pcg_solve(Ad, M, b, spmv_lanes=lanes)
    assert info.status == "ENONFINITE"
    xs = np.linalg.solve(A.to_dense(), w.rhs(256, 16))
    x, info = gpu.pcg_solve(Ad, M, w.rhs(256, 16), x0=xs, spmv_lanes=lanes)
    assert info.status == "OK" and info.iterations == 0


@BOTH_SOLVERS
def test_pcg_indefinite_breakdown(gpu, orc, lanes):
    n = 32
    rows, cols, vals = list(range(n)), list(range(n)), [1.0] * n
    for i in range(0, n, 2):
        j = (i + 17) % n
        rows += [i, j]; cols += [j, i]; vals += [3.0, 3.0]
    A = w.from_coo(n, np.array(rows), np.array(cols), np.array(vals))
    ev, vec = np.linalg.eigh(A.to_dense())
    Ad = dev(A)
    x, info = gpu.pcg_solve(Ad, gpu.precondition(Ad, block_size=8), vec[:, 0], spmv_lanes=lanes)
    assert info.status == "EBREAKDOWN" and info.iterations == 0


@BOTH_SOLVERS
def test_pcg_history_matches_oracle(gpu, orc, lanes):
    W = w.workload("poisson2d_32")
    hist = torch.full((W.A.n + 1,), float("nan"), dtype=torch.float64, device=DEV)
    x, info = gpu.pcg_solve(dev(W.A), gpu.precondition(dev(W.A), block_size=16), W.b, history=hist,
                            spmv_lanes=lanes)
    ref = orc.pcg(W.A, W.b, orc.Precond.uniform(W.A, 16), history=True)
    h = hist[: info.iterations + 1].cpu().numpy()
    k = min(len(h), len(ref.history))
    np.testing.assert_allclose(h[:k], ref.history[:k], rtol=1e-6)


def test_empty_system(gpu):
    from paper_2410_02408_amd import bjp

    A = bjp.DeviceCsr(0, torch.zeros(1, dtype=torch.int32, device=DEV),
                      torch.zeros(0, dtype=torch.int32, device=DEV),
                      torch.zeros(0, dtype=torch.float64, device=DEV))
    x, info = gpu.pcg_solve(A, None, torch.zeros(0, dtype=torch.float64, device=DEV))
    assert info.status == "OK" and x.numel() == 0


# ------------------------------------------------------------------ kappa

def test_kappa_cfg_small(gpu, orc):
    W = w.workload("poisson2d_32")
    A = dev(W.A)
    k = gpu.kappa_estimate(A, W.b, 100)
    ko = orc.kappa(W.A, W.b, 100)
    assert k.status == "OK" and k.steps == ko.steps
    assert abs(k.kappa - ko.kappa) <= 1e-6 * ko.kappa
    assert abs(k.kappa - 1 / np.tan(np.pi / 66) ** 2) <= 1e-6 * k.kappa
    M = gpu.precondition(A, block_size=16)
    k = gpu.kappa_estimate(A, W.b, 100, M)
    ko = orc.kappa(W.A, W.b, 100, orc.Precond.uniform(W.A, 16))
    assert k.steps == ko.steps and abs(k.kappa - ko.kappa) <= 1e-6 * ko.kappa
    assert abs(k.kappa - 234.53060475823) <= 1e-6 * k.kappa
    np.testing.assert_allclose(k.alpha, ko.alpha, rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("nb", [0, 64, 8])
def test_kappa_diffusion(gpu, orc, nb):
    W = w.workload("diffusion3d_16")
    A = dev(W.A)
    M = gpu.precondition(A, block_size=nb) if nb else None
    k = gpu.kappa_estimate(A, W.b, 60, M)
    ko = orc.kappa(W.A, W.b, 60, orc.Precond.uniform(W.A, nb) if nb else None)
    assert k.steps == ko.steps
    assert abs(k.kappa - ko.kappa) <= 1e-6 * ko.kappa


def test_kappa_single_block_and_breakdown(gpu):
    A = w.poisson2d(8)
    Ad = dev(A)
    k = gpu.kappa_estimate(Ad, w.rhs(64, 20), 30, gpu.precondition(Ad, block_size=64))
    assert k.status == "OK" and k.steps == 1 and abs(k.kappa - 1) < 1e-12
    k = gpu.kappa_estimate(Ad, np.zeros(64), 5)
    assert k.status == "EBREAKDOWN"


@pytest.mark.parametrize("n,steps", [(400, 300), (2100, 320)], ids=["one-workgroup", "multi-launch"])
def test_kappa_many_steps_tiles(gpu, orc, n, steps):
    """More than one group of Gram coefficients (j > 256): 400 rows take the
    one-workgroup estimate, 2100 the multi-launch one; equal step counts,
    kappa within 1e-6 and the tridiagonal within 1e-8 of the oracle's."""
    A = w.random_spd(n, np.random.default_rng(11), shift=0.3)
    Ad = dev(A)
    k = gpu.kappa_estimate(Ad, w.rhs(n, 21), steps)
    ko = orc.kappa(A, w.rhs(n, 21), steps)
    assert k.steps == ko.steps == steps
    assert abs(k.kappa - ko.kappa) <= 1e-6 * ko.kappa
    np.testing.assert_allclose(k.alpha, ko.alpha, rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("n,steps", [(1000, 60), (1000, 5000), (3000, 60), (3000, 5000)],
                         ids=["1000 rows, 60 steps (one workgroup)", "1000 rows, 5000 steps (multi-launch)",
                              "3000 rows, 60 steps", "3000 rows, 5000 steps"])
def test_kappa_tridiagonal_extremes(gpu, orc, n, steps):
    """A diagonal matrix with ten evenly spaced eigenvalues 1..10 (each n/10
    times): Lanczos breaks down after ten steps and its Ritz extremes are the
    exact extremes, kappa = 10.  The multisection's results equal the extreme
    eigenvalues of the returned tridiagonal (numpy), with the tridiagonal
    staged in LDS (60 steps) and read from global memory (5000 steps, above
    the staging limit)."""
    vals = np.repeat(np.linspace(1.0, 10.0, 10), n // 10)
    A = w.from_coo(n, np.arange(n), np.arange(n), vals)
    b = w.rhs(n, 95)
    k = gpu.kappa_estimate(dev(A), b, steps)
    ko = orc.kappa(A, b, steps)
    assert k.status == ko.status == "OK" and k.steps == ko.steps == 10
    T = np.diag(k.alpha) + np.diag(k.beta, 1) + np.diag(k.beta, -1)
    ev = np.linalg.eigvalsh(T)
    assert abs(k.theta_min - ev[0]) <= 1e-13 * ev[-1] and abs(k.theta_max - ev[-1]) <= 1e-13 * ev[-1]
    assert abs(k.kappa - 10.0) <= 1e-9 * 10.0
    assert abs(k.kappa - ko.kappa) <= 1e-10 * ko.kappa


KAPPA_SMALL = [("poisson2d_32 fp32-stored", lambda: (w.poisson2d(32), w.rhs(1024, 0)), 16, "fp32", 100),
               ("random_spd_777 explicit blocks", lambda: (w.random_spd(777, np.random.default_rng(81)),
                                                           w.rhs(777, 85)), 0, "explicit", 120),
               ("random_spd_2048/64", lambda: (w.random_spd(2048, np.random.default_rng(79)), w.rhs(2048, 86)),
                64, None, 150),
               ("diffusion3d_12/8", lambda: (w.diffusion3d(12, 1.5, 1), w.rhs(1728, 1)), 8, None, 100),
               ("diffusion3d_12 plain", lambda: (w.diffusion3d(12, 1.5, 1), w.rhs(1728, 1)), 0, None, 100),
               ("random_spd_2048 plain", lambda: (w.random_spd(2048, np.random.default_rng(87), shift=0.2),
                                                  w.rhs(2048, 88)), 0, None, 130)]


@pytest.mark.parametrize("name,make,nb,kind,steps", KAPPA_SMALL, ids=[c[0] for c in KAPPA_SMALL])
def test_kappa_one_workgroup_matches_oracle(gpu, orc, name, make, nb, kind, steps):
    """The one-workgroup estimate (systems of at most 2048 rows) against the
    oracle's CGS2 Lanczos: equal step counts, kappa within 1e-6, the
    tridiagonal within 1e-8."""
    print(f"case {name}", flush=True)
    A, b = make()
    Ad = dev(A)
    if kind == "explicit":
        sizes = np.random.default_rng(83).integers(1, 65, size=A.n)
        off = np.concatenate([[0], np.cumsum(sizes)])
        off = off[off < A.n].tolist() + [A.n]
        Md, Mo = gpu.precondition(Ad, offsets=off), orc.Precond(A, off)
    elif nb:
        Md = gpu.precondition(Ad, block_size=nb, precision="fp32" if kind == "fp32" else "fp64")
        Mo = orc.Precond.uniform(A, nb)
    else:
        Md = Mo = None
    k = gpu.kappa_estimate(Ad, b, steps, Md)
    ko = orc.kappa(A, b, steps, Mo)
    print(f"  gpu {k.kappa:.12g} ({k.steps} steps) oracle {ko.kappa:.12g} ({ko.steps})", flush=True)
    assert k.status == ko.status == "OK" and k.steps == ko.steps
    tol = 1e-5 if kind == "fp32" else 1e-6
    assert abs(k.kappa - ko.kappa) <= tol * ko.kappa
    if kind != "fp32":
        np.testing.assert_allclose(k.alpha, ko.alpha, rtol=1e-8, atol=1e-12)


@BOTH_SOLVERS
def test_pcg_max_iter_iterate_matches_oracle(gpu, orc, lanes):
    """Stopped after 7 iterations (ENOCONV), the returned x is the 7th iterate,
    x update of the last step included, as in the oracle."""
    W = w.workload("diffusion3d_12")
    M = gpu.precondition(dev(W.A), block_size=64)
    ref = orc.pcg(W.A, W.b, orc.Precond.uniform(W.A, 64), max_iter=7)
    for check_every in (1, 2, 16):
        x, info = gpu.pcg_solve(dev(W.A), M, W.b, max_iter=7, check_every=check_every, spmv_lanes=lanes)
        assert info.status == ref.status == "ENOCONV" and info.iterations == ref.iterations == 7
        xg = x.cpu().numpy()
        assert np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x) <= 1e-12
        assert abs(info.rel_res_true - ref.rel_res_true) <= 1e-12 * max(1.0, ref.rel_res_true)


def test_pcg_poll_cadence_does_not_change_result(gpu):
    """Polls only read the state: every poll cadence gives the same iterate
    bits and iteration count."""
    W = w.workload("diffusion3d_16")
    A = dev(W.A)
    M = gpu.precondition(A, block_size=64)
    x0, i0 = gpu.pcg_solve(A, M, W.b, check_every=16)
    for ce in (1, 3, 64):
        x, info = gpu.pcg_solve(A, M, W.b, check_every=ce)
        assert info.iterations == i0.iterations and info.status == "OK"
        assert torch.equal(x, x0)


@BOTH_SOLVERS
def test_pcg_warm_start_matches_oracle(gpu, orc, lanes):
    W = w.workload("diffusion3d_12")
    x0 = np.random.default_rng(21).standard_normal(W.A.n)
    M = gpu.precondition(dev(W.A), block_size=64)
    x, info = gpu.pcg_solve(dev(W.A), M, W.b, x0=x0, spmv_lanes=lanes)
    ref = orc.pcg(W.A, W.b, orc.Precond.uniform(W.A, 64), x0=x0)
    assert info.status == ref.status == "OK"
    print(f"  it gpu {info.iterations} oracle {ref.iterations}", flush=True)
    assert abs(info.iterations - ref.iterations) <= WIDE_ITERATION_BAR.get("diffusion3d_12/64 warm", 1)
    assert np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x) <= 1e-10


@pytest.mark.parametrize("n,hub_deg", [(4000, 3000), (2000, 1500)],
                         ids=["4000 rows (multi-launch)", "2000 rows (one workgroup with the automatic schedule)"])
def test_pcg_streaming_long_and_empty_rows(gpu, orc, n, hub_deg):
    """A row far longer than one LDS stage of the row-block streaming (a hub
    row coupled to most others) and rows with only a diagonal, under the
    streaming schedule and the automatic one (at 2000 rows the one-workgroup
    solver, whose thread takes the hub row alone)."""
    rng = np.random.default_rng(22)
    hub = 1234
    others = np.setdiff1d(rng.choice(n, hub_deg, replace=False), [hub])
    pi = np.concatenate([np.arange(n - 1), np.full(len(others), hub)])     # one entry per pair
    pj = np.concatenate([np.arange(1, n), others])
    keep = (pi < n - 100) & (pj < n - 100)                                  # the last 100 rows: diagonal only
    pi, pj = pi[keep], pj[keep]
    pv = -rng.random(len(pi))
    rows, cols, vals = np.concatenate([pi, pj]), np.concatenate([pj, pi]), np.concatenate([pv, pv])
    diag = np.bincount(rows, weights=np.abs(vals), minlength=n) + 0.5
    A = w.from_coo(n, np.concatenate([rows, np.arange(n)]), np.concatenate([cols, np.arange(n)]),
                   np.concatenate([vals, diag]))
    assert np.diff(A.row_ptr).max() > 1024 + 256 and A.nnz / n < 12
    b = w.rhs(n, 23)
    for lanes in (-1, 0):
        _pcg_parity(gpu, orc, A, b, 16, case=f"hub_{n}/16", spmv_lanes=lanes)


def test_torch_sparse_csr_input(gpu):
    """A torch sparse CSR tensor is accepted wherever a DeviceCsr is."""
    W = w.workload("poisson2d_32")
    A = W.A
    t = torch.sparse_csr_tensor(torch.as_tensor(A.row_ptr, dtype=torch.int64),
                                torch.as_tensor(A.col_idx, dtype=torch.int64),
                                torch.as_tensor(A.val), size=(A.n, A.n)).to(DEV)
    Mt = gpu.precondition(t, block_size=16)
    xt, it_ = gpu.pcg_solve(t, Mt, W.b)
    Md = gpu.precondition(dev(A), block_size=16)
    xd, id_ = gpu.pcg_solve(dev(A), Md, W.b)
    assert it_.iterations == id_.iterations and torch.equal(xt, xd)
    assert gpu.kappa_estimate(t, W.b, 20, M=Mt).kappa == gpu.kappa_estimate(dev(A), W.b, 20, M=Md).kappa


@pytest.mark.parametrize("stride", [1, 4])
def test_kernel_timer_stride(gpu, stride):
    """Every stride-th application is timed; timing leaves the result bitwise
    unchanged."""
    W = w.workload("diffusion3d_20")
    A = dev(W.A)
    M = gpu.precondition(A, block_size=64)
    x0, info0 = gpu.pcg_solve(A, M, W.b, tol=W.tol)
    tm = gpu.KernelTimer(gpu.KERNEL_APPLY, 512, stride=stride)
    x1, info1 = gpu.pcg_solve(A, M, W.b, tol=W.tol, timer=tm)
    assert info1.iterations == info0.iterations and torch.equal(x0, x1)
    n = tm.struct.recorded
    # launches past convergence may be timed too (polls overlap the iterations)
    assert -(-info1.iterations // stride) <= n <= 512
    d = tm.durations_ms()
    assert len(d) == n and all(v > 0 for v in d)


PANEL_CASES = [
    ("powerlaw_16k/32", lambda: w.powerlaw_spd(1 << 14, seed=7), 32, 0),
    ("powerlaw_4100/16", lambda: w.powerlaw_spd(4100, seed=8, max_offdiag=300), 16, 0),
    ("random_spd_9000/none", lambda: w.random_spd(9000, np.random.default_rng(12), pairs_per_row=7.0), 0, 0),
]


@pytest.mark.parametrize("name,make,nb,_", PANEL_CASES, ids=[c[0] for c in PANEL_CASES])
def test_pcg_column_panels(gpu, orc, name, make, nb, _):
    """The column-panel product (forced with spmv_lanes = -2; rows of the
    power-law family, ragged panel widths and scan blocks) gives
    oracle-parity results, the same iteration count as the CSR schedule, and
    bitwise the same result on a second solve."""
    print(f"case {name}", flush=True)
    A = make()
    b = w.rhs(A.n, 41)
    info, _ = _pcg_parity(gpu, orc, A, b, nb, case=name, spmv_lanes=-2)
    x1, info1 = gpu.pcg_solve(dev(A), gpu.precondition(dev(A), block_size=nb) if nb else None, b, spmv_lanes=-2)
    x2, info2 = gpu.pcg_solve(dev(A), gpu.precondition(dev(A), block_size=nb) if nb else None, b, spmv_lanes=-2)
    assert info1.iterations == info2.iterations and torch.equal(x1, x2)
    _, info_csr = gpu.pcg_solve(dev(A), gpu.precondition(dev(A), block_size=nb) if nb else None, b)
    print(f"  csr schedule: {info_csr.iterations} iterations", flush=True)
    assert abs(info_csr.iterations - info.iterations) <= 2 * WIDE_ITERATION_BAR.get(name, 1)


def test_pcg_column_panels_need_long_rows(gpu):
    """Forcing column panels on short rows (3D stencil, 7 per row) is an
    argument error."""
    W = w.workload("diffusion3d_16")
    with pytest.raises(gpu.BjpError):
        gpu.pcg_solve(dev(W.A), None, W.b, spmv_lanes=-2)


SWEEP_CASES = [(n, nb, lanes) for n, nb in [(513, 7), (777, 16), (1000, 33), (2049, 64), (4099, 1)]
               for lanes in (-2, -1, 0, 4, 16)]


@pytest.mark.parametrize("n,nb,lanes", SWEEP_CASES, ids=[f"n{c[0]}-nb{c[1]}-lanes{c[2]}" for c in SWEEP_CASES])
def test_pcg_odd_sizes_every_schedule(gpu, orc, n, nb, lanes):
    """Odd sizes (n not a multiple of the panel count, the scan block or the
    block size; ragged last blocks) under every product schedule, column
    panels included, against the oracle."""
    print(f"case n={n} nb={nb} lanes={lanes}", flush=True)
    A = w.random_spd(n, np.random.default_rng(n + nb), pairs_per_row=7.0)
    _pcg_parity(gpu, orc, A, w.rhs(n, n), nb, case=f"odd_{n}/{nb}", spmv_lanes=lanes)


def test_pcg_short_rows_far_columns(gpu, orc):
    """Short rows whose columns lie far from their row block (random pairs over
    100,000 rows): the 16-bit column offsets do not fit, the product falls back
    to the 32-bit indices, and the solve still matches the oracle."""
    A = w.random_spd(100000, np.random.default_rng(21), pairs_per_row=3.0)
    assert A.nnz < 12 * A.n
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    d = A.col_idx.astype(np.int64) - (rows - rows % 256)
    assert d.max() > 32767 or d.min() < -32768
    _pcg_parity(gpu, orc, A, w.rhs(A.n, 22), 16, case="random_spd_100000/16")


def split_and_shuffle(A, seed):
    """The same operator stored with every entry split into two duplicates
    (u a and (1 - u) a, u in [0.25, 0.75) chosen per unordered pair so A
    stays symmetric) and each row's entries in random order: the CSR the C
    ABI promises to accept (duplicates summed, unsorted columns)."""
    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.row_ptr))
    cols = A.col_idx.astype(np.int64)
    lo, hi = np.minimum(rows, cols), np.maximum(rows, cols)
    u = 0.25 + 0.5 * (((lo * 2654435761 + hi * 40503) % 1000) / 1000.0)
    r2 = np.concatenate([rows, rows])
    c2 = np.concatenate([cols, cols])
    v2 = np.concatenate([A.val * u, A.val * (1.0 - u)])
    order = np.lexsort((np.random.default_rng(seed).random(len(r2)), r2))
    rp = np.zeros(A.n + 1, np.int64)
    rp[1:] = np.cumsum(np.bincount(r2, minlength=A.n))
    return w.CsrMatrix(A.n, rp.astype(np.int32), c2[order].astype(np.int32), v2[order])


DUP_CASES = [("random_spd_3000 dup", lambda: w.random_spd(3000, np.random.default_rng(70), pairs_per_row=7.0),
              32, (-2, -1, 0, 4, 16)),
             ("poisson2d_32 dup", lambda: w.poisson2d(32), 16, (-1, 0, 4, 16))]


@pytest.mark.parametrize("name,make,nb,schedules", DUP_CASES, ids=[c[0] for c in DUP_CASES])
def test_duplicates_and_unsorted_columns(gpu, orc, name, make, nb, schedules):
    """Split duplicate entries and shuffled columns go through validation,
    block extraction and every product schedule (column panels, row-block
    streaming with 16- or 32-bit columns, lane groups) with oracle parity."""
    A = split_and_shuffle(make(), 71)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    key = rows.astype(np.int64) * A.n + A.col_idx
    assert len(np.unique(key)) < len(key)                       # duplicates present
    assert np.any(np.diff(A.col_idx)[np.diff(rows) == 0] < 0)   # unsorted rows present
    M = gpu.precondition(dev(A), block_size=nb)
    r = w.rhs(A.n, 72)
    z = gpu.apply(M, torch.as_tensor(r, device=DEV)).cpu().numpy()
    zo = orc.Precond.uniform(A, nb).apply(r)
    assert _rel(z, zo) <= 1e-10
    b = w.rhs(A.n, 73)
    for lanes in schedules:
        print(f"case {name} lanes={lanes}", flush=True)
        _pcg_parity(gpu, orc, A, b, nb, case=name, spmv_lanes=lanes)


# What the one-workgroup solver keeps in LDS besides its vectors (160 KB in
# all): poisson2d_32/16 the inverse packets and the CSR (FP64 and FP32),
# poisson2d_45/8 the packets only, poisson2d_32 plain CG and the explicit
# blocks the CSR only, the random 2048-row and 2001-row systems and
# diffusion3d_12/64 neither.
SMALL_CASES = [("poisson2d_32/16", lambda: w.workload("poisson2d_32"), 16, None),
               ("poisson2d_45/8 (2025 rows, packets in LDS)", lambda: w.poisson2d(45), 8, None),
               ("random_spd_2048 plain CG", lambda: w.random_spd(2048, np.random.default_rng(79)), 0, None),
               ("diffusion3d_12/64 (1728 rows)", lambda: w.workload("diffusion3d_12"), 64, None),
               ("random_spd_2048/64 (the largest one-workgroup size)", lambda: w.random_spd(2048, np.random.default_rng(79)), 64, None),
               ("random_spd_2001/24 (ragged last block)", lambda: w.random_spd(2001, np.random.default_rng(80)), 24, None),
               ("random_spd_777 explicit blocks", lambda: w.random_spd(777, np.random.default_rng(81)), 0, "explicit"),
               ("poisson2d_32 fp32-stored", lambda: w.workload("poisson2d_32"), 16, "fp32"),
               ("poisson2d_32 plain CG", lambda: w.workload("poisson2d_32"), 0, None)]


@pytest.mark.parametrize("name,make,nb,kind", SMALL_CASES, ids=[c[0] for c in SMALL_CASES])
def test_one_workgroup_solver_matches_oracle(gpu, orc, name, make, nb, kind):
    """Systems of at most 2048 rows (automatic schedule) are solved in one
    workgroup: a single host poll, x within 1e-10 of the oracle's, iteration
    counts within one, and the multi-launch solver on the same system agrees
    with both."""
    print(f"case {name}", flush=True)
    W = make()
    A_h = W.A if hasattr(W, "A") else W
    b = W.b if hasattr(W, "b") else w.rhs(A_h.n, 82)
    Ad = dev(A_h)
    if kind == "explicit":
        rng = np.random.default_rng(83)
        sizes = rng.integers(1, 65, size=A_h.n)
        off = np.concatenate([[0], np.cumsum(sizes)])
        off = off[off < A_h.n].tolist() + [A_h.n]
        Md = gpu.precondition(Ad, offsets=off)
        Mo = orc.Precond(A_h, off)
    elif nb:
        Md = gpu.precondition(Ad, block_size=nb, precision="fp32" if kind == "fp32" else "fp64")
        Mo = orc.Precond.uniform(A_h, nb)
    else:
        Md = Mo = None
    ref = orc.pcg(A_h, b, Mo)
    x, info = gpu.pcg_solve(Ad, Md, b)
    xm, im = gpu.pcg_solve(Ad, Md, b, spmv_lanes=-1)
    print(f"  it one-workgroup {info.iterations} multi-launch {im.iterations} oracle {ref.iterations}", flush=True)
    assert info.status == im.status == ref.status == "OK"
    assert info.polls == 1
    bar = WIDE_ITERATION_BAR.get(name.split(" ")[0], 1)
    assert abs(info.iterations - ref.iterations) <= bar and abs(im.iterations - ref.iterations) <= bar
    for xx in (x, xm):
        assert _rel(xx.cpu().numpy(), ref.x) <= 1e-10
    assert info.rel_res_true <= 1e-10
    true = np.linalg.norm(orc.spmv(A_h, x.cpu().numpy()) - b) / np.linalg.norm(b)
    assert abs(true - info.rel_res_true) <= 1e-13


@pytest.mark.parametrize("nb", [1, 4, 16])
def test_one_workgroup_register_application(gpu, nb):
    """Uniform blocks as wide as their lane group are applied in registers by
    the one-workgroup solver; the same blocks given as explicit offsets go
    through LDS.  Both are the same operations in the same order: equal
    iteration counts, residual histories and solutions, bit for bit (900 rows:
    a ragged last block)."""
    A = w.poisson2d(30)
    b = w.rhs(A.n, 91)
    Ad = dev(A)
    off = list(range(0, A.n, nb)) + [A.n]
    Mu = gpu.precondition(Ad, block_size=nb)
    Me = gpu.precondition(Ad, offsets=off)
    hu = torch.full((A.n + 1,), float("nan"), dtype=torch.float64, device=DEV)
    he = hu.clone()
    xu, iu = gpu.pcg_solve(Ad, Mu, b, history=hu)
    xe, ie = gpu.pcg_solve(Ad, Me, b, history=he)
    assert iu.status == ie.status == "OK" and iu.polls == ie.polls == 1
    assert iu.iterations == ie.iterations
    k = iu.iterations + 1
    assert torch.equal(hu[:k], he[:k])
    assert torch.equal(xu, xe)


def test_one_workgroup_limit(gpu):
    """2049 rows take the multi-launch solver (several polls at a cadence of
    one iteration), 2048 the one-workgroup solver."""
    for n, one in ((2048, True), (2049, False)):
        A = w.random_spd(n, np.random.default_rng(n))
        Ad = dev(A)
        _, info = gpu.pcg_solve(Ad, gpu.precondition(Ad, block_size=16), w.rhs(n, 84), check_every=1)
        assert info.status == "OK" and (info.polls == 1) == one, (n, info)
