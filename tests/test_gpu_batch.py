"""Batched solver (every system advancing in the same launches) against
per-system oracle solves."""
import numpy as np
import pytest
import torch

from paper_2410_02408_amd import workloads as w

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

def small_batch(count=12, seed=5):
    mats, nbs, rhs = w.random_spd_batch(count, seed=seed, n_lo=100, n_hi=3000)
    return mats, nbs, rhs


@pytest.mark.parametrize("lanes,tile_rows", [(0, 0), (-1, 256), (-1, 2048), (4, 256), (16, 1024), (32, 4096)])
def test_batch_matches_oracle(gpu, orc, lanes, tile_rows):
    mats, nbs, rhs = small_batch()
    B = gpu.Batch.from_systems(mats, nbs, DEV)
    M = gpu.batch_precondition(B)
    x, info = gpu.batch_pcg_solve(B, M, np.concatenate(rhs), lanes=lanes, tile_rows=tile_rows)
    assert info.status == "OK" and info.systems_ok == len(mats)
    xs = x.cpu().numpy()
    for s, (A, nb, b) in enumerate(zip(mats, nbs, rhs)):
        r0, r1 = B.sys_rows[s], B.sys_rows[s + 1]
        ref = orc.pcg(A, b, orc.Precond.uniform(A, nb))
        it = int(info.per_system["iterations"][s])
        assert abs(it - ref.iterations) <= max(1, int(np.ceil(0.03 * ref.iterations)))
        err = np.linalg.norm(xs[r0:r1] - ref.x) / np.linalg.norm(ref.x)
        res = np.linalg.norm(orc.spmv(A, xs[r0:r1]) - b) / np.linalg.norm(b)
        assert err <= 1e-10 and res <= 1e-10, (s, err, res)
        assert abs(info.per_system["rel_res_true"][s] - res) <= 1e-13


def test_batch_fp32_store(gpu, orc):
    mats, nbs, rhs = small_batch(6, seed=6)
    B = gpu.Batch.from_systems(mats, nbs, DEV)
    M = gpu.batch_precondition(B, precision="fp32")
    x, info = gpu.batch_pcg_solve(B, M, np.concatenate(rhs))
    assert info.status == "OK"
    xs = x.cpu().numpy()
    for s, (A, nb, b) in enumerate(zip(mats, nbs, rhs)):
        r0, r1 = B.sys_rows[s], B.sys_rows[s + 1]
        res = np.linalg.norm(orc.spmv(A, xs[r0:r1]) - b) / np.linalg.norm(b)
        assert res <= 1e-10


def test_batch_rejects_coupled_systems(gpu):
    mats, nbs, _ = small_batch(3, seed=7)
    B = gpu.Batch.from_systems(mats, nbs, DEV)
    ci = B.A.col_idx.clone()
    ci[5] = int(B.sys_rows[2])            # a row of system 0 pointing into system 2
    bad = gpu.Batch(gpu.DeviceCsr(B.A.n, B.A.row_ptr, ci, B.A.val), B.sys_rows, B.block_sizes)
    with pytest.raises(gpu.BjpError) as e:
        gpu.batch_precondition(bad)
    assert e.value.status == "EINVAL"


def test_batch_not_spd_global_block_index(gpu):
    mats, _, _ = small_batch(3, seed=8)
    nbs = [16, 16, 16]
    A = mats[1]
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    i = 2 * 16 + 3
    A.val[np.nonzero((rows == i) & (A.col_idx == i))[0]] = -5.0
    B = gpu.Batch.from_systems(mats, nbs, DEV)
    with pytest.raises(gpu.BjpError) as e:
        gpu.batch_precondition(B)
    assert e.value.status == "ENOTSPD"
    assert e.value.failed_block == (mats[0].n + 15) // 16 + 2


def test_batch_autotune_picks_a_candidate(gpu, tmp_path, monkeypatch):
    from paper_2410_02408_amd import autotune

    monkeypatch.setenv("BJP_CACHE_DIR", str(tmp_path))
    mats, nbs, rhs = small_batch(8, seed=9)
    B = gpu.Batch.from_systems(mats, nbs, DEV)
    M = gpu.batch_precondition(B)
    cfg, timings = autotune.tune_batch(B, M, np.concatenate(rhs), probe_iters=5,
                                       lanes=(4, 16), tile_rows=(256, 2048))
    assert cfg["lanes"] in (4, 16) and cfg["tile_rows"] in (256, 2048) and len(timings) == 4
    cfg2, t2 = autotune.tune_batch(B, M, np.concatenate(rhs))
    assert cfg2 == cfg and t2 is None
    x, info = gpu.batch_pcg_solve(B, M, np.concatenate(rhs), **cfg)
    assert info.status == "OK"


def test_batch_graph_replays_match_eager(gpu):
    """The captured-graph iterations reproduce the eagerly launched ones bit
    for bit: several replays per solve (polls every 3 iterations, with the
    host reading the states between replays), over two solves in a row."""
    mats, nbs, rhs = small_batch(10, seed=11)
    B = gpu.Batch.from_systems(mats, nbs, DEV)
    M = gpu.batch_precondition(B)
    b = np.concatenate(rhs)
    xe, ie = gpu.batch_pcg_solve(B, M, b, check_every=3, graph=False)
    ws = None
    for _ in range(2):
        xg, ig = gpu.batch_pcg_solve(B, M, b, check_every=3, graph=True, workspace=ws)
        torch.cuda.synchronize()
        assert torch.equal(xg, xe)
        assert np.array_equal(ig.per_system["iterations"], ie.per_system["iterations"])
        assert np.array_equal(ig.per_system["rel_res_true"], ie.per_system["rel_res_true"])
        assert ig.status == ie.status == "OK"
        xe2 = torch.empty_like(xe).copy_(xe)   # eager device work between the solves
        assert torch.equal(xe2, xe)
