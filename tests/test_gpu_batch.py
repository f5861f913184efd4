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


def _check_systems(orc, B, mats, nbs, rhs, x, info):
    """Every system against its own oracle solve: iteration counts within
    one (x then also compared with the oracle stopped at the GPU's count),
    x within 1e-10 of the oracle's, both true residuals below 1e-10."""
    assert info.status == "OK" and info.systems_ok == len(mats)
    xs = x.cpu().numpy()
    for s, (A, nb, b) in enumerate(zip(mats, nbs, rhs)):
        r0, r1 = B.sys_rows[s], B.sys_rows[s + 1]
        Mo = orc.Precond.uniform(A, nb)
        ref = orc.pcg(A, b, Mo)
        it = int(info.per_system["iterations"][s])
        assert abs(it - ref.iterations) <= 1, (s, it, ref.iterations)
        if it != ref.iterations:
            ref_k = orc.pcg(A, b, Mo, max_iter=it)
            assert np.linalg.norm(xs[r0:r1] - ref_k.x) / np.linalg.norm(ref_k.x) <= 1e-10
        err = np.linalg.norm(xs[r0:r1] - ref.x) / np.linalg.norm(ref.x)
        res = np.linalg.norm(orc.spmv(A, xs[r0:r1]) - b) / np.linalg.norm(b)
        assert err <= 1e-10 and res <= 1e-10, (s, err, res)
        assert abs(info.per_system["rel_res_true"][s] - res) <= 1e-13


@pytest.mark.parametrize("lanes,tile_rows", [(0, 0), (-1, 256), (-1, 2048), (4, 256), (16, 1024), (32, 4096)])
def test_batch_matches_oracle(gpu, orc, lanes, tile_rows):
    mats, nbs, rhs = small_batch()
    B = gpu.Batch.from_systems(mats, nbs, DEV)
    M = gpu.batch_precondition(B)
    x, info = gpu.batch_pcg_solve(B, M, np.concatenate(rhs), lanes=lanes, tile_rows=tile_rows)
    _check_systems(orc, B, mats, nbs, rhs, x, info)


def test_batch_per_system_schedules_match_oracle(gpu, orc):
    """Each system with its own product schedule and tile size (several
    product launches per iteration, one per schedule), graph-replayed, against
    per-system oracle solves; and bitwise equal to a solve in which every
    system's schedule is given batch-wide when all systems share one."""
    mats, nbs, rhs = small_batch(14, seed=12)
    B = gpu.Batch.from_systems(mats, nbs, DEV)
    M = gpu.batch_precondition(B)
    rng = np.random.default_rng(13)
    sys_lanes = rng.choice([-1, 4, 8, 16, 32, 0], size=len(mats))
    sys_tiles = rng.choice([256, 1024, 4096, 0], size=len(mats))
    b = np.concatenate(rhs)
    x, info = gpu.batch_pcg_solve(B, M, b, lanes=8, tile_rows=512, sys_lanes=sys_lanes, sys_tile_rows=sys_tiles)
    _check_systems(orc, B, mats, nbs, rhs, x, info)
    x1, i1 = gpu.batch_pcg_solve(B, M, b, sys_lanes=[16] * len(mats), sys_tile_rows=[1024] * len(mats))
    x2, i2 = gpu.batch_pcg_solve(B, M, b, lanes=16, tile_rows=1024)
    assert torch.equal(x1, x2)
    assert np.array_equal(i1.per_system["iterations"], i2.per_system["iterations"])


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


@pytest.mark.parametrize("where", ["first", "middle", "last"])
@pytest.mark.parametrize("side", ["below", "above"])
def test_batch_rejects_column_just_outside(gpu, where, side):
    """One entry of the middle system moved to the row just before or just
    after that system's rows, at its first, a middle or its last entry (the
    check scans each system's entries in rounds of four, then a tail)."""
    mats, nbs, _ = small_batch(3, seed=7)
    B = gpu.Batch.from_systems(mats, nbs, DEV)
    rp = B.A.row_ptr.cpu().numpy()
    lo, hi = int(B.sys_rows[1]), int(B.sys_rows[2])
    e0, e1 = int(rp[lo]), int(rp[hi])
    k = {"first": e0, "middle": (e0 + e1) // 2, "last": e1 - 1}[where]
    ci = B.A.col_idx.clone()
    ci[k] = lo - 1 if side == "below" else hi
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


def test_batch_autotune_per_class(gpu, orc, tmp_path, monkeypatch):
    """The tuner picks a candidate for every class of systems (block size x
    size x row length), times that assignment on the whole batch against every
    batch-wide schedule, keeps the fastest, caches everything, and the chosen
    schedule solves the batch with oracle parity."""
    from paper_2410_02408_amd import autotune

    monkeypatch.setenv("BJP_CACHE_DIR", str(tmp_path))
    mats, nbs, rhs = w.random_spd_batch(16, seed=9, n_lo=300, n_hi=20000)
    B = gpu.Batch.from_systems(mats, nbs, DEV)
    M = gpu.batch_precondition(B)
    b = np.concatenate(rhs)
    classes = autotune.system_classes(B)
    assert sorted(s for m in classes.values() for s in m) == list(range(len(mats)))
    assert len(classes) >= 3
    kw = dict(probe_iters=8, lanes=(-1, 4, 16), tile_rows=(256, 2048))
    cfg, report = autotune.tune_batch(B, M, b, **kw)
    assert set(report["classes"]) == set(classes)
    for key, members in classes.items():
        r = report["classes"][key]
        assert r["systems"] == len(members) and len(r["us_per_iteration"]) == 6
        assert r["lanes"] in (-1, 4, 16) and r["tile_rows"] in (256, 2048)
    whole = report["whole_batch_us_per_iteration"]
    assert len(whole) == 7 and report["chosen"] == min(whole, key=whole.get)
    if report["chosen"] == "per_class":
        for key, members in classes.items():
            r = report["classes"][key]
            assert all(cfg["sys_lanes"][s] == r["lanes"] and cfg["sys_tile_rows"][s] == r["tile_rows"]
                       for s in members)
    else:
        assert f"{cfg['lanes']},{cfg['tile_rows']}" == report["chosen"]
    cfg2, report2 = autotune.tune_batch(B, M, b, **kw)
    assert cfg2 == cfg and report2["whole_batch_us_per_iteration"] is None
    assert all(r["us_per_iteration"] is None for r in report2["classes"].values())
    x, info = gpu.batch_pcg_solve(B, M, b, **cfg)
    _check_systems(orc, B, mats, nbs, rhs, x, info)


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
