"""Host-side batch logic on the CPU: the sub-batch copy the autotuner times
its candidates on, and the grouping of systems into tuning classes."""
import numpy as np
import torch

from paper_2410_02408_amd import workloads as w


def test_subset_equals_batch_of_the_selected_systems():
    from paper_2410_02408_amd import bjp

    mats, nbs, rhs = w.random_spd_batch(7, seed=21, n_lo=50, n_hi=400)
    B = bjp.Batch.from_systems(mats, nbs, "cpu")
    b = torch.as_tensor(np.concatenate(rhs))
    pick = [5, 0, 3]
    sub, bsub = B.subset(pick, b)
    ref = bjp.Batch.from_systems([mats[s] for s in pick], [nbs[s] for s in pick], "cpu")
    assert sub.num_systems == 3 and sub.A.n == ref.A.n and sub.A.nnz == ref.A.nnz
    assert np.array_equal(sub.sys_rows, ref.sys_rows) and np.array_equal(sub.block_sizes, ref.block_sizes)
    assert torch.equal(sub.A.row_ptr, ref.A.row_ptr) and torch.equal(sub.A.col_idx, ref.A.col_idx)
    assert torch.equal(sub.A.val, ref.A.val)
    assert torch.equal(bsub, torch.as_tensor(np.concatenate([rhs[s] for s in pick])))


def test_system_classes_partition_the_batch():
    from paper_2410_02408_amd import autotune, bjp

    mats, nbs, _ = w.random_spd_batch(40, seed=22, n_lo=100, n_hi=30000)
    B = bjp.Batch.from_systems(mats, nbs, "cpu")
    cl = autotune.system_classes(B)
    members = sorted(s for m in cl.values() for s in m)
    assert members == list(range(40))
    for key, m in cl.items():
        assert len({int(nbs[s]) for s in m}) == 1 and key.startswith(f"nb{int(nbs[m[0]])}-")
        sizes = {int(np.searchsorted(autotune.SIZE_EDGES, mats[s].n, side="right")) for s in m}
        assert len(sizes) == 1
