"""Host-side parts of bench.py (no GPU): the one-GPU refusal and the
algorithmic byte counts that the roofline figures divide by."""
import importlib.util
import os
import subprocess
import sys

import numpy as np

from paper_2410_02408_amd import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert not r.stdout.strip()            # no JSON line


def test_apply_bytes_count_the_stored_triangles():
    """The packed inverses hold the lower triangle of every block: counted
    here block by block with numpy's triangle indices, on ragged blocks."""
    b = _bench()
    off = np.array([0, 5, 64, 70, 100, 133, 197, 250, 251, 300, 364, 400])
    tri = sum(len(np.tril_indices(e - s)[0]) for s, e in zip(off[:-1], off[1:]))
    for elem in (8, 4):
        assert b.apply_bytes(400, off, elem) == elem * tri + 4 * len(off) + 32 * 400


def test_apply_bytes_headline_workload():
    """128^3 rows in blocks of 64: 32,768 triangles of 2,080 entries, 32,769
    offsets, and the q, r reads and r, z writes."""
    b = _bench()
    n = 128 ** 3
    off = np.arange(0, n + 1, 64)
    assert b.apply_bytes(n, off, 8) == 32768 * 2080 * 8 + 4 * 32769 + 32 * n == 612_499_460


def test_column_offsets_decide_the_product_bytes():
    """Entries cost 10 bytes when every column lies within +-32K of its row's
    256-row block (the 16-bit offsets the product reads), else 12."""
    b = _bench()
    assert b.column_bytes(w.diffusion3d(16)) == 2           # plane neighbours 256 apart
    assert b.column_bytes(w.poisson2d(32)) == 2
    n = 70000
    rows = np.concatenate([np.arange(n), [0, n - 1]])
    cols = np.concatenate([np.arange(n), [n - 1, 0]])
    far = w.from_coo(n, rows, cols, np.ones(len(rows)))
    assert b.column_bytes(far) == 4                         # offset 69,999 does not fit
    rows = np.concatenate([np.arange(n), [300, 40000]])
    cols = np.concatenate([np.arange(n), [256 + 32767, 39936 - 32768]])   # blocks start at 256, 39936
    edge = w.from_coo(n, rows, cols, np.ones(len(rows)))
    assert b.column_bytes(edge) == 2                        # both ends of the 16-bit range
    d = 12 * n                                              # rows of 12 entries: 32-bit columns
    long_rows = w.CsrMatrix(n, np.arange(0, d + 1, 12, dtype=np.int32), np.zeros(d, dtype=np.int32), np.ones(d))
    assert b.column_bytes(long_rows) == 4
    assert b.spmv_bytes(n, d, 4) == 12 * d + 4 * (n + 1) + 16 * n
