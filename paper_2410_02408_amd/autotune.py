"""Autotuner for the batched solver's launch shape.

The batched solver has two free schedule parameters: lanes per CSR row (the
row-bundling of the SpMV: 4, 8, 16 or 32 lanes per row, i.e. 16..2 rows per
wavefront, or -1 for row blocks streamed through LDS) and rows per SpMV tile (the work of one workgroup).  ``tune_batch``
times every candidate on the actual batch for a short, fixed number of PCG
iterations per system (so each candidate does the same work), keeps the
fastest, and caches the choice in a JSON file keyed by the batch's shape
class (system count, mean row length, size range, block sizes).  The cache lives in $BJP_CACHE_DIR or
~/.cache/bjp.
"""
from __future__ import annotations

import itertools
import json
import os
import time

import numpy as np
import torch

from . import bjp

LANES = (-1, 4, 8, 16, 32)
TILE_ROWS = (1024, 2048, 4096)


def _cache_path() -> str:
    d = os.environ.get("BJP_CACHE_DIR", os.path.join(os.path.expanduser("~"), ".cache", "bjp"))
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, "batch_autotune.json")


def shape_key(B: bjp.Batch) -> str:
    n = np.diff(B.sys_rows.astype(np.int64))
    mean_row = B.A.nnz / max(B.A.n, 1)
    return (f"S{B.num_systems}-r{int(round(mean_row))}-n{int(n.min())}:{int(n.max())}"
            f"-nb{'.'.join(str(v) for v in sorted(set(B.block_sizes.tolist())))}")


def tune_batch(B: bjp.Batch, M: bjp.BatchPrecond, b, probe_iters: int = 20, use_cache: bool = True,
               lanes=LANES, tile_rows=TILE_ROWS):
    """Return (config dict, timings) for the fastest candidate."""
    key = shape_key(B)
    path = _cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return cache[key], None
    dev = B.A.device
    b = bjp._vec(b, dev)
    x = torch.empty(B.A.n, dtype=torch.float64, device=dev)
    n = bjp.C.c_size_t()
    bjp._load_batch(bjp.load()).bjp_batch_pcg_workspace(bjp.C.byref(B.A.struct()), bjp.C.byref(B.struct()),
                                                        bjp.C.byref(n))
    ws = bjp._workspace(n.value, dev)
    timings = {}
    for ln, tr in itertools.product(lanes, tile_rows):
        bjp.batch_pcg_solve(B, M, b, tol=1e-300, max_iter=2, lanes=ln, tile_rows=tr, out=x, workspace=ws)
        torch.cuda.synchronize()
        t = time.perf_counter()
        bjp.batch_pcg_solve(B, M, b, tol=1e-300, max_iter=probe_iters, lanes=ln, tile_rows=tr,
                            check_every=probe_iters, out=x, workspace=ws)
        torch.cuda.synchronize()
        timings[(ln, tr)] = time.perf_counter() - t
    best = min(timings, key=timings.get)
    cfg = {"lanes": best[0], "tile_rows": best[1]}
    cache[key] = cfg
    try:
        json.dump(cache, open(path, "w"), indent=1)
    except OSError:
        pass
    return cfg, timings
