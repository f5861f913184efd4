"""Autotuner for the batched solver's launch shape.

The persistent batched launch has three free parameters: lanes per CSR row
(4, 8, 16, 32), workgroup size (256, 512, 1024 threads) and the number of
persistent workgroups.  ``tune_batch`` times every candidate on the actual
batch for a short, fixed number of PCG iterations per system (so each
candidate does the same work), keeps the fastest, and caches the choice in a
JSON file keyed by the batch's shape class (system count, mean row length,
size range, block sizes).  The cache lives in $BJP_CACHE_DIR or
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

LANES = (4, 8, 16, 32)
THREADS = (256, 512, 1024)


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
               lanes=LANES, threads=THREADS, workgroups=(0,)):
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
    for ln, nt, wg in itertools.product(lanes, threads, workgroups):
        bjp.batch_pcg_solve(B, M, b, tol=1e-300, max_iter=2, lanes=ln, threads=nt, workgroups=wg,
                            out=x, workspace=ws)
        torch.cuda.synchronize()
        t = time.perf_counter()
        bjp.batch_pcg_solve(B, M, b, tol=1e-300, max_iter=probe_iters, lanes=ln, threads=nt,
                            workgroups=wg, out=x, workspace=ws)
        torch.cuda.synchronize()
        timings[(ln, nt, wg)] = time.perf_counter() - t
    best = min(timings, key=timings.get)
    cfg = {"lanes": best[0], "threads": best[1], "workgroups": best[2]}
    cache[key] = cfg
    try:
        json.dump(cache, open(path, "w"), indent=1)
    except OSError:
        pass
    return cfg, timings
