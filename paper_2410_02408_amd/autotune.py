"""Autotuner for the batched solver's product schedule, per class of systems.

The batched solver takes a product schedule per system: lanes per CSR row
(the row bundling of the SpMV: 4, 8, 16 or 32 lanes per row, i.e. 16..2 rows
per wavefront, or -1 for row blocks streamed through LDS) and rows per
product tile (the work of one workgroup).  Systems sharing a schedule share a
launch.  ``tune_batch`` groups the batch's systems into classes by block size,
size (rows below 4096, below 16384, above) and mean row length (rounded to a
power of two); for each class it builds a sub-batch of that class's systems
and times every candidate on it (eager launches, the same fixed number of PCG
iterations per system for every candidate, the difference of a long and a
short run so fixed costs cancel), keeps the fastest, and returns per-system
arrays for ``bjp.batch_pcg_solve``.  Systems tuned apart still run together,
and a schedule that wins on one class alone can lose inside the whole batch
(one more product launch per iteration, different co-scheduling), so the
per-class assignment is then timed on the whole batch against every single
batch-wide schedule and kept only if it is the fastest.  Choices are cached in
a JSON file keyed by class (or batch shape), precision and the library's
source digest, in $BJP_CACHE_DIR or ~/.cache/bjp.  Waves per workgroup are
not a separate dimension: every kernel runs four, and a tile of T rows on four
waves gives each wave the rows that a tile of 2T rows would on eight, so the
tile-row candidates already span what the wave count would change (the row
loops and reductions the batch shares with the single-system kernels are
written for four waves).
"""
from __future__ import annotations

import itertools
import json
import os
import time

import numpy as np
import torch

from . import bjp, build

LANES = (-1, 4, 8, 16, 32)
TILE_ROWS = (1024, 2048, 4096)
SIZE_EDGES = (4096, 16384)


def _cache_path() -> str:
    d = os.environ.get("BJP_CACHE_DIR", os.path.join(os.path.expanduser("~"), ".cache", "bjp"))
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, "batch_autotune.json")


def system_classes(B: bjp.Batch) -> dict:
    """Class key -> indices of the systems in that class."""
    n = np.diff(B.sys_rows.astype(np.int64))
    rp = B.A.row_ptr[torch.as_tensor(B.sys_rows.astype(np.int64), device=B.A.device)].cpu().numpy()
    mean_row = np.diff(rp.astype(np.int64)) / np.maximum(n, 1)
    classes = {}
    for s in range(B.num_systems):
        size = int(np.searchsorted(SIZE_EDGES, n[s], side="right"))
        row = int(round(np.log2(max(mean_row[s], 1.0))))
        key = f"nb{int(B.block_sizes[s])}-size{size}-row{1 << row}"
        classes.setdefault(key, []).append(s)
    return classes


def _probe(B, M, b, iters, x, ws, **sched):
    torch.cuda.synchronize()
    t = time.perf_counter()
    bjp.batch_pcg_solve(B, M, b, tol=1e-300, max_iter=iters, check_every=iters, out=x, workspace=ws,
                        graph=False, **sched)
    torch.cuda.synchronize()
    return time.perf_counter() - t


class _Prober:
    """Seconds per PCG iteration of one schedule on one batch: the difference
    of a long and a short run (every system runs exactly that many
    iterations), so the fixed costs of a solve cancel."""

    def __init__(self, B, M, b, probe_iters):
        self.B, self.M, self.b = B, M, b
        self.x = torch.empty(B.A.n, dtype=torch.float64, device=B.A.device)
        n = bjp.C.c_size_t()
        bjp._load_batch(bjp.load()).bjp_batch_pcg_workspace(bjp.C.byref(B.A.struct()), bjp.C.byref(B.struct()),
                                                            bjp.C.byref(n))
        self.ws = bjp._workspace(n.value, B.A.device)
        self.long, self.short = probe_iters, max(2, probe_iters // 4)

    def __call__(self, **sched):
        args = (self.B, self.M, self.b)
        _probe(*args, self.short, self.x, self.ws, **sched)           # warm-up
        dt = _probe(*args, self.long, self.x, self.ws, **sched) - _probe(*args, self.short, self.x, self.ws, **sched)
        return dt / (self.long - self.short)


def _tune_class(sub, Msub, bsub, probe_iters, lanes, tile_rows):
    probe = _Prober(sub, Msub, bsub, probe_iters)
    timings = {(ln, tr): probe(lanes=ln, tile_rows=tr) for ln, tr in itertools.product(lanes, tile_rows)}
    best = min(timings, key=timings.get)
    return {"lanes": best[0], "tile_rows": best[1]}, timings


def shape_key(B: bjp.Batch) -> str:
    n = np.diff(B.sys_rows.astype(np.int64))
    return (f"S{B.num_systems}-n{int(n.sum())}-nnz{B.A.nnz}-{int(n.min())}:{int(n.max())}"
            f"-nb{'.'.join(str(v) for v in sorted(set(B.block_sizes.tolist())))}")


def tune_batch(B: bjp.Batch, M: bjp.BatchPrecond, b, probe_iters: int = 20, use_cache: bool = True,
               lanes=LANES, tile_rows=TILE_ROWS):
    """Return (cfg, report).  cfg holds keyword arguments of
    bjp.batch_pcg_solve: {"sys_lanes": [...], "sys_tile_rows": [...]} when the
    per-class schedules win on the whole batch, else {"lanes": .., "tile_rows":
    ..}.  report = {"classes": {class key: {"systems", "lanes", "tile_rows",
    "us_per_iteration" (the timed candidates)}}, "whole_batch_us_per_iteration":
    {"per_class": .., "lanes,tile_rows": ..}, "chosen": "per_class" | "lanes,tile_rows"};
    the timings are None when a choice came from the cache."""
    precision = "fp32" if M.handle.precision == bjp.FP32_STORE else "fp64"
    tag = f"{precision}-{build.source_digest()}-lanes{'.'.join(map(str, lanes))}-tiles{'.'.join(map(str, tile_rows))}"
    path = _cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    b = bjp._vec(b, B.A.device)
    sys_lanes = np.zeros(B.num_systems, dtype=np.int32)
    sys_tiles = np.zeros(B.num_systems, dtype=np.int32)
    classes = {}
    for key, members in sorted(system_classes(B).items()):
        ck = f"{key}-{tag}"
        timings = None
        if use_cache and ck in cache:
            choice = cache[ck]
        else:
            sub, bsub = B.subset(members, b)
            Msub = bjp.batch_precondition(sub, precision=precision)
            choice, timings = _tune_class(sub, Msub, bsub, probe_iters, lanes, tile_rows)
            cache[ck] = choice
        sys_lanes[members] = choice["lanes"]
        sys_tiles[members] = choice["tile_rows"]
        classes[key] = {"systems": len(members), **choice,
                        "us_per_iteration": None if timings is None else
                        {f"{ln},{tr}": round(1e6 * t, 1) for (ln, tr), t in timings.items()}}
    per_class = {"sys_lanes": sys_lanes.tolist(), "sys_tile_rows": sys_tiles.tolist()}
    # the whole batch: the per-class assignment against every batch-wide schedule
    bk = f"batch-{shape_key(B)}-{tag}"
    whole = None
    if use_cache and bk in cache and cache[bk].get("per_class") == per_class["sys_lanes"] + per_class["sys_tile_rows"]:
        chosen = cache[bk]["chosen"]
    else:
        probe = _Prober(B, M, b, probe_iters)
        whole = {"per_class": probe(**per_class)}
        for ln, tr in itertools.product(lanes, tile_rows):
            whole[f"{ln},{tr}"] = probe(lanes=ln, tile_rows=tr)
        chosen = min(whole, key=whole.get)
        cache[bk] = {"chosen": chosen, "per_class": per_class["sys_lanes"] + per_class["sys_tile_rows"]}
    try:
        json.dump(cache, open(path, "w"), indent=1)
    except OSError:
        pass
    report = {"classes": classes, "chosen": chosen,
              "whole_batch_us_per_iteration": None if whole is None else
              {k: round(1e6 * t, 1) for k, t in whole.items()}}
    if chosen == "per_class":
        return per_class, report
    ln, tr = (int(v) for v in chosen.split(","))
    return {"lanes": ln, "tile_rows": tr}, report
