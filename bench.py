"""Benchmark: block-Jacobi PCG + Lanczos kappa on one MI355X.

One step = the whole hot path over one synthetic system already resident in
HBM: CSR validation and block extraction + batched Cholesky inversion
(bjp_precondition), PCG to a 1e-10 relative residual (bjp_pcg_solve), and the
Lanczos estimates kappa(A) and kappa(M^-1 A) (bjp_kappa_estimate, twice).

Headline value: PCG iterations per second over the timed solves.  The line
also carries the roofline of the dominant kernel (the block-inverse
application, timed live with HIP events around each of its launches) and the
CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload diffusion3d_128]
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
TIMER_STRIDE = 8       # every 8th block-inverse application is timed with events


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diffusion3d_128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--kappa-steps", type=int, default=0, help="override Lanczos steps (0 = workload's)")
    ap.add_argument("--mode", default="headline",
                    choices=["headline", "nb_sweep", "batch", "adjoint", "precision"],
                    help="headline: the metric's line; the others measure the extensions")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    return ap.parse_args()


def apply_bytes(n: int, offsets, elem: int) -> int:
    """Algorithmic bytes of one block-apply launch inside PCG: the packed
    block inverses (sum_t n_t(n_t+1)/2 scalars), the block offsets, and the
    vectors q, r read (16 N) and r, z written (16 N)."""
    import numpy as np

    nt = np.diff(np.asarray(offsets, dtype=np.int64))
    return int(elem * np.sum(nt * (nt + 1) // 2) + 4 * len(offsets) + 32 * n)


def spmv_bytes(n: int, nnz: int, col_bytes: int = 4) -> int:
    """Algorithmic bytes of one SpMV launch: CSR ((8 + col_bytes) nnz +
    4(N+1)), p read (8 N), q written (8 N).  col_bytes is 2 when the product
    reads 16-bit column offsets (short rows whose columns all lie within
    +-32K of their 256-row block), else 4."""
    return (8 + col_bytes) * nnz + 4 * (n + 1) + 16 * n


def column_bytes(A) -> int:
    """Bytes per column index the iteration's product reads for A."""
    import numpy as np

    if A.n == 0 or A.nnz >= 12 * A.n:
        return 4
    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.row_ptr))
    d = A.col_idx.astype(np.int64) - (rows - rows % 256)
    return 2 if d.min() >= -32768 and d.max() <= 32767 else 4


def direction_bytes(n: int) -> int:
    """Algorithmic bytes of one direction update: x, p_old, z read (24 N),
    x, p_new written (16 N)."""
    return 40 * n


def read_traffic(kernel_tag: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_sha256:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t:
        return None
    from paper_2410_02408_amd import build

    if m.group(1) != build.source_digest():
        return None
    return float(t.group(1))


def _timed(fn):
    import torch

    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    out = fn()
    e1.record()
    torch.cuda.synchronize()
    return out, e0.elapsed_time(e1)


def mode_nb_sweep(args):
    """kappa(M^-1 A), PCG iterations and time per block size (the paper's
    block-size question, answered by measurement; n_b = 1 is its point Jacobi)."""
    import numpy as np
    import torch

    from paper_2410_02408_amd import bjp, workloads

    W = workloads.workload(args.workload)
    steps = args.kappa_steps or W.lanczos_steps
    dev = torch.device("cuda:0")
    A = bjp.DeviceCsr.from_host(W.A, dev)
    b = torch.as_tensor(W.b, device=dev)
    ws = bjp.PcgWorkspace(A)
    kws = bjp.KappaWorkspace(A, steps)
    kA = bjp.kappa_estimate(A, b, steps, None, workspace=kws)
    for nb in (1, 8, 16, 32, 64):
        M, setup_ms = _timed(lambda: bjp.precondition(A, block_size=nb, precision=args.precision))
        bjp.pcg_solve(A, M, b, tol=W.tol, workspace=ws)
        (x, info), ms = _timed(lambda: bjp.pcg_solve(A, M, b, tol=W.tol, workspace=ws))
        k = bjp.kappa_estimate(A, b, steps, M, workspace=kws)
        print(json.dumps({"mode": "nb_sweep", "workload": args.workload, "block_size": nb,
                          "precision": args.precision, "kappa_A": kA.kappa, "kappa_MA": k.kappa,
                          "lanczos_steps": steps, "pcg_iterations": info.iterations,
                          "pcg_ms": round(ms, 3), "us_per_iteration": round(1e3 * ms / info.iterations, 2),
                          "setup_ms": round(setup_ms, 3), "rel_res_true": info.rel_res_true,
                          "status": info.status}), flush=True)


def mode_batch(args):
    """512 uneven random SPD systems solved together (every system advancing in
    the same tile launches, iterations replayed from a captured hipGraph)."""
    import numpy as np
    import torch

    from paper_2410_02408_amd import autotune, bjp, workloads

    t0 = time.time()
    mats, nbs, rhs = workloads.random_spd_batch(512, seed=2)
    gen_s = time.time() - t0
    dev = torch.device("cuda:0")
    B = bjp.Batch.from_systems(mats, nbs, dev)
    b = torch.as_tensor(np.concatenate(rhs), device=dev)
    M, setup_ms = _timed(lambda: bjp.batch_precondition(B, precision=args.precision))
    cfg, timings = autotune.tune_batch(B, M, b, probe_iters=10)
    bjp.batch_pcg_solve(B, M, b, **cfg)
    (x, info), ms = _timed(lambda: bjp.batch_pcg_solve(B, M, b, **cfg))
    n = np.diff(B.sys_rows.astype(np.int64))
    nnz = np.array([m.nnz for m in mats], dtype=np.int64)
    nbv = np.array(nbs, dtype=np.int64)
    it = info.per_system["iterations"].astype(np.int64)
    msz = 4 if args.precision == "fp32" else 8
    # per system per iteration: CSR, packed inverses, vectors (direction 24 N,
    # product 16 N, x/r update with the block application 56 N)
    per_it = 12 * nnz + 4 * n + msz * n * (nbv + 1) // 2 + 96 * n
    total_bytes = float(np.sum(per_it * it))
    print(json.dumps({"mode": "batch", "workload": "random_spd_batch_512", "precision": args.precision,
                      "systems": len(mats), "rows_total": int(n.sum()), "nnz_total": int(nnz.sum()),
                      "status": info.status, "systems_ok": info.systems_ok,
                      "total_iterations": int(info.total_iterations), "max_iterations": info.max_iterations,
                      "solve_ms": round(ms, 3),
                      "system_iterations_per_s": round(info.total_iterations / (ms / 1e3), 1),
                      "achieved_gbps": round(total_bytes / (ms / 1e3) / 1e9, 1),
                      "max_rel_res_true": info.max_rel_res_true, "setup_ms": round(setup_ms, 3),
                      "launch": cfg, "gen_s": round(gen_s, 1)}), flush=True)


def mode_adjoint(args):
    """Forward + adjoint solve on the 2D edge-conductivity Poisson problem."""
    import numpy as np
    import torch

    from paper_2410_02408_amd import autograd as ad, workloads

    n = 1024
    g = workloads.edge_graph2d(n)
    c = workloads.edge_conductivities(g, seed=3)
    A = workloads.edge_poisson2d(g, c)
    b, xt = workloads.rhs(A.n, 3), workloads.target(A.n, 3)
    dev = torch.device("cuda:0")
    pat = ad.Pattern.from_host(A, dev)
    asm = ad.EdgeAssembly(g, A, dev)
    ct = torch.as_tensor(c, device=dev).requires_grad_(True)
    bt = torch.as_tensor(b, device=dev).requires_grad_(True)
    xtt = torch.as_tensor(xt, device=dev)

    def run():
        infos = []
        x = ad.pcg_solve_diff(asm.assemble(ct), bt, pat, 32, tol=1e-10, info_out=infos)
        loss = torch.sum((x - xtt) ** 2)
        loss.backward()
        return infos, loss

    run()
    ct.grad = None
    bt.grad = None
    (infos, loss), ms = _timed(run)
    its = [i.iterations for i in infos]
    print(json.dumps({"mode": "adjoint", "workload": "edge_poisson2d_1024", "n": A.n, "nnz": A.nnz,
                      "block_size": 32, "forward_iterations": its[0], "adjoint_iterations": its[1],
                      "forward_plus_backward_ms": round(ms, 3),
                      "pcg_iterations_per_s": round(sum(its) / (ms / 1e3), 1),
                      "loss": loss.item(), "grad_c_norm": float(ct.grad.norm()),
                      "status": [i.status for i in infos]}), flush=True)


def mode_precision(args):
    """FP32-stored block inverses inside the FP64 PCG vs the plain FP64 path,
    both to the 1e-10 true residual, on the power-law workload."""
    import numpy as np
    import torch

    from paper_2410_02408_amd import bjp, workloads

    t0 = time.time()
    A_h = workloads.powerlaw_spd(1 << 22, seed=4)
    b_h = workloads.rhs(A_h.n, 4)
    gen_s = time.time() - t0
    dev = torch.device("cuda:0")
    A = bjp.DeviceCsr.from_host(A_h, dev)
    b = torch.as_tensor(b_h, device=dev)
    ws = bjp.PcgWorkspace(A)
    deg = np.diff(A_h.row_ptr)
    res = {}
    for prec in ("fp64", "fp32"):
        M, setup_ms = _timed(lambda: bjp.precondition(A, block_size=32, precision=prec))
        bjp.pcg_solve(A, M, b, workspace=ws)
        (x, info), ms = _timed(lambda: bjp.pcg_solve(A, M, b, workspace=ws))
        # the application's duration from a second solve with every launch
        # timed (the events would otherwise lengthen the timed solve)
        tm = bjp.KernelTimer(bjp.KERNEL_APPLY, 4096)
        bjp.pcg_solve(A, M, b, workspace=ws, timer=tm)
        apply_us = 1e3 * float(np.median(tm.durations_ms()[: info.iterations]))
        res[prec] = (x.clone(), info, ms, setup_ms, apply_us)
    x64 = res["fp64"][0]
    for prec in ("fp64", "fp32"):
        x, info, ms, setup_ms, apply_us = res[prec]
        err = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
        elem = 4 if prec == "fp32" else 8
        ab = elem * A_h.n * 33 // 2 + 32 * A_h.n
        print(json.dumps({"mode": "precision", "workload": "powerlaw_4m", "precision": prec,
                          "n": A_h.n, "nnz": A_h.nnz, "mean_nnz_row": round(float(deg.mean()), 2),
                          "max_nnz_row": int(deg.max()), "block_size": 32,
                          "pcg_iterations": info.iterations, "status": info.status,
                          "rel_res_true": info.rel_res_true, "pcg_ms": round(ms, 3),
                          "us_per_iteration": round(1e3 * ms / info.iterations, 2),
                          "apply_us": round(apply_us, 2),
                          "apply_gbps": round(ab / (apply_us * 1e-6) / 1e9, 1),
                          "rel_err_vs_fp64_path": err, "setup_ms": round(setup_ms, 3),
                          "gen_s": round(gen_s, 1)}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(the solver runs on a single MI355X).", file=sys.stderr)
        sys.exit(2)
    if args.mode != "headline":
        {"nb_sweep": mode_nb_sweep, "batch": mode_batch, "adjoint": mode_adjoint,
         "precision": mode_precision}[args.mode](args)
        return

    import numpy as np
    import torch

    from paper_2410_02408_amd import bjp, workloads

    t0 = time.time()
    W = workloads.workload(args.workload)
    gen_s = time.time() - t0
    steps_k = args.kappa_steps or W.lanczos_steps
    dev = torch.device("cuda:0")
    A = bjp.DeviceCsr.from_host(W.A, dev)
    b = torch.as_tensor(W.b, device=dev)
    pcg_ws = bjp.PcgWorkspace(A)
    kap_ws = bjp.KappaWorkspace(A, steps_k)
    torch.cuda.synchronize()

    def step(timer=None):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record()
        M = bjp.precondition(A, block_size=W.block_size, precision=args.precision)
        ev[1].record()
        x, info = bjp.pcg_solve(A, M, b, tol=W.tol, workspace=pcg_ws, timer=timer)
        ev[2].record()
        kA = bjp.kappa_estimate(A, b, steps_k, None, workspace=kap_ws)
        ev[3].record()
        kM = bjp.kappa_estimate(A, b, steps_k, M, workspace=kap_ws)
        ev[4].record()
        return M, info, kA, kM, ev

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # device-to-device copy of 1 GiB: the calibration for "achieved" bandwidth
    # and the known-size kernel the HBM byte counters are scaled against
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    (_, copy_ms) = _timed(lambda: [dst.copy_(src) for _ in range(5)])
    copy_gbps = 2 * src.numel() * 8 * 5 / (copy_ms * 1e-3) / 1e9
    del src, dst

    # every 8th application is bracketed by events (each event pair delays the
    # launches around it by a few microseconds, which would otherwise be
    # charged to the solve being timed)
    cap = 4096
    timers = [bjp.KernelTimer(bjp.KERNEL_APPLY, cap, stride=TIMER_STRIDE) for _ in range(args.steps)]
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t_wall = time.time()
    start.record()
    results = [step(timers[i]) for i in range(args.steps)]
    end.record()
    torch.cuda.synchronize()
    wall_s = time.time() - t_wall
    total_ms = start.elapsed_time(end)

    setup_ms = [r[4][0].elapsed_time(r[4][1]) for r in results]
    pcg_ms = [r[4][1].elapsed_time(r[4][2]) for r in results]
    kapA_ms = [r[4][2].elapsed_time(r[4][3]) for r in results]
    kapM_ms = [r[4][3].elapsed_time(r[4][4]) for r in results]
    iters = [r[1].iterations for r in results]
    M, info, kA, kM, _ = results[-1]
    for r in results:
        assert r[1].status == "OK" and r[1].rel_res_true <= W.tol, r[1]
        assert r[2].status == "OK" and r[3].status == "OK"

    value = sum(iters) / (sum(pcg_ms) / 1e3)
    durs = []
    for tmr, r in zip(timers, results):
        # launches past the converged iteration return at once: leave them out
        durs.extend(tmr.durations_ms()[: -(-r[1].iterations // TIMER_STRIDE)])
    apply_avg_ms = float(np.mean(durs))
    off = M.offsets()
    elem = 4 if M.precision == bjp.FP32_STORE else 8
    ab = apply_bytes(W.A.n, off, elem)
    achieved = ab / (apply_avg_ms * 1e-3) / 1e9
    B_iter = ab + spmv_bytes(W.A.n, W.A.nnz, column_bytes(W.A)) + direction_bytes(W.A.n)
    iter_gbs = B_iter * sum(iters) / (sum(pcg_ms) / 1e3) / 1e9
    traffic = read_traffic(f"apply_{args.workload}")

    line = {
        "metric": "PCG iters/s + achieved HBM GB/s at 1e-10 rel residual; κ(A)/κ(M⁻¹A)",
        "value": round(value, 2),
        "unit": "PCG iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32-block-inverses",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": W.A.n, "nnz": W.A.nnz,
                   "block_size": W.block_size, "tol": W.tol, "lanczos_steps": steps_k,
                   "parallelism": "single GPU"},
        "pcg_iterations": iters[-1],
        "pcg_ms": round(float(np.median(pcg_ms)), 3),
        "us_per_iteration": round(1e3 * sum(pcg_ms) / sum(iters), 2),
        "iteration_hbm_gbps": round(iter_gbs, 1),
        "iteration_bytes": B_iter,
        "setup_ms": round(float(np.median(setup_ms)), 3),
        "kappa_A_ms": round(float(np.median(kapA_ms)), 3),
        "kappa_MA_ms": round(float(np.median(kapM_ms)), 3),
        "kappa_A": kA.kappa,
        "kappa_MA": kM.kappa,
        "rel_res_true": info.rel_res_true,
        "roofline": {"bound": "hbm", "kernel": "k_apply (block inverse + r update)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": ab, "avg_launch_us": round(apply_avg_ms * 1e3, 3),
                     "launches_timed": len(durs)},
        "copy_gbps": round(copy_gbps, 1),
        "frac_of_copy": round(achieved / copy_gbps, 4),
        "wall_s": round(wall_s, 3),
        "gen_s": round(gen_s, 2),
    }

    if not args.no_cpu_baseline:
        import oracle

        Mo_t = time.time()
        Mo = oracle.Precond.uniform(W.A, W.block_size)
        setup_cpu = time.time() - Mo_t
        t = time.time()
        r = oracle.pcg(W.A, W.b, Mo, tol=W.tol, max_iter=args.cpu_iters, max_replacements=0)
        dt = time.time() - t
        line["cpu_baseline"] = {
            "value": round(r.iterations / dt, 3), "unit": "PCG iterations/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{r.iterations} PCG iterations of the same {args.workload} system "
                      f"(single-threaded FP64 C oracle; its setup took {setup_cpu:.1f} s, not included)"}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
