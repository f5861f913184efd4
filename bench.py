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
SMALL_MAX_ROWS = 2048  # systems the library solves in one workgroup (automatic schedule)
TIMER_STRIDE = 8       # every 8th block-inverse application is timed with events


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diffusion3d_128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=100,
                    help="iterations of the single-threaded oracle sample")
    ap.add_argument("--cpu-single-full", action="store_true",
                    help="time the single-threaded oracle over the full solve too")
    ap.add_argument("--cpu-min-s", type=float, default=5.0,
                    help="repeat each oracle sample until it lasts this long (small systems)")
    ap.add_argument("--oracle-check", action="store_true",
                    help="solve with the (sequential) oracle and report the GPU's error against it")
    ap.add_argument("--no-oracle", action="store_true",
                    help="precision mode: skip the oracle solve (profiling runs)")
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


def gram_pass_bytes(n: int, j: int) -> dict:
    """Algorithmic bytes of the three Gram passes of Lanczos step j (0-based,
    j+1 stored basis vectors), as the CGS2 passes stream them:
      first   r~ = w - alpha u_j - beta u_{j-1}; c = V^T r~:
              8(j+1)N (V) + 24N (w, u_j, u_{j-1}; 16N at j = 0) + 8N (r~ written)
      second  r~ -= U c; c = V^T r~: 16(j+1)N (U and V) + 16N (r~ read, written)
      final   r~ -= U c: 8(j+1)N + 16N
    (The per-workgroup coefficient partials, a few KB, stay in the caches.)"""
    return {"first": 8 * (j + 1) * n + (24 if j > 0 else 16) * n + 8 * n,
            "second": 16 * (j + 1) * n + 16 * n,
            "final": 8 * (j + 1) * n + 16 * n}


def kappa_bytes(n: int, nnz: int, steps: int, m_bytes: int | None) -> int:
    """Algorithmic bytes of one m-step Lanczos estimate (m_bytes: bytes of the
    packed block inverses and offsets, None for kappa(A)).  Per step: the
    product (CSR 12 nnz + 4(N+1); z~ read, v_j, w written, and with M also r~
    read and u_j written: 40N, else 24N), the three Gram passes
    (gram_pass_bytes), and with M the application z~ = M^-1 r~ (m_bytes +
    16N).  The start (one application, one normalisation) is left out."""
    total = 0
    for j in range(steps):
        total += 12 * nnz + 4 * (n + 1) + (40 if m_bytes is not None else 24) * n
        total += sum(gram_pass_bytes(n, j).values())
        if m_bytes is not None:
            total += m_bytes + 16 * n
    return total


def host_cpu() -> dict:
    """The host's CPU model and the logical CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": avail, "cpu_count": os.cpu_count()}


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
    bjp.batch_precondition(B, precision=args.precision)       # first use loads the kernels
    M, setup_ms = _timed(lambda: bjp.batch_precondition(B, precision=args.precision))
    t0 = time.time()
    cfg, report = autotune.tune_batch(B, M, b, probe_iters=12)
    tune_s = time.time() - t0
    bjp.batch_pcg_solve(B, M, b, **cfg)
    (x, info), ms = _timed(lambda: bjp.batch_pcg_solve(B, M, b, **cfg))
    # reference: one schedule for the whole batch (row blocks streamed
    # through LDS, 1024-row tiles)
    bjp.batch_pcg_solve(B, M, b, lanes=-1, tile_rows=1024)
    (_, info_u), ms_u = _timed(lambda: bjp.batch_pcg_solve(B, M, b, lanes=-1, tile_rows=1024))
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
                      "launch": {"chosen": report["chosen"],
                                 "classes": {k: {"systems": r["systems"], "lanes": r["lanes"],
                                                 "tile_rows": r["tile_rows"]}
                                             for k, r in report["classes"].items()},
                                 "whole_batch_us_per_iteration": report["whole_batch_us_per_iteration"]},
                      "tune_s": round(tune_s, 1),
                      "one_schedule_solve_ms": round(ms_u, 3), "one_schedule": {"lanes": -1, "tile_rows": 1024},
                      "gen_s": round(gen_s, 1)}), flush=True)


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
    both to the 1e-10 true residual, on the power-law workload; each result's
    error against the FP64 oracle's solve; the random-gather product against
    the GPU's measured gather rates."""
    import numpy as np
    import torch

    import oracle
    from paper_2410_02408_amd import bjp, workloads

    t0 = time.time()
    A_h = workloads.powerlaw_spd(1 << 22, seed=4)
    b_h = workloads.rhs(A_h.n, 4)
    gen_s = time.time() - t0
    print(f"generated the power-law system in {gen_s:.0f} s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    refs = bandwidth_references(dev, gather_log2=(22, 19))
    A = bjp.DeviceCsr.from_host(A_h, dev)
    b = torch.as_tensor(b_h, device=dev)
    ws = bjp.PcgWorkspace(A)
    deg = np.diff(A_h.row_ptr)
    res = {}
    for prec in ("fp64", "fp32"):
        bjp.precondition(A, block_size=32, precision=prec)    # first use: kernel loading, allocation
        M, setup_ms = _timed(lambda: bjp.precondition(A, block_size=32, precision=prec))
        bjp.pcg_solve(A, M, b, workspace=ws)
        (x, info), ms = _timed(lambda: bjp.pcg_solve(A, M, b, workspace=ws))
        # kernel durations from further solves with every launch of one kernel
        # timed (the events would otherwise lengthen the timed solve)
        dur = {}
        for kid in (bjp.KERNEL_APPLY, bjp.KERNEL_SPMV):
            tm = bjp.KernelTimer(kid, 4096)
            bjp.pcg_solve(A, M, b, workspace=ws, timer=tm)
            dur[kid] = 1e3 * float(np.median(tm.durations_ms()[: info.iterations]))
        res[prec] = (x.cpu().numpy(), info, ms, setup_ms, dur)
    # the FP64 oracle's solve of the same system (sequential parity build)
    ref, oracle_s = None, 0.0
    if not args.no_oracle:
        print("GPU solves done; oracle solve", file=sys.stderr, flush=True)
        t = time.time()
        ref = oracle.pcg(A_h, b_h, oracle.Precond.uniform(A_h, 32), tol=1e-10)
        oracle_s = time.time() - t
    n, nnz = A_h.n, A_h.nnz
    # the column-panel product: CSR copy 12 nnz, 8 panel row-pointer arrays,
    # p gathered (8N), 8 partial vectors written and read (128N), q written
    # and p read by the row finish (16N)
    spmv_alg = 12 * nnz + 4 * 8 * (n + 1) + 8 * n + 2 * 64 * n + 16 * n
    for prec in ("fp64", "fp32"):
        x, info, ms, setup_ms, dur = res[prec]
        apply_us, spmv_us = dur[bjp.KERNEL_APPLY], dur[bjp.KERNEL_SPMV]
        elem = 4 if prec == "fp32" else 8
        ab = elem * n * 33 // 2 + 32 * n
        gps = nnz / (spmv_us * 1e-6) / 1e9
        print(json.dumps({"mode": "precision", "workload": "powerlaw_4m", "precision": prec,
                          "n": n, "nnz": nnz, "mean_nnz_row": round(float(deg.mean()), 2),
                          "max_nnz_row": int(deg.max()), "block_size": 32,
                          "pcg_iterations": info.iterations, "status": info.status,
                          "rel_res_true": info.rel_res_true, "pcg_ms": round(ms, 3),
                          "us_per_iteration": round(1e3 * ms / info.iterations, 2),
                          "apply_us": round(apply_us, 2),
                          "apply_gbps": round(ab / (apply_us * 1e-6) / 1e9, 1),
                          "spmv_us": round(spmv_us, 2),
                          "spmv": {"algorithmic_bytes": spmv_alg,
                                   "gbps": round(spmv_alg / (spmv_us * 1e-6) / 1e9, 1),
                                   "frac_hbm": round(spmv_alg / (spmv_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                                   "gathers_per_s_G": round(gps, 1),
                                   "frac_of_gather_rate_32MB": round(gps / refs["gather_G_per_s"]["32MB"], 4),
                                   "frac_of_gather_rate_4MB": round(gps / refs["gather_G_per_s"]["4MB"], 4)},
                          "vs_oracle": None if ref is None else {
                              "rel_err": float(np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)),
                              "oracle_iterations": ref.iterations, "oracle_status": ref.status,
                              "oracle_rel_res_true": ref.rel_res_true,
                              "iteration_delta": info.iterations - ref.iterations},
                          "rel_err_vs_fp64_path": float(np.linalg.norm(x - res["fp64"][0]) /
                                                        np.linalg.norm(res["fp64"][0])),
                          "references": refs, "setup_ms": round(setup_ms, 3),
                          "gen_s": round(gen_s, 1), "oracle_s": round(oracle_s, 1)}), flush=True)


def bandwidth_references(dev, gather_log2=()) -> dict:
    """What this GPU's memory system delivers for the solver's two access
    patterns, from the calibration kernels (calib/calib.hip): a read stream
    over 2 GiB (the best of five grid sizes, one to sixteen 256-thread
    workgroups per compute unit, x 4, 8 or 16 loads in flight per thread) and
    2^27 random 8-byte gathers from regions of 2^k doubles."""
    import ctypes as C

    import torch

    from paper_2410_02408_amd import build

    L = C.CDLL(build.CALIB_LIB)
    L.bjpcal_read_stream.argtypes = [C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    L.bjpcal_gather.argtypes = [C.c_void_p, C.c_int, C.c_longlong, C.c_int, C.c_void_p, C.c_void_p]
    stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    out = torch.empty(65536, dtype=torch.float64, device=dev)
    buf = torch.ones(1 << 28, dtype=torch.float64, device=dev)
    nbytes = buf.numel() * 8
    best = 0.0
    for grid in (256, 512, 1024, 2048, 4096):
        for inflight in (4, 8, 16):
            def run():
                for _ in range(5):
                    assert L.bjpcal_read_stream(C.c_void_p(buf.data_ptr()), nbytes, grid, inflight,
                                                C.c_void_p(out.data_ptr()), stream) == 0
            run()
            _, ms = _timed(run)
            best = max(best, 5 * nbytes / (ms * 1e-3) / 1e9)
    del buf
    refs = {"read_stream_gbps": round(best, 1)}
    if gather_log2:
        src = torch.ones(1 << max(gather_log2), dtype=torch.float64, device=dev)
        count = 1 << 27
        rates = {}
        for k in gather_log2:
            def run():
                for _ in range(3):
                    assert L.bjpcal_gather(C.c_void_p(src.data_ptr()), k, count, 8192,
                                           C.c_void_p(out.data_ptr()), stream) == 0
            run()
            _, ms = _timed(run)
            rates[f"{(8 << k) >> 20}MB" if k >= 17 else f"{(8 << k) >> 10}KB"] = round(
                3 * count / (ms * 1e-3) / 1e9, 1)
        refs["gather_G_per_s"] = rates
        del src
    return refs


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
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
        return M, info, kA, kM, ev, x

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # bandwidth references measured on this GPU: a device-to-device copy of
    # 1 GiB (read + write; also the known-size kernel the HBM byte counters
    # are scaled against) and a read stream of 2 GiB
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    (_, copy_ms) = _timed(lambda: [dst.copy_(src) for _ in range(5)])
    copy_gbps = 2 * src.numel() * 8 * 5 / (copy_ms * 1e-3) / 1e9
    del src, dst
    read_gbps = bandwidth_references(dev)["read_stream_gbps"]

    # every 8th application is bracketed by events (each event pair delays the
    # launches around it by a few microseconds, which would otherwise be
    # charged to the solve being timed)
    # (systems the one-workgroup solver takes, n <= SMALL_MAX_ROWS, have no
    # separate application launch to time: their roofline is the whole solve's)
    cap = 4096
    small = W.A.n <= SMALL_MAX_ROWS
    timers = [None if small else bjp.KernelTimer(bjp.KERNEL_APPLY, cap, stride=TIMER_STRIDE)
              for _ in range(args.steps)]
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
    M, info, kA, kM, _, _ = results[-1]
    for r in results:
        assert r[1].status == "OK" and r[1].rel_res_true <= W.tol, r[1]
        assert r[2].status == "OK" and r[3].status == "OK"

    value = sum(iters) / (sum(pcg_ms) / 1e3)
    off = M.offsets()
    elem = 4 if M.precision == bjp.FP32_STORE else 8
    ab = apply_bytes(W.A.n, off, elem)
    B_iter = ab + spmv_bytes(W.A.n, W.A.nnz, column_bytes(W.A)) + direction_bytes(W.A.n)
    durs = []
    if small:
        # one launch per solve: the whole iteration's bytes over its time
        kernel, per_launch = "k_pcg_small (the whole solve in one workgroup; latency-bound)", B_iter
        apply_avg_ms = sum(pcg_ms) / sum(iters)
    else:
        for tmr, r in zip(timers, results):
            # launches past the converged iteration return at once: leave them out
            durs.extend(tmr.durations_ms()[: -(-r[1].iterations // TIMER_STRIDE)])
        kernel, per_launch = "k_apply (block inverse + r update)", ab
        apply_avg_ms = float(np.mean(durs))
    achieved = per_launch / (apply_avg_ms * 1e-3) / 1e9
    iter_gbs = B_iter * sum(iters) / (sum(pcg_ms) / 1e3) / 1e9
    # the committed counters were taken on the FP64 application of this workload
    traffic = read_traffic(f"apply_{args.workload}") if args.precision == "fp64" else None
    m_bytes = ab - 32 * W.A.n          # packed inverses + offsets
    kb_A = kappa_bytes(W.A.n, W.A.nnz, kA.steps, None)
    kb_M = kappa_bytes(W.A.n, W.A.nnz, kM.steps, m_bytes)
    kA_s = float(np.median(kapA_ms)) / 1e3
    kM_s = float(np.median(kapM_ms)) / 1e3

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
        "roofline": {"bound": "hbm", "kernel": kernel,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_source": (f"profiles/apply_{args.workload}_counters.md (rocprofv3 FETCH_SIZE/"
                                        "WRITE_SIZE taken on the same kernel sources)" if traffic else None),
                     "bytes_per_launch": per_launch,
                     "avg_launch_us" if not small else "us_per_iteration": round(apply_avg_ms * 1e3, 3),
                     "launches_timed": len(durs)},
        "kappa_roofline": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                           "bytes_A": kb_A, "bytes_MA": kb_M,
                           "achieved_A": round(kb_A / kA_s / 1e9, 1), "achieved_MA": round(kb_M / kM_s / 1e9, 1),
                           "frac_A": round(kb_A / kA_s / 1e9 / HBM_PEAK_GBS, 4),
                           "frac_MA": round(kb_M / kM_s / 1e9 / HBM_PEAK_GBS, 4),
                           "gram_bytes_last_step": gram_pass_bytes(W.A.n, kA.steps - 1)},
        "copy_gbps": round(copy_gbps, 1),
        "read_stream_gbps": round(read_gbps, 1),
        "frac_of_copy": round(achieved / copy_gbps, 4),
        "frac_of_read_stream": round(achieved / read_gbps, 4),
        "wall_s": round(wall_s, 3),
        "gen_s": round(gen_s, 2),
    }

    if args.oracle_check:
        import oracle

        # the sequential (parity) oracle's solve of the same system
        ref = oracle.pcg(W.A, W.b, oracle.Precond.uniform(W.A, W.block_size), tol=W.tol)
        xg = results[-1][5].cpu().numpy()
        line["vs_oracle"] = {"rel_err": float(np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)),
                             "oracle_iterations": ref.iterations, "oracle_rel_res_true": ref.rel_res_true,
                             "gpu_iterations": iters[-1]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(W, args)
    print(json.dumps(line))


def cpu_baseline(W, args) -> dict:
    """The oracle on this host's cores, on the same system: the OpenMP timing
    build over the full solve to tol on all available threads (the value),
    and the sequential build over a bounded sample of iterations (or the full
    solve with --cpu-single-full), each repeated until it lasts --cpu-min-s.
    Setup is timed separately."""
    import oracle

    def repeated(solve):
        # the same solve again until the sample lasts --cpu-min-s (small
        # systems), unless one more would take it past 1.5 times that
        reps, t0 = 0, time.time()
        while True:
            r = solve()
            reps += 1
            dt = time.time() - t0
            if dt >= args.cpu_min_s or dt * (reps + 1) / reps > 1.5 * args.cpu_min_s:
                return r, reps, dt

    def times(reps):
        return "" if reps == 1 else f", {reps} times"

    host = host_cpu()
    with oracle.timing_threads(0) as threads:
        t = time.time()
        Mo = oracle.Precond.uniform(W.A, W.block_size)
        setup_s = time.time() - t
        r, reps, dt = repeated(lambda: oracle.pcg(W.A, W.b, Mo, tol=W.tol))
    del Mo
    Mo = oracle.Precond.uniform(W.A, W.block_size)
    single_iters = None if args.cpu_single_full else args.cpu_iters
    r1, reps1, dt1 = repeated(lambda: oracle.pcg(W.A, W.b, Mo, tol=W.tol, max_iter=single_iters,
                                                 max_replacements=3 if single_iters is None else 0))
    what1 = "the full solve" if single_iters is None or r1.iterations < single_iters else f"{r1.iterations} iterations"
    return {
        "value": round(reps * r.iterations / dt, 3), "unit": "PCG iterations/s", "cores": threads, "kind": "oracle",
        "sample": (f"full solve of the same {args.workload} system to {W.tol:g} ({r.iterations} iterations, "
                   f"{r.status}{times(reps)}, {dt:.1f} s) by the oracle's OpenMP timing build on {threads} "
                   f"threads; its block setup took {setup_s:.1f} s, not included"),
        "host": host,
        "single_thread": {"value": round(reps1 * r1.iterations / dt1, 3), "cores": 1,
                          "sample": (f"{what1} of the same system by the sequential oracle"
                                     f"{times(reps1)} ({dt1:.1f} s)")},
    }


if __name__ == "__main__":
    main()
