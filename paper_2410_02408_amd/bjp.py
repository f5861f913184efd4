"""Python binding of libbjp (include/bjp.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels; PyTorch
provides device memory (tensors) and the stream (the current stream of the
tensors' device).  Names follow the C entry points without the ``bjp_``
prefix: ``precondition``, ``apply``, ``pcg_solve``, ``kappa_estimate``.
The library must be built (``python -m paper_2410_02408_amd.build``); there
is no fallback when it is missing.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbjp.so")

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOTSPD", -3: "ENOCONV", -4: "EBREAKDOWN",
          -5: "ENONFINITE", -6: "EWORKSPACE", -7: "EHIP"}
FP64, FP32_STORE = 0, 1
MAX_BLOCK = 64


class CsrT(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p)]


class BlockSpecT(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("num_blocks", C.c_int32), ("offsets", C.c_void_p)]


class PrecondT(C.Structure):
    _fields_ = [("n", C.c_int32), ("block_size", C.c_int32), ("num_blocks", C.c_int32),
                ("precision", C.c_int32), ("group", C.c_int32), ("num_packets", C.c_int32),
                ("packet_elems", C.c_int32), ("pad", C.c_int32),
                ("offsets", C.c_void_p), ("tiles", C.c_void_p)]


class TimingT(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("capacity", C.c_int32), ("recorded", C.c_int32),
                ("stride", C.c_int32), ("events", C.c_void_p)]


class PcgOptsT(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("x0_given", C.c_int32),
                ("max_replacements", C.c_int32), ("check_every", C.c_int32),
                ("spmv_lanes", C.c_int32), ("pad", C.c_int32),
                ("history", C.c_void_p), ("timing", C.c_void_p)]


KERNEL_APPLY, KERNEL_SPMV = 0, 1


class KernelTimer:
    """Event pairs that the solver records around one kernel class.

    Uses torch.cuda.Event objects (HIP events); durations are read after the
    solve with Event.elapsed_time.  With stride k only every k-th launch is
    timed (each event pair delays the launches it brackets by a few
    microseconds)."""

    def __init__(self, kernel: int, capacity: int, stride: int = 1):
        self.events = [torch.cuda.Event(enable_timing=True) for _ in range(2 * capacity)]
        for e in self.events:
            e.record()          # materialise the underlying HIP event
        torch.cuda.synchronize()
        self._handles = (C.c_void_p * (2 * capacity))(*[e.cuda_event for e in self.events])
        self.struct = TimingT(kernel, capacity, 0, max(int(stride), 1), C.cast(self._handles, C.c_void_p))

    def durations_ms(self) -> list:
        torch.cuda.synchronize()
        n = self.struct.recorded
        return [self.events[2 * i].elapsed_time(self.events[2 * i + 1]) for i in range(n)]


class PcgInfoT(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("replacements", C.c_int32),
                ("polls", C.c_int32), ("rel_res_recursive", C.c_double),
                ("rel_res_true", C.c_double)]


class KappaInfoT(C.Structure):
    _fields_ = [("status", C.c_int32), ("steps_done", C.c_int32), ("theta_min", C.c_double),
                ("theta_max", C.c_double), ("kappa", C.c_double)]


_lib = None


def load():
    """Load libbjp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2410_02408_amd.build")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp, sz = C.c_void_p, C.c_size_t
    L.bjp_status_string.argtypes = [C.c_int]
    L.bjp_status_string.restype = C.c_char_p
    L.bjp_precondition_workspace.argtypes = [P(CsrT), P(BlockSpecT), C.c_int, P(sz)]
    L.bjp_precondition.argtypes = [P(CsrT), P(BlockSpecT), C.c_int, vp, sz, P(PrecondT),
                                   P(C.c_int32), vp]
    L.bjp_apply.argtypes = [P(PrecondT), vp, vp, vp]
    L.bjp_pcg_workspace.argtypes = [P(CsrT), P(sz)]
    L.bjp_pcg_solve.argtypes = [P(CsrT), P(PrecondT), vp, vp, P(PcgOptsT), vp, sz, P(PcgInfoT), vp]
    L.bjp_pcg_solve_noalloc.argtypes = [P(CsrT), P(PrecondT), vp, vp, P(PcgOptsT), P(PcgInfoT), vp]
    L.bjp_kappa_workspace.argtypes = [P(CsrT), C.c_int, P(sz)]
    L.bjp_kappa_estimate.argtypes = [P(CsrT), P(PrecondT), vp, C.c_int, vp, vp, vp, sz,
                                     P(KappaInfoT), vp]
    L.bjp_value_grad.argtypes = [P(CsrT), vp, vp, vp, vp]
    _lib = L
    return L


class BjpError(RuntimeError):
    def __init__(self, status: int, what: str, failed_block: int = -1):
        self.status = STATUS.get(status, str(status))
        self.failed_block = failed_block
        super().__init__(f"{what}: BJP_{self.status}" + (f" (block {failed_block})" if failed_block >= 0 else ""))


def _stream(device: torch.device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor | None):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _vec(v, device) -> torch.Tensor:
    if isinstance(v, torch.Tensor):
        t = v.to(device=device, dtype=torch.float64)
    else:
        t = torch.as_tensor(np.asarray(v, dtype=np.float64), device=device)
    return t.contiguous()


class DeviceCsr:
    """A CSR matrix resident on the GPU (int32 indices, float64 values)."""

    def __init__(self, n: int, row_ptr: torch.Tensor, col_idx: torch.Tensor, val: torch.Tensor):
        self.n = int(n)
        self.row_ptr = row_ptr.contiguous()
        self.col_idx = col_idx.contiguous()
        self.val = val.contiguous()
        assert self.row_ptr.dtype == torch.int32 and self.col_idx.dtype == torch.int32
        assert self.val.dtype == torch.float64
        assert self.row_ptr.numel() == self.n + 1
        self.nnz = int(self.col_idx.numel())
        self.device = self.val.device

    @classmethod
    def from_host(cls, A, device="cuda"):
        """From any object with n, row_ptr, col_idx, val (NumPy arrays)."""
        dev = torch.device(device)
        return cls(A.n, torch.as_tensor(np.asarray(A.row_ptr, np.int32), device=dev),
                   torch.as_tensor(np.asarray(A.col_idx, np.int32), device=dev),
                   torch.as_tensor(np.asarray(A.val, np.float64), device=dev))

    @classmethod
    def from_torch(cls, t: torch.Tensor):
        """From a square torch sparse CSR tensor on the GPU (indices converted
        to int32 and values to float64; the tensor itself is not modified)."""
        if t.layout != torch.sparse_csr or t.dim() != 2 or t.shape[0] != t.shape[1]:
            raise TypeError("expected a square torch.sparse_csr tensor")
        return cls(t.shape[0], t.crow_indices().to(torch.int32), t.col_indices().to(torch.int32),
                   t.values().to(torch.float64))

    def struct(self) -> CsrT:
        return CsrT(self.n, self.nnz, self.row_ptr.data_ptr(),
                    self.col_idx.data_ptr() if self.nnz else 0,
                    self.val.data_ptr() if self.nnz else 0)


def as_csr(A) -> DeviceCsr:
    """A DeviceCsr as is, or a torch sparse CSR tensor converted to one."""
    if isinstance(A, DeviceCsr):
        return A
    if isinstance(A, torch.Tensor) and A.layout == torch.sparse_csr:
        return DeviceCsr.from_torch(A)
    raise TypeError("expected a DeviceCsr or a torch.sparse_csr tensor")


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Precond:
    """Block-Jacobi preconditioner; owns the workspace its handle points into."""

    def __init__(self, handle: PrecondT, ws: torch.Tensor):
        self.handle = handle
        self.ws = ws

    @property
    def n(self):
        return self.handle.n

    @property
    def num_blocks(self):
        return self.handle.num_blocks

    @property
    def precision(self):
        return self.handle.precision

    def offsets(self) -> np.ndarray:
        start = self.handle.offsets - self.ws.data_ptr()
        nbytes = 4 * (self.handle.num_blocks + 1)
        return self.ws[start:start + nbytes].view(torch.int32).cpu().numpy()

    def tiles(self) -> torch.Tensor:
        """The raw packet storage (diagonal packets of the block inverses)."""
        base = self.ws.data_ptr()
        start = self.handle.tiles - base
        s = 4 if self.handle.precision == FP32_STORE else 8
        count = self.handle.num_packets * self.handle.packet_elems
        dt = torch.float32 if s == 4 else torch.float64
        return self.ws[start:start + count * s].view(dt)


def _spec(block_size, offsets):
    if offsets is not None:
        off = np.ascontiguousarray(offsets, dtype=np.int32)
        return BlockSpecT(0, len(off) - 1, off.ctypes.data), off
    return BlockSpecT(int(block_size), 0, None), None


def precondition(A: DeviceCsr, block_size: int | None = None, offsets=None,
                 precision: str | int = "fp64") -> Precond:
    """bjp_precondition: extract, factor and invert the diagonal blocks."""
    L = load()
    A = as_csr(A)
    prec = {"fp64": FP64, "fp32": FP32_STORE}.get(precision, precision)
    csr = A.struct()
    spec, keep = _spec(block_size, offsets)
    nbytes = C.c_size_t()
    st = L.bjp_precondition_workspace(C.byref(csr), C.byref(spec), prec, C.byref(nbytes))
    if st:
        raise BjpError(st, "bjp_precondition_workspace")
    ws = _workspace(nbytes.value, A.device)
    h = PrecondT()
    fb = C.c_int32(-1)
    st = L.bjp_precondition(C.byref(csr), C.byref(spec), prec, _ptr(ws), ws.numel(), C.byref(h),
                            C.byref(fb), _stream(A.device))
    del keep
    if st:
        raise BjpError(st, "bjp_precondition", fb.value)
    return Precond(h, ws)


def apply(M: Precond, r: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """bjp_apply: z = M^-1 r (asynchronous on the current stream)."""
    L = load()
    r = _vec(r, M.ws.device)
    z = torch.empty_like(r) if out is None else out
    st = L.bjp_apply(C.byref(M.handle), _ptr(r), _ptr(z), _stream(M.ws.device))
    if st:
        raise BjpError(st, "bjp_apply")
    return z


@dataclasses.dataclass
class PcgInfo:
    status: str
    iterations: int
    replacements: int
    polls: int
    rel_res_recursive: float
    rel_res_true: float


class PcgWorkspace:
    """Reusable solver workspace for one matrix size."""

    def __init__(self, A: DeviceCsr):
        A = as_csr(A)
        n = C.c_size_t()
        st = load().bjp_pcg_workspace(C.byref(A.struct()), C.byref(n))
        if st:
            raise BjpError(st, "bjp_pcg_workspace")
        self.ws = _workspace(n.value, A.device)


def pcg_solve(A: DeviceCsr, M: Precond | None, b, tol: float = 1e-10, max_iter: int | None = None,
              x0=None, out: torch.Tensor | None = None, max_replacements: int = 3,
              check_every: int = 0, spmv_lanes: int = 0,
              history: torch.Tensor | None = None, workspace: PcgWorkspace | None = None,
              timer: KernelTimer | None = None):
    """bjp_pcg_solve.  Returns (x, PcgInfo); solver failures are reported in
    info.status, argument/workspace/runtime errors raise BjpError."""
    L = load()
    A = as_csr(A)
    dev = A.device
    b = _vec(b, dev)
    if out is not None:
        x = out
        if x0 is not None:
            x.copy_(_vec(x0, dev))
    else:
        x = _vec(x0, dev).clone() if x0 is not None else torch.empty(A.n, dtype=torch.float64, device=dev)
    ws = workspace or PcgWorkspace(A)
    opts = PcgOptsT(tol, int(max_iter or 0), 1 if x0 is not None else 0,
                    -1 if max_replacements == 0 else int(max_replacements), int(check_every),
                    int(spmv_lanes), 0,
                    history.data_ptr() if history is not None else None,
                    C.cast(C.pointer(timer.struct), C.c_void_p) if timer is not None else None)
    info = PcgInfoT()
    st = L.bjp_pcg_solve(C.byref(A.struct()), C.byref(M.handle) if M is not None else None,
                         _ptr(b), _ptr(x), C.byref(opts), _ptr(ws.ws), ws.ws.numel(), C.byref(info),
                         _stream(dev))
    if st in (-1, -6, -7):
        raise BjpError(st, "bjp_pcg_solve")
    return x, PcgInfo(STATUS[info.status], info.iterations, info.replacements, info.polls,
                      info.rel_res_recursive, info.rel_res_true)


NOALLOC_SCRATCH_BYTES = 128 << 20


def pcg_solve_noalloc(A: DeviceCsr, M: Precond | None, b: torch.Tensor, x: torch.Tensor,
                      tol: float = 1e-10, max_iter: int | None = None, x0_given: bool = False,
                      max_replacements: int = 3, check_every: int = 0, spmv_lanes: int = 0,
                      history: torch.Tensor | None = None):
    """bjp_pcg_solve_noalloc: the solve on the library's static scratch.  b and
    x are caller-owned device tensors of n float64 (x holds x0 when
    x0_given); nothing is allocated here or in the library.  Returns
    PcgInfo; argument/size/runtime errors raise BjpError."""
    L = load()
    A = as_csr(A)
    opts = PcgOptsT(tol, int(max_iter or 0), 1 if x0_given else 0,
                    -1 if max_replacements == 0 else int(max_replacements), int(check_every),
                    int(spmv_lanes), 0, history.data_ptr() if history is not None else None, None)
    info = PcgInfoT()
    st = L.bjp_pcg_solve_noalloc(C.byref(A.struct()), C.byref(M.handle) if M is not None else None,
                                 _ptr(b), _ptr(x), C.byref(opts), C.byref(info), _stream(A.device))
    if st in (-1, -6, -7):
        raise BjpError(st, "bjp_pcg_solve_noalloc")
    return PcgInfo(STATUS[info.status], info.iterations, info.replacements, info.polls,
                   info.rel_res_recursive, info.rel_res_true)


@dataclasses.dataclass
class KappaInfo:
    status: str
    steps: int
    theta_min: float
    theta_max: float
    kappa: float
    alpha: np.ndarray
    beta: np.ndarray


class KappaWorkspace:
    def __init__(self, A: DeviceCsr, steps: int):
        n = C.c_size_t()
        st = load().bjp_kappa_workspace(C.byref(A.struct()), int(steps), C.byref(n))
        if st:
            raise BjpError(st, "bjp_kappa_workspace")
        self.steps = steps
        self.ws = _workspace(n.value, A.device)


def kappa_estimate(A: DeviceCsr, v0, steps: int, M: Precond | None = None,
                   workspace: KappaWorkspace | None = None) -> KappaInfo:
    """bjp_kappa_estimate: Lanczos estimate of kappa(M^-1 A) (kappa(A) if M is None)."""
    L = load()
    A = as_csr(A)
    dev = A.device
    v0 = _vec(v0, dev)
    ws = workspace if workspace is not None and workspace.steps >= steps else KappaWorkspace(A, steps)
    al = torch.zeros(steps, dtype=torch.float64, device=dev)
    be = torch.zeros(steps, dtype=torch.float64, device=dev)
    info = KappaInfoT()
    st = L.bjp_kappa_estimate(C.byref(A.struct()), C.byref(M.handle) if M is not None else None,
                              _ptr(v0), int(steps), _ptr(al), _ptr(be), _ptr(ws.ws), ws.ws.numel(),
                              C.byref(info), _stream(dev))
    if st in (-1, -6, -7):
        raise BjpError(st, "bjp_kappa_estimate")
    s = info.steps_done
    return KappaInfo(STATUS[info.status], s, info.theta_min, info.theta_max, info.kappa,
                     al[:s].cpu().numpy(), be[:max(s - 1, 0)].cpu().numpy())


def value_grad(A: DeviceCsr, lam: torch.Tensor, x: torch.Tensor, out: torch.Tensor | None = None):
    """bjp_value_grad: -lambda_i x_j on every stored entry of A (CSR order)."""
    L = load()
    A = as_csr(A)
    g = torch.empty(A.nnz, dtype=torch.float64, device=A.device) if out is None else out
    st = L.bjp_value_grad(C.byref(A.struct()), _ptr(_vec(lam, A.device)), _ptr(_vec(x, A.device)),
                          _ptr(g), _stream(A.device))
    if st:
        raise BjpError(st, "bjp_value_grad")
    return g


# ---------------------------------------------------------------------------
# batches of independent systems
# ---------------------------------------------------------------------------

class BatchT(C.Structure):
    _fields_ = [("num_systems", C.c_int32), ("sys_rows", C.c_void_p), ("block_size", C.c_void_p)]


class BatchPrecondT(C.Structure):
    _fields_ = [("num_systems", C.c_int32), ("precision", C.c_int32), ("systems", C.c_void_p),
                ("tiles", C.c_void_p)]


class BatchOptsT(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("max_replacements", C.c_int32),
                ("lanes", C.c_int32), ("tile_rows", C.c_int32), ("check_every", C.c_int32),
                ("eager", C.c_int32), ("sys_lanes", C.c_void_p), ("sys_tile_rows", C.c_void_p)]


class SystemInfoT(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("replacements", C.c_int32),
                ("pad", C.c_int32), ("rel_res_recursive", C.c_double), ("rel_res_true", C.c_double)]


class BatchInfoT(C.Structure):
    _fields_ = [("status", C.c_int32), ("systems_ok", C.c_int32), ("max_iterations", C.c_int32),
                ("pad", C.c_int32), ("total_iterations", C.c_int64), ("max_rel_res_true", C.c_double)]


def _load_batch(L):
    if getattr(L, "_batch_ready", False):
        return L
    P = C.POINTER
    vp, sz = C.c_void_p, C.c_size_t
    L.bjp_batch_precondition_workspace.argtypes = [P(CsrT), P(BatchT), C.c_int, P(sz)]
    L.bjp_batch_precondition.argtypes = [P(CsrT), P(BatchT), C.c_int, vp, sz, P(BatchPrecondT),
                                         P(C.c_int32), vp]
    L.bjp_batch_pcg_workspace.argtypes = [P(CsrT), P(BatchT), P(sz)]
    L.bjp_batch_pcg_solve.argtypes = [P(CsrT), P(BatchT), P(BatchPrecondT), vp, vp, P(BatchOptsT), vp,
                                      sz, P(BatchInfoT), vp, vp]
    L._batch_ready = True
    return L


class Batch:
    """A batch of independent systems stored as one block-diagonal CSR on
    the device (system s = rows sys_rows[s]:sys_rows[s+1]) with a block size
    per system."""

    def __init__(self, A: DeviceCsr, sys_rows, block_sizes):
        self.A = A
        self.sys_rows = np.ascontiguousarray(sys_rows, dtype=np.int32)
        self.block_sizes = np.ascontiguousarray(block_sizes, dtype=np.int32)
        self.num_systems = len(self.block_sizes)

    @classmethod
    def from_systems(cls, mats, block_sizes, device="cuda"):
        """Concatenate host CSR systems (columns shifted to global rows)."""
        rows = np.zeros(len(mats) + 1, dtype=np.int64)
        for s, M in enumerate(mats):
            rows[s + 1] = rows[s] + M.n
        nnz = np.zeros(len(mats) + 1, dtype=np.int64)
        for s, M in enumerate(mats):
            nnz[s + 1] = nnz[s] + M.nnz
        rp = np.empty(int(rows[-1]) + 1, dtype=np.int64)
        ci = np.empty(int(nnz[-1]), dtype=np.int32)
        va = np.empty(int(nnz[-1]), dtype=np.float64)
        for s, M in enumerate(mats):
            rp[rows[s]:rows[s + 1]] = M.row_ptr[:-1].astype(np.int64) + nnz[s]
            ci[nnz[s]:nnz[s + 1]] = M.col_idx + rows[s]
            va[nnz[s]:nnz[s + 1]] = M.val
        rp[-1] = nnz[-1]
        if nnz[-1] >= 2 ** 31:
            raise ValueError("batch nnz does not fit int32 indices")
        dev = torch.device(device)
        A = DeviceCsr(int(rows[-1]), torch.as_tensor(rp.astype(np.int32), device=dev),
                      torch.as_tensor(ci, device=dev), torch.as_tensor(va, device=dev))
        return cls(A, rows.astype(np.int32), block_sizes)

    def struct(self) -> BatchT:
        return BatchT(self.num_systems, self.sys_rows.ctypes.data, self.block_sizes.ctypes.data)

    def subset(self, systems, b: torch.Tensor | None = None):
        """A batch of the listed systems (copied on the device, in the given
        order) and, if b is given, the matching slices of b."""
        dev = self.A.device
        sr = self.sys_rows.astype(np.int64)
        ep = self.A.row_ptr[torch.as_tensor(sr, device=dev)].cpu().numpy().astype(np.int64)
        rps, cis, vals, bs, rows = [], [], [], [], [0]
        nnz0 = 0
        for s in systems:
            r0, r1, e0, e1 = sr[s], sr[s + 1], ep[s], ep[s + 1]
            rps.append(self.A.row_ptr[r0:r1].to(torch.int64) - int(e0) + nnz0)
            cis.append(self.A.col_idx[e0:e1] - int(r0 - rows[-1]))
            vals.append(self.A.val[e0:e1])
            if b is not None:
                bs.append(b[r0:r1])
            nnz0 += int(e1 - e0)
            rows.append(rows[-1] + int(r1 - r0))
        rps.append(torch.tensor([nnz0], dtype=torch.int64, device=dev))
        A = DeviceCsr(rows[-1], torch.cat(rps).to(torch.int32), torch.cat(cis), torch.cat(vals))
        sub = Batch(A, np.asarray(rows, dtype=np.int32), self.block_sizes[np.asarray(systems)])
        return sub, (torch.cat(bs) if b is not None else None)


class BatchPrecond:
    def __init__(self, handle: BatchPrecondT, ws: torch.Tensor):
        self.handle = handle
        self.ws = ws


def batch_precondition(B: Batch, precision: str | int = "fp64") -> BatchPrecond:
    """bjp_batch_precondition: per-system block-Jacobi setup for the whole batch."""
    L = _load_batch(load())
    prec = {"fp64": FP64, "fp32": FP32_STORE}.get(precision, precision)
    csr, bs = B.A.struct(), B.struct()
    n = C.c_size_t()
    st = L.bjp_batch_precondition_workspace(C.byref(csr), C.byref(bs), prec, C.byref(n))
    if st:
        raise BjpError(st, "bjp_batch_precondition_workspace")
    ws = _workspace(n.value, B.A.device)
    h = BatchPrecondT()
    fb = C.c_int32(-1)
    st = L.bjp_batch_precondition(C.byref(csr), C.byref(bs), prec, _ptr(ws), ws.numel(), C.byref(h),
                                  C.byref(fb), _stream(B.A.device))
    if st:
        raise BjpError(st, "bjp_batch_precondition", fb.value)
    return BatchPrecond(h, ws)


@dataclasses.dataclass
class BatchInfo:
    status: str
    systems_ok: int
    total_iterations: int
    max_iterations: int
    max_rel_res_true: float
    per_system: np.ndarray      # structured: status, iterations, replacements, rel_res_*


def batch_pcg_solve(B: Batch, M: BatchPrecond, b, tol: float = 1e-10, max_iter: int = 0,
                    lanes: int = 0, tile_rows: int = 0, check_every: int = 0,
                    out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                    graph: bool = True, sys_lanes=None, sys_tile_rows=None):
    """bjp_batch_pcg_solve: every system advances in the same launches (the
    iterations between polls replayed from a captured hipGraph unless
    graph=False).  sys_lanes / sys_tile_rows (one int per system, 0 = the
    batch-wide value) set each system's product schedule."""
    L = _load_batch(load())
    dev = B.A.device
    b = _vec(b, dev)
    x = torch.empty(B.A.n, dtype=torch.float64, device=dev) if out is None else out
    csr, bs = B.A.struct(), B.struct()
    if workspace is None:
        n = C.c_size_t()
        st = L.bjp_batch_pcg_workspace(C.byref(csr), C.byref(bs), C.byref(n))
        if st:
            raise BjpError(st, "bjp_batch_pcg_workspace")
        workspace = _workspace(n.value, dev)
    sl = None if sys_lanes is None else np.ascontiguousarray(sys_lanes, dtype=np.int32)
    st_ = None if sys_tile_rows is None else np.ascontiguousarray(sys_tile_rows, dtype=np.int32)
    for arr in (sl, st_):
        if arr is not None and len(arr) != B.num_systems:
            raise ValueError("per-system schedule arrays need one entry per system")
    opts = BatchOptsT(tol, int(max_iter), 0, int(lanes), int(tile_rows), int(check_every), 0 if graph else 1,
                      sl.ctypes.data if sl is not None else None, st_.ctypes.data if st_ is not None else None)
    info = BatchInfoT()
    per = (SystemInfoT * B.num_systems)()
    st = L.bjp_batch_pcg_solve(C.byref(csr), C.byref(bs), C.byref(M.handle), _ptr(b), _ptr(x),
                               C.byref(opts), _ptr(workspace), workspace.numel(), C.byref(info),
                               C.cast(per, C.c_void_p), _stream(dev))
    if st in (-1, -6, -7):
        raise BjpError(st, "bjp_batch_pcg_solve")
    arr = np.array([(p.status, p.iterations, p.replacements, p.rel_res_recursive, p.rel_res_true)
                    for p in per], dtype=[("status", "i4"), ("iterations", "i4"), ("replacements", "i4"),
                                          ("rel_res_recursive", "f8"), ("rel_res_true", "f8")])
    return x, BatchInfo(STATUS[info.status], info.systems_ok, info.total_iterations,
                        info.max_iterations, info.max_rel_res_true, arr)
