"""ctypes shim over the plain-C FP64 oracle (``bjp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark.  The GPU library never imports,
links or calls anything here, and nothing here calls the GPU library.

Each wrapper takes NumPy arrays and returns NumPy arrays; the arithmetic
(all of it FP64, sequential sums, no FMA contraction) happens in C.

Two builds of the same source: ``liboracle.so`` (sequential; every parity
check uses it) and ``liboracle_omp.so`` (OpenMP, used only to time the oracle
on all host cores: its dot products sum fixed per-thread chunks in thread
order, so it rounds differently).  Calls go to the sequential build unless
they run inside ``with timing_threads(k):``.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bjp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
# A test that plants a mistake in a copy of the oracle points this at the
# mutant's build; it is never set by the product or the benchmark.
_LIB_OVERRIDE = os.environ.get("BJP_ORACLE_LIB")

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOTSPD", -3: "ENOCONV", -4: "EBREAKDOWN", -5: "ENONFINITE"}

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


GCC_FLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]


def _compile(out: str, extra, force: bool) -> str:
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, *extra, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction): the sequential
    build and the OpenMP timing build."""
    _compile(_LIB_OMP, ["-fopenmp"], force)
    return _compile(_LIB, ["-Wno-unknown-pragmas"], force)


class _PcgInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("replacements", C.c_int),
                ("rel_res_recursive", C.c_double), ("rel_res_true", C.c_double)]


_libs = {}
_timing = None   # the OpenMP build while inside timing_threads()


def _load(path: str):
    if path not in _libs:
        L = C.CDLL(path)
        L.orc_csr_validate.argtypes = [C.c_int, _i32p, _i32p, _f64p]
        L.orc_spmv.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.orc_dot.argtypes = [C.c_int, _f64p, _f64p]
        L.orc_dot.restype = C.c_double
        L.orc_uniform_offsets.argtypes = [C.c_int, C.c_int, _i32p]
        L.orc_extract_block.argtypes = [_i32p, _i32p, _f64p, C.c_int, C.c_int, _f64p]
        L.orc_cholesky.argtypes = [C.c_int, _f64p]
        L.orc_chol_solve.argtypes = [C.c_int, _f64p, _f64p, _f64p]
        L.orc_precondition.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, _i32p,
                                       C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_precondition.restype = C.c_void_p
        L.orc_precond_free.argtypes = [C.c_void_p]
        L.orc_apply.argtypes = [C.c_void_p, _f64p, _f64p]
        L.orc_precond_block.argtypes = [C.c_void_p, C.c_int, _f64p]
        L.orc_pcg.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_void_p, _f64p, _f64p,
                              C.c_double, C.c_int, C.c_int, C.c_int, C.POINTER(_PcgInfo),
                              C.c_void_p]
        L.orc_lanczos.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_void_p, _f64p, C.c_int,
                                  _f64p, _f64p, C.POINTER(C.c_int)]
        L.orc_sturm_count.argtypes = [C.c_int, _f64p, _f64p, C.c_double]
        L.orc_tridiag_extremes.argtypes = [C.c_int, _f64p, _f64p, C.POINTER(C.c_double),
                                           C.POINTER(C.c_double)]
        L.orc_value_grad.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.orc_edge_grad.argtypes = [C.c_int, _i32p, _i32p, C.c_int, _i32p, _f64p, _f64p, _f64p]
        L.orc_set_threads.argtypes = [C.c_int]
        _libs[path] = L
    return _libs[path]


def lib():
    """The build the next call goes to (sequential unless timing_threads)."""
    if _timing is not None:
        return _timing
    if _LIB_OVERRIDE:
        return _load(_LIB_OVERRIDE)
    build(force=False)
    return _load(_LIB)


@contextlib.contextmanager
def timing_threads(threads: int = 0):
    """Route the oracle calls inside the block to the OpenMP timing build with
    `threads` threads (0: OpenMP's default).  Yields the thread count used.
    For timing only: its dot products round differently from the parity
    build."""
    global _timing
    _compile(_LIB_OMP, ["-fopenmp"], False)
    L = _load(_LIB_OMP)
    used = L.orc_set_threads(int(threads))
    prev, _timing = _timing, L
    try:
        yield used
    finally:
        _timing = prev


def _csr(A):
    return (int(A.n), np.ascontiguousarray(A.row_ptr, np.int32),
            np.ascontiguousarray(A.col_idx, np.int32), np.ascontiguousarray(A.val, np.float64))


def _vec(v):
    return np.ascontiguousarray(v, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, status, failed_block=-1):
        super().__init__(f"oracle status {STATUS.get(status, status)} (block {failed_block})")
        self.status = STATUS.get(status, status)
        self.failed_block = failed_block


def validate(A) -> str:
    n, rp, ci, v = _csr(A)
    return STATUS[lib().orc_csr_validate(n, rp, ci, v)]


def spmv(A, x) -> np.ndarray:
    n, rp, ci, v = _csr(A)
    y = np.empty(n)
    lib().orc_spmv(n, rp, ci, v, _vec(x), y)
    return y


def dot(a, b) -> float:
    a, b = _vec(a), _vec(b)
    return lib().orc_dot(len(a), a, b)


def uniform_offsets(n: int, block_size: int) -> np.ndarray:
    off = np.zeros(n // block_size + 2, dtype=np.int32)
    k = lib().orc_uniform_offsets(n, block_size, off)
    if k < 0:
        raise ValueError("bad block size")
    return off[: k + 1].copy()


def extract_block(A, s: int, e: int) -> np.ndarray:
    _, rp, ci, v = _csr(A)
    tile = np.zeros((e - s) * (e - s))
    lib().orc_extract_block(rp, ci, v, s, e, tile)
    return tile.reshape(e - s, e - s)


def cholesky(tile) -> np.ndarray:
    a = np.array(tile, dtype=np.float64, order="C", copy=True)
    st = lib().orc_cholesky(a.shape[0], a.ravel())
    if st != 0:
        raise OracleError(st)
    return a


def chol_solve(L, r) -> np.ndarray:
    """Solve (L L^T) z = r with the oracle's forward/backward substitution."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    z = np.empty(L.shape[0])
    lib().orc_chol_solve(L.shape[0], L.ravel(), _vec(r), z)
    return z


class Precond:
    """Block-Jacobi preconditioner held as per-block Cholesky factors."""

    def __init__(self, A, offsets):
        n, rp, ci, v = _csr(A)
        self.offsets = np.ascontiguousarray(offsets, np.int32)
        self.n = n
        st, fb = C.c_int(0), C.c_int(-1)
        self._lib = lib()
        self._h = self._lib.orc_precondition(n, rp, ci, v, len(self.offsets) - 1, self.offsets,
                                             C.byref(st), C.byref(fb))
        if not self._h:
            raise OracleError(st.value, fb.value)

    @classmethod
    def uniform(cls, A, block_size: int):
        return cls(A, uniform_offsets(A.n, block_size))

    def apply(self, r) -> np.ndarray:
        z = np.empty(self.n)
        lib().orc_apply(self._h, _vec(r), z)
        return z

    def factor(self, t: int) -> np.ndarray:
        m = int(self.offsets[t + 1] - self.offsets[t])
        out = np.empty(m * m)
        lib().orc_precond_block(self._h, t, out)
        return out.reshape(m, m)

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.orc_precond_free(self._h)
            self._h = None


@dataclasses.dataclass
class PcgResult:
    x: np.ndarray
    status: str
    iterations: int
    replacements: int
    rel_res_recursive: float
    rel_res_true: float
    history: np.ndarray | None = None


def pcg(A, b, M: Precond | None = None, tol: float = 1e-10, max_iter: int | None = None,
        x0=None, max_replacements: int = 3, history: bool = False) -> PcgResult:
    n, rp, ci, v = _csr(A)
    b = _vec(b)
    max_iter = n if max_iter is None else int(max_iter)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    info = _PcgInfo()
    hist = np.full(max_iter + 1, np.nan) if history else None
    lib().orc_pcg(n, rp, ci, v, M._h if M is not None else None, b, x, tol, max_iter,
                  0 if x0 is None else 1, max_replacements, C.byref(info),
                  hist.ctypes.data if hist is not None else None)
    if hist is not None:
        hist = hist[: info.iterations + 1]
    return PcgResult(x, STATUS[info.status], info.iterations, info.replacements,
                     info.rel_res_recursive, info.rel_res_true, hist)


@dataclasses.dataclass
class LanczosResult:
    status: str
    steps: int
    alpha: np.ndarray
    beta: np.ndarray


def lanczos(A, v0, steps: int, M: Precond | None = None) -> LanczosResult:
    n, rp, ci, v = _csr(A)
    al = np.zeros(max(steps, 1))
    be = np.zeros(max(steps, 1))
    sd = C.c_int(0)
    st = lib().orc_lanczos(n, rp, ci, v, M._h if M is not None else None, _vec(v0), steps,
                           al, be, C.byref(sd))
    s = sd.value
    return LanczosResult(STATUS[st], s, al[:s].copy(), be[: max(s - 1, 0)].copy())


def sturm_count(alpha, beta, x: float) -> int:
    alpha, beta = _vec(alpha), _vec(np.append(beta, 0.0))
    return lib().orc_sturm_count(len(alpha), alpha, beta, float(x))


def tridiag_extremes(alpha, beta):
    alpha, beta = _vec(alpha), _vec(np.append(beta, 0.0))
    lo, hi = C.c_double(), C.c_double()
    st = lib().orc_tridiag_extremes(len(alpha), alpha, beta, C.byref(lo), C.byref(hi))
    if st != 0:
        raise OracleError(st)
    return lo.value, hi.value


@dataclasses.dataclass
class KappaResult:
    status: str
    steps: int
    theta_min: float
    theta_max: float
    kappa: float
    alpha: np.ndarray
    beta: np.ndarray


def kappa(A, v0, steps: int, M: Precond | None = None) -> KappaResult:
    lz = lanczos(A, v0, steps, M)
    if lz.status != "OK":
        return KappaResult(lz.status, lz.steps, np.nan, np.nan, np.nan, lz.alpha, lz.beta)
    lo, hi = tridiag_extremes(lz.alpha, lz.beta)
    return KappaResult("OK", lz.steps, lo, hi, hi / lo, lz.alpha, lz.beta)


def value_grad(A, lam, x) -> np.ndarray:
    n, rp, ci, _ = _csr(A)
    g = np.empty(len(ci))
    lib().orc_value_grad(n, rp, ci, _vec(lam), _vec(x), g)
    return g


def edge_grad(graph, lam, x) -> np.ndarray:
    ei = np.ascontiguousarray(graph.ei, np.int32)
    ej = np.ascontiguousarray(graph.ej, np.int32)
    bi = np.ascontiguousarray(graph.bi, np.int32)
    g = np.empty(len(ei) + len(bi))
    lib().orc_edge_grad(len(ei), ei, ej, len(bi), bi, _vec(lam), _vec(x), g)
    return g
