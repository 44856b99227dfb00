"""CPU oracle for the AAR solver: plain FP64 C (``aar_oracle.c``) behind ctypes.

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously correct
reference the GPU solver is checked against.  Only ``tests/``, the package
smoke check and the benchmark's CPU-baseline leg may import it; the solver
never does, and it shares no code with the GPU path.

Every function cites the part of the paper (arXiv:1606.08740) it follows;
the readings taken where the paper is silent are listed at the top of
``aar_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aar_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, BREAKDOWN, BAD_ARG = 0, 1, 2, -1


# gcc flags of the oracle: optimized, ISO C (no floating-point contraction or
# reassociation, so every build computes the same bits), OpenMP static loops
CFLAGS = ["-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (CFLAGS) into oracle/liboracle.so (portable:
    no -march, so the library runs on any x86-64 host it is copied to)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def load_native(dirpath: str):
    """Build the oracle with CFLAGS plus -march=native for the host that runs
    this (the CPU baseline's build) into `dirpath`, load it, and make it the
    library every function here calls.  Returns the flags used."""
    flags = CFLAGS + ["-march=native"]
    path = os.path.join(dirpath, "liboracle_native.so")
    subprocess.check_call(["gcc", *flags, "-o", path, _SRC, "-lm"])
    _load_from(path)
    return flags


class _Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3), ("bc", ctypes.c_int32 * 3),
                ("radius", ctypes.c_int32), ("diffusion", ctypes.c_double),
                ("shift", ctypes.c_double), ("velocity", ctypes.c_void_p)]


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


_lib = None


def _load():
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _load_from(_LIB)
    return _lib


def _load_from(path: str):
    global _lib
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(_Problem)
    lib.oracle_fd_weights.argtypes = [ctypes.c_int, dp]
    lib.oracle_apply.argtypes = [pp, dp, dp]
    lib.oracle_diagonal.argtypes = [pp, dp]
    lib.oracle_jacobi_eigen.argtypes = [ctypes.c_int, dp, dp]
    lib.oracle_pinv_solve.argtypes = [ctypes.c_int, dp, dp, dp]
    lib.oracle_pinv_solve.restype = ctypes.c_int
    lib.oracle_aar_solve.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_int64), dp, dp, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_aar_solve.restype = ctypes.c_int
    lib.oracle_relative_residual.argtypes = [pp, dp, dp]
    lib.oracle_relative_residual.restype = ctypes.c_double
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_deflate_constant.argtypes = [pp, dp, dp]
    lib.oracle_deflate_constant.restype = ctypes.c_int
    lib.oracle_apply_complex.argtypes = [pp, ctypes.c_double, dp, dp]
    lib.oracle_aar_solve_complex.argtypes = [pp, ctypes.c_double, dp, dp, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), dp,
                                             dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_aar_solve_complex.restype = ctypes.c_int
    cp = ctypes.POINTER(_Csr)
    lib.oracle_csr_check.argtypes = [cp]
    lib.oracle_csr_check.restype = ctypes.c_int
    lib.oracle_csr_apply.argtypes = [cp, dp, dp]
    lib.oracle_ilu0.argtypes = [cp, ctypes.c_int, dp]
    lib.oracle_ilu0.restype = ctypes.c_int
    lib.oracle_ilu0_solve.argtypes = [cp, ctypes.c_int, dp, dp, dp]
    lib.oracle_csr_precondition.argtypes = [cp, ctypes.c_int, ctypes.c_int, dp, dp]
    lib.oracle_csr_precondition.restype = ctypes.c_int
    lib.oracle_aar_solve_csr.argtypes = [cp, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64), dp, dp, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_aar_solve_csr.restype = ctypes.c_int
    lib.oracle_relative_residual_csr.argtypes = [cp, dp, dp]
    lib.oracle_relative_residual_csr.restype = ctypes.c_double
    _lib = lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class _Bound:
    """A ctypes problem struct plus the arrays it points into (kept alive)."""

    def __init__(self, prob):
        self.vel = None if prob.velocity is None else _f64(prob.velocity)
        s = _Problem()
        s.n = (ctypes.c_int32 * 3)(*[int(v) for v in prob.n])
        s.h = (ctypes.c_double * 3)(*[float(v) for v in prob.h])
        s.bc = (ctypes.c_int32 * 3)(*[int(v) for v in prob.bc])
        s.radius = int(prob.radius)
        s.diffusion = float(prob.diffusion)
        s.shift = float(prob.shift)
        s.velocity = None if self.vel is None else self.vel.ctypes.data
        self.s = s
        self.size = int(prob.n[0]) * int(prob.n[1]) * int(prob.n[2])

    @property
    def ref(self):
        return ctypes.byref(self.s)


def fd_weights(r: int) -> np.ndarray:
    """Order-2r central second-difference weights w_0..w_r (the paper's
    sixth-order discretization, Secs. 3.2-3.3, is r = 3)."""
    w = np.zeros(7)
    _load().oracle_fd_weights(int(r), _ptr(w))
    return w[: r + 1].copy()


def apply(prob, x) -> np.ndarray:
    """y = A x for the finite-difference operator of `prob` (Eq. 1)."""
    b = _Bound(prob)
    x = _f64(x)
    y = np.empty(b.size)
    _load().oracle_apply(b.ref, _ptr(x), _ptr(y))
    return y


def diagonal(prob) -> np.ndarray:
    """D = diag(A): the Jacobi preconditioner M = D (Sec. 2, AAJ special case)."""
    b = _Bound(prob)
    d = np.empty(b.size)
    _load().oracle_diagonal(b.ref, _ptr(d))
    return d


def jacobi_eigen(S) -> tuple:
    """Cyclic Jacobi eigendecomposition of a symmetric matrix: (eigenvalues, V)."""
    S = _f64(S).copy()
    l = S.shape[0]
    V = np.empty((l, l))
    _load().oracle_jacobi_eigen(l, _ptr(S), _ptr(V))
    return np.diag(S).copy(), V


def pinv_solve(G, c) -> tuple:
    """gamma = pinv(F^T F) F^T f given G = F^T F and c = F^T f (Eq. 3 with the
    Moore-Penrose pseudoinverse, Sec. 3.2).  Returns (gamma, rank)."""
    G = _f64(G)
    c = _f64(c)
    l = c.shape[0]
    g = np.zeros(max(l, 1))
    rank = _load().oracle_pinv_solve(l, _ptr(G), _ptr(c), _ptr(g))
    return g[:l].copy(), rank


def aar_solve(prob, b, x0=None, omega=0.6, beta=0.6, m=7, p=6, tol=1e-10, max_iter=1_000_000,
              trace_cap: int = 0) -> dict:
    """Jacobi-preconditioned AAR (Eqs. 2-6) in FP64.

    Returns a dict with x, status, iterations, relres (last measured
    ||b - A x_k|| / ||b||) and, when trace_cap > 0, `trace`: one row per
    Anderson step [k, r_k, ||f_k||, ||f_k - F_k gamma_k||, rank,
    cond(F_k^T F_k) over the kept eigenvalues].
    """
    bd = _Bound(prob)
    b = _f64(b)
    x = np.zeros(bd.size) if x0 is None else _f64(x0).copy()
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    tl = ctypes.c_int64(0)
    tr = np.zeros((max(trace_cap, 1), 6))
    st = _load().oracle_aar_solve(bd.ref, _ptr(b), _ptr(x), float(omega), float(beta), int(m), int(p),
                                  float(tol), int(max_iter), ctypes.byref(it), ctypes.byref(rr),
                                  _ptr(tr) if trace_cap > 0 else None, int(trace_cap),
                                  ctypes.byref(tl))
    out = {"x": x, "status": st, "iterations": it.value, "relres": rr.value}
    if trace_cap > 0:
        out["trace"] = tr[: tl.value].copy()
    return out


def deflate_constant(prob, b, x0=None) -> np.ndarray:
    """The solver's optional constant-mode step (not in the paper): for an
    all-periodic system with sigma > 0, x0 + (mean(b - A x0) / sigma) 1, whose
    residual has zero mean (A 1 = sigma 1).  Raises ValueError otherwise."""
    bd = _Bound(prob)
    x = np.zeros(bd.size) if x0 is None else _f64(x0).copy()
    if _load().oracle_deflate_constant(bd.ref, _ptr(_f64(b)), _ptr(x)) != OK:
        raise ValueError("the constant-mode step needs every axis periodic and shift > 0")
    return x


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def apply_complex(prob, shift_im, x) -> np.ndarray:
    """y = A x for the complex operator A = A_r + i shift_im I (A_r: the real
    operator of `prob`, its real shift included): Eq. 1 over C, the form of
    the periodic Helmholtz problem of Sec. 3.2 (Eq. 7)."""
    bd = _Bound(prob)
    xc = _c128(x)
    y = np.empty(bd.size, dtype=np.complex128)
    _load().oracle_apply_complex(bd.ref, float(shift_im), _ptr(xc.view(np.float64)), _ptr(y.view(np.float64)))
    return y


def aar_solve_complex(prob, b, shift_im, x0=None, omega=0.6, beta=0.6, m=7, p=6, tol=1e-10,
                      max_iter=1_000_000, trace_cap: int = 0) -> dict:
    """Complex AAR (Eqs. 2-6 over C, T the conjugate transpose) with the
    complex Jacobi preconditioner D = diag(A); omega and beta may be complex.
    Returns x (complex), status, iterations, relres and, with trace_cap > 0,
    trace rows [k, r_k, ||f_k||, ||f_k - F_k gamma_k||, rank, cond]."""
    bd = _Bound(prob)
    bc = _c128(b)
    x = np.zeros(bd.size, dtype=np.complex128) if x0 is None else _c128(x0).copy()
    omega, beta = complex(omega), complex(beta)
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    tl = ctypes.c_int64(0)
    tr = np.zeros((max(trace_cap, 1), 6))
    st = _load().oracle_aar_solve_complex(bd.ref, float(shift_im), _ptr(bc.view(np.float64)),
                                          _ptr(x.view(np.float64)), omega.real, omega.imag, beta.real, beta.imag,
                                          int(m), int(p), float(tol), int(max_iter), ctypes.byref(it),
                                          ctypes.byref(rr), _ptr(tr) if trace_cap > 0 else None, int(trace_cap),
                                          ctypes.byref(tl))
    out = {"x": x, "status": st, "iterations": it.value, "relres": rr.value}
    if trace_cap > 0:
        out["trace"] = tr[: tl.value].copy()
    return out


def relative_residual_complex(prob, shift_im, b, x) -> float:
    """||b - A x|| / ||b|| for the complex operator, from apply_complex."""
    r = _c128(b) - apply_complex(prob, shift_im, x)
    return float(np.linalg.norm(r) / np.linalg.norm(_c128(b)))


def relative_residual(prob, b, x) -> float:
    """||b - A x|| / ||b|| in FP64 with the oracle's own operator (Sec. 2)."""
    bd = _Bound(prob)
    return float(_load().oracle_relative_residual(bd.ref, _ptr(_f64(b)), _ptr(_f64(x))))


# ---- general sparse A (Sec. 3.1; block-Jacobi ILU(0), Secs. 3.2-3.3) ----

PRECOND_JACOBI, PRECOND_ILU0 = 0, 1


class _BoundCsr:
    """A ctypes CSR struct plus the arrays it points into (kept alive).
    `A` is any object with rowptr, col, val arrays (n = len(rowptr) - 1)."""

    def __init__(self, A):
        self.rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(A.col, dtype=np.int32)
        self.val = _f64(A.val)
        s = _Csr()
        s.n = len(self.rowptr) - 1
        s.rowptr = self.rowptr.ctypes.data
        s.col = self.col.ctypes.data
        s.val = self.val.ctypes.data
        self.s = s
        self.n = int(s.n)

    @property
    def ref(self):
        return ctypes.byref(self.s)


def csr_check(A) -> bool:
    """True when A's arrays form a valid CSR matrix (sorted columns in range,
    diagonal present in every row)."""
    return _load().oracle_csr_check(_BoundCsr(A).ref) == OK


def csr_apply(A, x) -> np.ndarray:
    """y = A x for a CSR matrix."""
    bd = _BoundCsr(A)
    x = _f64(x)
    y = np.empty(bd.n)
    _load().oracle_csr_apply(bd.ref, _ptr(x), _ptr(y))
    return y


def ilu0(A, nblocks: int = 1) -> np.ndarray:
    """ILU(0) factors of each of the `nblocks` contiguous diagonal blocks of A
    (block Jacobi with ILU(0) per block; nblocks = 1 is ILU(0) of A), stored in
    A's pattern: strictly lower entries hold L (unit diagonal not stored), the
    others U.  Entries that couple two blocks keep A's values and are unused.
    Raises ZeroDivisionError on a zero or non-finite pivot."""
    bd = _BoundCsr(A)
    lu = np.empty(len(bd.val))
    st = _load().oracle_ilu0(bd.ref, int(nblocks), _ptr(lu))
    if st == BREAKDOWN:
        raise ZeroDivisionError("ILU(0) met a zero or non-finite pivot")
    if st != OK:
        raise ValueError("bad matrix or block count")
    return lu


def ilu0_solve(A, lu, r, nblocks: int = 1) -> np.ndarray:
    """z = (L U)^-1 r block by block for factors from ilu0()."""
    bd = _BoundCsr(A)
    lu = _f64(lu)
    r = _f64(r)
    z = np.empty(bd.n)
    _load().oracle_ilu0_solve(bd.ref, int(nblocks), _ptr(lu), _ptr(r), _ptr(z))
    return z


def precondition(A, r, precond: int = PRECOND_ILU0, nblocks: int = 1) -> np.ndarray:
    """z = M^-1 r for the Jacobi diagonal or block ILU(0) of A."""
    bd = _BoundCsr(A)
    r = _f64(r)
    z = np.empty(bd.n)
    st = _load().oracle_csr_precondition(bd.ref, int(precond), int(nblocks), _ptr(r), _ptr(z))
    if st == BREAKDOWN:
        raise ZeroDivisionError("ILU(0) met a zero or non-finite pivot")
    if st != OK:
        raise ValueError("bad matrix, preconditioner or block count")
    return z


def aar_solve_csr(A, b, x0=None, precond: int = PRECOND_ILU0, nblocks: int = 1, omega=0.6, beta=0.6, m=9, p=8,
                  tol=1e-6, max_iter=1_000_000, trace_cap: int = 0) -> dict:
    """Preconditioned AAR (Eqs. 2-6) for a CSR matrix with the Jacobi or
    block ILU(0) preconditioner; the paper's defaults for its sparse study
    (Sec. 3.1) are omega = beta = 0.6, m = 9, p = 8, tol 1e-6.  Returns the
    same dict as aar_solve."""
    bd = _BoundCsr(A)
    b = _f64(b)
    x = np.zeros(bd.n) if x0 is None else _f64(x0).copy()
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    tl = ctypes.c_int64(0)
    tr = np.zeros((max(trace_cap, 1), 6))
    st = _load().oracle_aar_solve_csr(bd.ref, int(precond), int(nblocks), _ptr(b), _ptr(x), float(omega),
                                      float(beta), int(m), int(p), float(tol), int(max_iter), ctypes.byref(it),
                                      ctypes.byref(rr), _ptr(tr) if trace_cap > 0 else None, int(trace_cap),
                                      ctypes.byref(tl))
    out = {"x": x, "status": st, "iterations": it.value, "relres": rr.value}
    if trace_cap > 0:
        out["trace"] = tr[: tl.value].copy()
    return out


def relative_residual_csr(A, b, x) -> float:
    """||b - A x|| / ||b|| for a CSR matrix."""
    bd = _BoundCsr(A)
    return float(_load().oracle_relative_residual_csr(bd.ref, _ptr(_f64(b)), _ptr(_f64(x))))


def threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(_load().oracle_threads())


def solve_workload_params(params) -> dict:
    """Keyword arguments of aar_solve taken from an inputs.Params."""
    return dict(omega=params.omega, beta=params.beta, m=params.m, p=params.p, tol=params.tol,
                max_iter=params.max_iter)


__all__ = ["build", "fd_weights", "apply", "diagonal", "jacobi_eigen", "pinv_solve", "aar_solve",
           "relative_residual", "threads", "solve_workload_params", "csr_check", "csr_apply", "ilu0",
           "ilu0_solve", "precondition", "aar_solve_csr", "relative_residual_csr", "PRECOND_JACOBI", "PRECOND_ILU0",
           "OK", "NOT_CONVERGED", "BREAKDOWN", "BAD_ARG"]

