"""ctypes binding of the HIP AAR solver library (C ABI in include/aar.h).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  Functions carry the C names (aar_create, aar_solve, ...);
:class:`Solver` wraps a handle for torch tensors on the GPU.  PyTorch
supplies device memory and the stream; it is imported before the library is
loaded so both share one HIP runtime.  The library must have been built
(``python -m paper_1606_08740_amd.build``): there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libaar_hip.so")
HEADER = os.path.join(ROOT, "include", "aar.h")

AAR_OK, AAR_NOT_CONVERGED, AAR_BREAKDOWN = 0, 1, 2
AAR_ERR_INVALID_ARG, AAR_ERR_UNSUPPORTED, AAR_ERR_DEVICE, AAR_ERR_OUT_OF_MEMORY = -1, -2, -3, -4
AAR_BC_ZERO_DIRICHLET, AAR_BC_PERIODIC = 0, 1
AAR_FP64, AAR_MIXED_FP32, AAR_MIXED_FP32_BF16HIST, AAR_FP64_FP32HIST, AAR_FP64_BF16HIST = 0, 1, 2, 3, 4
AAR_FLAG_RECORD_RESIDUALS, AAR_FLAG_DEFLATE_CONSTANT, AAR_FLAG_NO_GRAPH, AAR_FLAG_NO_AUTOTUNE = 1, 2, 4, 8
AAR_FLAG_FORCE_PINV, AAR_FLAG_RECYCLE_HISTORY = 16, 32
AAR_PRECOND_JACOBI, AAR_PRECOND_ILU0 = 0, 1

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "BREAKDOWN", -1: "INVALID_ARG", -2: "UNSUPPORTED",
                -3: "DEVICE", -4: "OUT_OF_MEMORY"}


class aar_problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3), ("bc", ctypes.c_int32 * 3),
                ("radius", ctypes.c_int32), ("diffusion", ctypes.c_double), ("shift", ctypes.c_double),
                ("velocity", ctypes.c_void_p)]


class aar_params(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("beta", ctypes.c_double), ("m", ctypes.c_int32),
                ("p", ctypes.c_int32), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class aar_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int64),
                ("outer_steps", ctypes.c_int32), ("rel_residual", ctypes.c_double)]


_lib = None


def header_functions() -> list:
    """Names of the functions include/aar.h declares."""
    text = open(HEADER).read()
    return re.findall(r"^(?:aar_status|const char \*)\s*(aar_\w+)\s*\(", text, flags=re.M)


def load_library():
    """Load libaar_hip.so (after torch, so both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP solver library not built: {LIB_PATH} is missing "
                           "(run python -m paper_1606_08740_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i32, i64, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int
    lib.aar_create.argtypes = [P(vp), P(aar_problem), i32, P(aar_params), vp]
    lib.aar_solve.argtypes = [vp, vp, vp, P(aar_result)]
    lib.aar_solve_batched.argtypes = [vp, vp, vp, P(i64), P(aar_result)]
    lib.aar_apply.argtypes = [vp, i32, vp, vp]
    lib.aar_residual_log.argtypes = [vp, i32, P(ctypes.c_double), i64, P(i64)]
    lib.aar_rank_log.argtypes = [vp, i32, P(i32), i64, P(i64)]
    lib.aar_solve_noalloc.argtypes = [P(aar_problem), P(aar_params), vp, vp, P(aar_result), vp]
    d = ctypes.c_double
    lib.aar_create_complex.argtypes = [P(vp), P(aar_problem), P(aar_params), d, d, d, vp]
    lib.aar_select_parameters.argtypes = [P(aar_problem), P(aar_params), vp, P(d), i32, P(i32), i32, i64, vp,
                                          P(d), P(i32), P(d)]
    lib.aar_create_csr.argtypes = [P(vp), i64, vp, vp, vp, i32, i32, P(aar_params), vp]
    lib.aar_precondition.argtypes = [vp, vp, vp]
    lib.aar_workspace_bytes.argtypes = [P(aar_problem), i32, P(aar_params), P(ctypes.c_size_t)]
    lib.aar_destroy.argtypes = [vp]
    lib.aar_last_error.argtypes = []
    lib.aar_last_error.restype = ctypes.c_char_p
    lib.aar_set_timing.argtypes = [vp, i32]
    lib.aar_sweep_time.argtypes = [vp, P(ctypes.c_double), P(i64)]
    for name in ["aar_create", "aar_solve", "aar_solve_batched", "aar_apply", "aar_residual_log",
                 "aar_rank_log", "aar_solve_noalloc", "aar_create_complex", "aar_create_csr", "aar_precondition",
                 "aar_select_parameters", "aar_workspace_bytes", "aar_destroy", "aar_set_timing", "aar_sweep_time"]:
        getattr(lib, name).restype = st
    _lib = lib
    return lib


class AarError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = load_library().aar_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def _check(status: int, where: str) -> int:
    if status < 0:
        raise AarError(status, where)
    return status


# ---------------------------------------------------------------------------
# C-named entry points (marshalling only)
# ---------------------------------------------------------------------------
def aar_create(problems, params, hip_stream: int = 0):
    lib = load_library()
    arr = (aar_problem * len(problems))(*problems)
    h = ctypes.c_void_p()
    _check(lib.aar_create(ctypes.byref(h), arr, len(problems), ctypes.byref(params),
                          ctypes.c_void_p(hip_stream)), "aar_create")
    return h


def aar_create_complex(problem, params, shift_imag: float, omega_imag: float = 0.0, beta_imag: float = 0.0,
                       hip_stream: int = 0):
    h = ctypes.c_void_p()
    _check(load_library().aar_create_complex(ctypes.byref(h), ctypes.byref(problem), ctypes.byref(params),
                                             float(shift_imag), float(omega_imag), float(beta_imag),
                                             ctypes.c_void_p(hip_stream)), "aar_create_complex")
    return h


def aar_create_csr(rowptr, col, val, preconditioner: int, nblocks: int, params, hip_stream: int = 0):
    """rowptr (int64), col (int32), val (float64): host numpy arrays."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(load_library().aar_create_csr(ctypes.byref(h), len(rowptr) - 1, rowptr.ctypes.data, col.ctypes.data,
                                         val.ctypes.data, int(preconditioner), int(nblocks), ctypes.byref(params),
                                         ctypes.c_void_p(hip_stream)), "aar_create_csr")
    return h


def aar_precondition(handle, r_ptr: int, z_ptr: int) -> None:
    _check(load_library().aar_precondition(handle, ctypes.c_void_p(r_ptr), ctypes.c_void_p(z_ptr)),
           "aar_precondition")


def aar_select_parameters(problem, params, b_ptr: int, betas, ps, trial_iterations: int, hip_stream: int = 0):
    """Returns (beta, p, scores[len(ps)][len(betas)])."""
    nb, npp = len(betas), len(ps)
    bet = (ctypes.c_double * nb)(*[float(v) for v in betas])
    pp = (ctypes.c_int32 * npp)(*[int(v) for v in ps])
    sc = (ctypes.c_double * (nb * npp))()
    bo, po = ctypes.c_double(0.0), ctypes.c_int32(0)
    _check(load_library().aar_select_parameters(ctypes.byref(problem), ctypes.byref(params), ctypes.c_void_p(b_ptr),
                                                bet, nb, pp, npp, int(trial_iterations), ctypes.c_void_p(hip_stream),
                                                ctypes.byref(bo), ctypes.byref(po), sc), "aar_select_parameters")
    return bo.value, po.value, np.array(list(sc)).reshape(npp, nb)


def aar_solve(handle, b_ptr: int, x_ptr: int) -> aar_result:
    r = aar_result()
    _check(load_library().aar_solve(handle, ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_ptr),
                                    ctypes.byref(r)), "aar_solve")
    return r


def aar_solve_batched(handle, b_ptr: int, x_ptr: int, offsets, count: int) -> list:
    offs = (ctypes.c_int64 * (count + 1))(*[int(v) for v in offsets])
    res = (aar_result * count)()
    _check(load_library().aar_solve_batched(handle, ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_ptr),
                                            offs, res), "aar_solve_batched")
    return list(res)


def aar_solve_noalloc(problem: aar_problem, params: aar_params, b_ptr: int, x_ptr: int,
                      hip_stream: int = 0) -> aar_result:
    r = aar_result()
    _check(load_library().aar_solve_noalloc(ctypes.byref(problem), ctypes.byref(params), ctypes.c_void_p(b_ptr),
                                            ctypes.c_void_p(x_ptr), ctypes.byref(r), ctypes.c_void_p(hip_stream)),
           "aar_solve_noalloc")
    return r


def aar_apply(handle, instance: int, x_ptr: int, y_ptr: int) -> None:
    _check(load_library().aar_apply(handle, int(instance), ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr)),
           "aar_apply")


def aar_residual_log(handle, instance: int = 0, cap: int = 1 << 20) -> np.ndarray:
    out = np.zeros(max(cap, 1))
    cnt = ctypes.c_int64(0)
    _check(load_library().aar_residual_log(handle, int(instance),
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           int(cap), ctypes.byref(cnt)), "aar_residual_log")
    return out[: min(cnt.value, cap)].copy()


def aar_rank_log(handle, instance: int = 0, cap: int = 1 << 20) -> np.ndarray:
    out = np.zeros(max(cap, 1), dtype=np.int32)
    cnt = ctypes.c_int64(0)
    _check(load_library().aar_rank_log(handle, int(instance),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       int(cap), ctypes.byref(cnt)), "aar_rank_log")
    return out[: min(cnt.value, cap)].copy()


def aar_workspace_bytes(problems, params) -> int:
    arr = (aar_problem * len(problems))(*problems)
    n = ctypes.c_size_t(0)
    _check(load_library().aar_workspace_bytes(arr, len(problems), ctypes.byref(params), ctypes.byref(n)),
           "aar_workspace_bytes")
    return int(n.value)


def aar_destroy(handle) -> None:
    if handle:
        _check(load_library().aar_destroy(handle), "aar_destroy")


def aar_last_error() -> str:
    return load_library().aar_last_error().decode(errors="replace")


def aar_set_timing(handle, enable: bool) -> None:
    _check(load_library().aar_set_timing(handle, 1 if enable else 0), "aar_set_timing")


def aar_sweep_time(handle) -> tuple:
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(load_library().aar_sweep_time(handle, ctypes.byref(ms), ctypes.byref(n)), "aar_sweep_time")
    return ms.value, n.value


# ---------------------------------------------------------------------------
# Convenience wrapper for torch tensors
# ---------------------------------------------------------------------------
def make_problem(prob, velocity_ptr: int = 0) -> aar_problem:
    s = aar_problem()
    s.n = (ctypes.c_int32 * 3)(*[int(v) for v in prob.n])
    s.h = (ctypes.c_double * 3)(*[float(v) for v in prob.h])
    s.bc = (ctypes.c_int32 * 3)(*[int(v) for v in prob.bc])
    s.radius = int(prob.radius)
    s.diffusion = float(prob.diffusion)
    s.shift = float(prob.shift)
    s.velocity = velocity_ptr or None
    return s


def make_params(params) -> aar_params:
    s = aar_params()
    s.omega = float(params.omega)
    s.beta = float(params.beta)
    s.m = int(params.m)
    s.p = int(params.p)
    s.tol = float(params.tol)
    s.max_iter = int(params.max_iter)
    s.precision = int(params.precision)
    s.inner_tol = float(params.inner_tol)
    s.max_outer = int(params.max_outer)
    s.flags = int(params.flags)
    return s


def result_dict(r: aar_result) -> dict:
    return {"status": int(r.status), "iterations": int(r.iterations), "rel_residual": float(r.rel_residual),
            "outer_steps": int(r.outer_steps)}


class Solver:
    """A solver handle for one or more systems (inputs.Problem) sharing params.

    Velocities (numpy) are uploaded for creation only; the library copies
    them.  Vectors are float64 CUDA tensors of each system's size.
    """

    def __init__(self, problems, params, device=None, stream=None):
        import torch
        load_library()
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.device = torch.device(device or "cuda:0")
        self.problems = list(problems)
        self.params = params
        self.stream = stream or torch.cuda.current_stream(self.device)
        vel_tensors = []
        structs = []
        for prob in self.problems:
            vptr = 0
            if prob.velocity is not None:
                v = torch.as_tensor(np.ascontiguousarray(prob.velocity, dtype=np.float64), device=self.device)
                vel_tensors.append(v)
                vptr = v.data_ptr()
            structs.append(make_problem(prob, vptr))
        with torch.cuda.device(self.device):
            self.handle = aar_create(structs, make_params(params), self.stream.cuda_stream)
        self.sizes = [p.size for p in self.problems]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        del vel_tensors

    def solve(self, b, x) -> dict:
        self._check_vec(b, self.sizes[0])
        self._check_vec(x, self.sizes[0])
        return result_dict(aar_solve(self.handle, b.data_ptr(), x.data_ptr()))

    def solve_batched(self, b, x) -> list:
        total = int(self.offsets[-1])
        self._check_vec(b, total)
        self._check_vec(x, total)
        res = aar_solve_batched(self.handle, b.data_ptr(), x.data_ptr(), self.offsets, len(self.sizes))
        return [result_dict(r) for r in res]

    def apply(self, x, instance: int = 0):
        import torch
        self._check_vec(x, self.sizes[instance])
        y = torch.empty_like(x)
        aar_apply(self.handle, instance, x.data_ptr(), y.data_ptr())
        return y

    def residual_log(self, instance: int = 0) -> np.ndarray:
        return aar_residual_log(self.handle, instance)

    def rank_log(self, instance: int = 0) -> np.ndarray:
        return aar_rank_log(self.handle, instance)

    def set_timing(self, enable: bool) -> None:
        aar_set_timing(self.handle, enable)

    def sweep_time(self) -> tuple:
        return aar_sweep_time(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            aar_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_vec(self, t, n):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.numel() == n):
            raise ValueError(f"expected a contiguous float64 CUDA tensor of {n} elements")


class ComplexSolver:
    """A solver handle for one complex-valued system (aar_create_complex):
    A = A_r + i shift_imag I with A_r the real operator of `problem`; omega and
    beta may be complex.  Vectors are complex128 CUDA tensors (interleaved
    re, im in memory)."""

    def __init__(self, problem, params, shift_imag, omega=None, beta=None, device=None, stream=None):
        import torch
        load_library()
        self.device = torch.device(device or "cuda:0")
        self.problem = problem
        self.params = params
        self.stream = stream or torch.cuda.current_stream(self.device)
        omega = complex(params.omega if omega is None else omega)
        beta = complex(params.beta if beta is None else beta)
        pm = make_params(params)
        pm.omega, pm.beta = omega.real, beta.real
        with torch.cuda.device(self.device):
            self.handle = aar_create_complex(make_problem(problem), pm, shift_imag, omega.imag, beta.imag,
                                             self.stream.cuda_stream)
        self.size = problem.size

    def solve(self, b, x) -> dict:
        self._check_vec(b)
        self._check_vec(x)
        return result_dict(aar_solve(self.handle, b.data_ptr(), x.data_ptr()))

    def apply(self, x):
        import torch
        self._check_vec(x)
        y = torch.empty_like(x)
        aar_apply(self.handle, 0, x.data_ptr(), y.data_ptr())
        return y

    def residual_log(self) -> np.ndarray:
        return aar_residual_log(self.handle, 0)

    def rank_log(self) -> np.ndarray:
        return aar_rank_log(self.handle, 0)

    def close(self) -> None:
        if getattr(self, "handle", None):
            aar_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_vec(self, t):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
                and t.numel() == self.size):
            raise ValueError(f"expected a contiguous complex128 CUDA tensor of {self.size} elements")


class CsrSolver:
    """A solver handle for one general sparse system (aar_create_csr): A in
    compressed sparse rows (any object with rowptr, col, val arrays), the
    Jacobi (AAR_PRECOND_JACOBI) or block ILU(0) (AAR_PRECOND_ILU0, `nblocks`
    contiguous row blocks) preconditioner.  Vectors are float64 CUDA tensors of
    n elements."""

    def __init__(self, A, params, preconditioner=AAR_PRECOND_ILU0, nblocks=1, device=None, stream=None):
        import torch
        load_library()
        self.device = torch.device(device or "cuda:0")
        self.params = params
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.size = len(A.rowptr) - 1
        with torch.cuda.device(self.device):
            self.handle = aar_create_csr(A.rowptr, A.col, A.val, preconditioner, nblocks, make_params(params),
                                         self.stream.cuda_stream)

    def solve(self, b, x) -> dict:
        self._check_vec(b)
        self._check_vec(x)
        return result_dict(aar_solve(self.handle, b.data_ptr(), x.data_ptr()))

    def apply(self, x):
        import torch
        self._check_vec(x)
        y = torch.empty_like(x)
        aar_apply(self.handle, 0, x.data_ptr(), y.data_ptr())
        return y

    def precondition(self, r):
        import torch
        self._check_vec(r)
        z = torch.empty_like(r)
        aar_precondition(self.handle, r.data_ptr(), z.data_ptr())
        return z

    def residual_log(self) -> np.ndarray:
        return aar_residual_log(self.handle, 0)

    def rank_log(self) -> np.ndarray:
        return aar_rank_log(self.handle, 0)

    def set_timing(self, enable: bool) -> None:
        aar_set_timing(self.handle, enable)

    def sweep_time(self) -> tuple:
        return aar_sweep_time(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            aar_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_vec(self, t):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.numel() == self.size):
            raise ValueError(f"expected a contiguous float64 CUDA tensor of {self.size} elements")
