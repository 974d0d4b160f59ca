"""Python binding of libmscg (the recursive multi-scale PCG on MI355X).

Argument marshalling only: every computation runs in the HIP kernels of
libmscg.so.  PyTorch supplies device memory (tensors) and the stream.  There is
no fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmscg.so")
MAX_LEVELS = 8

OK, NOT_CONVERGED = 0, 1
E_ARG, E_NOMEM, E_DEVICE, E_BREAKDOWN, E_STATE, E_SINGULAR = -1, -2, -3, -4, -5, -6
NEUMANN, DIRICHLET = 0, 1
FP64, MIXED = 0, 1
SPLIT_SGS, SPLIT_JACOBI = 0, 1
CYCLE_RECURSIVE, CYCLE_MGCG, CYCLE_POLY = 0, 1, 2
INTERP_LINEAR, INTERP_CONSTANT = 0, 1

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "E_ARG", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_BREAKDOWN",
                -5: "E_STATE", -6: "E_SINGULAR"}


class MscgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("length", ctypes.c_double * 3),
                ("bc_type", ctypes.c_int * 6), ("bc_value", ctypes.c_double * 6)]


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("scale", ctypes.c_int), ("smooth_steps", ctypes.c_int),
                ("level_factor", ctypes.c_double), ("min_coarse_side", ctypes.c_int), ("max_levels", ctypes.c_int),
                ("max_outer_iters", ctypes.c_int), ("max_inner_iters", ctypes.c_int), ("interp", ctypes.c_int),
                ("flexible", ctypes.c_int), ("inner_rel_floor", ctypes.c_double), ("semi_coarsen", ctypes.c_int),
                ("axis_weight", ctypes.c_double * 3), ("splitting", ctypes.c_int), ("cycle", ctypes.c_int),
                ("frac_scale", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("outer_iters", ctypes.c_int), ("n_levels", ctypes.c_int),
                ("level_n", (ctypes.c_int * 3) * MAX_LEVELS), ("level_iters", ctypes.c_longlong * MAX_LEVELS),
                ("level_calls", ctypes.c_longlong * MAX_LEVELS), ("rel_residual_true", ctypes.c_double),
                ("b_norm", ctypes.c_double), ("solve_ms", ctypes.c_double)]


EXPORTS = [
    "mscg_default_options", "mscg_footprint_bytes", "mscg_create_problem", "mscg_set_permeability", "mscg_solve",
    "mscg_solve_batch", "mscg_destroy_problem", "mscg_last_error", "mscg_level_info", "mscg_get_transmissibility",
    "mscg_apply_operator", "mscg_apply_smoother", "mscg_restrict_residual", "mscg_prolong_add",
    "mscg_apply_preconditioner", "mscg_time_kernel", "mscg_enable_kernel_timing", "mscg_small_level_timing",
]
(KERNEL_SMOOTH_HALF, KERNEL_SPMV, KERNEL_RESTRICT, KERNEL_PROLONG, KERNEL_CG_UPDATE, KERNEL_SMOOTH_PRE,
 KERNEL_SMOOTH_POST) = range(7)

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libmscg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -m paper_math_9809043_amd.build_lib)")
    L = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    L.mscg_default_options.argtypes = [ctypes.POINTER(_Options)]
    L.mscg_default_options.restype = None
    L.mscg_footprint_bytes.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Options)]
    L.mscg_footprint_bytes.restype = ctypes.c_size_t
    L.mscg_create_problem.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Options), vp, ctypes.c_size_t, vp,
                                      ctypes.POINTER(vp)]
    L.mscg_create_problem.restype = ctypes.c_int
    L.mscg_set_permeability.argtypes = [vp, vp, vp, vp]
    L.mscg_set_permeability.restype = ctypes.c_int
    L.mscg_solve.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(_Stats)]
    L.mscg_solve.restype = ctypes.c_int
    L.mscg_solve_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), dp, ctypes.c_int,
                                   ctypes.POINTER(_Stats)]
    L.mscg_solve_batch.restype = ctypes.c_int
    L.mscg_destroy_problem.argtypes = [vp]
    L.mscg_destroy_problem.restype = ctypes.c_int
    L.mscg_last_error.argtypes = []
    L.mscg_last_error.restype = ctypes.c_char_p
    L.mscg_level_info.argtypes = [vp, ctypes.c_int, ip]
    L.mscg_level_info.restype = ctypes.c_int
    L.mscg_get_transmissibility.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.mscg_get_transmissibility.restype = ctypes.c_int
    L.mscg_apply_operator.argtypes = [vp, ctypes.c_int, vp, vp]
    L.mscg_apply_operator.restype = ctypes.c_int
    L.mscg_apply_smoother.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int]
    L.mscg_apply_smoother.restype = ctypes.c_int
    L.mscg_restrict_residual.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.mscg_restrict_residual.restype = ctypes.c_int
    L.mscg_prolong_add.argtypes = [vp, ctypes.c_int, vp, vp]
    L.mscg_prolong_add.restype = ctypes.c_int
    L.mscg_apply_preconditioner.argtypes = [vp, vp, vp, ctypes.c_double]
    L.mscg_apply_preconditioner.restype = ctypes.c_int
    L.mscg_time_kernel.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
    L.mscg_time_kernel.restype = ctypes.c_int
    L.mscg_enable_kernel_timing.argtypes = [vp, ctypes.c_int]
    L.mscg_enable_kernel_timing.restype = ctypes.c_int
    L.mscg_small_level_timing.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong),
                                          dp]
    L.mscg_small_level_timing.restype = ctypes.c_int
    _lib = L
    return L


def last_error() -> str:
    return load_library().mscg_last_error().decode()


def _check(code: int, allow=(OK,)):
    if code not in allow:
        raise MscgError(code, last_error())
    return code


@dataclass
class Grid:
    dim: int
    n: tuple
    bc_type: list = field(default_factory=lambda: [DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, NEUMANN, NEUMANN])
    bc_value: list = field(default_factory=lambda: [0.0, 1.0, 0.0, 0.0, 0.0, 0.0])
    length: tuple = (1.0, 1.0, 1.0)

    def _c(self) -> _Grid:
        g = _Grid()
        g.dim = self.dim
        n = tuple(self.n) + (1,) * (3 - len(self.n))
        for a in range(3):
            g.n[a] = int(n[a])
            g.length[a] = float(self.length[a])
        for f in range(6):
            g.bc_type[f] = int(self.bc_type[f])
            g.bc_value[f] = float(self.bc_value[f])
        return g

    @property
    def N(self) -> int:
        n = tuple(self.n) + (1,) * (3 - len(self.n))
        return int(n[0] * n[1] * (n[2] if self.dim == 3 else 1))


@dataclass
class Options:
    precision: int = FP64
    scale: int = 4
    smooth_steps: int = 0
    level_factor: float = 0.1
    min_coarse_side: int = 8
    max_levels: int = MAX_LEVELS
    max_outer_iters: int = 200
    max_inner_iters: int = 200
    interp: int = INTERP_LINEAR
    flexible: int = 0
    inner_rel_floor: float = 1e-6
    semi_coarsen: int = 0
    axis_weight: tuple = (1.0, 1.0, 1.0)
    splitting: int = 0  # SPLIT_SGS or SPLIT_JACOBI
    cycle: int = 0  # CYCLE_RECURSIVE (eq. 2.10), CYCLE_MGCG (eq. 2.9) or CYCLE_POLY (Section 2.1)
    frac_scale: float = 0.0  # > 1: coarsening factor that need not be an integer (Section 3)

    def _c(self) -> _Options:
        o = _Options()
        for name, _ in _Options._fields_:
            if name == "axis_weight":
                for a in range(3):
                    o.axis_weight[a] = float(self.axis_weight[a])
            else:
                setattr(o, name, getattr(self, name))
        if o.smooth_steps <= 0:
            o.smooth_steps = o.scale
        return o


@dataclass
class Stats:
    status: int
    outer_iters: int
    n_levels: int
    level_n: list
    level_iters: list
    level_calls: list
    rel_residual_true: float
    b_norm: float
    solve_ms: float

    @staticmethod
    def _from(s: _Stats) -> "Stats":
        nl = s.n_levels
        return Stats(status=s.status, outer_iters=s.outer_iters, n_levels=nl,
                     level_n=[tuple(s.level_n[l]) for l in range(nl)],
                     level_iters=[int(s.level_iters[l]) for l in range(nl)],
                     level_calls=[int(s.level_calls[l]) for l in range(nl)],
                     rel_residual_true=s.rel_residual_true, b_norm=s.b_norm, solve_ms=s.solve_ms)


def _ptr(t):
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _f64(t):
    import torch
    if t.dtype != torch.float64:
        raise ValueError("expected a float64 tensor")
    return _ptr(t)


def footprint_bytes(grid: Grid, options: Options | None = None) -> int:
    L = load_library()
    o = (options or Options())._c()
    g = grid._c()
    b = L.mscg_footprint_bytes(ctypes.byref(g), ctypes.byref(o))
    if b == 0:
        raise MscgError(E_ARG, last_error())
    return int(b)


class Problem:
    """A grid + options + device workspace (a torch uint8 tensor) + stream."""

    def __init__(self, grid: Grid, options: Options | None = None, stream=None, device=None):
        import torch
        self.grid = grid
        self.options = options or Options()
        L = load_library()
        self._L = L
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        nbytes = footprint_bytes(grid, self.options)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        g = grid._c()
        o = self.options._c()
        with torch.cuda.device(dev):
            _check(L.mscg_create_problem(ctypes.byref(g), ctypes.byref(o), ctypes.c_void_p(aligned), nbytes,
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.n_levels = L.mscg_level_info(h, 0, None)

    def close(self):
        if getattr(self, "_h", None):
            self._L.mscg_destroy_problem(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_dims(self, level: int) -> tuple:
        d = (ctypes.c_int * 3)()
        _check(self._L.mscg_level_info(self._h, level, d), allow=tuple(range(1, MAX_LEVELS + 1)))
        return tuple(d)

    def set_permeability(self, kx, ky=None, kz=None):
        _check(self._L.mscg_set_permeability(self._h, _f64(kx), _f64(ky) if ky is not None else None,
                                             _f64(kz) if kz is not None else None))

    def solve(self, f, p, tol: float, use_x0: bool = False) -> Stats:
        st = _Stats()
        rc = self._L.mscg_solve(self._h, _f64(f), _f64(p), float(tol), int(use_x0), ctypes.byref(st))
        if rc < 0 and st.n_levels == 0:
            raise MscgError(rc, last_error())
        return Stats._from(st)

    def transmissibility(self, level: int):
        import torch
        nx, ny, nz = self.level_dims(level)
        tx = torch.empty((nx + 1) * ny * nz, dtype=torch.float64, device=self.device)
        ty = torch.empty(nx * (ny + 1) * nz, dtype=torch.float64, device=self.device)
        tz = torch.empty(nx * ny * (nz + 1), dtype=torch.float64, device=self.device) if self.grid.dim == 3 else None
        _check(self._L.mscg_get_transmissibility(self._h, level, _ptr(tx), _ptr(ty), _ptr(tz)))
        return tx, ty, tz

    def apply_operator(self, level: int, x, y):
        _check(self._L.mscg_apply_operator(self._h, level, _f64(x), _f64(y)))

    def apply_smoother(self, level: int, r, x, steps: int):
        _check(self._L.mscg_apply_smoother(self._h, level, _f64(r), _f64(x), int(steps)))

    def restrict_residual(self, level: int, r, x, g):
        _check(self._L.mscg_restrict_residual(self._h, level, _f64(r), _f64(x) if x is not None else None, _f64(g)))

    def prolong_add(self, level: int, y, x):
        _check(self._L.mscg_prolong_add(self._h, level, _f64(y), _f64(x)))

    def time_kernel(self, kernel: int, level: int = 0, reps: int = 20):
        """(average microseconds per launch, algorithmic bytes per launch)."""
        us, b = ctypes.c_double(), ctypes.c_double()
        _check(self._L.mscg_time_kernel(self._h, kernel, level, reps, ctypes.byref(us), ctypes.byref(b)))
        return us.value, b.value

    def enable_kernel_timing(self, on: bool = True):
        """Brackets each launch of the one-workgroup last-inner-level solver with
        HIP events in the following solves (clears the totals)."""
        _check(self._L.mscg_enable_kernel_timing(self._h, 1 if on else 0))

    def small_level_timing(self) -> dict:
        """Totals since enable_kernel_timing: ms, launches, iterations, FP64 flops."""
        ms, fl = ctypes.c_double(), ctypes.c_double()
        nl, it = ctypes.c_longlong(), ctypes.c_longlong()
        _check(self._L.mscg_small_level_timing(self._h, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(it),
                                               ctypes.byref(fl)))
        return {"total_ms": ms.value, "launches": nl.value, "iterations": it.value, "flops": fl.value}

    def apply_preconditioner(self, r, z, eps2: float = 0.0):
        _check(self._L.mscg_apply_preconditioner(self._h, _f64(r), _f64(z), float(eps2)), allow=(OK, E_BREAKDOWN))


def solve_batch(problems, fs, ps, tols) -> list:
    L = load_library()
    n = len(problems)
    H = (ctypes.c_void_p * n)(*[p._h for p in problems])
    F = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
    P = (ctypes.c_void_p * n)(*[p.data_ptr() for p in ps])
    T = (ctypes.c_double * n)(*[float(t) for t in tols])
    S = (_Stats * n)()
    L.mscg_solve_batch(H, F, P, T, n, S)
    return [Stats._from(S[i]) for i in range(n)]
