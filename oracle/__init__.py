"""CPU oracle for the recursive multi-scale PCG -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library never loads it.

`mscg_oracle.c` is a plain FP64 C implementation of the method, built here with
gcc into `liboracle.so` next to this file; this module is a thin ctypes
wrapper around it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mscg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAX_LEVELS = 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, serial)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class _Stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("outer_iters", ctypes.c_int),
        ("nlev", ctypes.c_int),
        ("level_n", (ctypes.c_int * 3) * MAX_LEVELS),
        ("level_iters", ctypes.c_longlong * MAX_LEVELS),
        ("level_calls", ctypes.c_longlong * MAX_LEVELS),
        ("rel_residual_true", ctypes.c_double),
        ("b_norm", ctypes.c_double),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_solve.argtypes = [ctypes.c_int, ip, dp, dp, dp, dp, dp, ip, dp, ctypes.c_double, ip, dp, dp,
                                   ctypes.POINTER(_Stats), dp]
        L.oracle_solve.restype = ctypes.c_int
        L.oracle_level_plan.argtypes = [ctypes.c_int, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip]
        L.oracle_level_plan.restype = ctypes.c_int
        L.oracle_level_plan_semi.argtypes = [ctypes.c_int, ip, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip]
        L.oracle_level_plan_semi.restype = ctypes.c_int
        L.oracle_face_T.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double] * 3 + [dp, dp, dp, ip, dp, dp, dp]
        L.oracle_face_T.restype = None
        L.oracle_coarsen_T.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp, dp, dp, dp]
        L.oracle_coarsen_T.restype = None
        L.oracle_apply_A.argtypes = [ctypes.c_int] * 4 + [dp, dp, dp, dp, dp]
        L.oracle_apply_A.restype = None
        L.oracle_sgs.argtypes = [ctypes.c_int] * 4 + [dp, dp, dp, dp, dp, ctypes.c_int]
        L.oracle_sgs.restype = None
        L.oracle_gs_colour.argtypes = [ctypes.c_int] * 4 + [dp, dp, dp, dp, dp, ctypes.c_int]
        L.oracle_gs_colour.restype = None
        L.oracle_mjac.argtypes = [ctypes.c_int] * 4 + [dp, dp, dp, dp, dp, ctypes.c_int]
        L.oracle_mjac.restype = None
        L.oracle_prolong_add.argtypes = [ctypes.c_int, ip, ip, ctypes.c_int, dp, dp]
        L.oracle_prolong_add.restype = None
        L.oracle_restrict.argtypes = [ctypes.c_int, ip, ip, ctypes.c_int, dp, dp]
        L.oracle_restrict.restype = None
        L.oracle_cholesky.argtypes = [ctypes.c_int, dp, dp]
        L.oracle_cholesky.restype = ctypes.c_int
        L.oracle_cholesky_solve.argtypes = [ctypes.c_int, dp, dp, dp]
        L.oracle_cholesky_solve.restype = None
        L.oracle_precond.argtypes = [ctypes.c_int, ip, dp, dp, dp, dp, ip, ip, ctypes.c_double, ctypes.c_double,
                                     dp, dp, dp]
        L.oracle_precond.restype = ctypes.c_int
        L.oracle_hierarchy_T.argtypes = [ctypes.c_int, ip, dp, dp, dp, dp, ip, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, dp, ctypes.c_size_t, dp]
        L.oracle_hierarchy_T.restype = ctypes.c_int
        L.oracle_prolong_add_dims.argtypes = [ctypes.c_int, ip, ip, ctypes.c_int, dp, dp]
        L.oracle_prolong_add_dims.restype = None
        L.oracle_restrict_dims.argtypes = [ctypes.c_int, ip, ip, ctypes.c_int, dp, dp]
        L.oracle_restrict_dims.restype = None
        L.oracle_set_frac_scale.argtypes = [ctypes.c_double]
        L.oracle_set_frac_scale.restype = None
        L.oracle_level_plan_frac.argtypes = [ctypes.c_int, ip, ctypes.c_double, ctypes.c_int, ctypes.c_int, ip]
        L.oracle_level_plan_frac.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(v):
    a = (ctypes.c_int * len(v))(*[int(x) for x in v])
    return ctypes.cast(a, ctypes.POINTER(ctypes.c_int)), a


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Result:
    p: np.ndarray
    status: int
    outer_iters: int
    nlev: int
    level_n: list
    level_iters: list
    level_calls: list
    rel_residual_true: float
    b_norm: float


LINEAR = 0
CONSTANT = 1


SGS = 0
JACOBI = 1


RECURSIVE = 0  # recursive multi-scale PCG (eq. 2.10)
MGCG = 1       # Tatebe's multigrid preconditioner (eq. 2.9)
POLY = 2       # polynomial preconditioner (Section 2.1, W = P^-1)


def _opts(scale=4, min_side=8, m=0, max_outer=200, max_inner=200, max_levels=MAX_LEVELS, interp=LINEAR,
          splitting=SGS, cycle=RECURSIVE):
    return [scale, min_side, m, max_outer, max_inner, max_levels, interp, splitting, cycle]


def _axis_w(axis_weight):
    return None if axis_weight is None else np.ascontiguousarray(axis_weight, dtype=np.float64)


def solve_arrays(dim, n, kx, ky, kz, f, bc_type, bc_value, tol, length=(1.0, 1.0, 1.0), flvl=0.1,
                 axis_weight=None, frac_scale=0.0, **opt) -> Result:
    """Solve -div(K grad p) = f with the oracle's recursive multi-scale PCG.  axis_weight:
    per-axis permeability scale for the aspect-ratio-aware level plan (None: uniform plan)."""
    L = lib()
    aw = _axis_w(axis_weight)
    nx, ny, nz = n
    N = nx * ny * (nz if dim == 3 else 1)
    kx = _f64(kx)
    ky = _f64(ky if ky is not None else kx)
    kz = _f64(kz if (kz is not None or dim != 3) else kx)
    f = _f64(f)
    assert kx.size == N and ky.size == N and f.size == N
    p = np.zeros(N)
    st = _Stats()
    npt, _a = _i(n)
    bct, _b = _i(bc_type)
    opt_p, _c = _i(_opts(**opt))
    bcv = np.asarray(bc_value, dtype=np.float64)
    Ld = np.asarray(length, dtype=np.float64)
    fl = np.array([flvl])
    L.oracle_set_frac_scale(float(frac_scale))
    try:
        L.oracle_solve(dim, npt, _d(Ld), _d(kx), _d(ky), _d(kz), _d(f), bct, _d(bcv), float(tol), opt_p, _d(fl),
                       _d(p), ctypes.byref(st), _d(aw))
    finally:
        L.oracle_set_frac_scale(0.0)
    nl = st.nlev
    return Result(p=p, status=st.status, outer_iters=st.outer_iters, nlev=nl,
                  level_n=[tuple(st.level_n[l]) for l in range(nl)],
                  level_iters=[int(st.level_iters[l]) for l in range(nl)],
                  level_calls=[int(st.level_calls[l]) for l in range(nl)],
                  rel_residual_true=st.rel_residual_true, b_norm=st.b_norm)


def solve(problem, tol=None, **opt) -> Result:
    """Solve a `synth.Problem`-like object (dim, n, kx, ky, kz, f, bc_type, bc_value, length, tol)."""
    return solve_arrays(problem.dim, problem.n, problem.kx, problem.ky, problem.kz, problem.f, problem.bc_type,
                        problem.bc_value, problem.tol if tol is None else tol, length=problem.length, **opt)


def level_plan(dim, n, scale=4, min_side=8, max_levels=MAX_LEVELS, axis_weight=None, length=(1.0, 1.0, 1.0),
               frac_scale=0.0):
    L = lib()
    dims = (ctypes.c_int * (3 * MAX_LEVELS))()
    npt, _a = _i(n)
    if frac_scale > 0.0:
        nl = L.oracle_level_plan_frac(dim, npt, float(frac_scale), min_side, max_levels,
                                      ctypes.cast(dims, ctypes.POINTER(ctypes.c_int)))
    elif axis_weight is None:
        nl = L.oracle_level_plan(dim, npt, scale, min_side, max_levels, ctypes.cast(dims, ctypes.POINTER(ctypes.c_int)))
    else:
        Ld = np.asarray(length, dtype=np.float64)
        aw = _axis_w(axis_weight)
        nl = L.oracle_level_plan_semi(dim, npt, _d(Ld), _d(aw), scale, min_side, max_levels,
                                      ctypes.cast(dims, ctypes.POINTER(ctypes.c_int)))
    return [tuple(dims[3 * l:3 * l + 3]) for l in range(nl)]


def face_T(dim, n, h, kx, ky, kz, bc_type):
    """Face transmissibilities (tx, ty, tz) on the finest grid."""
    L = lib()
    nx, ny, nz = n
    nz = nz if dim == 3 else 1
    kx = _f64(kx)
    ky = _f64(ky if ky is not None else kx)
    kz = _f64(kz) if dim == 3 else None
    tx = np.zeros((nx + 1) * ny * nz)
    ty = np.zeros(nx * (ny + 1) * nz)
    tz = np.zeros(nx * ny * (nz + 1)) if dim == 3 else None
    bct, _b = _i(bc_type)
    L.oracle_face_T(dim, nx, ny, nz, h[0], h[1], h[2] if dim == 3 else 1.0, _d(kx), _d(ky), _d(kz), bct, _d(tx),
                    _d(ty), _d(tz))
    return tx, ty, tz


def coarsen_T(dim, fd, s, tx, ty, tz):
    L = lib()
    fd3 = (fd[0], fd[1], fd[2] if dim == 3 else 1)
    s3 = (s[0], s[1], s[2] if dim == 3 else 1)
    cd = (fd3[0] // s3[0], fd3[1] // s3[1], fd3[2] // s3[2])
    ctx = np.zeros((cd[0] + 1) * cd[1] * cd[2])
    cty = np.zeros(cd[0] * (cd[1] + 1) * cd[2])
    ctz = np.zeros(cd[0] * cd[1] * (cd[2] + 1)) if dim == 3 else None
    a, _a = _i(fd3)
    b, _b = _i(s3)
    L.oracle_coarsen_T(dim, a, b, _d(_f64(tx)), _d(_f64(ty)), _d(_f64(tz)), _d(ctx), _d(cty), _d(ctz))
    return ctx, cty, ctz


def apply_A(dim, n, T, x):
    L = lib()
    tx, ty, tz = (_f64(t) for t in T) if T[2] is not None else (_f64(T[0]), _f64(T[1]), None)
    y = np.zeros_like(x, dtype=np.float64)
    L.oracle_apply_A(dim, n[0], n[1], n[2] if dim == 3 else 1, _d(tx), _d(ty), _d(tz), _d(_f64(x)), _d(y))
    return y


def sgs(dim, n, T, r, x, m):
    """m symmetric Gauss-Seidel steps in red-black order; returns the new x."""
    L = lib()
    tx, ty, tz = (_f64(T[0]), _f64(T[1]), _f64(T[2]) if T[2] is not None else None)
    x = np.array(x, dtype=np.float64, copy=True)
    L.oracle_sgs(dim, n[0], n[1], n[2] if dim == 3 else 1, _d(tx), _d(ty), _d(tz), _d(_f64(r)), _d(x), int(m))
    return x


def mjac(dim, n, T, r, x, m):
    """m modified Jacobi steps (P = 2D); returns the new x."""
    L = lib()
    tx, ty, tz = (_f64(T[0]), _f64(T[1]), _f64(T[2]) if T[2] is not None else None)
    x = np.array(x, dtype=np.float64, copy=True)
    L.oracle_mjac(dim, n[0], n[1], n[2] if dim == 3 else 1, _d(tx), _d(ty), _d(tz), _d(_f64(r)), _d(x), int(m))
    return x


def gs_colour(dim, n, T, r, x, colour):
    L = lib()
    tx, ty, tz = (_f64(T[0]), _f64(T[1]), _f64(T[2]) if T[2] is not None else None)
    x = np.array(x, dtype=np.float64, copy=True)
    L.oracle_gs_colour(dim, n[0], n[1], n[2] if dim == 3 else 1, _d(tx), _d(ty), _d(tz), _d(_f64(r)), _d(x),
                       int(colour))
    return x


def prolong_add(dim, fd, s, yc, xf, interp=LINEAR):
    L = lib()
    a, _a = _i((fd[0], fd[1], fd[2] if dim == 3 else 1))
    b, _b = _i((s[0], s[1], s[2] if dim == 3 else 1))
    xf = np.array(xf, dtype=np.float64, copy=True)
    L.oracle_prolong_add(dim, a, b, int(interp), _d(_f64(yc)), _d(xf))
    return xf


def restrict(dim, fd, s, rf, interp=LINEAR):
    L = lib()
    fd3 = (fd[0], fd[1], fd[2] if dim == 3 else 1)
    s3 = (s[0], s[1], s[2] if dim == 3 else 1)
    nc = (fd3[0] // s3[0]) * (fd3[1] // s3[1]) * (fd3[2] // s3[2])
    a, _a = _i(fd3)
    b, _b = _i(s3)
    g = np.zeros(nc)
    L.oracle_restrict(dim, a, b, int(interp), _d(_f64(rf)), _d(g))
    return g


def prolong_add_dims(dim, fd, cd, yc, xf, interp=LINEAR):
    """xf + E yc between a fine grid fd and a coarser grid cd (factors need not be integers)."""
    L = lib()
    a, _a = _i((fd[0], fd[1], fd[2] if dim == 3 else 1))
    b, _b = _i((cd[0], cd[1], cd[2] if dim == 3 else 1))
    xf = np.array(xf, dtype=np.float64, copy=True)
    L.oracle_prolong_add_dims(dim, a, b, int(interp), _d(_f64(yc)), _d(xf))
    return xf


def restrict_dims(dim, fd, cd, rf, interp=LINEAR):
    """E^T rf from a fine grid fd to a coarser grid cd."""
    L = lib()
    a, _a = _i((fd[0], fd[1], fd[2] if dim == 3 else 1))
    b, _b = _i((cd[0], cd[1], cd[2] if dim == 3 else 1))
    g = np.zeros(cd[0] * cd[1] * (cd[2] if dim == 3 else 1))
    L.oracle_restrict_dims(dim, a, b, int(interp), _d(_f64(rf)), _d(g))
    return g


def cholesky(A):
    L = lib()
    A = _f64(A)
    n = A.shape[0]
    Lf = np.zeros_like(A)
    rc = L.oracle_cholesky(n, _d(A), _d(Lf))
    return rc, Lf


def cholesky_solve(Lf, b):
    L = lib()
    x = np.zeros(b.size)
    L.oracle_cholesky_solve(Lf.shape[0], _d(_f64(Lf)), _d(_f64(b)), _d(x))
    return x


def precond(problem, r, eps2=0.0, flvl=0.1, axis_weight=None, frac_scale=0.0, **opt):
    """z = M_0^-1 r on the problem's hierarchy (level-0 preconditioner of eq. 2.10)."""
    L = lib()
    aw = _axis_w(axis_weight)
    dim, n = problem.dim, problem.n
    kx = _f64(problem.kx)
    ky = _f64(problem.ky)
    kz = _f64(problem.kz) if dim == 3 else None
    npt, _a = _i(n)
    bct, _b = _i(problem.bc_type)
    o, _c = _i(_opts(**opt))
    z = np.zeros(problem.N)
    Ld = np.asarray(problem.length, dtype=np.float64)
    L.oracle_set_frac_scale(float(frac_scale))
    try:
        rc = L.oracle_precond(dim, npt, _d(Ld), _d(kx), _d(ky), _d(kz), bct, o, float(flvl), float(eps2),
                              _d(_f64(r)), _d(z), _d(aw))
    finally:
        L.oracle_set_frac_scale(0.0)
    if rc != 0:
        raise RuntimeError(f"oracle_precond failed: {rc}")
    return z


def hierarchy_T(problem, scale=4, min_side=8, max_levels=MAX_LEVELS, axis_weight=None, frac_scale=0.0):
    """Per-level face arrays [(dims, tx, ty, tz), ...] of the problem's hierarchy."""
    L = lib()
    dim, n = problem.dim, problem.n
    aw = _axis_w(axis_weight)
    plan = level_plan(dim, n, scale, min_side, max_levels, axis_weight=aw, length=problem.length,
                      frac_scale=frac_scale)
    sizes = []
    total = 0
    for d in plan:
        a = (d[0] + 1) * d[1] * d[2]
        b = d[0] * (d[1] + 1) * d[2]
        c = d[0] * d[1] * (d[2] + 1) if dim == 3 else 0
        sizes.append((a, b, c))
        total += a + b + c
    out = np.zeros(total)
    npt, _a = _i(n)
    bct, _b = _i(problem.bc_type)
    Ld = np.asarray(problem.length, dtype=np.float64)
    kz = _f64(problem.kz) if dim == 3 else None
    L.oracle_set_frac_scale(float(frac_scale))
    try:
        nl = L.oracle_hierarchy_T(dim, npt, _d(Ld), _d(_f64(problem.kx)), _d(_f64(problem.ky)), _d(kz), bct, scale,
                                  min_side, max_levels, _d(out), out.size, _d(aw))
    finally:
        L.oracle_set_frac_scale(0.0)
    assert nl == len(plan), (nl, plan)
    res = []
    off = 0
    for d, (a, b, c) in zip(plan, sizes):
        tx = out[off:off + a]; off += a
        ty = out[off:off + b]; off += b
        tz = out[off:off + c] if c else None; off += c
        res.append((d, tx.copy(), ty.copy(), None if tz is None else tz.copy()))
    return res
