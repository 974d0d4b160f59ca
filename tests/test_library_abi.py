"""Host-side checks of libmscg: it loads, exports every function include/mscg.h
declares, and rejects bad grids and options before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_math_9809043_amd import mscg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "mscg.h")).read()
    return sorted(set(re.findall(r"\b(mscg_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("mscg_create_problem", "mscg_set_permeability", "mscg_solve", "mscg_solve_batch"):
        assert required in names
    assert set(names) == set(mscg.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = mscg.load_library()
    for name in header_functions():
        assert hasattr(L, name), name


def test_default_options():
    L = mscg.load_library()
    o = mscg._Options()
    L.mscg_default_options(ctypes.byref(o))
    assert (o.precision, o.scale, o.smooth_steps, o.min_coarse_side, o.interp) == (0, 4, 4, 8, 0)
    assert o.level_factor == pytest.approx(0.1)


def test_footprint_and_argument_errors():
    g = mscg.Grid(dim=2, n=(1024, 1024))
    b = mscg.footprint_bytes(g)
    # five vectors per level plus faces, rhs and the 256x256 coarsest inverse
    assert 1024 * 1024 * 8 * 7 < b < 1024 * 1024 * 8 * 12
    with pytest.raises(mscg.MscgError, match="coarsest level"):
        mscg.footprint_bytes(mscg.Grid(dim=2, n=(50, 50)))
    with pytest.raises(mscg.MscgError, match="dim"):
        mscg.footprint_bytes(mscg.Grid(dim=4, n=(8, 8)))
    with pytest.raises(mscg.MscgError, match="bc_type"):
        mscg.footprint_bytes(mscg.Grid(dim=2, n=(32, 32), bc_type=[3, 1, 0, 0, 0, 0]))
    with pytest.raises(mscg.MscgError, match="interp"):
        mscg.footprint_bytes(g, mscg.Options(interp=7))
    mixed = mscg.footprint_bytes(g, mscg.Options(precision=mscg.MIXED))
    assert mixed > b


def test_create_rejects_small_workspace_before_any_launch():
    L = mscg.load_library()
    g = mscg.Grid(dim=2, n=(32, 32))._c()
    o = mscg.Options()._c()
    h = ctypes.c_void_p()
    rc = L.mscg_create_problem(ctypes.byref(g), ctypes.byref(o), ctypes.c_void_p(256), 16, None, ctypes.byref(h))
    assert rc == mscg.E_NOMEM
    assert "workspace" in mscg.last_error()


def test_default_cycle_and_scale():
    L = mscg.load_library()
    o = mscg._Options()
    L.mscg_default_options(ctypes.byref(o))
    assert (o.cycle, o.splitting) == (mscg.CYCLE_RECURSIVE, mscg.SPLIT_SGS)
    assert o.frac_scale == 0.0


def test_cycle_and_fractional_scale_arguments():
    # a 50^2 grid cannot be divided by 4, but the rounded factor plans it: 50 -> 13 (-> 3 < 8 stops)
    g = mscg.Grid(dim=2, n=(50, 50))
    assert mscg.footprint_bytes(g, mscg.Options(frac_scale=4.0)) > 0
    # 1001^2 with the factor of Table 1 gives levels 1001, 252, 63, 16 (and 4 with min side 4)
    big = mscg.footprint_bytes(mscg.Grid(dim=2, n=(1001, 1001)), mscg.Options(frac_scale=3.98, min_coarse_side=4))
    assert 1001 * 1001 * 8 * 7 < big < 1001 * 1001 * 8 * 12
    with pytest.raises(mscg.MscgError, match="frac_scale"):
        mscg.footprint_bytes(g, mscg.Options(frac_scale=0.5))
    with pytest.raises(mscg.MscgError, match="frac_scale"):
        mscg.footprint_bytes(g, mscg.Options(frac_scale=17.0))
    with pytest.raises(mscg.MscgError, match="semi_coarsen"):
        mscg.footprint_bytes(g, mscg.Options(frac_scale=3.0, semi_coarsen=1))
    with pytest.raises(mscg.MscgError, match="cycle"):
        mscg.footprint_bytes(mscg.Grid(dim=2, n=(32, 32)), mscg.Options(cycle=3))
    for cyc in (mscg.CYCLE_RECURSIVE, mscg.CYCLE_MGCG, mscg.CYCLE_POLY):
        assert mscg.footprint_bytes(mscg.Grid(dim=2, n=(32, 32)), mscg.Options(cycle=cyc)) > 0
