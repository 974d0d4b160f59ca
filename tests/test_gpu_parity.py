"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Operators element by element, then full solves: relative residual <= 1e-10,
solution within 1e-8 relative of the oracle's, outer iterations within 2.
"""
import numpy as np
import pytest

import oracle
from paper_math_9809043_amd import synth

from conftest import gpu_available
from test_oracle_pins import rhs

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _torch():
    import torch
    return torch


def dev_tensor(a):
    torch = _torch()
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def make_problem(P, **opt):
    from paper_math_9809043_amd import mscg
    grid = mscg.Grid(dim=P.dim, n=P.n, bc_type=P.bc_type, bc_value=P.bc_value, length=P.length)
    prob = mscg.Problem(grid, mscg.Options(**opt))
    prob.set_permeability(dev_tensor(P.kx), dev_tensor(P.ky), dev_tensor(P.kz) if P.dim == 3 else None)
    return prob


def gpu_solve(P, tol=None, **opt):
    torch = _torch()
    prob = make_problem(P, **opt)
    p = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    st = prob.solve(dev_tensor(P.f), p, P.tol if tol is None else tol)
    torch.cuda.synchronize()
    return st, p.cpu().numpy(), prob


def case(name):
    print(f"\n[case] {name}", flush=True)


def oracle_opts(opt):
    out = {}
    if "interp" in opt:
        out["interp"] = opt["interp"]
    if "min_coarse_side" in opt:
        out["min_side"] = opt["min_coarse_side"]
    if "max_levels" in opt:
        out["max_levels"] = opt["max_levels"]
    return out


# ------------------------------------------------------------------ operators

HIER_CASES = [
    ("small32", lambda: synth.small_case(0), {}),
    ("ragged96x40", lambda: synth.smoothed_lognormal_2d(4, 96, 40, lo=-3, hi=3), {}),
    ("channel128", lambda: synth.channelised_2d(1, 128), {"interp": 1}),
    ("layered32", lambda: synth.layered_3d(2, 32, n_layers=8), {"interp": 1}),
    ("smooth512", lambda: synth.smoothed_lognormal_2d(5, 512, lo=-3, hi=3), {}),
]


@pytest.mark.parametrize("name,make,opt", HIER_CASES, ids=[c[0] for c in HIER_CASES])
def test_transmissibility_hierarchy(name, make, opt):
    case(f"hierarchy {name}")
    P = make()
    prob = make_problem(P, **opt)
    ref = oracle.hierarchy_T(P, min_side=opt.get("min_coarse_side", 8))
    assert prob.n_levels == len(ref)
    for lvl, (dims, tx, ty, tz) in enumerate(ref):
        assert prob.level_dims(lvl) == dims
        gx, gy, gz = prob.transmissibility(lvl)
        for g, r in ((gx, tx), (gy, ty), (gz, tz)):
            if r is None:
                continue
            g = g.cpu().numpy()
            assert np.allclose(g, r, rtol=1e-13, atol=0), (lvl, np.abs(g - r).max())


@pytest.mark.parametrize("name,make,opt", HIER_CASES[:4], ids=[c[0] for c in HIER_CASES[:4]])
def test_operator_smoother_transfers(name, make, opt):
    case(f"operators {name}")
    torch = _torch()
    P = make()
    prob = make_problem(P, **opt)
    ref = oracle.hierarchy_T(P, min_side=opt.get("min_coarse_side", 8))
    rng = np.random.default_rng(11)
    interp = opt.get("interp", 0)
    for lvl, (dims, tx, ty, tz) in enumerate(ref):
        n = dims[0] * dims[1] * dims[2]
        T = (tx, ty, tz)
        x = rng.standard_normal(n)
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        prob.apply_operator(lvl, dev_tensor(x), y)
        ya = oracle.apply_A(P.dim, dims, T, x)
        assert np.allclose(y.cpu().numpy(), ya, rtol=0, atol=1e-13 * np.abs(ya).max())
        r = rng.standard_normal(n)
        x0 = rng.standard_normal(n)
        xs = dev_tensor(x0)
        prob.apply_smoother(lvl, dev_tensor(r), xs, 4)
        xo = oracle.sgs(P.dim, dims, T, r, x0, 4)
        assert np.allclose(xs.cpu().numpy(), xo, rtol=0, atol=1e-11 * np.abs(xo).max())
        if lvl + 1 < len(ref):
            cd = ref[lvl + 1][0]
            s = (dims[0] // cd[0], dims[1] // cd[1], dims[2] // cd[2])
            nc = cd[0] * cd[1] * cd[2]
            g = torch.empty(nc, dtype=torch.float64, device="cuda")
            prob.restrict_residual(lvl, dev_tensor(r), dev_tensor(x0), g)
            res = r - oracle.apply_A(P.dim, dims, T, x0)
            go = oracle.restrict(P.dim, dims, s, res, interp)
            assert np.allclose(g.cpu().numpy(), go, rtol=0, atol=1e-12 * np.abs(go).max())
            yc = rng.standard_normal(nc)
            xf = dev_tensor(x0)
            prob.prolong_add(lvl, dev_tensor(yc), xf)
            xo = oracle.prolong_add(P.dim, dims, s, yc, x0, interp)
            assert np.allclose(xf.cpu().numpy(), xo, rtol=0, atol=1e-14 * np.abs(xo).max())


@pytest.mark.parametrize("name,make,opt", [HIER_CASES[0], HIER_CASES[2], HIER_CASES[3]],
                         ids=["small32", "channel128", "layered32"])
def test_preconditioner(name, make, opt):
    case(f"preconditioner {name}")
    torch = _torch()
    P = make()
    prob = make_problem(P, **opt)
    rng = np.random.default_rng(5)
    r = rng.standard_normal(P.N)
    z = torch.empty(P.N, dtype=torch.float64, device="cuda")
    eps2 = 1e-3
    prob.apply_preconditioner(dev_tensor(r), z, eps2)
    zo = oracle.precond(P, r, eps2=eps2, **oracle_opts(opt))
    # two levels: exact coarse solve, only rounding differs.  Three levels: an
    # inner PCG on a 1e9-contrast operator amplifies the rounding differences of
    # its reductions by its condition number (~1e9 * 1e-16).
    tol = 1e-10 if prob.n_levels == 2 else 1e-6
    assert np.linalg.norm(z.cpu().numpy() - zo) / np.linalg.norm(zo) < tol


# ------------------------------------------------------------------ full solves

SOLVE_CASES = [(f"small32_s{s}", (lambda s=s: synth.small_case(s)), {}) for s in range(10)] + [
    ("small32_fonly", lambda: synth.smoothed_lognormal_2d(3, 32, bc_value=(0.0, 0.0)), {}),
    ("ragged96x40", lambda: synth.smoothed_lognormal_2d(4, 96, 40, lo=-3, hi=3), {}),
    ("rect128x64", lambda: synth.smoothed_lognormal_2d(6, 128, 64, lo=-2, hi=2), {}),
    ("smooth256", lambda: synth.smoothed_lognormal_2d(1, 256, lo=-3, hi=3), {}),
    ("smooth512", lambda: synth.smoothed_lognormal_2d(5, 512, lo=-3, hi=3), {}),
    ("smooth256_const", lambda: synth.smoothed_lognormal_2d(1, 256, lo=-3, hi=3), {"interp": 1}),
    ("channel64_const", lambda: synth.channelised_2d(0, 64), {"interp": 1}),
    ("layered32_const", lambda: synth.layered_3d(2, 32, n_layers=8), {"interp": 1}),
]


@pytest.mark.parametrize("name,make,opt", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_solve_parity(name, make, opt):
    case(f"solve {name}")
    P = make()
    st, x, _ = gpu_solve(P, **opt)
    ref = oracle.solve(P, **oracle_opts(opt))
    err = np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p)
    print(f"  gpu outer={st.outer_iters} levels={st.level_iters} res={st.rel_residual_true:.2e} | "
          f"oracle outer={ref.outer_iters} levels={ref.level_iters} | rel err {err:.2e}", flush=True)
    assert ref.status == 0
    assert st.status == 0
    assert st.rel_residual_true <= 1e-10
    assert err <= 1e-8
    assert abs(st.outer_iters - ref.outer_iters) <= 2
    # residual of the GPU result recomputed on the CPU from the oracle's operator
    h = tuple(P.length[a] / P.n[a] for a in range(3))
    T = oracle.face_T(P.dim, P.n, h, P.kx, P.ky, P.kz, P.bc_type)
    b = rhs(P, *T)
    Ax = oracle.apply_A(P.dim, P.n, T, x)
    assert np.linalg.norm(Ax - b) / np.linalg.norm(b) <= 1.5e-10


@pytest.mark.parametrize("side,opt", [(16, {}), (24, {"max_levels": 1}), (32, {"max_levels": 1})],
                         ids=["16x16", "24x24", "32x32"])
def test_single_level_direct_solve(side, opt):
    """One level, solved by the coarsest factorisation and inverse alone: band
    in LDS (16 x 16, 24 x 24), band through a window (32 x 32)."""
    case(f"solve single level {side}x{side} direct")
    P = synth.smoothed_lognormal_2d(2, side)
    st, x, prob = gpu_solve(P, **opt)
    assert prob.n_levels == 1 and st.outer_iters == 0
    ref = oracle.solve(P, **oracle_opts(opt))
    assert np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p) < 1e-10


def test_constant_K_linear_ramp():
    case("solve constant K ramp")
    P = synth.small_case(0)
    P.kx[:] = 2.5
    P.ky[:] = 2.5
    P.f[:] = 0.0
    st, x, _ = gpu_solve(P)
    xc = (np.arange(32) + 0.5) / 32
    assert st.outer_iters == 0
    assert np.abs(x.reshape(32, 32) - xc[None, :]).max() < 1e-14


# ------------------------------------------------------------------ errors

def test_error_paths():
    case("error paths")
    torch = _torch()
    from paper_math_9809043_amd import mscg
    P = synth.small_case(0)
    grid = mscg.Grid(dim=2, n=P.n, bc_type=P.bc_type, bc_value=P.bc_value)
    prob = mscg.Problem(grid)
    f = dev_tensor(P.f)
    p = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    with pytest.raises(mscg.MscgError, match="E_STATE"):
        prob.solve(f, p, 1e-10)
    bad = P.kx.copy()
    bad[17] = -1.0
    with pytest.raises(mscg.MscgError, match="E_ARG"):
        prob.set_permeability(dev_tensor(bad))
    bad[17] = np.nan
    with pytest.raises(mscg.MscgError, match="E_ARG"):
        prob.set_permeability(dev_tensor(bad))
    neu = mscg.Problem(mscg.Grid(dim=2, n=P.n, bc_type=[0] * 6))
    with pytest.raises(mscg.MscgError, match="E_SINGULAR"):
        neu.set_permeability(dev_tensor(P.kx))
    capped = mscg.Problem(grid, mscg.Options(max_outer_iters=1))
    capped.set_permeability(dev_tensor(P.kx), dev_tensor(P.ky))
    st = capped.solve(f, p, 1e-10)
    assert st.status == mscg.NOT_CONVERGED and st.outer_iters == 1 and st.rel_residual_true > 1e-10


def test_batch_matches_single():
    case("batch of mixed sizes")
    torch = _torch()
    from paper_math_9809043_amd import mscg
    Ps = [synth.request_problem(synth.Request(i, 0.0, side, 1000 + i)) for i, side in enumerate((64, 128, 64, 256))]
    probs, fs, ps, singles = [], [], [], []
    for P in Ps:
        prob = make_problem(P)
        probs.append(prob)
        fs.append(dev_tensor(P.f))
        ps.append(torch.zeros(P.N, dtype=torch.float64, device="cuda"))
        q = torch.zeros(P.N, dtype=torch.float64, device="cuda")
        prob.solve(fs[-1], q, P.tol)
        singles.append(q.cpu().numpy())
    stats = mscg.solve_batch(probs, fs, ps, [P.tol for P in Ps])
    torch.cuda.synchronize()
    for st, p, s in zip(stats, ps, singles):
        assert st.status == 0 and st.rel_residual_true <= 1e-8
        assert np.array_equal(p.cpu().numpy(), s)


@pytest.mark.parametrize("name,make,opt", [
    ("ragged96x40", lambda: synth.smoothed_lognormal_2d(4, 96, 40, lo=-3, hi=3), {}),
    ("smooth512", lambda: synth.smoothed_lognormal_2d(5, 512, lo=-3, hi=3), {}),
    ("channel128_const", lambda: synth.channelised_2d(1, 128), {"interp": 1}),
], ids=["ragged96x40", "smooth512", "channel128_const"])
def test_tiled_smoother_matches_half_sweeps(name, make, opt, monkeypatch):
    """The LDS-tiled smoother, in every tile shape, reproduces the grid-wide
    half sweeps bitwise (a missing barrier, a short halo or a wrong ragged
    tile edge would break this)."""
    P = make()
    # r . z from the same grid-wide reduction on both sides
    monkeypatch.setenv("MSCG_FUSED_DOT", "0")
    monkeypatch.setenv("MSCG_UNTILED", "1")
    case(f"untiled {name}")
    st_u, x_u, _ = gpu_solve(P, **opt)
    monkeypatch.delenv("MSCG_UNTILED")
    for shape in ("auto", "0", "1", "2", "3"):
        case(f"tiled shape {shape} {name}")
        if shape == "auto":
            monkeypatch.delenv("MSCG_TILE_SHAPE", raising=False)
        else:
            monkeypatch.setenv("MSCG_TILE_SHAPE", shape)
        st_t, x_t, _ = gpu_solve(P, **opt)
        assert st_t.level_iters == st_u.level_iters
        assert np.array_equal(x_t, x_u), (shape, np.abs(x_t - x_u).max())


@pytest.mark.parametrize("name,make,opt", [
    ("ragged96x40", lambda: synth.smoothed_lognormal_2d(4, 96, 40, lo=-3, hi=3), {}),
    ("smooth512", lambda: synth.smoothed_lognormal_2d(5, 512, lo=-3, hi=3), {}),
    ("smooth512_mixed", lambda: synth.smoothed_lognormal_2d(5, 512, lo=-3, hi=3), {"precision": 1}),
], ids=["ragged96x40", "smooth512", "smooth512_mixed"])
def test_fused_rho_matches_grid_wide_dot(name, make, opt, monkeypatch):
    """r . z summed per tile by the post-smoother (one partial per tile) gives
    the solve of the grid-wide reduction up to rounding, and matches the oracle."""
    P = make()
    ref = oracle.solve(P)
    out = {}
    for fused in ("0", "1"):
        case(f"fused r.z {fused} {name}")
        monkeypatch.setenv("MSCG_FUSED_DOT", fused)
        st, x, _ = gpu_solve(P, **opt)
        assert st.status == 0 and st.rel_residual_true <= 1e-10
        assert abs(st.outer_iters - ref.outer_iters) <= 2
        assert np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p) <= 1e-8
        out[fused] = (st, x)
    assert abs(out["0"][0].outer_iters - out["1"][0].outer_iters) <= 1
    assert np.linalg.norm(out["0"][1] - out["1"][1]) / np.linalg.norm(out["0"][1]) <= 1e-9


@pytest.mark.parametrize("name,make,opt", [
    ("smooth512", lambda: synth.smoothed_lognormal_2d(5, 512, lo=-3, hi=3), {}),
    ("smooth512_mixed", lambda: synth.smoothed_lognormal_2d(5, 512, lo=-3, hi=3), {"precision": 1}),
    ("layered32_semi", lambda: synth.layered_3d(2, 32, n_layers=4),
     {"interp": 1, "semi_coarsen": 1, "axis_weight": (1, 1, 0.01)}),
], ids=["smooth512", "smooth512_mixed", "layered32_semi"])
def test_folded_finishes_match_finish_kernels_bitwise(name, make, opt, monkeypatch):
    """r.z and p.q summed inside the SpMV and update kernels (every workgroup
    the same partials in the same order) give the bits of the path with a
    finish kernel after each reduction."""
    P = make()
    out = {}
    for ff in ("0", "1"):
        case(f"folded finishes {ff} {name}")
        monkeypatch.setenv("MSCG_FUSED_FINISH", ff)
        st, x, _ = gpu_solve(P, **opt)
        assert st.status == 0 and st.rel_residual_true <= 1e-10
        out[ff] = (st, x)
    assert out["0"][0].level_iters == out["1"][0].level_iters
    assert np.array_equal(out["0"][1], out["1"][1])


@pytest.mark.parametrize("name,make,opt", [
    ("smooth256", lambda: synth.smoothed_lognormal_2d(1, 256, lo=-3, hi=3), {}),
    ("rect288x160", lambda: synth.smoothed_lognormal_2d(7, 288, 160, lo=-3, hi=3), {}),
    ("smooth256_const", lambda: synth.smoothed_lognormal_2d(1, 256, lo=-3, hi=3), {"interp": 1}),
    # last inner level 56 x 40: part of the 64 x 64 block grid is ghosts
    ("rect224x160", lambda: synth.smoothed_lognormal_2d(8, 224, 160, lo=-3, hi=3), {}),
], ids=["smooth256", "rect288x160", "smooth256_const", "rect224x160"])
def test_small_level_kernels_agree(name, make, opt, monkeypatch):
    """The 2x2-block, the colour-split and the cell-strided one-workgroup
    solvers of the last inner level give the same solve up to rounding, and
    all match the oracle."""
    P = make()
    ref = oracle.solve(P, **oracle_opts(opt))
    out = {}
    for variant in ("0", "1", "2"):
        case(f"small-level kernel {variant} {name}")
        monkeypatch.setenv("MSCG_SMALL_VARIANT", variant)
        st, x, prob = gpu_solve(P, **opt)
        assert prob.n_levels >= 3
        assert st.status == 0 and st.rel_residual_true <= 1e-10
        assert abs(st.outer_iters - ref.outer_iters) <= 2
        assert np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p) <= 1e-8
        out[variant] = x
    for v in ("0", "2"):
        assert np.linalg.norm(out[v] - out["1"]) / np.linalg.norm(out["1"]) <= 1e-8


SEMI_CASES = [
    ("layered32_linear", lambda: synth.layered_3d(2, 32, n_layers=4), (1, 1, 0.01), {}),
    ("layered32_const", lambda: synth.layered_3d(3, 32, n_layers=8), (1, 1, 0.01), {"interp": 1}),
    ("strip256x64", lambda: synth.anisotropic_strip_2d(1, 256, 64), (1, 100, 1), {}),
    ("strip512x128", lambda: synth.anisotropic_strip_2d(4, 512, 128), (1, 100, 1), {}),
    # last inner level 64 x 33 (y not coarsened): an odd side, ghost cells inside 2x2 blocks
    ("strip256x132", lambda: synth.anisotropic_strip_2d(2, 256, 132), (1, 100, 1), {}),
    # the bench's 3-D workload at full size.  Its layers (contrast 1e6, kz = kx/100)
    # make the operator ill-conditioned enough that two iterates with relative
    # residual 1e-10 differ by ~1e-7, so both sides solve to 1e-12 here
    ("layered128_const", lambda: synth.layered_128(0), (1, 1, 0.01), {"interp": 1, "tol": 1e-12}),
]


@pytest.mark.parametrize("name,make,w,opt", SEMI_CASES, ids=[c[0] for c in SEMI_CASES])
def test_semi_coarsening_parity(name, make, w, opt):
    """Aspect-ratio-aware level plan (Section 5): same levels as the oracle, and
    the solve matches it."""
    case(f"semi-coarsened solve {name}")
    P = make()
    opt = dict(opt)
    tol = opt.pop("tol", P.tol)
    st, x, prob = gpu_solve(P, tol=tol, semi_coarsen=1, axis_weight=w, **opt)
    ref = oracle.solve(P, tol=tol, axis_weight=w, **oracle_opts(opt))
    err = np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p)
    print(f"  gpu outer={st.outer_iters} levels={st.level_iters} dims={st.level_n} | oracle outer={ref.outer_iters} "
          f"levels={ref.level_iters} | rel err {err:.2e}", flush=True)
    assert [tuple(d) for d in st.level_n] == [tuple(d) for d in ref.level_n]
    assert ref.status == 0 and st.status == 0
    assert st.rel_residual_true <= max(tol, 1e-10)
    assert err <= 1e-8
    assert abs(st.outer_iters - ref.outer_iters) <= 2


JACOBI_CASES = [
    ("small32", lambda: synth.small_case(3), {}),
    ("smooth256", lambda: synth.smoothed_lognormal_2d(1, 256, lo=-3, hi=3), {}),
    ("rect288x160_const", lambda: synth.smoothed_lognormal_2d(7, 288, 160, lo=-2, hi=2), {"interp": 1}),
    ("layered32_semi", lambda: synth.layered_3d(3, 32, n_layers=8), {"interp": 1, "semi": (1, 1, 0.01)}),
]


@pytest.mark.parametrize("name,make,opt", JACOBI_CASES, ids=[c[0] for c in JACOBI_CASES])
def test_modified_jacobi_parity(name, make, opt):
    """Modified Jacobi splitting (P = 2D, Section 3) on every level, against the oracle."""
    case(f"modified Jacobi solve {name}")
    from paper_math_9809043_amd import mscg
    P = make()
    opt = dict(opt)
    semi = opt.pop("semi", None)
    gopt = dict(opt, splitting=mscg.SPLIT_JACOBI)
    if semi:
        gopt.update(semi_coarsen=1, axis_weight=semi)
    st, x, _ = gpu_solve(P, **gopt)
    ref = oracle.solve(P, splitting=oracle.JACOBI, axis_weight=semi, **oracle_opts(opt))
    err = np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p)
    print(f"  gpu outer={st.outer_iters} levels={st.level_iters} | oracle outer={ref.outer_iters} "
          f"levels={ref.level_iters} | rel err {err:.2e}", flush=True)
    assert ref.status == 0 and st.status == 0
    assert st.rel_residual_true <= 1e-10
    assert err <= 1e-8
    assert abs(st.outer_iters - ref.outer_iters) <= 2


def test_one_row_grids():
    """Degenerate 2-D grids one cell tall: with every axis coarsened together
    they cannot coarsen (a single, directly solved level, or an error when it
    exceeds the dense limit); the aspect-ratio-aware plan coarsens x alone."""
    from paper_math_9809043_amd import mscg
    case("one-row grids")
    P = synth.smoothed_lognormal_2d(3, 64, 1, lo=-2, hi=2)
    st, x, prob = gpu_solve(P)
    ref = oracle.solve(P)
    assert prob.n_levels == 1 and st.status == 0
    assert np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p) <= 1e-8
    Q = synth.smoothed_lognormal_2d(3, 4096, 1, lo=-2, hi=2)
    with pytest.raises(mscg.MscgError):
        make_problem(Q)
    st, x, prob = gpu_solve(Q, semi_coarsen=1)
    ref = oracle.solve(Q, axis_weight=(1, 1, 1))
    assert [tuple(d) for d in st.level_n] == [tuple(d) for d in ref.level_n] and prob.n_levels == 5
    assert st.status == 0 and st.rel_residual_true <= 1e-10
    assert np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p) <= 1e-8
    assert abs(st.outer_iters - ref.outer_iters) <= 2


def test_full_size_1024_matches_oracle():
    """The bench's workload at full size (1024^2, contrast 1e6, tol 1e-10) in
    the bench's launch configuration, FP64 and mixed, against the oracle's full
    solution."""
    from paper_math_9809043_amd import mscg
    case("full-size smooth1024")
    P = synth.smoothed_lognormal_2d(0, 1024, lo=-3.0, hi=3.0, tol=1e-10, name="smooth1024")
    ref = oracle.solve(P)
    assert ref.status == 0
    for prec in (mscg.FP64, mscg.MIXED):
        st, x, _ = gpu_solve(P, precision=prec)
        err = np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p)
        print(f"  precision {prec}: outer {st.outer_iters} (oracle {ref.outer_iters}) levels {st.level_iters} "
              f"(oracle {ref.level_iters}) res {st.rel_residual_true:.2e} err {err:.2e}", flush=True)
        assert st.status == 0 and st.rel_residual_true <= 1e-10
        assert err <= 1e-8
        assert abs(st.outer_iters - ref.outer_iters) <= 2


# ------------------------------------------- Tatebe's multigrid preconditioner (eq. 2.9)

@pytest.mark.parametrize("name,make,opt", [
    ("small32_3lev", lambda: synth.small_case(2), {"min_coarse_side": 2}),
    ("smooth256", lambda: synth.smoothed_lognormal_2d(1, 256, lo=-3, hi=3), {}),
    ("layered32_const", lambda: synth.layered_3d(2, 32, n_layers=8), {"interp": 1, "min_coarse_side": 2}),
], ids=["small32_3lev", "smooth256", "layered32_const"])
def test_mgcg_preconditioner(name, make, opt):
    """M_0^-1 r of eq. 2.9 (one pass down and up the hierarchy, no inner PCG):
    only rounding differs from the oracle."""
    from paper_math_9809043_amd import mscg
    case(f"MGCG preconditioner {name}")
    torch = _torch()
    P = make()
    prob = make_problem(P, cycle=mscg.CYCLE_MGCG, **opt)
    assert prob.n_levels >= 3
    r = np.random.default_rng(8).standard_normal(P.N)
    z = torch.empty(P.N, dtype=torch.float64, device="cuda")
    prob.apply_preconditioner(dev_tensor(r), z, 0.0)
    zo = oracle.precond(P, r, cycle=oracle.MGCG, **oracle_opts(opt))
    err = np.linalg.norm(z.cpu().numpy() - zo) / np.linalg.norm(zo)
    print(f"  rel diff {err:.2e}", flush=True)
    assert err < 1e-10


MGCG_CASES = [
    ("small32_3lev", lambda: synth.small_case(4), {"min_coarse_side": 2}),
    ("ragged176x48", lambda: synth.smoothed_lognormal_2d(4, 176, 48, lo=-3, hi=3), {"min_coarse_side": 2}),
    ("smooth256", lambda: synth.smoothed_lognormal_2d(1, 256, lo=-3, hi=3), {}),
    ("smooth512", lambda: synth.smoothed_lognormal_2d(5, 512, lo=-3, hi=3), {}),
    ("rect288x160_const", lambda: synth.smoothed_lognormal_2d(7, 288, 160, lo=-2, hi=2), {"interp": 1}),
    ("layered32_const", lambda: synth.layered_3d(2, 32, n_layers=8), {"interp": 1, "min_coarse_side": 2}),
    ("smooth256_jacobi", lambda: synth.smoothed_lognormal_2d(1, 256, lo=-3, hi=3), {"jacobi": True}),
    ("smooth1024", lambda: synth.smoothed_lognormal_2d(0, 1024, lo=-3.0, hi=3.0, tol=1e-10), {}),
]


@pytest.mark.parametrize("name,make,opt", MGCG_CASES, ids=[c[0] for c in MGCG_CASES])
def test_mgcg_parity(name, make, opt):
    """Full solves with Tatebe's preconditioner, FP64 and mixed, against the
    oracle's: residual, solution, outer iterations, and one visit of every
    inner level per application of the level above."""
    from paper_math_9809043_amd import mscg
    case(f"MGCG solve {name}")
    P = make()
    opt = dict(opt)
    jac = opt.pop("jacobi", False)
    gopt = dict(opt, cycle=mscg.CYCLE_MGCG)
    oopt = dict(oracle_opts(opt), cycle=oracle.MGCG)
    if jac:
        gopt["splitting"] = mscg.SPLIT_JACOBI
        oopt["splitting"] = oracle.JACOBI
    ref = oracle.solve(P, **oopt)
    assert ref.status == 0 and ref.nlev >= 3
    for prec in (mscg.FP64, mscg.MIXED):
        st, x, _ = gpu_solve(P, precision=prec, **gopt)
        err = np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p)
        print(f"  precision {prec}: outer {st.outer_iters} (oracle {ref.outer_iters}) calls "
              f"{st.level_calls} (oracle {ref.level_calls}) res {st.rel_residual_true:.2e} err {err:.2e}", flush=True)
        assert st.status == 0 and st.rel_residual_true <= 1e-10
        assert err <= 1e-8
        assert abs(st.outer_iters - ref.outer_iters) <= 2
        assert list(st.level_iters[1:]) == [0] * (st.n_levels - 1)
        assert [st.level_calls[k] for k in range(1, st.n_levels)] == [st.outer_iters] * (st.n_levels - 1)


# ------------------------------------------- polynomial preconditioner (Section 2.1)

POLY_CASES = [
    ("small32", lambda: synth.small_case(5), {}),
    ("rect96x40", lambda: synth.smoothed_lognormal_2d(4, 96, 40, lo=-3, hi=3), {}),
    ("smooth128", lambda: synth.smoothed_lognormal_2d(2, 128, lo=-3, hi=3), {}),
    ("smooth64_jacobi", lambda: synth.smoothed_lognormal_2d(2, 64, lo=-3, hi=3), {"jacobi": True}),
    ("layered16", lambda: synth.layered_3d(2, 16, n_layers=4), {"min_coarse_side": 2}),
]


@pytest.mark.parametrize("name,make,opt", POLY_CASES, ids=[c[0] for c in POLY_CASES])
def test_polynomial_parity(name, make, opt):
    """W = P^-1 (2m+1 steps of the splitting from zero): the preconditioner
    itself to rounding, and full solves in FP64 and mixed against the oracle's."""
    from paper_math_9809043_amd import mscg
    case(f"polynomial preconditioner {name}")
    torch = _torch()
    P = make()
    opt = dict(opt)
    jac = opt.pop("jacobi", False)
    gopt = dict(opt, cycle=mscg.CYCLE_POLY, max_outer_iters=3000)
    oopt = dict(oracle_opts(opt), cycle=oracle.POLY, max_outer=3000)
    if jac:
        gopt["splitting"] = mscg.SPLIT_JACOBI
        oopt["splitting"] = oracle.JACOBI
    prob = make_problem(P, **gopt)
    r = np.random.default_rng(3).standard_normal(P.N)
    z = torch.empty(P.N, dtype=torch.float64, device="cuda")
    prob.apply_preconditioner(dev_tensor(r), z, 0.0)
    zo = oracle.precond(P, r, **oopt)
    assert np.linalg.norm(z.cpu().numpy() - zo) / np.linalg.norm(zo) < 1e-12
    ref = oracle.solve(P, **oopt)
    assert ref.status == 0
    for prec in (mscg.FP64, mscg.MIXED):
        st, x, _ = gpu_solve(P, precision=prec, **gopt)
        err = np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p)
        print(f"  precision {prec}: outer {st.outer_iters} (oracle {ref.outer_iters}) res "
              f"{st.rel_residual_true:.2e} err {err:.2e}", flush=True)
        assert st.status == 0 and st.rel_residual_true <= 1e-10
        assert err <= 1e-8
        assert list(st.level_calls[1:]) == [0] * (st.n_levels - 1)
        # FP64 follows the oracle's iteration to rounding; the FP32 preconditioner may move the
        # count of this slowly converging iteration a little further
        assert abs(st.outer_iters - ref.outer_iters) <= (2 if prec == mscg.FP64 else max(2, ref.outer_iters // 10))


# ------------------------------------------- non-integer scale factors (Section 3)

FRAC_CASES = [
    ("smooth1001_s3.98", lambda: synth.smoothed_lognormal_2d(2, 1001, lo=-3, hi=3), 3.98, {"min_coarse_side": 4}),
    ("rect250x170_s2.5", lambda: synth.smoothed_lognormal_2d(3, 250, 170, lo=-3, hi=3), 2.5, {}),
    ("small45_s3_const", lambda: synth.smoothed_lognormal_2d(4, 45, lo=-2, hi=2), 3.0,
     {"min_coarse_side": 2, "interp": 1}),
    ("smooth256_s4", lambda: synth.smoothed_lognormal_2d(1, 256, lo=-3, hi=3), 4.0, {}),
    ("layered30_s2.5_const", lambda: synth.layered_3d(2, 30, n_layers=6), 2.5, {"min_coarse_side": 4, "interp": 1}),
]


@pytest.mark.parametrize("name,make,fs,opt", FRAC_CASES, ids=[c[0] for c in FRAC_CASES])
def test_fractional_scale_parity(name, make, fs, opt):
    """Hierarchies whose factors need not be integers (coarse graining with
    partial overlaps, fractional extension weights): the level sizes, full
    solves in FP64 and mixed against the oracle's, and eq. 2.9's
    preconditioner over the whole hierarchy to rounding."""
    from paper_math_9809043_amd import mscg
    case(f"fractional scale {name}")
    torch = _torch()
    P = make()
    gopt = dict(opt, frac_scale=fs)
    oopt = dict(oracle_opts(opt), frac_scale=fs)
    ref = oracle.solve(P, **oopt)
    assert ref.status == 0 and ref.nlev >= 3
    for prec in (mscg.FP64, mscg.MIXED):
        st, x, _ = gpu_solve(P, precision=prec, **gopt)
        err = np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p)
        print(f"  precision {prec}: levels {st.level_n} outer {st.outer_iters} (oracle {ref.outer_iters}) iters "
              f"{st.level_iters} (oracle {ref.level_iters}) res {st.rel_residual_true:.2e} err {err:.2e}", flush=True)
        assert [tuple(d) for d in st.level_n] == [tuple(d) for d in ref.level_n]
        assert st.status == 0 and st.rel_residual_true <= 1e-10
        assert err <= 1e-8
        assert abs(st.outer_iters - ref.outer_iters) <= 2
    # Tatebe's preconditioner over the whole hierarchy has no inner PCG, so M^-1 r differs from
    # the oracle's by rounding only: every level's fractional transfers and coarse graining
    prob = make_problem(P, cycle=mscg.CYCLE_MGCG, **gopt)
    r = np.random.default_rng(9).standard_normal(P.N)
    z = torch.empty(P.N, dtype=torch.float64, device="cuda")
    prob.apply_preconditioner(dev_tensor(r), z, 0.0)
    zo = oracle.precond(P, r, cycle=oracle.MGCG, **oopt)
    err = np.linalg.norm(z.cpu().numpy() - zo) / np.linalg.norm(zo)
    print(f"  eq. 2.9 preconditioner rel diff {err:.2e}", flush=True)
    assert err < 1e-10


def test_batch_matches_single_for_every_cycle_and_fractional_plans():
    """mscg_solve_batch with problems of different cycles, splittings and level
    plans in one call: each result is bitwise the one it gets alone."""
    from paper_math_9809043_amd import mscg
    case("batch of mixed cycles and plans")
    torch = _torch()
    jobs = [
        (synth.smoothed_lognormal_2d(1, 256, lo=-3, hi=3), {"cycle": mscg.CYCLE_MGCG}),
        (synth.smoothed_lognormal_2d(2, 64, lo=-2, hi=2), {"cycle": mscg.CYCLE_POLY, "max_outer_iters": 2000}),
        (synth.smoothed_lognormal_2d(3, 250, 170, lo=-3, hi=3), {"frac_scale": 2.5}),
        (synth.smoothed_lognormal_2d(4, 128, lo=-3, hi=3), {}),
        (synth.smoothed_lognormal_2d(5, 128, lo=-3, hi=3), {"precision": mscg.MIXED, "cycle": mscg.CYCLE_MGCG}),
    ]
    probs, fs, ps, singles = [], [], [], []
    for P, opt in jobs:
        prob = make_problem(P, **opt)
        probs.append(prob)
        fs.append(dev_tensor(P.f))
        ps.append(torch.zeros(P.N, dtype=torch.float64, device="cuda"))
        q = torch.zeros(P.N, dtype=torch.float64, device="cuda")
        st = prob.solve(fs[-1], q, P.tol)
        assert st.status == 0
        singles.append(q.cpu().numpy())
    stats = mscg.solve_batch(probs, fs, ps, [P.tol for P, _ in jobs])
    torch.cuda.synchronize()
    for st, p, s in zip(stats, ps, singles):
        assert st.status == 0 and st.rel_residual_true <= 1e-10
        assert np.array_equal(p.cpu().numpy(), s)


SCALE_CASES = [
    ("smooth96_s2", lambda: synth.smoothed_lognormal_2d(3, 96, lo=-3, hi=3), 2),
    ("smooth128_s2", lambda: synth.smoothed_lognormal_2d(3, 128, lo=-3, hi=3), 2),
    ("smooth216_s3", lambda: synth.smoothed_lognormal_2d(3, 216, lo=-3, hi=3), 3),
    ("smooth512_s8", lambda: synth.smoothed_lognormal_2d(3, 512, lo=-3, hi=3), 8),
]


@pytest.mark.parametrize("name,make,sc", SCALE_CASES, ids=[c[0] for c in SCALE_CASES])
def test_integer_scale_factors_parity(name, make, sc):
    """Integer factors other than 4 (with m = s smoothing steps, Section 3):
    grid-wide smoothing, the generic transfer footprints and the one-workgroup
    solvers' factor checks, FP64 and mixed, against the oracle."""
    from paper_math_9809043_amd import mscg
    case(f"integer scale {name}")
    P = make()
    ref = oracle.solve(P, scale=sc)
    assert ref.status == 0 and ref.nlev >= 3
    for prec in (mscg.FP64, mscg.MIXED):
        st, x, _ = gpu_solve(P, precision=prec, scale=sc)
        err = np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p)
        print(f"  precision {prec}: levels {st.level_n} outer {st.outer_iters} (oracle {ref.outer_iters}) iters "
              f"{st.level_iters} (oracle {ref.level_iters}) res {st.rel_residual_true:.2e} err {err:.2e}", flush=True)
        assert [tuple(d) for d in st.level_n] == [tuple(d) for d in ref.level_n]
        assert st.status == 0 and st.rel_residual_true <= 1e-10
        assert err <= 1e-8
        assert abs(st.outer_iters - ref.outer_iters) <= 2


KNOB_CASES = [
    ("smooth256_m2", {"smooth_steps": 2}, {"m": 2}),
    ("smooth256_m6", {"smooth_steps": 6}, {"m": 6}),
    ("smooth256_f0.3", {"level_factor": 0.3}, {"flvl": 0.3}),
    ("smooth256_f0.02", {"level_factor": 0.02}, {"flvl": 0.02}),
]


@pytest.mark.parametrize("name,gopt,oopt", KNOB_CASES, ids=[c[0] for c in KNOB_CASES])
def test_smoothing_steps_and_level_factor_parity(name, gopt, oopt):
    """The other knobs of the method (Section 3): m smoothing steps away from
    the tiled smoother's m = 4, and the level factor f of the per-level
    criterion, FP64 and mixed, against the oracle."""
    from paper_math_9809043_amd import mscg
    case(f"knobs {name}")
    P = synth.smoothed_lognormal_2d(1, 256, lo=-3, hi=3)
    ref = oracle.solve(P, **oopt)
    assert ref.status == 0
    for prec in (mscg.FP64, mscg.MIXED):
        st, x, _ = gpu_solve(P, precision=prec, **gopt)
        err = np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p)
        print(f"  precision {prec}: outer {st.outer_iters} (oracle {ref.outer_iters}) iters {st.level_iters} "
              f"(oracle {ref.level_iters}) res {st.rel_residual_true:.2e} err {err:.2e}", flush=True)
        assert st.status == 0 and st.rel_residual_true <= 1e-10
        assert err <= 1e-8
        assert abs(st.outer_iters - ref.outer_iters) <= 2


def test_dense_coarsest_factorisation():
    """Coarsest levels whose band (nx) is wider than 64 are factored densely
    (`k_chol_factor`, `k_chol_inverse`); the coarsest product reads the full
    inverse row by row.  A two-level 400 x 40 hierarchy (coarsest 100 x 10) in
    FP64 and mixed, and a single-level 80 x 12 direct solve."""
    from paper_math_9809043_amd import mscg
    case("dense coarsest factorisation")
    P = synth.smoothed_lognormal_2d(8, 400, 40, lo=-2, hi=2)
    ref = oracle.solve(P)
    assert ref.status == 0 and ref.level_n[-1][:2] == (100, 10)
    for prec in (mscg.FP64, mscg.MIXED):
        st, x, _ = gpu_solve(P, precision=prec)
        err = np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p)
        print(f"  precision {prec}: outer {st.outer_iters} (oracle {ref.outer_iters}) res {st.rel_residual_true:.2e} "
              f"err {err:.2e}", flush=True)
        assert st.status == 0 and st.rel_residual_true <= 1e-10
        assert err <= 1e-8
        assert abs(st.outer_iters - ref.outer_iters) <= 2
    Q = synth.smoothed_lognormal_2d(9, 80, 12, lo=-2, hi=2)
    st, x, prob = gpu_solve(Q, max_levels=1)
    assert prob.n_levels == 1 and st.outer_iters == 0
    refq = oracle.solve(Q, max_levels=1)
    assert np.linalg.norm(x - refq.p) / np.linalg.norm(refq.p) < 1e-10
