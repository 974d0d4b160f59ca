"""Serving: continuous batching of solves of different sizes on one GPU, and
mixed precision against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_math_9809043_amd import synth

from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def case(name):
    print(f"\n[case] {name}", flush=True)


def test_serving_mix_matches_alone_and_respects_budget():
    case("serving 48 requests, 4 slots, small budget")
    import torch
    from paper_math_9809043_amd import mscg, serve
    opts = mscg.Options(precision=mscg.MIXED)
    reqs = synth.request_stream(48, rate_per_s=5000.0, sides=(64, 128, 256, 512), arrival_seed=3, first_seed=500)
    srv = serve.Server(slots=4, budget_bytes=0, options=opts, tol=1e-8)
    budget = srv.footprint(512) + srv.footprint(256)
    srv.budget = budget
    keep = [r.idx for r in reqs[::6]]
    rep = srv.run(reqs, keep=keep)
    s = rep.summary()
    print(" ", s, flush=True)
    assert s["ok"] == len(reqs)
    assert all(r.rel_residual_true <= 1e-8 for r in rep.results)
    assert rep.peak_inflight_bytes <= budget or rep.peak_inflight == 1
    assert rep.max_queue > 0          # the budget made requests wait
    assert rep.peak_inflight >= 2     # and still let several run together
    by_idx = {r.idx: r for r in rep.results}
    for req in reqs:
        if req.idx not in keep:
            continue
        st, p, k, f = serve.solve_alone(req, opts, tol=1e-8)
        mixed = by_idx[req.idx].solution.cpu().numpy()
        alone = p.cpu().numpy()
        assert st.status == 0
        assert np.array_equal(mixed, alone), (req.idx, np.abs(mixed - alone).max())


def test_serving_result_matches_oracle():
    case("served request vs FP64 oracle")
    from paper_math_9809043_amd import mscg, serve
    opts = mscg.Options(precision=mscg.MIXED)
    for side in (64, 256):
        req = synth.Request(0, 0.0, side, 4242 + side)
        st, p, k, f = serve.solve_alone(req, opts, tol=1e-8)
        ref = oracle.solve_arrays(2, (side, side, 1), k.cpu().numpy(), k.cpu().numpy(), None, f.cpu().numpy(),
                                  [1, 1, 0, 0, 0, 0], [0.0, 1.0, 0, 0, 0, 0], 1e-8)
        x = p.cpu().numpy()
        err = np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p)
        print(f"  side {side}: mixed outer {st.outer_iters} oracle {ref.outer_iters} err {err:.2e} "
              f"res {st.rel_residual_true:.2e}", flush=True)
        # mixed precision: the residual target holds; the error against the FP64
        # oracle is reported, bounded by conditioning times the tolerance
        assert st.status == 0 and st.rel_residual_true <= 1e-8 and err <= 1e-5
        assert st.outer_iters <= 1.5 * ref.outer_iters + 1


MIXED_CASES = [
    ("smooth256", lambda: synth.smoothed_lognormal_2d(1, 256, lo=-3, hi=3), {}),
    ("smooth512", lambda: synth.smoothed_lognormal_2d(5, 512, lo=-3, hi=3), {}),
    ("layered32", lambda: synth.layered_3d(2, 32, n_layers=8), {"interp": 1}),
    ("smooth512_flexible", lambda: synth.smoothed_lognormal_2d(5, 512, lo=-3, hi=3), {"flexible": 1}),
]


@pytest.mark.parametrize("name,make,opt", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_mixed_precision_reaches_fp64_accuracy(name, make, opt):
    case(f"mixed {name}")
    import torch
    from paper_math_9809043_amd import mscg
    P = make()
    grid = mscg.Grid(dim=P.dim, n=P.n, bc_type=P.bc_type, bc_value=P.bc_value)
    prob = mscg.Problem(grid, mscg.Options(precision=mscg.MIXED, **opt))
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda")
    prob.set_permeability(dev(P.kx), dev(P.ky), dev(P.kz) if P.dim == 3 else None)
    p = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    st = prob.solve(dev(P.f), p, 1e-10)
    ref = oracle.solve(P, **({"interp": opt["interp"]} if "interp" in opt else {}))  # FP64, Fletcher-Reeves
    x = p.cpu().numpy()
    err = np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p)
    print(f"  mixed outer={st.outer_iters} levels={st.level_iters} res={st.rel_residual_true:.2e} | "
          f"oracle outer={ref.outer_iters} | rel err vs FP64 oracle {err:.2e}", flush=True)
    assert st.status == 0
    assert st.rel_residual_true <= 1e-10
    # the error against the FP64 oracle is stated per solve; at 1e-10 residual it
    # is bounded by the operator's conditioning (layered 3-D: ~1e-7)
    assert err <= 1e-6
    assert st.outer_iters <= 1.5 * ref.outer_iters + 1


def test_batch_overlaps_on_own_streams():
    case("solve_batch on separate streams")
    import torch
    from paper_math_9809043_amd import mscg
    Ps = [synth.request_problem(synth.Request(i, 0.0, side, 900 + i)) for i, side in enumerate((512, 256, 128, 64))]
    probs, fs, ps, singles = [], [], [], []
    for P in Ps:
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            prob = mscg.Problem(mscg.Grid(dim=2, n=P.n), mscg.Options(), stream=s)
            prob.set_permeability(torch.tensor(P.kx, device="cuda"), torch.tensor(P.ky, device="cuda"))
            f = torch.tensor(P.f, device="cuda")
            q = torch.zeros(P.N, dtype=torch.float64, device="cuda")
        prob.solve(f, q, P.tol)
        torch.cuda.synchronize()
        probs.append(prob)
        fs.append(f)
        singles.append(q.cpu().numpy())
        with torch.cuda.stream(s):
            ps.append(torch.zeros(P.N, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    stats = mscg.solve_batch(probs, fs, ps, [P.tol for P in Ps])
    torch.cuda.synchronize()
    for st, p, s in zip(stats, ps, singles):
        assert st.status == 0 and st.rel_residual_true <= 1e-8
        assert np.array_equal(p.cpu().numpy(), s)


def test_repeated_solves_are_bitwise_identical():
    case("repeatability of one-workgroup inner solvers")
    from paper_math_9809043_amd import mscg, serve
    for prec in (mscg.FP64, mscg.MIXED):
        for side in (128, 256, 512):
            req = synth.Request(0, 0.0, side, 502)
            ref = None
            for rep in range(4):
                st, p, k, f = serve.solve_alone(req, mscg.Options(precision=prec), tol=1e-8)
                x = p.cpu().numpy()
                assert st.status == 0, (prec, side, rep, mscg.last_error())
                if ref is None:
                    ref = x
                else:
                    assert np.array_equal(ref, x), (prec, side, rep)


def test_one_workgroup_solvers_ignore_what_lds_held_before():
    """Solves of a 3-D semi-coarsened problem (last inner level in the cell-
    strided one-workgroup kernel) give the same bits whatever ran before them:
    other problems' kernels leave arbitrary data in LDS, which a boundary cell
    must never read (it once did, through a zero coefficient times a stale
    value, and 0 * NaN is NaN)."""
    case("one-workgroup solvers after other kernels")
    import torch
    from paper_math_9809043_amd import mscg
    cube = synth.layered_3d(2, 32, n_layers=4)
    strip = synth.anisotropic_strip_2d(4, 512, 128)

    def run(P, prec, **o):
        grid = mscg.Grid(dim=P.dim, n=P.n, bc_type=P.bc_type, bc_value=P.bc_value, length=P.length)
        prob = mscg.Problem(grid, mscg.Options(precision=prec, semi_coarsen=1, **o))
        prob.set_permeability(torch.tensor(P.kx, device="cuda"), torch.tensor(P.ky, device="cuda"),
                              torch.tensor(P.kz, device="cuda") if P.dim == 3 else None)
        p = torch.zeros(P.N, dtype=torch.float64, device="cuda")
        st = prob.solve(torch.tensor(P.f, device="cuda"), p, P.tol)
        torch.cuda.synchronize()
        return st, p.cpu().numpy()

    for prec in (mscg.FP64, mscg.MIXED):
        ref = None
        for rep in range(3):
            run(strip, prec, axis_weight=(1, 100, 1))
            st, x = run(cube, prec, axis_weight=(1, 1, 0.01), interp=1)
            assert st.status == 0 and st.rel_residual_true <= 1e-10, (prec, rep, mscg.last_error())
            if ref is None:
                ref = x
            assert np.array_equal(ref, x), (prec, rep)
