"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
solutions, dense linear algebra built independently in numpy from the
definitions, identities of Section 2 (eqs. 2.5, 2.7a, 2.10), or physical
invariants of the coarse graining of Section 3.
"""
import numpy as np
import pytest

import oracle
from paper_math_9809043_amd import synth

RNG = np.random.default_rng(12345)


def dense_from_T(dim, n, tx, ty, tz=None):
    """Independent dense assembly of the finite-volume operator from face arrays."""
    nx, ny = n[0], n[1]
    nz = n[2] if dim == 3 else 1
    N = nx * ny * nz
    A = np.zeros((N, N))
    TX = tx.reshape(nz, ny, nx + 1)
    TY = ty.reshape(nz, ny + 1, nx)
    TZ = tz.reshape(nz + 1, ny, nx) if dim == 3 else None

    def idx(i, j, k):
        return i + nx * (j + ny * k)

    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = idx(i, j, k)
                faces = [(TX[k, j, i], (i - 1, j, k)), (TX[k, j, i + 1], (i + 1, j, k)),
                         (TY[k, j, i], (i, j - 1, k)), (TY[k, j + 1, i], (i, j + 1, k))]
                if dim == 3:
                    faces += [(TZ[k, j, i], (i, j, k - 1)), (TZ[k + 1, j, i], (i, j, k + 1))]
                for t, (a, b, cc) in faces:
                    A[c, c] += t
                    if 0 <= a < nx and 0 <= b < ny and 0 <= cc < nz:
                        A[c, idx(a, b, cc)] -= t
    return A


def problem_2d(n, lo=-1, hi=1, seed=0, bc_value=(0.0, 1.0)):
    return synth.smoothed_lognormal_2d(seed, n[0], n[1], lo=lo, hi=hi, bc_value=bc_value)


def rhs(P, tx, ty, tz=None):
    """b = f |V| + T_b p_D on Dirichlet faces, written out independently."""
    nx, ny = P.n[0], P.n[1]
    nz = P.n[2] if P.dim == 3 else 1
    h = [P.length[a] / P.n[a] for a in range(3)]
    vol = h[0] * h[1] * (h[2] if P.dim == 3 else 1.0)
    b = (P.f * vol).reshape(nz, ny, nx).copy()
    TX = tx.reshape(nz, ny, nx + 1)
    TY = ty.reshape(nz, ny + 1, nx)
    if P.bc_type[0]:
        b[:, :, 0] += TX[:, :, 0] * P.bc_value[0]
    if P.bc_type[1]:
        b[:, :, -1] += TX[:, :, -1] * P.bc_value[1]
    if P.bc_type[2]:
        b[:, 0, :] += TY[:, 0, :] * P.bc_value[2]
    if P.bc_type[3]:
        b[:, -1, :] += TY[:, -1, :] * P.bc_value[3]
    if P.dim == 3:
        TZ = tz.reshape(nz + 1, ny, nx)
        if P.bc_type[4]:
            b[0] += TZ[0] * P.bc_value[4]
        if P.bc_type[5]:
            b[-1] += TZ[-1] * P.bc_value[5]
    return b.reshape(-1)


# ---------------------------------------------------------------- level plan

def test_level_plan_matches_configs():
    # 32x32 recurses to an 8x8 coarsest grid (the small configuration)
    assert oracle.level_plan(2, (32, 32, 1)) == [(32, 32, 1), (8, 8, 1)]
    assert oracle.level_plan(2, (1024, 1024, 1)) == [(1024, 1024, 1), (256, 256, 1), (64, 64, 1), (16, 16, 1)]
    assert oracle.level_plan(3, (128, 128, 128)) == [(128, 128, 128), (32, 32, 32), (8, 8, 8)]
    assert oracle.level_plan(2, (96, 40, 1)) == [(96, 40, 1), (24, 10, 1)]  # 10 is not divisible by 4
    assert oracle.level_plan(2, (128, 64, 1)) == [(128, 64, 1), (32, 16, 1)]


# ---------------------------------------------------------------- face T (Section 3)

def test_face_T_harmonic_and_boundaries():
    nx, ny = 4, 3
    kx = RNG.uniform(0.5, 2.0, nx * ny)
    ky = RNG.uniform(0.5, 2.0, nx * ny)
    h = (1.0 / nx, 1.0 / ny, 1.0)
    tx, ty, _ = oracle.face_T(2, (nx, ny, 1), h, kx, ky, None, [1, 0, 1, 0, 0, 0])
    K = kx.reshape(ny, nx)
    TX = tx.reshape(ny, nx + 1)
    ax = h[1] / h[0]
    for j in range(ny):
        assert TX[j, 0] == pytest.approx(2 * ax * K[j, 0], rel=1e-15)  # Dirichlet: value at the face
        assert TX[j, nx] == 0.0                                        # Neumann: no flow
        for i in range(1, nx):
            a, b = K[j, i - 1], K[j, i]
            # series resistance of two half cells = 1/harmonic mean
            assert 1.0 / TX[j, i] == pytest.approx((0.5 / a + 0.5 / b) / ax, rel=1e-14)
    TY = ty.reshape(ny + 1, nx)
    KY = ky.reshape(ny, nx)
    ay = h[0] / h[1]
    assert np.allclose(TY[0], 2 * ay * KY[0], rtol=1e-15)
    assert np.all(TY[ny] == 0.0)


def test_operator_is_symmetric_and_positive_definite():
    P = problem_2d((12, 8), lo=-3, hi=3)
    tx, ty, _ = oracle.face_T(2, P.n, (1 / 12, 1 / 8, 1), P.kx, P.ky, None, P.bc_type)
    A = dense_from_T(2, P.n, tx, ty)
    # the oracle's operator equals the independent assembly
    cols = np.stack([oracle.apply_A(2, P.n, (tx, ty, None), e) for e in np.eye(P.N)], axis=1)
    assert np.allclose(cols, A, rtol=0, atol=1e-13 * np.abs(A).max())
    assert np.allclose(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0


# ---------------------------------------------------------------- closed-form solutions

def test_constant_K_gives_linear_ramp_with_zero_iterations():
    P = problem_2d((32, 32))
    P.kx[:] = 3.7
    P.ky[:] = 3.7
    P.f[:] = 0
    r = oracle.solve(P)
    xc = (np.arange(32) + 0.5) / 32
    assert r.outer_iters == 0 and r.status == 0
    assert np.abs(r.p.reshape(32, 32) - xc[None, :]).max() < 1e-14


def test_layered_in_y_gives_linear_ramp():
    P = problem_2d((32, 16))
    K = 10.0 ** RNG.uniform(-3, 3, 16)
    P.kx = np.repeat(K, 32)
    P.ky = P.kx.copy()
    P.f[:] = 0
    r = oracle.solve(P)
    xc = (np.arange(32) + 0.5) / 32
    assert np.abs(r.p.reshape(16, 32) - xc[None, :]).max() < 1e-12


def test_layered_in_x_matches_series_resistance():
    n = 32
    P = problem_2d((n, n), bc_value=(0.25, 2.0))
    Kc = 10.0 ** RNG.uniform(-2, 2, n)
    P.kx = np.tile(Kc, n)
    P.ky = P.kx.copy()
    P.f[:] = 0
    r = oracle.solve(P, tol=1e-13)
    # 1-D: resistances from the left face to each centre, in series
    h = 1.0 / n
    res = np.zeros(n)
    acc = 0.5 * h / Kc[0]
    res[0] = acc
    for i in range(1, n):
        acc += 0.5 * h / Kc[i - 1] + 0.5 * h / Kc[i]
        res[i] = acc
    total = acc + 0.5 * h / Kc[-1]
    p_exact = 0.25 + (2.0 - 0.25) * res / total
    assert np.abs(r.p.reshape(n, n) - p_exact[None, :]).max() < 1e-11


def test_continuous_manufactured_solution_second_order():
    # -lap p = f with p = sin(pi x) cos(pi y): p = 0 on x = 0, 1; dp/dy = 0 on y = 0, 1
    errs = []
    for n in (32, 64):
        P = problem_2d((n, n), bc_value=(0.0, 0.0))
        P.kx[:] = 1.0
        P.ky[:] = 1.0
        xc = (np.arange(n) + 0.5) / n
        X, Y = np.meshgrid(xc, xc)
        P.f = (2 * np.pi ** 2 * np.sin(np.pi * X) * np.cos(np.pi * Y)).reshape(-1)
        r = oracle.solve(P, tol=1e-12)
        exact = (np.sin(np.pi * X) * np.cos(np.pi * Y)).reshape(-1)
        errs.append(np.sqrt(np.mean((r.p - exact) ** 2)))
    assert errs[0] / errs[1] > 3.5  # O(h^2)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("n,interp,lo,hi", [((32, 32), 0, -1, 1), ((64, 32), 0, -3, 3), ((32, 32), 1, -3, 3),
                                             ((64, 64), 1, -1, 1)])
def test_solve_matches_dense_solution(n, interp, lo, hi):
    P = problem_2d(n, lo=lo, hi=hi, seed=3)
    h = (1 / n[0], 1 / n[1], 1)
    tx, ty, _ = oracle.face_T(2, P.n, h, P.kx, P.ky, None, P.bc_type)
    A = dense_from_T(2, P.n, tx, ty)
    b = rhs(P, tx, ty)
    x = np.linalg.solve(A, b)
    r = oracle.solve(P, tol=1e-10, interp=interp)
    assert r.status == 0
    assert np.linalg.norm(b - A @ r.p) / np.linalg.norm(b) < 1e-10
    assert r.rel_residual_true < 1e-10
    assert np.linalg.norm(r.p - x) / np.linalg.norm(x) < 1e-8


def test_solve_3d_matches_dense_solution():
    P = synth.layered_3d(1, 16, n_layers=4, amp=1.0)
    h = (1 / 16, 1 / 16, 1 / 16)
    tx, ty, tz = oracle.face_T(3, P.n, h, P.kx, P.ky, P.kz, P.bc_type)
    A = dense_from_T(3, P.n, tx, ty, tz)
    b = rhs(P, tx, ty, tz)
    x = np.linalg.solve(A, b)
    r = oracle.solve(P, tol=1e-10, min_side=2, interp=1)
    assert r.nlev == 2 and r.status == 0
    assert np.linalg.norm(r.p - x) / np.linalg.norm(x) < 1e-8


def test_discrete_manufactured_solution():
    # Section 4 accuracy test: put the residual of a known field into the source
    n = 64
    P = problem_2d((n, n), lo=-2, hi=2, bc_value=(0.0, 0.0))
    h = 1.0 / n
    tx, ty, _ = oracle.face_T(2, P.n, (h, h, 1), P.kx, P.ky, None, P.bc_type)
    A = dense_from_T(2, P.n, tx, ty)
    xc = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xc, xc)
    pstar = (np.sin(3 * X) * np.cos(2 * Y) + 0.1 * RNG.standard_normal((n, n))).reshape(-1)
    P.f = A @ pstar / (h * h)
    r = oracle.solve(P, tol=1e-12)
    assert np.abs(r.p - pstar).max() < 1e-9


# ---------------------------------------------------------------- coarse graining (Section 3)

def test_coarsening_uniform_2d():
    n = 16
    P = problem_2d((n, n))
    P.kx[:] = 1.0
    P.ky[:] = 1.0
    hier = oracle.hierarchy_T(P, min_side=2)
    (d1, tx, ty, _) = hier[1]
    assert d1 == (4, 4, 1)
    TX = tx.reshape(4, 5)
    TY = ty.reshape(5, 4)
    # 2-D transmissibility is scale invariant; Dirichlet faces keep 2K, Neumann 0
    assert np.allclose(TX, np.array([2, 1, 1, 1, 2])[None, :], rtol=1e-14)
    assert np.allclose(TY, np.array([0, 1, 1, 1, 0])[:, None], rtol=1e-14)


def test_coarsening_uniform_3d():
    P = synth.layered_3d(0, 16, n_layers=1, amp=0.0, kz_ratio=1.0)
    hier = oracle.hierarchy_T(P, min_side=2)
    d0, tx0, _, _ = hier[0]
    d1, tx1, ty1, tz1 = hier[1]
    h = 1 / 16
    assert np.allclose(tx0.reshape(16, 16, 17)[:, :, 1:-1], h)     # T = K h
    TX = tx1.reshape(4, 4, 5)
    assert np.allclose(TX[:, :, 1:-1], 4 * h, rtol=1e-14)          # K H with H = 4h
    assert np.allclose(TX[:, :, 0], 8 * h, rtol=1e-14)             # Dirichlet 2 K H
    TZ = tz1.reshape(5, 4, 4)
    assert np.allclose(TZ[1:-1], 4 * h, rtol=1e-14) and np.all(TZ[0] == 0) and np.all(TZ[-1] == 0)  # Neumann z


@pytest.mark.parametrize("dim", [2, 3])
def test_coarsening_reproduces_coarse_discretisation(dim):
    """K constant on every coarse cell: coarse graining gives exactly the faces
    of the coarse grid's own discretisation (harmonic means, Dirichlet 2K)."""
    nc = 4
    n = 4 * nc
    if dim == 2:
        Kc = 10.0 ** RNG.uniform(-3, 3, (nc, nc))
        K = np.kron(Kc, np.ones((4, 4))).reshape(-1)
        P = problem_2d((n, n))
        P.kx, P.ky = K.copy(), K.copy()
        P.bc_type = [1, 1, 1, 0, 0, 0]
        hc = (1 / nc, 1 / nc, 1.0)
        expect = oracle.face_T(2, (nc, nc, 1), hc, Kc.reshape(-1), Kc.reshape(-1), None, P.bc_type)
    else:
        Kc = 10.0 ** RNG.uniform(-3, 3, (nc, nc, nc))
        K = np.kron(Kc, np.ones((4, 4, 4))).reshape(-1)
        P = synth.layered_3d(0, n, n_layers=1)
        P.kx, P.ky, P.kz = K.copy(), K.copy() * 2, K.copy() * 0.5
        P.bc_type = [1, 1, 0, 1, 1, 0]
        hc = (1 / nc, 1 / nc, 1 / nc)
        expect = oracle.face_T(3, (nc, nc, nc), hc, Kc.reshape(-1), 2 * Kc.reshape(-1), 0.5 * Kc.reshape(-1),
                               P.bc_type)
    hier = oracle.hierarchy_T(P, min_side=2)
    got = hier[1][1:]
    for g, e in zip(got, expect):
        if e is None:
            continue
        assert np.allclose(g, e, rtol=1e-13, atol=0)


def test_coarsening_parallel_layers_exact():
    # K(y) layers along the flow: coarse x-transmissivity = arithmetic mean of the rows
    n = 16
    P = problem_2d((n, n))
    K = 10.0 ** RNG.uniform(-2, 2, n)
    P.kx = np.repeat(K, n)
    P.ky = P.kx.copy()
    hier = oracle.hierarchy_T(P, min_side=2)
    TX = hier[1][1].reshape(4, 5)
    expect = K.reshape(4, 4).mean(axis=1)
    assert np.allclose(TX[:, 1:-1], expect[:, None], rtol=1e-13)


# ---------------------------------------------------------------- transfers (Section 3)

@pytest.mark.parametrize("interp", [oracle.LINEAR, oracle.CONSTANT])
def test_transfer_identities(interp):
    fd, s = (32, 16, 1), (4, 4, 1)
    nc = 8 * 4
    ones_c = np.ones(nc)
    assert np.allclose(oracle.prolong_add(2, fd, s, ones_c, np.zeros(512), interp), 1.0, rtol=0, atol=1e-15)
    u = RNG.standard_normal(nc)
    v = RNG.standard_normal(512)
    Eu = oracle.prolong_add(2, fd, s, u, np.zeros(512), interp)
    Rv = oracle.restrict(2, fd, s, v, interp)
    assert abs(Eu @ v - u @ Rv) < 1e-12 * np.abs(Eu).sum() * np.abs(v).max()


def test_linear_extension_weights():
    fd, s = (32, 32, 1), (4, 4, 1)
    e = np.zeros(64)
    e[2 + 8 * 3] = 1.0  # interior coarse cell (2, 3)
    Ee = oracle.prolong_add(2, fd, s, e, np.zeros(1024)).reshape(32, 32)
    w = np.array([1, 3, 5, 7, 7, 5, 3, 1]) / 8.0
    expect = np.zeros((32, 32))
    expect[3 * 4 - 2:3 * 4 + 6, 2 * 4 - 2:2 * 4 + 6] = np.outer(w, w)
    assert np.array_equal(Ee, expect)  # k/8 weights are exact in binary
    # boundary coarse cell: zero slope => fine cells 0, 1 take the coarse value
    e = np.zeros(64)
    e[0] = 1.0
    Ee = oracle.prolong_add(2, fd, s, e, np.zeros(1024)).reshape(32, 32)
    wb = np.array([1, 1, 7 / 8, 5 / 8, 3 / 8, 1 / 8])
    assert np.array_equal(Ee[:6, :6], np.outer(wb, wb))
    # affine functions are reproduced away from the clamped boundary cells
    Xc = (np.arange(8) + 0.5) * 4
    y = (1.5 + 0.25 * Xc)[None, :] * np.ones((8, 1))
    Ey = oracle.prolong_add(2, fd, s, y.reshape(-1), np.zeros(1024)).reshape(32, 32)
    xf = np.arange(32) + 0.5
    assert np.allclose(Ey[:, 2:30], (1.5 + 0.25 * xf[2:30])[None, :], rtol=0, atol=1e-14)


# ---------------------------------------------------------------- smoother (eq. 2.3, Section 3)

def splitting_dense(A, nx, ny, nz=1):
    """P = (D+L) D^-1 (D+U) of symmetric Gauss-Seidel in red-black order, built
    from the dense operator: permute reds first, split, permute back."""
    N = A.shape[0]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    colour = ((i + j + k) % 2).reshape(-1)
    perm = np.concatenate([np.where(colour == 0)[0], np.where(colour == 1)[0]])
    Ap = A[np.ix_(perm, perm)]
    D = np.diag(np.diag(Ap))
    L = np.tril(Ap, -1)
    U = np.triu(Ap, 1)
    Pp = (D + L) @ np.linalg.inv(D) @ (D + U)
    inv = np.argsort(perm)
    Pm = Pp[np.ix_(inv, inv)]
    return Pm, Pm - A


def test_sgs_splitting():
    n = (8, 6, 1)
    P = problem_2d(n[:2], lo=-2, hi=2)
    tx, ty, _ = oracle.face_T(2, n, (1 / 8, 1 / 6, 1), P.kx, P.ky, None, P.bc_type)
    A = dense_from_T(2, n, tx, ty)
    Pm, Qm = splitting_dense(A, 8, 6)
    T = (tx, ty, None)
    # one oracle step from zero applies P^-1
    Pinv = np.stack([oracle.sgs(2, n, T, e, np.zeros(48), 1) for e in np.eye(48)], axis=1)
    assert np.allclose(Pinv @ Pm, np.eye(48), atol=1e-12)
    # and from any x it is x + P^-1 (r - A x)
    x = RNG.standard_normal(48)
    r = RNG.standard_normal(48)
    assert np.allclose(oracle.sgs(2, n, T, r, x, 1), x + np.linalg.solve(Pm, r - A @ x), atol=1e-12)
    # P symmetric positive definite, Q symmetric positive semi-definite (Section 2)
    assert np.allclose(Pm, Pm.T, atol=1e-12)
    assert np.linalg.eigvalsh((Pm + Pm.T) / 2).min() > 0
    assert np.linalg.eigvalsh((Qm + Qm.T) / 2).min() > -1e-10
    # a repeated colour is a no-op, bitwise: R,B,B,R,R,B,B,R == R,B,R,B,R from zero
    xa = oracle.sgs(2, n, T, r, np.zeros(48), 2)
    xb = np.zeros(48)
    for c in (0, 1, 0, 1, 0):
        xb = oracle.gs_colour(2, n, T, r, xb, c)
    assert np.array_equal(xa, xb)


# ---------------------------------------------------------------- preconditioner (eqs. 2.5, 2.7a, 2.10)

def test_modified_jacobi_splitting():
    """P = 2D, Q = D - U - L (Section 3): a step applies x + (2D)^-1 (r - A x),
    P - Q = A, and unlike plain Jacobi the iteration damps the checkerboard
    mode (the spectrum of P^-1 Q stays inside (-1, 1))."""
    n = (8, 6, 1)
    P = problem_2d(n[:2], lo=-2, hi=2, seed=4)
    tx, ty, _ = oracle.face_T(2, n, (1 / 8, 1 / 6, 1), P.kx, P.ky, None, P.bc_type)
    A = dense_from_T(2, n, tx, ty)
    D = np.diag(np.diag(A))
    Pm, Qm = 2 * D, D - (A - D)
    assert np.allclose(Pm - Qm, A)
    T = (tx, ty, None)
    x = RNG.standard_normal(48)
    r = RNG.standard_normal(48)
    assert np.allclose(oracle.mjac(2, n, T, r, x, 1), x + np.linalg.solve(Pm, r - A @ x), atol=1e-12)
    x3 = x.copy()
    for _ in range(3):
        x3 = x3 + np.linalg.solve(Pm, r - A @ x3)
    assert np.allclose(oracle.mjac(2, n, T, r, x, 3), x3, atol=1e-12)
    ev = np.linalg.eigvals(np.linalg.solve(Pm, Qm)).real
    assert ev.max() < 1 and ev.min() > -1
    ev_plain = np.linalg.eigvals(np.linalg.solve(D, D - A)).real
    assert ev_plain.min() < ev.min()  # plain Jacobi leaves the checkerboard mode near -1


def two_level_dense(P, interp, m=4):
    n = P.n
    h = (1 / n[0], 1 / n[1], 1)
    hier = oracle.hierarchy_T(P, min_side=2, max_levels=2)
    (d0, tx, ty, _), (d1, ctx, cty, _) = hier
    A = dense_from_T(2, d0, tx, ty)
    Ac = dense_from_T(2, d1, ctx, cty)

    def e1(nf, s):
        nc = nf // s
        E = np.zeros((nf, nc))
        for i in range(nf):
            if interp == oracle.CONSTANT:
                E[i, i // s] = 1
                continue
            xi = (i + 0.5) / s - 0.5
            if xi <= 0:
                E[i, 0] = 1
            elif xi >= nc - 1:
                E[i, nc - 1] = 1
            else:
                b = int(np.floor(xi))
                E[i, b] += 1 - (xi - b)
                E[i, b + 1] += xi - b
        return E

    E = np.kron(e1(n[1], 4), e1(n[0], 4))
    Pm, Qm = splitting_dense(A, n[0], n[1])
    return A, Ac, E, Pm, Qm


@pytest.mark.parametrize("interp,splitting", [(oracle.LINEAR, oracle.SGS), (oracle.CONSTANT, oracle.SGS),
                                              (oracle.LINEAR, oracle.JACOBI)])
def test_preconditioner_is_eq_2_10(interp, splitting):
    P = problem_2d((16, 16), lo=-3, hi=3, seed=7)
    m = 4
    A, Ac, E, Pm, Qm = two_level_dense(P, interp, m)
    if splitting == oracle.JACOBI:
        D = np.diag(np.diag(A))
        Pm, Qm = 2 * D, D - (A - D)
    N = A.shape[0]
    Pinv = np.linalg.inv(Pm)
    H = Pinv @ Qm
    W = E @ np.linalg.solve(Ac, E.T)
    Hm = np.linalg.matrix_power(H, m)
    Minv = Hm @ W @ Hm.T + sum(np.linalg.matrix_power(H, j) @ Pinv for j in range(2 * m))
    got = np.stack([oracle.precond(P, e, interp=interp, max_levels=2, min_side=2, splitting=splitting)
                    for e in np.eye(N)], axis=1)
    assert np.allclose(got, Minv, rtol=0, atol=1e-10 * np.abs(Minv).max())
    # symmetric positive definite (Tatebe's condition, Section 2)
    assert np.allclose(got, got.T, atol=1e-12 * np.abs(got).max())
    assert np.linalg.eigvalsh((got + got.T) / 2).min() > 0
    # eq. 2.7a and the norm bound
    lhs = A @ got - np.eye(N)
    QP = Qm @ Pinv
    QPm = np.linalg.matrix_power(QP, m)
    rhs7 = QPm @ (A @ W - np.eye(N)) @ QPm
    assert np.allclose(lhs, rhs7, atol=1e-8 * np.abs(lhs).max())
    # eq. 2.5: W = A^-1 turns the same construction into A^-1
    Ainv = np.linalg.inv(A)
    M5 = Hm @ Ainv @ Hm.T + sum(np.linalg.matrix_power(H, j) @ Pinv for j in range(2 * m))
    assert np.allclose(M5, Ainv, atol=1e-9 * np.abs(Ainv).max())


def test_polynomial_special_case():
    # W = P^-1 gives the first 2m+1 terms of the Neumann series (Section 2.1)
    P = problem_2d((8, 8), lo=-1, hi=1, seed=2)
    A, Ac, E, Pm, Qm = two_level_dense(P, oracle.LINEAR, 2)
    Pinv = np.linalg.inv(Pm)
    H = Pinv @ Qm
    m = 2
    Hm = np.linalg.matrix_power(H, m)
    M = Hm @ Pinv @ Hm.T + sum(np.linalg.matrix_power(H, j) @ Pinv for j in range(2 * m))
    series = sum(np.linalg.matrix_power(H, j) @ Pinv for j in range(2 * m + 1))
    assert np.allclose(M, series, atol=1e-12 * np.abs(series).max())


# ---------------------------------------------------------------- Cholesky

def test_cholesky_matches_numpy():
    B = RNG.standard_normal((30, 30))
    S = B @ B.T + 30 * np.eye(30)
    rc, Lf = oracle.cholesky(S)
    assert rc == 0
    assert np.allclose(Lf, np.linalg.cholesky(S), rtol=1e-13, atol=1e-13)
    b = RNG.standard_normal(30)
    assert np.allclose(oracle.cholesky_solve(Lf, b), np.linalg.solve(S, b), rtol=1e-12)
    rc, _ = oracle.cholesky(-S)
    assert rc == -6


# ---------------------------------------------------------------- behaviour (Section 4 expectations)

def test_iterations_nearly_constant_in_N():
    its = []
    for n in (64, 128, 256):
        P = synth.smoothed_lognormal_2d(1, n, lo=-3, hi=3)
        its.append(oracle.solve(P, tol=1e-8).outer_iters)
    assert max(its) - min(its) <= 3


def test_all_neumann_is_singular():
    P = problem_2d((32, 32))
    P.bc_type = [0, 0, 0, 0, 0, 0]
    r = oracle.solve(P)
    assert r.status == -6


# ------------------------------------------------------- semi-coarsening (Section 5)

@pytest.mark.parametrize("n", [(32, 32), (64, 32)])
def test_jacobi_solve_matches_dense_solution(n):
    P = problem_2d(n, lo=-2, hi=2, seed=5)
    h = (1 / n[0], 1 / n[1], 1)
    tx, ty, _ = oracle.face_T(2, P.n, h, P.kx, P.ky, None, P.bc_type)
    A = dense_from_T(2, P.n, tx, ty)
    b = rhs(P, tx, ty)
    x = np.linalg.solve(A, b)
    r = oracle.solve(P, tol=1e-10, splitting=oracle.JACOBI, min_side=2)
    assert r.status == 0 and r.nlev >= 3
    assert np.linalg.norm(r.p - x) / np.linalg.norm(x) < 1e-8


@pytest.mark.parametrize("dim,n,length", [(2, (1024, 1024, 1), (1, 1, 1)), (2, (32, 32, 1), (1, 1, 1)),
                                          (2, (288, 160, 1), (1, 1, 1)), (3, (128, 128, 128), (1, 1, 1)),
                                          (3, (32, 32, 32), (1, 1, 1))])
def test_semi_plan_with_equal_weights_is_the_uniform_plan(dim, n, length):
    """With no anisotropy and near-square cells every axis is coarsened together."""
    assert oracle.level_plan(dim, n, axis_weight=(1, 1, 1), length=length) == oracle.level_plan(dim, n)


def effective_sizes(dims, length, w):
    return [length[a] / dims[a] / np.sqrt(w[a]) for a in range(len(w))]


@pytest.mark.parametrize("dim,n,length,w", [(2, (512, 128, 1), (4, 1, 1), (1, 100, 1)),
                                            (2, (2048, 512, 1), (4, 1, 1), (1, 100, 1)),
                                            (3, (128, 128, 128), (1, 1, 1), (1, 1, 0.01)),
                                            (3, (32, 32, 32), (1, 1, 1), (1, 1, 0.01))])
def test_semi_plan_coarsens_the_finest_direction_first(dim, n, length, w):
    """Section 5: coarsening aims at cells of aspect ratio one, so the direction
    in which cells are effectively smallest (the strongly coupled one) is
    coarsened first.  At every level, an axis left alone while it could have
    been coarsened is effectively coarser than every axis that was coarsened;
    while no axis has reached its minimum side, the effective aspect ratio never
    grows beyond its start or the factor 4."""
    plan = oracle.level_plan(dim, n, axis_weight=w, length=length)
    assert len(plan) >= 3
    start = effective_sizes(plan[0], length, w[:dim])
    first = [a for a in range(dim) if plan[1][a] != plan[0][a]]
    assert first == [int(np.argmin(start[:dim]))] or (dim == 3 and first == [0, 1])
    for cur, nxt in zip(plan, plan[1:]):
        e = effective_sizes(cur, length, w[:dim])
        done = [a for a in range(dim) if nxt[a] != cur[a]]
        assert all(cur[a] == 4 * nxt[a] for a in done) and done
        left = [a for a in range(dim) if a not in done and cur[a] % 4 == 0 and cur[a] // 4 >= 8]
        for a in left:
            assert all(e[a] > e[b] for b in done)
        if all(cur[a] % 4 == 0 and cur[a] // 4 >= 8 for a in range(dim)):  # no axis at its limit yet
            en = effective_sizes(nxt, length, w[:dim])
            assert max(en) / min(en) <= max(max(start) / min(start), 4.0) + 1e-12


def test_semi_coarsened_solve_matches_dense_solution():
    """A 4:1 strip with ky = 100 kx, four semi-coarsened levels, against the
    dense solution."""
    P = synth.anisotropic_strip_2d(2, 64, 16)
    h = (P.length[0] / 64, 1 / 16, 1)
    tx, ty, _ = oracle.face_T(2, P.n, h, P.kx, P.ky, None, P.bc_type)
    A = dense_from_T(2, P.n, tx, ty)
    b = rhs(P, tx, ty)
    x = np.linalg.solve(A, b)
    for interp in (oracle.LINEAR, oracle.CONSTANT):
        r = oracle.solve(P, tol=1e-10, min_side=2, interp=interp, axis_weight=(1, 100, 1))
        assert r.status == 0 and r.nlev == 4
        assert r.level_n == [(64, 16, 1), (64, 4, 1), (16, 4, 1), (4, 4, 1)]
        assert np.linalg.norm(r.p - x) / np.linalg.norm(x) < 1e-8


def test_semi_coarsening_helps_anisotropic_problems():
    """The paper's observation on the anisotropic strip: aspect-ratio-aware
    coarsening keeps the outer iteration count small where uniform coarsening
    does not (here 7 against 61 on the strip, 5 against 200+ on the layered
    cube with linear extension)."""
    strip = synth.anisotropic_strip_2d(1, 512, 128)
    uni = oracle.solve(strip)
    semi = oracle.solve(strip, axis_weight=(1, 100, 1))
    assert semi.status == 0 and semi.rel_residual_true < 1e-10
    assert semi.outer_iters * 4 < uni.outer_iters
    cube = synth.layered_3d(2, 32, n_layers=4)
    semi3 = oracle.solve(cube, axis_weight=(1, 1, 0.01))
    assert semi3.status == 0 and semi3.outer_iters <= 8


# ------------------------------------------------- Tatebe's multigrid preconditioner (eq. 2.9)

def ext_1d(nf, s, interp):
    """Dense 1-D extension operator (fine nf cells from nf / s coarse cells), written out from
    its definition: cell-centred linear interpolation with zero slope at the boundary, or
    piecewise constant."""
    nc = nf // s
    E = np.zeros((nf, nc))
    for i in range(nf):
        if interp == oracle.CONSTANT:
            E[i, i // s] = 1
            continue
        xi = (i + 0.5) / s - 0.5
        if xi <= 0:
            E[i, 0] = 1
        elif xi >= nc - 1:
            E[i, nc - 1] = 1
        else:
            b = int(np.floor(xi))
            E[i, b] += 1 - (xi - b)
            E[i, b + 1] += xi - b
    return E


@pytest.mark.parametrize("interp", [oracle.LINEAR, oracle.CONSTANT])
def test_mgcg_preconditioner_is_eq_2_9(interp):
    # three levels (32^2, 8^2, 2^2): M_2^-1 = A_2^-1 exactly, and each finer level applies
    # M_k^-1 = H^m (E M_{k+1}^-1 R) (H^T)^m + sum_{j<2m} H^j P^-1 with H = P^-1 Q (eq. 2.9)
    P = problem_2d((32, 32), lo=-2, hi=2, seed=11)
    m = 2
    hier = oracle.hierarchy_T(P, min_side=2, max_levels=3)
    assert [d[:2] for d, *_ in hier] == [(32, 32), (8, 8), (2, 2)]
    As = [dense_from_T(2, d, tx, ty) for d, tx, ty, _ in hier]
    Minv = np.linalg.inv(As[2])
    for k in (1, 0):
        d = hier[k][0]
        E = np.kron(ext_1d(d[1], 4, interp), ext_1d(d[0], 4, interp))
        Pm, Qm = splitting_dense(As[k], d[0], d[1])
        Pinv = np.linalg.inv(Pm)
        H = Pinv @ Qm
        Hm = np.linalg.matrix_power(H, m)
        Minv = Hm @ (E @ Minv @ E.T) @ Hm.T + sum(np.linalg.matrix_power(H, j) @ Pinv for j in range(2 * m))
    N = As[0].shape[0]
    got = np.stack([oracle.precond(P, e, interp=interp, m=m, min_side=2, max_levels=3, cycle=oracle.MGCG)
                    for e in np.eye(N)], axis=1)
    assert np.allclose(got, Minv, rtol=0, atol=1e-10 * np.abs(Minv).max())
    # Tatebe's condition (Section 2): symmetric positive definite
    assert np.allclose(got, got.T, atol=1e-12 * np.abs(got).max())
    assert np.linalg.eigvalsh((got + got.T) / 2).min() > 0
    # with three levels the recursive form differs: its level-1 coarse part is a PCG solve
    rec = oracle.precond(P, np.eye(N)[0], interp=interp, m=m, min_side=2, max_levels=3, eps2=1e-30)
    assert np.abs(rec - got[:, 0]).max() > 1e-6 * np.abs(got[:, 0]).max()


def test_mgcg_two_levels_is_the_recursive_method():
    # with one coarse level both forms use the exact coarse inverse (eq. 2.9 with M_1 = A_1, eq. 2.10)
    P = problem_2d((64, 64), lo=-3, hi=3, seed=4)
    a = oracle.solve(P, tol=1e-10, max_levels=2)
    b = oracle.solve(P, tol=1e-10, max_levels=2, cycle=oracle.MGCG)
    assert a.outer_iters == b.outer_iters and np.array_equal(a.p, b.p)


@pytest.mark.parametrize("n,interp", [((32, 32), oracle.LINEAR), ((64, 32), oracle.LINEAR),
                                      ((64, 64), oracle.CONSTANT)])
def test_mgcg_solve_matches_dense_solution(n, interp):
    P = problem_2d(n, lo=-2, hi=2, seed=9)
    h = (1 / n[0], 1 / n[1], 1)
    tx, ty, _ = oracle.face_T(2, P.n, h, P.kx, P.ky, None, P.bc_type)
    A = dense_from_T(2, P.n, tx, ty)
    x = np.linalg.solve(A, rhs(P, tx, ty))
    r = oracle.solve(P, tol=1e-10, min_side=2, interp=interp, cycle=oracle.MGCG)
    assert r.status == 0 and r.nlev >= 3
    assert r.rel_residual_true < 1e-10
    assert np.linalg.norm(r.p - x) / np.linalg.norm(x) < 1e-8
    # every inner level is visited once per application of the level above; no inner CG iterations
    assert r.level_iters[1:] == [0] * (r.nlev - 1)
    assert r.level_calls[1] == r.outer_iters
    for k in range(2, r.nlev):
        assert r.level_calls[k] == r.level_calls[k - 1]


def test_mgcg_needs_more_iterations_than_recursive():
    # Section 4 expectation: Tatebe's algorithm takes more outer iterations than the recursive
    # multi-scale PCG.  On these smoothed fields the gap shows with light smoothing (m = 1: 26
    # against 24 at 256^2); with m = 4 both take 12.
    P = synth.smoothed_lognormal_2d(2, 256, lo=-3, hi=3)
    rec = oracle.solve(P, tol=1e-10, m=1)
    mg = oracle.solve(P, tol=1e-10, m=1, cycle=oracle.MGCG)
    assert rec.status == 0 and mg.status == 0
    assert mg.outer_iters > rec.outer_iters


# ------------------------------------------------- polynomial preconditioner (Section 2.1)

@pytest.mark.parametrize("splitting", [oracle.SGS, oracle.JACOBI])
def test_polynomial_preconditioner_is_the_series(splitting):
    # W = P^-1: M^-1 is the first 2m+1 terms of the series of eq. 2.4, sum_{j<=2m} (P^-1 Q)^j P^-1
    P = problem_2d((16, 16), lo=-3, hi=3, seed=3)
    m = 2
    A, _, _, Pm, Qm = two_level_dense(P, oracle.LINEAR, m)
    if splitting == oracle.JACOBI:
        D = np.diag(np.diag(A))
        Pm, Qm = 2 * D, D - (A - D)
    Pinv = np.linalg.inv(Pm)
    H = Pinv @ Qm
    series = sum(np.linalg.matrix_power(H, j) @ Pinv for j in range(2 * m + 1))
    N = A.shape[0]
    got = np.stack([oracle.precond(P, e, m=m, max_levels=2, min_side=2, splitting=splitting, cycle=oracle.POLY)
                    for e in np.eye(N)], axis=1)
    assert np.allclose(got, series, rtol=0, atol=1e-11 * np.abs(series).max())
    assert np.allclose(got, got.T, atol=1e-12 * np.abs(got).max())
    assert np.linalg.eigvalsh((got + got.T) / 2).min() > 0


@pytest.mark.parametrize("n", [(32, 32), (64, 32)])
def test_polynomial_solve_matches_dense_solution(n):
    P = problem_2d(n, lo=-2, hi=2, seed=6)
    h = (1 / n[0], 1 / n[1], 1)
    tx, ty, _ = oracle.face_T(2, P.n, h, P.kx, P.ky, None, P.bc_type)
    A = dense_from_T(2, P.n, tx, ty)
    x = np.linalg.solve(A, rhs(P, tx, ty))
    r = oracle.solve(P, tol=1e-10, min_side=2, cycle=oracle.POLY, max_outer=2000)
    assert r.status == 0 and r.rel_residual_true < 1e-10
    assert np.linalg.norm(r.p - x) / np.linalg.norm(x) < 1e-8
    # one level only: no coarse level is visited
    assert r.level_calls[1:] == [0] * (r.nlev - 1) and r.level_iters[1:] == [0] * (r.nlev - 1)


def test_polynomial_iterations_grow_with_the_grid():
    # Section 2.1: with a purely local preconditioner the iteration count grows rapidly with
    # the dimension of the system (here about twofold per doubling of the side), unlike the
    # recursive method's nearly constant count
    its = []
    for n in (32, 64, 128):
        P = synth.smoothed_lognormal_2d(2, n, lo=-3, hi=3)
        r = oracle.solve(P, tol=1e-10, cycle=oracle.POLY, max_outer=2000)
        assert r.status == 0
        its.append(r.outer_iters)
    assert its[1] > 1.6 * its[0] and its[2] > 1.6 * its[1]


# ------------------------------------------------- non-integer scale factors (Section 3)

def test_fractional_plan_reproduces_table_1_sizes():
    # Table 1: a 1001^2 grid coarsened by a factor of about 4 gives 252^2, 63^2, 16^2, 4^2
    assert oracle.level_plan(2, (1001, 1001, 1), min_side=4, frac_scale=3.98) == \
        [(1001, 1001, 1), (252, 252, 1), (63, 63, 1), (16, 16, 1), (4, 4, 1)]


def test_fractional_path_with_integer_factors_is_the_integer_method():
    # with exact division the fractional overlaps, weights and plan reduce to the integer ones, bit for bit
    P = problem_2d((64, 64), lo=-3, hi=3, seed=5)
    a = oracle.solve(P, tol=1e-10)
    b = oracle.solve(P, tol=1e-10, frac_scale=4.0)
    assert a.level_n == b.level_n and a.outer_iters == b.outer_iters and np.array_equal(a.p, b.p)


@pytest.mark.parametrize("n,fs", [((25, 25), 2.5), ((30, 20), 3.0), ((44, 44), 3.5)])
def test_fractional_coarsening_of_uniform_K_is_the_coarse_discretisation(n, fs):
    # uniform K on square cells: the coarse grid's own faces (1 inside, 2K on the Dirichlet faces,
    # 0 on the no-flow faces), whatever fraction of a fine cell each coarse cell covers
    nx, ny = n
    P = problem_2d(n, seed=0)
    P.kx = np.ones(nx * ny)
    P.ky = P.kx.copy()
    hier = oracle.hierarchy_T(P, min_side=2, max_levels=2, frac_scale=fs)
    (d0, *_), (d1, tx, ty, _) = hier
    cx, cy = d1[0], d1[1]
    assert (cx, cy) == (int(np.floor(nx / fs + 0.5)), int(np.floor(ny / fs + 0.5)))
    TX = tx.reshape(cy, cx + 1)
    TY = ty.reshape(cy + 1, cx)
    ratio_x = (1 / cy) / (1 / cx)  # coarse cell height / width (unit square)
    ratio_y = 1 / ratio_x
    assert np.allclose(TX[:, 1:-1], ratio_x, rtol=1e-12)
    assert np.allclose(TX[:, [0, -1]], 2 * ratio_x, rtol=1e-12)
    assert np.allclose(TY[1:-1, :], ratio_y, rtol=1e-12)
    assert np.all(TY[[0, -1], :] == 0.0)


@pytest.mark.parametrize("fd,cd", [((25, 1), (10, 1)), ((31, 7), (9, 3)), ((20, 12), (6, 5))])
def test_fractional_transfers(fd, cd):
    rng = np.random.default_rng(1)
    nf, nc = fd[0] * fd[1], cd[0] * cd[1]
    for interp in (oracle.LINEAR, oracle.CONSTANT):
        # E 1 = 1
        assert np.allclose(oracle.prolong_add_dims(2, fd, cd, np.ones(nc), np.zeros(nf), interp), 1.0, rtol=1e-14)
        # <E u, v> = <u, R v>
        u, v = rng.standard_normal(nc), rng.standard_normal(nf)
        Eu = oracle.prolong_add_dims(2, fd, cd, u, np.zeros(nf), interp)
        assert np.isclose(Eu @ v, u @ oracle.restrict_dims(2, fd, cd, v, interp), rtol=1e-12)
    # linear E reproduces a linear field between the outermost coarse centres: coarse centre I
    # sits at fine-index coordinate (I + 1/2) f - 1/2 with f = nf / nc
    f = fd[0] / cd[0]
    Xc = (np.arange(cd[0]) + 0.5) * f - 0.5
    yc = np.tile(Xc, cd[1])
    got = oracle.prolong_add_dims(2, fd, cd, yc, np.zeros(nf), oracle.LINEAR).reshape(fd[1], fd[0])
    i = np.arange(fd[0])
    inside = (i >= Xc[0]) & (i <= Xc[-1])
    assert np.allclose(got[:, inside], i[inside], rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,fs,interp", [((45, 45), 3.0, oracle.LINEAR), ((50, 30), 2.5, oracle.LINEAR),
                                         ((63, 63), 3.98, oracle.CONSTANT)])
def test_fractional_solve_matches_dense_solution(n, fs, interp):
    P = problem_2d(n, lo=-2, hi=2, seed=12)
    h = (1 / n[0], 1 / n[1], 1)
    tx, ty, _ = oracle.face_T(2, P.n, h, P.kx, P.ky, None, P.bc_type)
    A = dense_from_T(2, P.n, tx, ty)
    x = np.linalg.solve(A, rhs(P, tx, ty))
    r = oracle.solve(P, tol=1e-10, min_side=2, interp=interp, frac_scale=fs)
    assert r.status == 0 and r.nlev >= 3 and r.rel_residual_true < 1e-10
    assert np.linalg.norm(r.p - x) / np.linalg.norm(x) < 1e-8


def test_fractional_preconditioner_is_symmetric_positive_definite():
    # eq. 2.10 with a coarse grid that does not divide the fine one: W = E A_c^-1 R stays symmetric
    P = problem_2d((20, 20), lo=-2, hi=2, seed=3)
    N = P.N
    got = np.stack([oracle.precond(P, e, m=2, min_side=2, max_levels=2, frac_scale=2.5) for e in np.eye(N)], axis=1)
    assert np.allclose(got, got.T, atol=1e-12 * np.abs(got).max())
    assert np.linalg.eigvalsh((got + got.T) / 2).min() > 0
