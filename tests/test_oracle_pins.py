"""Pins of the CPU oracle against facts fixed by the mathematics.

Every check here is independent of the oracle's own code path: closed forms
derived by hand from the benchmark stencils of Sec. 3.1 (fixtures under
``tests/golden/``), invariants, dense library solves of small systems,
brute-force Jacobians and finite differences.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle_py
from paper_2311_08322_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")
COEFF = inputs.COEFF
DT_DZ = inputs.DT_DZ


def _grid(ni, nj, nk):
    """Interior-relative (i, j) index arrays on the padded (nk, nj+4, ni+4) grid."""
    i = np.arange(-2, ni + 2, dtype=np.float64)
    j = np.arange(-2, nj + 2, dtype=np.float64)
    J, I = np.meshgrid(j, i, indexing="ij")
    return (np.broadcast_to(I, (nk,) + I.shape).copy(), np.broadcast_to(J, (nk,) + J.shape).copy())


def _interior(a):
    return a[:, 2:-2, 2:-2]


def _golden(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _case(doc, name):
    return next(c for c in doc["cases"] if c["name"] == name)


# ---------------------------------------------------------------- P1-P5
def test_p1_laplacian_of_quadratic_is_constant(oracle):
    c = _case(_golden("hdiff_closed_forms.json"), "quadratic")
    I, J = _grid(9, 7, 2)
    u = c["A"] * I**2 + c["B"] * J**2 + c["C"] * I * J + c["D"] * I + c["E"] * J + c["F"]
    lap = oracle.laplacian(u)
    assert lap.shape == (2, 9, 11)
    assert np.all(lap == c["lap"])
    # a quadratic has constant lap, so every flux difference is zero: out == u
    out, _, _ = oracle.hdiff(u, COEFF)
    assert np.array_equal(out, u)


def test_p2_constant_field_is_not_diffused(oracle):
    u = np.full((3, 10, 12), 0.7353)
    out, mx, my = oracle.hdiff(u, COEFF)
    assert np.array_equal(out, u)
    # zero flux ties count as kept (strict > 0 zeroes)
    assert mx.all() and my.all()
    # with w = 0 the tridiagonal matrix is the identity and data = 0
    nk, nj, ni = 3, 6, 8
    nxt, _, _ = oracle.step(u, np.zeros((nk, nj, ni)), np.zeros((nk + 1, nj, ni)), COEFF, DT_DZ)
    assert np.array_equal(nxt, u)


def test_p3_linear_field_has_zero_laplacian(oracle):
    I, J = _grid(8, 6, 3)
    u = 2.0 * I - 3.0 * J + 5.0
    assert np.all(oracle.laplacian(u) == 0.0)
    out, _, _ = oracle.hdiff(u, COEFF)
    assert np.array_equal(out, u)


def test_p4_checkerboard_limiter_zeroes_every_x_flux(oracle):
    c = _case(_golden("hdiff_closed_forms.json"), "checkerboard in i")
    I, _ = _grid(10, 6, 2)
    u = np.where(I.astype(np.int64) % 2 == 0, 1.0, -1.0)
    out, mx, my = oracle.hdiff(u, c["coeff"])
    assert not mx.any(), "every x-flux has the sign of the gradient and must be zeroed"
    assert my.all(), "y-fluxes are zero (ties) and kept"
    assert np.array_equal(out, u * c["limited_factor"])
    # the same stencil with the limiter switched off (all masks 1)
    ones_x = np.ones_like(mx)
    ones_y = np.ones_like(my)
    h = oracle.hdiff_tangent(u, ones_x, ones_y, c["coeff"])
    np.testing.assert_allclose(h, _interior(u) * c["unlimited_factor"], rtol=0, atol=1e-15)


@pytest.mark.parametrize("axis", ["i", "j"])
def test_p5_quartic_keeps_every_flux_and_adds_24_coeff(oracle, axis):
    c = _case(_golden("hdiff_closed_forms.json"), "quartic in i")
    ni, nj, nk = 9, 8, 2
    I, J = _grid(ni, nj, nk)
    x = (I if axis == "i" else J) + 4.0
    u = x**4
    out, mx, my = oracle.hdiff(u, c["coeff"])
    if axis == "i":
        assert mx.all()
    else:
        assert my.all()
    d = _interior(out) - _interior(u)
    np.testing.assert_allclose(d, c["increment"], rtol=0, atol=1e-9)


# ---------------------------------------------------------------- P6
def test_p6_limiter_predicate_on_random_field(oracle):
    f = inputs.fields_sized(37, 29, 5, seed=7)
    u = f.u
    lap = oracle.laplacian(u)  # box [-1, ni] x [-1, nj]
    mx, my = oracle.hdiff_masks(u)
    # x-fluxes on [-1, ni) x [0, nj)
    fx = lap[:, 1:-1, 1:] - lap[:, 1:-1, :-1]
    gx = u[:, 2:-2, 2:-1] - u[:, 2:-2, 1:-2]
    zeroed_x = fx * gx > 0
    assert np.array_equal(mx == 0, zeroed_x)
    fy = lap[:, 1:, 1:-1] - lap[:, :-1, 1:-1]
    gy = u[:, 2:-1, 2:-2] - u[:, 1:-2, 2:-2]
    zeroed_y = fy * gy > 0
    assert np.array_equal(my == 0, zeroed_y)
    # roughly 90% of the fluxes are zeroed on a U[0,1) field
    frac = (zeroed_x.sum() + zeroed_y.sum()) / (zeroed_x.size + zeroed_y.size)
    assert 0.8 < frac < 0.97


def test_p6_f32_decisions_differ_only_at_near_ties(oracle):
    f = inputs.fields_sized(64, 48, 6, seed=8)
    u32 = f.u.astype(np.float32).astype(np.float64)
    mx64, my64 = oracle.hdiff_masks(u32, decide_f32=False)
    mx32, my32 = oracle.hdiff_masks(u32, decide_f32=True)
    lap = oracle.laplacian(u32)
    fx = lap[:, 1:-1, 1:] - lap[:, 1:-1, :-1]
    bound_x = 64 * np.finfo(np.float32).eps * (np.abs(lap[:, 1:-1, 1:]) + np.abs(lap[:, 1:-1, :-1]))
    diff = mx64 != mx32
    assert np.all(np.abs(fx[diff]) <= bound_x[diff])
    fy = lap[:, 1:, 1:-1] - lap[:, :-1, 1:-1]
    bound_y = 64 * np.finfo(np.float32).eps * (np.abs(lap[:, 1:, 1:-1]) + np.abs(lap[:, :-1, 1:-1]))
    diff = my64 != my32
    assert np.all(np.abs(fy[diff]) <= bound_y[diff])


# ---------------------------------------------------------------- P7-P9
def _dense_T(wcol, dt_dz):
    """Tridiagonal matrix of one column, written out from the definition."""
    nk = len(wcol) - 1
    T = np.zeros((nk, nk))
    for k in range(nk):
        a = -0.25 * dt_dz * wcol[k] if k >= 1 else 0.0
        c = 0.25 * dt_dz * wcol[k + 1] if k <= nk - 2 else 0.0
        T[k, k] = 1.0 + abs(a) + abs(c)
        if k >= 1:
            T[k, k - 1] = a
        if k <= nk - 2:
            T[k, k + 1] = c
    return T


def test_p7_thomas_residual_full_size(oracle):
    wl = inputs.STEP_256
    f = inputs.fields_for(wl)
    d = _interior(f.u) + f.data
    x = oracle.vadv(_interior(f.u), f.data, f.w, DT_DZ)
    r = oracle.tridiag_apply(x, f.w, DT_DZ) - d
    assert np.max(np.abs(r)) < 1e-13


@pytest.mark.parametrize("nk", [1, 2, 3, 5, 8])
def test_p8_dense_solve_agrees(oracle, nk):
    f = inputs.fields_sized(5, 4, nk, seed=20 + nk)
    uin = _interior(f.u)
    x = oracle.vadv(uin, f.data, f.w, DT_DZ)
    xb = inputs.cotangent(5, 4, nk, child=30 + nk)
    lam = oracle.vadv_adjoint(xb, f.w, DT_DZ)
    for j in range(4):
        for i in range(5):
            T = _dense_T(f.w[:, j, i], DT_DZ)
            ref = np.linalg.solve(T, uin[:, j, i] + f.data[:, j, i])
            np.testing.assert_allclose(x[:, j, i], ref, rtol=0, atol=1e-14)
            refT = np.linalg.solve(T.T, xb[:, j, i])
            np.testing.assert_allclose(lam[:, j, i], refT, rtol=0, atol=1e-14)


def test_p9_zero_velocity_is_identity(oracle):
    f = inputs.fields_sized(6, 5, 7, seed=40)
    w0 = np.zeros_like(f.w)
    uin = _interior(f.u)
    x = oracle.vadv(uin, f.data, w0, DT_DZ)
    assert np.array_equal(x, uin + f.data)
    assert np.array_equal(oracle.vadv_adjoint(f.data, w0, DT_DZ), f.data)


def _cramer(sub, diag, sup, d):
    n = len(diag)
    M = [[Fraction(0)] * n for _ in range(n)]
    for k in range(n):
        M[k][k] = Fraction(str(diag[k]))
    for k in range(n - 1):
        M[k + 1][k] = Fraction(str(sub[k]))
        M[k][k + 1] = Fraction(str(sup[k]))

    def det(A):
        if len(A) == 1:
            return A[0][0]
        return sum((-1) ** c * A[0][c] * det([row[:c] + row[c + 1:] for row in A[1:]])
                   for c in range(len(A)))

    D = det(M)
    xs = []
    for c in range(n):
        Mc = [row[:] for row in M]
        for r in range(n):
            Mc[r][c] = Fraction(str(d[r]))
        xs.append(det(Mc) / D)
    return xs


def test_p9_hand_solved_columns(oracle):
    doc = _golden("vadv_columns.json")
    for case in doc["cases"]:
        nk = case["nk"]
        w = np.array(case["w"], dtype=np.float64).reshape(nk + 1, 1, 1)
        d = np.array(case["d"], dtype=np.float64).reshape(nk, 1, 1)
        x = oracle.vadv(d, np.zeros_like(d), w, case["dt_dz"])[:, 0, 0]
        ref = _cramer(case["sub"], case["diag"], case["sup"], case["d"])
        for k in range(nk):
            assert abs(x[k] - float(ref[k])) <= 4e-16 * max(1.0, abs(float(ref[k]))), (case, k)
        # the transposed system (adjoint) on the same hand matrix
        lam = oracle.vadv_adjoint(d, w, case["dt_dz"])[:, 0, 0]
        refT = _cramer(case["sup"], case["diag"], case["sub"], case["d"])
        for k in range(nk):
            assert abs(lam[k] - float(refT[k])) <= 4e-16 * max(1.0, abs(float(refT[k])))


# ---------------------------------------------------------------- the step's forcing term
# Inside the step the right-hand side of each column is d_k = u_k + data_k
# with u_k the diffused field (the implicit vertical advection of the
# benchmark, its right-hand side taken from the horizontal stage).  These pins
# compose the step from pieces pinned above (hdiff: closed forms; the column
# solve: dense LU, Cramer's rule) and check the forcing enters with its sign.
def test_step_forcing_at_zero_velocity_is_added_once(oracle):
    # w = 0 makes T the identity: the new interior is the diffused field plus
    # data, bit for bit (one rounding, in the same order as the definition)
    f = inputs.fields_sized(9, 7, 5, seed=41)
    w0 = np.zeros_like(f.w)
    nxt, mx, my = oracle.step(f.u, f.data, w0, COEFF, DT_DZ)
    h, hmx, hmy = oracle.hdiff(f.u, COEFF)
    assert np.array_equal(_interior(nxt), _interior(h) + f.data)
    assert np.array_equal(mx, hmx) and np.array_equal(my, hmy)
    # the halo is carried from u, not diffused or forced
    nxt[:, 2:-2, 2:-2] = 0.0
    ref = f.u.copy()
    ref[:, 2:-2, 2:-2] = 0.0
    assert np.array_equal(nxt, ref)
    # data = 0 leaves the diffused field itself; doubling data doubles the
    # increment exactly (data ~ U[-0.1, 0.1] doubles without rounding)
    n0, _, _ = oracle.step(f.u, np.zeros_like(f.data), w0, COEFF, DT_DZ)
    assert np.array_equal(_interior(n0), _interior(h))
    n2, _, _ = oracle.step(f.u, 2.0 * f.data, w0, COEFF, DT_DZ)
    assert np.array_equal(_interior(n2), _interior(h) + 2.0 * f.data)


def test_step_is_vadv_of_hdiff_with_forcing(oracle):
    # random w and non-zero data: the step equals vadv applied to hdiff's
    # interior with the same forcing, bit for bit, and each column solves the
    # dense tridiagonal system written out from its definition
    ni, nj, nk = 7, 6, 9
    f = inputs.fields_sized(ni, nj, nk, seed=42)
    assert np.max(np.abs(f.data)) > 0.05
    nxt, _, _ = oracle.step(f.u, f.data, f.w, COEFF, DT_DZ)
    h, _, _ = oracle.hdiff(f.u, COEFF)
    x = oracle.vadv(_interior(h), f.data, f.w, DT_DZ)
    assert np.array_equal(_interior(nxt), x)
    for j in range(nj):
        for i in range(ni):
            T = _dense_T(f.w[:, j, i], DT_DZ)
            ref = np.linalg.solve(T, _interior(h)[:, j, i] + f.data[:, j, i])
            np.testing.assert_allclose(_interior(nxt)[:, j, i], ref, rtol=0, atol=1e-14)
            # and not the unforced or oppositely forced solve
            bad = np.linalg.solve(T, _interior(h)[:, j, i] - f.data[:, j, i])
            assert np.max(np.abs(_interior(nxt)[:, j, i] - bad)) > 1e-6


# ---------------------------------------------------------------- independent pure-Python copy
def test_pure_python_copy_agrees(oracle):
    f = inputs.fields_sized(6, 5, 3, seed=50)
    out, mx, my = oracle.hdiff(f.u, COEFF)
    out_py, mx_py, my_py = oracle_py.hdiff(f.u.tolist(), COEFF)
    assert np.array_equal(mx, np.array(mx_py, np.uint8))
    assert np.array_equal(my, np.array(my_py, np.uint8))
    np.testing.assert_allclose(_interior(out), np.array(out_py), rtol=0, atol=1e-15)
    uin = _interior(f.u)
    x = oracle.vadv(uin, f.data, f.w, DT_DZ)
    for j in range(5):
        for i in range(6):
            ref = oracle_py.thomas_column(list(uin[:, j, i] + f.data[:, j, i]), list(f.w[:, j, i]), DT_DZ)
            np.testing.assert_allclose(x[:, j, i], ref, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- P10-P12 (adjoint)
def _brute_jacobian(fn, nin):
    cols = []
    for p in range(nin):
        e = np.zeros(nin)
        e[p] = 1.0
        cols.append(fn(e).ravel())
    return np.stack(cols, axis=1)


def test_p10_step_adjoint_is_transpose_of_tangent(oracle):
    ni, nj, nk = 5, 4, 3
    f = inputs.fields_sized(ni, nj, nk, seed=60)
    _, mx, my = oracle.step(f.u, f.data, f.w, COEFF, DT_DZ)
    shp = (nk, nj + 4, ni + 4)
    J = _brute_jacobian(lambda e: oracle.step_tangent(e.reshape(shp), f.w, mx, my, COEFF, DT_DZ),
                        int(np.prod(shp)))
    ob = inputs.cotangent(ni, nj, nk, child=61)
    ubar, dbar = oracle.step_adjoint(ob, f.w, mx, my, COEFF, DT_DZ)
    np.testing.assert_allclose(ubar.ravel(), J.T @ ob.ravel(), rtol=0, atol=1e-14)
    # d out / d data = T^{-1}: brute force through vadv with zero u_in
    Jd = _brute_jacobian(lambda e: oracle.vadv(np.zeros((nk, nj, ni)), e.reshape(nk, nj, ni), f.w, DT_DZ),
                         nk * nj * ni)
    np.testing.assert_allclose(dbar.ravel(), Jd.T @ ob.ravel(), rtol=0, atol=1e-14)


def test_p10_hdiff_adjoint_is_transpose_of_tangent(oracle):
    ni, nj, nk = 6, 5, 2
    f = inputs.fields_sized(ni, nj, nk, seed=62)
    mx, my = oracle.hdiff_masks(f.u)
    shp = (nk, nj + 4, ni + 4)
    J = _brute_jacobian(lambda e: oracle.hdiff_tangent(e.reshape(shp), mx, my, COEFF), int(np.prod(shp)))
    lam = inputs.cotangent(ni, nj, nk, child=63)
    ubar = oracle.hdiff_adjoint(lam, mx, my, COEFF)
    np.testing.assert_allclose(ubar.ravel(), J.T @ lam.ravel(), rtol=0, atol=1e-14)
    # the limiter mask matters: the two corners never read are exactly zero
    for k in range(nk):
        for (jj, ii) in [(0, 0), (0, 1), (1, 0)]:
            assert ubar[k, jj, ii] == 0.0


def test_tangent_is_derivative_of_forward(oracle):
    """Masks fixed, the step is affine in u: central differences reproduce
    the tangent wherever the masks of u +- h v agree with those of u."""
    ni, nj, nk = 12, 10, 6
    f = inputs.fields_sized(ni, nj, nk, seed=64)
    _, mx, my = oracle.step(f.u, f.data, f.w, COEFF, DT_DZ)
    v, _ = inputs.dot_vectors(ni, nj, nk)
    h = 1e-7
    up, mxp, myp = oracle.step(f.u + h * v, f.data, f.w, COEFF, DT_DZ)
    um, mxm, mym = oracle.step(f.u - h * v, f.data, f.w, COEFF, DT_DZ)
    assert np.array_equal(mxp, mx) and np.array_equal(mxm, mx)
    assert np.array_equal(myp, my) and np.array_equal(mym, my)
    fd = (_interior(up) - _interior(um)) / (2 * h)
    tl = oracle.step_tangent(v, f.w, mx, my, COEFF, DT_DZ)
    np.testing.assert_allclose(fd, tl, rtol=0, atol=1e-7)


def test_p11_dot_test(oracle):
    ni, nj, nk = 48, 40, 24
    f = inputs.fields_sized(ni, nj, nk, seed=65)
    _, mx, my = oracle.step(f.u, f.data, f.w, COEFF, DT_DZ)
    v, wv = inputs.dot_vectors(ni, nj, nk)
    Jv = oracle.step_tangent(v, f.w, mx, my, COEFF, DT_DZ)
    JTw, _ = oracle.step_adjoint(wv, f.w, mx, my, COEFF, DT_DZ)
    lhs = math.fsum((Jv * wv).ravel())
    rhs = math.fsum((v * JTw).ravel())
    assert abs(lhs - rhs) / max(abs(lhs), abs(rhs)) <= 1e-10


def test_p12_central_finite_differences(oracle):
    """Central differences of <ob, step(u)> at 64 seeded points, h = 1e-6."""
    ni, nj, nk = 40, 36, 24
    f = inputs.fields_sized(ni, nj, nk, seed=66)
    _, mx, my = oracle.step(f.u, f.data, f.w, COEFF, DT_DZ)
    ob = inputs.cotangent(ni, nj, nk)
    ubar, _ = oracle.step_adjoint(ob, f.w, mx, my, COEFF, DT_DZ)
    h = 1e-6
    checked = 0
    for p in inputs.fd_points(ni, nj, nk, 64):
        up = f.u.copy().ravel()
        um = f.u.copy().ravel()
        up[p] += h
        um[p] -= h
        sp, mxp, myp = oracle.step(up.reshape(f.u.shape), f.data, f.w, COEFF, DT_DZ)
        sm, mxm, mym = oracle.step(um.reshape(f.u.shape), f.data, f.w, COEFF, DT_DZ)
        if not (np.array_equal(mxp, mx) and np.array_equal(mxm, mx) and np.array_equal(myp, my)
                and np.array_equal(mym, my)):
            continue  # a limiter kink lies within h: the a.e. derivative does not apply
        fd = (math.fsum((_interior(sp) * ob).ravel()) - math.fsum((_interior(sm) * ob).ravel())) / (2 * h)
        g = ubar.ravel()[p]
        assert abs(fd - g) <= 1e-7 * max(1.0, abs(g)), (p, fd, g)
        checked += 1
    assert checked >= 56


# ---------------------------------------------------------------- semantics
def test_halo_is_carried_not_computed(oracle):
    f = inputs.fields_sized(7, 6, 4, seed=70)
    nxt, _, _ = oracle.step(f.u, f.data, f.w, COEFF, DT_DZ)
    mask = np.ones(f.u.shape, bool)
    mask[:, 2:-2, 2:-2] = False
    assert np.array_equal(nxt[mask], f.u[mask])


def test_corner_halo_points_never_read(oracle):
    """Only the radius-2 diamond of each output point is read: the three
    corner-most halo points of each corner do not influence the step."""
    f = inputs.fields_sized(7, 6, 3, seed=71)
    base, _, _ = oracle.step(f.u, f.data, f.w, COEFF, DT_DZ)
    u2 = f.u.copy()
    for (jj, ii) in [(0, 0), (0, 1), (1, 0), (0, -1), (0, -2), (1, -1), (-1, 0), (-2, 0), (-1, 1),
                     (-1, -1), (-1, -2), (-2, -1)]:
        u2[:, jj, ii] = 1e6
    nxt, _, _ = oracle.step(u2, f.data, f.w, COEFF, DT_DZ)
    assert np.array_equal(_interior(nxt), _interior(base))


# ---------------------------------------------------------------- parameter gradients
def _loss(oracle, f, ob, coeff, w):
    nxt, _, _ = oracle.step(f.u, f.data, w, coeff, DT_DZ)
    return math.fsum((_interior(nxt) * ob).ravel())


def test_divergence_closed_forms(oracle):
    """D(u) = (u - hdiff(u)) / coeff: 0 for a linear field, -24 for the
    quartic (i+4)^4 whose fluxes are all kept (P5)."""
    ni, nj, nk = 9, 8, 2
    I, J = _grid(ni, nj, nk)
    lin = 3.0 * I - 7.0 * J + 2.0  # integers: every stage is exact
    mx, my = oracle.hdiff_masks(lin)
    assert np.all(oracle.hdiff_divergence(lin, mx, my) == 0.0)
    q = (I + 4.0) ** 4
    mx, my = oracle.hdiff_masks(q)
    np.testing.assert_allclose(oracle.hdiff_divergence(q, mx, my), -24.0, rtol=0, atol=1e-9)


def test_coeff_gradient_is_exact_difference_quotient(oracle):
    """The limiter decisions do not depend on coeff, so <ob, step> is affine
    in coeff: its central difference quotient is exact up to rounding, and
    L(c) = L(0) + c dL/dcoeff."""
    ni, nj, nk = 14, 11, 9
    f = inputs.fields_sized(ni, nj, nk, seed=80)
    ob = inputs.cotangent(ni, nj, nk)
    mx, my = oracle.hdiff_masks(f.u)
    lam = oracle.vadv_adjoint(ob, f.w, DT_DZ)
    g = oracle.coeff_grad(f.u, lam, mx, my)
    h = 0.01
    fd = (_loss(oracle, f, ob, COEFF + h, f.w) - _loss(oracle, f, ob, COEFF - h, f.w)) / (2 * h)
    assert abs(fd - g) <= 1e-9 * max(1.0, abs(g)), (fd, g)
    l0 = _loss(oracle, f, ob, 0.0, f.w)
    lc = _loss(oracle, f, ob, COEFF, f.w)
    assert abs((lc - l0) - COEFF * g) <= 1e-11 * max(1.0, abs(lc))


def test_w_gradient_central_differences_every_level(oracle):
    """Central differences (h = 1e-6) of <ob, step(w)> for every staggered
    level of every column, including w_0 and w_nk, which do not enter T."""
    ni, nj, nk = 5, 4, 6
    f = inputs.fields_sized(ni, nj, nk, seed=81)
    ob = inputs.cotangent(ni, nj, nk)
    nxt, _, _ = oracle.step(f.u, f.data, f.w, COEFF, DT_DZ)
    lam = oracle.vadv_adjoint(ob, f.w, DT_DZ)
    wbar = oracle.w_grad(f.w, _interior(nxt), lam, DT_DZ)
    assert np.all(wbar[0] == 0.0) and np.all(wbar[nk] == 0.0)
    h = 1e-6
    checked = 0
    for p in range(f.w.size):
        if abs(f.w.ravel()[p]) < 1e-3:
            continue  # |a| or |c| has a kink at w = 0
        wp = f.w.copy().ravel()
        wm = f.w.copy().ravel()
        wp[p] += h
        wm[p] -= h
        fd = (_loss(oracle, f, ob, COEFF, wp.reshape(f.w.shape)) -
              _loss(oracle, f, ob, COEFF, wm.reshape(f.w.shape))) / (2 * h)
        g = wbar.ravel()[p]
        assert abs(fd - g) <= 1e-7 * max(1.0, abs(g)), (p, fd, g)
        checked += 1
    assert checked >= f.w.size - 4


def test_w_gradient_at_zero_velocity(oracle):
    """w = 0: T = I, x = d, lam = ob, and with d|t|/dt = 0 at 0 only the
    off-diagonal entries contribute: wbar_j = r/4 (lam_j x_{j-1} - lam_{j-1} x_j)."""
    ni, nj, nk = 3, 2, 5
    f = inputs.fields_sized(ni, nj, nk, seed=82)
    w0 = np.zeros_like(f.w)
    ob = inputs.cotangent(ni, nj, nk)
    nxt, _, _ = oracle.step(f.u, f.data, w0, COEFF, DT_DZ)
    x = _interior(nxt)
    lam = oracle.vadv_adjoint(ob, w0, DT_DZ)
    assert np.array_equal(lam, ob)
    wbar = oracle.w_grad(w0, x, lam, DT_DZ)
    want = np.zeros_like(w0)
    want[1:nk] = 0.25 * DT_DZ * (lam[1:] * x[:-1] - lam[:-1] * x[1:])
    np.testing.assert_allclose(wbar, want, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- periodic boundaries
def test_periodic_halo_closed_form(oracle):
    """Integer pattern u = 1e6 k + 1000 (i mod ni) + (j mod nj): after the
    fill every padded point holds the pattern at its wrapped index, also for
    domains narrower than the halo."""
    for ni, nj, nk in [(7, 5, 3), (1, 1, 2), (2, 3, 1)]:
        i = np.arange(-2, ni + 2)
        j = np.arange(-2, nj + 2)
        k = np.arange(nk)
        K, J, I = np.meshgrid(k, j, i, indexing="ij")
        want = 1e6 * K + 1000.0 * np.mod(I, ni) + np.mod(J, nj)
        u = np.full((nk, nj + 4, ni + 4), -1.0)
        u[:, 2:-2, 2:-2] = want[:, 2:-2, 2:-2]
        got = oracle.halo_periodic(u)
        assert np.array_equal(got, want), (ni, nj, nk)
        assert np.array_equal(oracle.halo_periodic(got), got)  # idempotent


def test_periodic_diffusion_conserves_mass(oracle):
    """With periodic halos the flux form telescopes: w = 0 and data = 0 make
    the column solve the identity, so the interior sum is kept by every step
    (to rounding)."""
    ni, nj, nk = 24, 20, 3
    f = inputs.fields_sized(ni, nj, nk, seed=90)
    u = oracle.halo_periodic(f.u)
    s0 = math.fsum(_interior(u).ravel())
    zero_w = np.zeros_like(f.w)
    zero_d = np.zeros_like(f.data)
    for _ in range(10):
        nxt, _, _ = oracle.step(u, zero_d, zero_w, COEFF, DT_DZ)
        u = oracle.halo_periodic(nxt)
    s1 = math.fsum(_interior(u).ravel())
    assert abs(s1 - s0) <= 1e-13 * math.fsum(np.abs(_interior(u)).ravel())


def test_openmp_build_is_identical_to_serial(oracle):
    """The CPU baseline's OpenMP build splits independent levels and columns
    over threads with per-thread temporaries; every result must equal the
    serial build's bit for bit (same operations, same order)."""
    ni, nj, nk = 37, 29, 23
    f = inputs.fields_sized(ni, nj, nk, seed=950)
    ob = inputs.cotangent(ni, nj, nk)
    kap = inputs.coeff_field(ni, nj, nk)
    ser = [oracle.step(f.u, f.data, f.w, inputs.COEFF, inputs.DT_DZ, kappa=kap, damping=True),
           oracle.step(f.u, f.data, f.w, inputs.COEFF, inputs.DT_DZ, decide_f32=True)]
    ser_adj = oracle.step_adjoint(ob, f.w, ser[0][1], ser[0][2], inputs.COEFF, inputs.DT_DZ, kappa=kap)
    with oracle.threaded():
        assert oracle.threads() >= 1
        par = [oracle.step(f.u, f.data, f.w, inputs.COEFF, inputs.DT_DZ, kappa=kap, damping=True),
               oracle.step(f.u, f.data, f.w, inputs.COEFF, inputs.DT_DZ, decide_f32=True)]
        par_adj = oracle.step_adjoint(ob, f.w, ser[0][1], ser[0][2], inputs.COEFF, inputs.DT_DZ, kappa=kap)
    assert oracle.threads() == 1
    for a, b in zip(ser, par):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    for x, y in zip(ser_adj, par_adj):
        assert np.array_equal(x, y)


# ---------------------------------------------------------------- the NumPy-backend analogue
@pytest.mark.parametrize("dims", [(1, 1, 1), (6, 5, 3), (17, 9, 2), (33, 20, 13), (64, 48, 16)],
                         ids=lambda d: "x".join(map(str, d)))
def test_numpy_step_equals_oracle(oracle, dims):
    # the whole-array NumPy step (CPU context for the benchmark) is the
    # oracle's step bit for bit, halo included
    from oracle import numpy_step

    ni, nj, nk = dims
    f = inputs.fields_sized(ni, nj, nk, seed=60 + nk)
    ref, _, _ = oracle.step(f.u, f.data, f.w, COEFF, DT_DZ)
    got = numpy_step.step(f.u, f.data, f.w, COEFF, DT_DZ)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)
