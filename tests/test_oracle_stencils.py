"""Pins of the oracle's finite-difference operators (P1, P3, P4, P6).

The weights come from the oracle's own Fornberg recurrence; these tests tie
them to textbook values, to exact rational weights from an independent
Vandermonde solve (sympy), and to exactness on polynomials through the RHS.
"""
import math

import numpy as np
import pytest
import sympy

import oracle
import z4c_inputs as zi


def exact_weights(deriv, pts):
    """Exact rational FD weights: solve sum_k w_k x_k^q = q! delta_{q,deriv}."""
    n = len(pts)
    V = sympy.Matrix(n, n, lambda q, k: sympy.Integer(pts[k]) ** q)
    rhs = sympy.Matrix(n, 1, lambda q, _: sympy.factorial(deriv) if q == deriv else 0)
    return [sympy.Rational(x) for x in V.LUsolve(rhs)]


TEXTBOOK = [
    (1, range(-2, 3), [1, -8, 0, 8, -1], 12),
    (1, range(-3, 4), [-1, 9, -45, 0, 45, -9, 1], 60),
    (2, range(-2, 3), [-1, 16, -30, 16, -1], 12),
    (2, range(-3, 4), [2, -27, 270, -490, 270, -27, 2], 180),
    (1, range(-2, 5), [2, -24, -35, 80, -30, 8, -1], 60),   # 6th-order lopsided (+)
    (1, range(-1, 4), [-3, -10, 18, -6, 1], 12),           # 4th-order lopsided (+)
]


@pytest.mark.parametrize("deriv,pts,num,den", TEXTBOOK)
def test_textbook_weights(deriv, pts, num, den):
    w = oracle.fd_weights(deriv, list(pts))
    np.testing.assert_allclose(w * den, num, rtol=0, atol=1e-12)


@pytest.mark.parametrize("N", [2, 3, 4])
def test_weights_match_exact_rationals(N):
    sets = [(1, list(range(-N, N + 1))), (2, list(range(-N, N + 1))),
            (1, list(range(-(N - 1), N + 2))), (1, list(range(-(N + 1), N)))]
    for deriv, pts in sets:
        w = oracle.fd_weights(deriv, pts)
        ex = np.array([float(x) for x in exact_weights(deriv, pts)])
        np.testing.assert_allclose(w, ex, rtol=4e-15, atol=4e-15)


def _mesh_user(n, g, lo=-1.0, hi=1.0):
    return zi.uniform_mesh((1, 1, 1), n, g, (lo,) * 3, (hi,) * 3, zi.BC_USER)


def _ghosted_axes(mesh):
    from z4c_inputs import analytic as an
    return an.ghosted_grid(mesh, 0)


@pytest.mark.parametrize("order", [4, 6, 8])
def test_polynomial_shift_exactness(order):
    """P3: flat conformal metric, chi = alpha = 1 and a polynomial shift of
    per-axis degree 2N: d_t Gamma~^i = lap beta^i + (1/3) d_i div beta and
    d_t g~_ij = d_i beta_j + d_j beta_i - (2/3) delta_ij div beta hold
    exactly, because every operator involved is exact on such polynomials."""
    N = order // 2
    g = N + 1
    mesh = _mesh_user(8, g)
    X, Y, Z = _ghosted_axes(mesh)
    rng = np.random.default_rng(11 + order)
    deg = 2 * N
    coef = rng.uniform(-1, 1, size=(3, deg + 1, deg + 1, deg + 1)) / (deg + 1) ** 3
    # keep total degree modest in magnitude: scale high powers down
    P = [np.polynomial.polynomial.polyval3d(X, Y, Z, coef[i]) for i in range(3)]

    def d(c, ax, k=1):
        return np.polynomial.polynomial.polyder(c, m=k, axis=ax)

    u = np.zeros((22,) + X.shape)
    u[0] = 1.0
    u[18] = 1.0
    for c in (1, 4, 6):
        u[c] = 1.0
    for i in range(3):
        u[19 + i] = P[i]
    om = oracle.OracleMesh(mesh)
    U = om.scatter_ghosted([u])
    p = zi.params_default(order)
    p["terms"] = 1  # PHYS only: no advection, dissipation or gauge
    r = oracle.rhs(om, p, U, fill=False)[0]
    Xi, Yi, Zi = mesh.grid(0)

    def ev(c):
        return np.polynomial.polynomial.polyval3d(Xi, Yi, Zi, c)
    db = [[ev(d(coef[i], j)) for j in range(3)] for i in range(3)]  # db[i][j] = d_j beta^i
    div = db[0][0] + db[1][1] + db[2][2]
    for i in range(3):
        lap = sum(ev(d(coef[i], j, 2)) for j in range(3))
        grad_div = sum(ev(d(d(coef[k], k), i)) for k in range(3))
        exp = lap + grad_div / 3.0
        scale = max(1.0, np.abs(exp).max())
        np.testing.assert_allclose(r[14 + i], exp, rtol=0, atol=2e-11 * scale)
    for i in range(3):
        for j in range(i, 3):
            exp = db[j][i] + db[i][j] - (2.0 / 3.0 if i == j else 0.0) * div
            np.testing.assert_allclose(r[1 + zi.SYM[i][j]], exp, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r[0], -2.0 / 3.0 * div, rtol=0, atol=1e-12)
    for f in (7, 8, 9, 10, 11, 12, 13, 17):
        assert np.abs(r[f]).max() < 1e-12


@pytest.mark.parametrize("order", [4, 6, 8])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_lopsided_advection_polynomial_exact(order, sign):
    """Advection alone with a constant shift: d_t f = beta^k d_k f exactly
    for polynomials of per-axis degree 2N, whichever way beta points."""
    N = order // 2
    mesh = _mesh_user(8, N + 1)
    X, Y, Z = _ghosted_axes(mesh)
    rng = np.random.default_rng(3)
    deg = 2 * N
    coef = rng.uniform(-1, 1, size=(deg + 1, deg + 1, deg + 1)) / (deg + 1) ** 3
    beta = sign * np.array([0.3, -0.2, 0.45])
    u = np.zeros((22,) + X.shape)
    for f in range(18):
        u[f] = np.polynomial.polynomial.polyval3d(X, Y, Z, coef) * (1 + 0.1 * f)
    for i in range(3):
        u[19 + i] = beta[i]
    u[18] = 1.0
    om = oracle.OracleMesh(mesh)
    p = zi.params_default(order)
    p["terms"] = 4  # ADVECT only
    r = oracle.rhs(om, p, om.scatter_ghosted([u]), fill=False)[0]
    Xi, Yi, Zi = mesh.grid(0)
    grad = [np.polynomial.polynomial.polyval3d(
        Xi, Yi, Zi, np.polynomial.polynomial.polyder(coef, axis=a)) for a in range(3)]
    exp = sum(beta[a] * grad[a] for a in range(3))
    for f in range(18):
        np.testing.assert_allclose(r[f], exp * (1 + 0.1 * f), rtol=0, atol=5e-12)
    for f in range(18, 22):
        assert np.all(r[f] == 0.0)


@pytest.mark.parametrize("order", [4, 6, 8])
def test_ko_nyquist_eigenvalue(order):
    """P4: the Nyquist mode (-1)^(i+j+k) is an eigenvector of the
    dissipation operator with eigenvalue -3 sigma/h, exactly."""
    N = order // 2
    mesh = zi.uniform_mesh((1, 1, 1), 16, N + 1, (0,) * 3, (1,) * 3, zi.BC_PERIODIC)
    data = zi.flat(mesh)
    I = np.indices((16, 16, 16)).sum(0)
    mode = np.where(I % 2 == 0, 1.0, -1.0) * 2.0 ** -20
    for f in range(22):
        data[0][f] += mode
    om = oracle.OracleMesh(mesh)
    p = zi.params_default(order)
    p["terms"] = 8  # DISSIP only
    r = oracle.rhs(om, p, om.scatter(data))[0]
    h = mesh.dx0
    for f in range(22):
        np.testing.assert_array_equal(r[f], -3 * p["ko_sigma"] / h * mode)


@pytest.mark.parametrize("order", [4, 6, 8])
def test_upwinding_is_dissipative(order):
    """P6: with a constant shift, one RK4 step of pure advection multiplies a
    Fourier mode by R(dt * s(k)), s the stencil symbol.  Upwinded lopsided
    stencils keep |R| <= 1 at CFL 0.25 for every resolved k; the downwind
    choice would amplify.  Checked numerically through the oracle, on a
    periodic block, against the exact advection phase at low k."""
    N = order // 2
    n = 16
    mesh = zi.uniform_mesh((1, 1, 1), n, N + 1, (0,) * 3, (1,) * 3, zi.BC_PERIODIC)
    h = mesh.dx0
    p = zi.params_default(order)
    p["terms"] = 4
    p["enforce"] = 0
    for beta in (0.8, -0.8):
        for kk in (1, 4, 7):
            data = zi.flat(mesh)
            X, Y, Z = mesh.grid(0)
            for i in range(3):
                data[0][19 + i][:] = 0.0
            data[0][19][:] = beta
            data[0][17] = np.cos(2 * math.pi * kk * X)
            data[0][7] = np.sin(2 * math.pi * kk * X)
            om = oracle.OracleMesh(mesh)
            regs = oracle.Registers(om, data)
            dt = 0.25 * h
            oracle.rk4_steps(regs, p, dt, 1)
            out = om.interiors(regs.U)[0]
            c = out[17] + 1j * out[7]
            c0 = data[0][17] + 1j * data[0][7]
            Rk = (c / c0).mean()
            assert abs(Rk) <= 1.0 + 1e-13, (beta, kk, abs(Rk))
            if kk == 1:
                # exact solution f(x + beta t): phase e^{i k beta dt}
                k = 2 * math.pi * kk
                ex = np.exp(1j * k * beta * dt)
                assert abs(Rk - ex) < 10 * dt * abs(beta) * k * (k * h) ** (2 * N) + 1e-13
