"""Pins of the reference extraction and tracking (oracle/extract.py):
cubic interpolation exact for per-axis cubics and not quartics, taken in
the finest block; the spin-weight -2 harmonics equal their closed forms
for l = 2 and are orthonormal under the geodesic-sphere quadrature; the
projection recovers the coefficients of a known mode sum; the RK4 tracker
in flat space with a uniform shift equals the RK4 polynomial of the joint
linear system beta' = -eta beta, x' = -beta exactly."""
import math

import numpy as np
import pytest

import oracle
import z4c_inputs as zi
from oracle import extract as ex


def two_level():
    m0 = zi.uniform_mesh((2, 2, 2), 8, 4, (0.0,) * 3, (2.0,) * 3, zi.BC_OUTFLOW)
    return zi.refine_blocks(m0, [0, 3])


def poly(X, Y, Z, deg, seed):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((deg + 1, deg + 1, deg + 1))
    return np.polynomial.polynomial.polyval3d(X, Y, Z, c)


@pytest.mark.parametrize("deg,exact", [(3, True), (4, False)])
def test_interpolation_order(deg, exact):
    mesh = two_level()
    inter = [np.stack([poly(*mesh.grid(b), deg, 1), poly(*mesh.grid(b), deg, 2)]) for b in range(mesh.nb)]
    rng = np.random.default_rng(3)
    pts = rng.uniform(0.01, 1.99, size=(200, 3))
    got = ex.interpolate(mesh, inter, pts)
    want = np.stack([poly(pts[:, 0], pts[:, 1], pts[:, 2], deg, 1), poly(pts[:, 0], pts[:, 1], pts[:, 2], deg, 2)], 1)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    assert (err < 1e-12) if exact else (err > 1e-6), err


def test_interpolation_uses_the_finest_block():
    mesh = two_level()
    inter = [np.full((1, 8, 8, 8), float(mesh.level[b])) for b in range(mesh.nb)]
    pts = np.array([[0.3, 0.4, 0.2], [1.7, 1.6, 0.3], [1.2, 0.3, 1.5]])   # blocks 0, 3 refined
    got = ex.interpolate(mesh, inter, pts)[:, 0]
    np.testing.assert_allclose(got, [1.0, 1.0, 0.0], rtol=0, atol=1e-14)


def test_swsh_closed_forms_l2():
    th = np.linspace(0.1, 3.0, 17)
    ph = np.linspace(-3.0, 3.0, 17)
    c, s = np.cos(th), np.sin(th)
    closed = {2: math.sqrt(5 / (64 * math.pi)) * (1 + c) ** 2 * np.exp(2j * ph),
              1: math.sqrt(5 / (16 * math.pi)) * s * (1 + c) * np.exp(1j * ph),
              0: math.sqrt(15 / (32 * math.pi)) * s ** 2,
              -1: math.sqrt(5 / (16 * math.pi)) * s * (1 - c) * np.exp(-1j * ph),
              -2: math.sqrt(5 / (64 * math.pi)) * (1 - c) ** 2 * np.exp(-2j * ph)}
    for m, want in closed.items():
        np.testing.assert_allclose(ex.swsh(-2, 2, m, th, ph), want, rtol=0, atol=1e-14)


def test_swsh_orthonormal_on_geodesic_sphere():
    P, w = zi.geodesic_sphere(5)
    th, ph = ex.angles(P, (0.0, 0.0, 0.0))
    modes = [(l, m) for l in range(2, 5) for m in range(-l, l + 1)]
    Y = np.array([ex.swsh(-2, l, m, th, ph) for l, m in modes])
    G = (Y * w) @ np.conj(Y).T
    assert np.max(np.abs(G - np.eye(len(modes)))) < 2e-3


def test_projection_recovers_mode_sum():
    P, w = zi.geodesic_sphere(5, 3.0, (0.5, -0.2, 0.1))
    th, ph = ex.angles(P, (0.5, -0.2, 0.1))
    rng = np.random.default_rng(7)
    coef = {(l, m): complex(*rng.standard_normal(2)) for l in range(2, 4) for m in range(-l, l + 1)}
    vals = sum(c * ex.swsh(-2, l, m, th, ph) for (l, m), c in coef.items())
    got = ex.project(vals, P, w, (0.5, -0.2, 0.1), 4)
    for key in got:
        assert abs(got[key] - coef.get(key, 0.0)) < 5e-3, key


def test_tracker_matches_rk4_of_the_linear_system():
    mesh = zi.uniform_mesh((2, 2, 2), 8, 4, (0.0,) * 3, (2.0,) * 3, zi.BC_PERIODIC)
    p = zi.params_default(6, eta=2.0)
    beta0 = np.array([0.3, -0.2, 0.1])
    data = zi.flat(mesh)
    for blk in data:
        for a in range(3):
            blk[19 + a] = beta0[a]
    om = oracle.OracleMesh(mesh)
    regs = oracle.Registers(om, data)
    x0 = np.array([[0.7, 1.1, 0.9], [1.5, 0.4, 1.2]])
    dt, nsteps = 0.05, 6
    x = x0.copy()
    for _ in range(nsteps):
        x = ex.rk4_step_with_tracker(regs, p, dt, x)
    # joint system y = (beta, x) per component: y' = A y
    A = np.array([[-p["eta"], 0.0], [-1.0, 0.0]]) * dt
    Rm = np.eye(2) + A + A @ A / 2 + A @ A @ A / 6 + A @ A @ A @ A / 24
    Rn = np.linalg.matrix_power(Rm, nsteps)
    for q in range(2):
        for a in range(3):
            want = Rn @ np.array([beta0[a], x0[q, a]])
            assert abs(x[q, a] - want[1]) < 1e-14, (q, a, x[q, a], want[1])
    beta = om.interiors(regs.U)[0][19:22, 0, 0, 0]
    np.testing.assert_allclose(beta, (Rn @ np.array([beta0, np.zeros(3)]))[0], rtol=0, atol=1e-15)
