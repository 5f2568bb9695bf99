"""Pins of the reference Psi4 (oracle or_psi4) against what general
relativity fixes: zero in flat space; for a linear outgoing TT wave, on the
tetrad's radial axis, Psi4 = d2h+/dt2 - i d2hx/dt2 with h+ = h_(theta theta),
hx = h_(theta phi) (both polarisations, two propagation directions), to the
order of the differencing; zero for Schwarzschild in isotropic and in
Kerr-Schild coordinates with the tetrad centred on the hole (Petrov type D
with radial principal null directions), converging with resolution."""
import math

import numpy as np
import pytest

import oracle
import z4c_inputs as zi
from z4c_inputs import analytic as an


def tt_wave(axis, Ap, Ax, L):
    """Linear TT wave along +axis on a periodic cube of side L: the two
    transverse axes (a, b) carry h_aa = -h_bb = Ap sin(k(s - t)) and
    h_ab = Ax cos(k(s - t)); alpha = 1, beta = 0, K_ij = -dh_ij/dt / 2."""
    k = 2.0 * math.pi / L
    a, b = [d for d in range(3) if d != axis]

    def fn(t, X, Y, Z):
        P = (X, Y, Z)
        ph = k * (P[axis] - t)
        one = an._ones(X) * (1.0 + 0 * t) * (1.0 + 0 * ph)
        gamma = np.zeros((3, 3) + np.shape(one), dtype=one.dtype)
        K = np.zeros_like(gamma)
        for d in range(3):
            gamma[d, d] = one
        gamma[a, a] = one + Ap * np.sin(ph)
        gamma[b, b] = one - Ap * np.sin(ph)
        gamma[a, b] = gamma[b, a] = Ax * np.cos(ph) * one
        # K = -1/2 dh/dt
        K[a, a] = -0.5 * (-Ap * k * np.cos(ph))
        K[b, b] = 0.5 * (-Ap * k * np.cos(ph))
        K[a, b] = K[b, a] = -0.5 * (Ax * k * np.sin(ph))
        return gamma, K, one, [0 * one, 0 * one, 0 * one]
    return fn, k, (a, b)


def psi4_on_mesh(mesh, fn, origin, order=6):
    om = oracle.OracleMesh(mesh)
    data = [an.adm_to_z4c(fn, 0.0, *mesh.grid(b)) for b in range(mesh.nb)]
    return oracle.psi4(om, zi.params_default(order), om.scatter(data), origin)


def test_flat_space_psi4_is_zero():
    mesh = zi.uniform_mesh((2, 1, 1), 8, 4, (0.0,) * 3, (2.0, 1.0, 1.0), zi.BC_OUTFLOW)
    om = oracle.OracleMesh(mesh)
    out = oracle.psi4(om, zi.params_default(6), om.scatter(zi.flat(mesh)), (0.3, 0.2, 0.1))
    assert all(np.all(b == 0.0) for b in out)


@pytest.mark.parametrize("axis,pol", [(0, "+"), (0, "x"), (1, "+"), (1, "x")])
def test_linear_wave_psi4_on_axis(axis, pol):
    """On the line through the tetrad origin along the propagation axis the
    coordinate tetrad is e_r = propagation direction, and Psi4 must equal
    d2h+/dt2 - i d2hx/dt2 of the wave."""
    L, A = 1.0, 1e-6
    Ap, Ax = (A, 0.0) if pol == "+" else (0.0, A)
    fn, k, (a, b) = tt_wave(axis, Ap, Ax, L)
    errs = []
    # 8 and 16 cells per wavelength: truncation dominates (at 32 the O(A)
    # nonlinear terms of the wave, ~1e-6 relative, take over)
    for n in (8, 16):
        mesh = zi.uniform_mesh((1, 1, 1), n, 4, (0.0,) * 3, (L,) * 3, zi.BC_PERIODIC)
        h = L / n
        # origin below the domain on the axis line through a row of zone centres
        c = (n // 2 + 0.5) * h
        origin = [c, c, c]
        origin[axis] = -0.3
        out = psi4_on_mesh(mesh, fn, origin)[0]
        # the zones on that line
        idx = [n // 2] * 3
        sl = [idx[2], idx[1], idx[0]]
        sl[2 - axis] = slice(None)
        re, im = out[0][tuple(sl)], out[1][tuple(sl)]
        s = (np.arange(n) + 0.5) * h
        # tetrad on the axis: e_theta, e_phi; h+ = h_(th th), hx = h_(th ph)
        e_r = np.eye(3)[axis]
        u = np.array([-e_r[1], e_r[0], 0.0])          # (-v_y, v_x, 0) direction
        if np.allclose(u, 0.0):
            pytest.skip("axis along z: the tetrad is degenerate there")
        e_ph = u / np.linalg.norm(u)
        w = np.cross(u, e_r)                           # w^a = eps_abc u^b v^c (flat)
        e_th = w / np.linalg.norm(w)
        H = np.zeros((3, 3, n))
        H[a, a] = Ap * np.sin(k * s)
        H[b, b] = -Ap * np.sin(k * s)
        H[a, b] = H[b, a] = Ax * np.cos(k * s)
        hdd = -k * k * H                               # d2/dt2 of f(s - t) = k^2 f''
        hp = np.einsum("i,j,ijn->n", e_th, e_th, hdd)
        hx = np.einsum("i,j,ijn->n", e_th, e_ph, hdd)
        want_re, want_im = hp, -hx
        scale = A * k * k
        errs.append(max(np.max(np.abs(re - want_re)), np.max(np.abs(im - want_im))) / scale)
    rate = math.log(errs[0] / errs[1]) / math.log(2.0)
    assert errs[1] < 1e-4 and rate > 5.0, (errs, rate)


@pytest.mark.parametrize("metric", ["isotropic", "kerr_schild"])
def test_schwarzschild_psi4_vanishes_with_centred_tetrad(metric):
    M = 1.0
    fn = an.schwarzschild_isotropic(M) if metric == "isotropic" else an.kerr_schild(M)
    res = []
    for n in (16, 32):
        # a block of the exterior, r in about [3.5, 7.5]
        mesh = zi.uniform_mesh((1, 1, 1), n, 4, (3.0, 2.0, 0.5), (7.0, 6.0, 4.5), zi.BC_OUTFLOW)
        out = psi4_on_mesh(mesh, fn, (0.0, 0.0, 0.0))[0]
        g = 4
        X, Y, Z = mesh.grid(0)
        r = np.sqrt(X * X + Y * Y + Z * Z)
        core = (slice(g, n - g),) * 3
        mag = np.hypot(out[0], out[1])[core] / (M / r[core] ** 3)
        res.append(float(np.max(mag)))
    rate = math.log(res[0] / res[1]) / math.log(2.0)
    assert res[1] < 1e-4 and rate > 4.5, (res, rate)
