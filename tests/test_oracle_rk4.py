"""Pins of the oracle's RK4 stages and algebraic enforcement (P5, P12, gauge
ODEs in closed form)."""
import numpy as np
import pytest

import oracle
import z4c_inputs as zi


def periodic(n=16, g=4, lo=0.0, hi=1.0):
    return zi.uniform_mesh((1, 1, 1), n, g, (lo,) * 3, (hi,) * 3, zi.BC_PERIODIC)


def test_rk4_stability_polynomial_on_nyquist_mode():
    """P5: dissipation only, Nyquist mode on Theta over flat space, sigma 0.5,
    CFL 0.25: one step multiplies the mode by R(z) = 1+z+z^2/2+z^3/6+z^4/24 at
    z = -3 sigma CFL = -0.375, R = 22523/32768; other fields stay untouched."""
    mesh = periodic()
    data = zi.flat(mesh)
    I = np.indices((16, 16, 16)).sum(0)
    mode = np.where(I % 2 == 0, 1.0, -1.0) * 2.0 ** -20
    data[0][17] += mode
    p = zi.params_default(4)
    p["terms"] = 8
    p["enforce"] = 0
    om = oracle.OracleMesh(mesh)
    regs = oracle.Registers(om, data)
    oracle.rk4_steps(regs, p, 0.25 * mesh.dx0, 1)
    out = om.interiors(regs.U)[0]
    R = 22523.0 / 32768.0
    np.testing.assert_allclose(out[17], R * mode, rtol=4 * 2.0 ** -52, atol=0)
    for f in range(22):
        if f != 17:
            np.testing.assert_array_equal(out[f], data[0][f])


def test_rk4_fourth_order_in_time():
    """P12: at fixed h the semi-discrete system is an ODE; halving dt must cut
    the time-integration error by 2^4 (Richardson ratio of 16)."""
    mesh, p, data, dt, _ = zi.workload("periodic16")
    mesh = periodic(8, 4)
    data = zi.add_perturbation(mesh, zi.flat(mesh), seed=3, amp=1e-3, periodic_box=1.0)
    for b in data:
        b[19:22] += 0.2
    p = zi.params_default(4)
    p["enforce"] = 0
    om = oracle.OracleMesh(mesh)
    T = 0.25
    res = []
    for nst in (4, 8, 16):
        regs = oracle.Registers(om, data)
        oracle.rk4_steps(regs, p, T / nst, nst)
        res.append(om.interiors(regs.U)[0])
    e1 = np.abs(res[0] - res[1]).max()
    e2 = np.abs(res[1] - res[2]).max()
    assert 13.0 < e1 / e2 < 19.0, (e1, e2)


def test_gauge_odes_closed_form():
    """Gauge terms only on spatially constant data: alpha' = -2 alpha Khat and
    beta' = mu_S Gamma - eta beta with Khat and Gamma frozen, so
    alpha(T) = alpha0 exp(-2 Khat T) and
    beta(T) = mu_S Gamma/eta + (beta0 - mu_S Gamma/eta) exp(-eta T)."""
    mesh = periodic(8, 4)
    data = zi.flat(mesh)
    K0, a0, G0, b0 = 0.3, 0.8, np.array([0.1, -0.2, 0.05]), np.array([0.4, 0.0, -0.3])
    data[0][7] = K0
    data[0][18] = a0
    for i in range(3):
        data[0][14 + i] = G0[i]
        data[0][19 + i] = b0[i]
    p = zi.params_default(4)
    p["terms"] = 2
    p["enforce"] = 0
    p["eta"] = 1.7
    p["mu_S"] = 0.75
    om = oracle.OracleMesh(mesh)
    T, nst = 1.0, 64
    regs = oracle.Registers(om, data)
    oracle.rk4_steps(regs, p, T / nst, nst)
    out = om.interiors(regs.U)[0]
    dt = T / nst
    assert abs(out[18].mean() - a0 * np.exp(-2 * K0 * T)) < 2 * (2 * K0 * dt) ** 4 * T
    for i in range(3):
        bi = p["mu_S"] * G0[i] / p["eta"]
        ex = bi + (b0[i] - bi) * np.exp(-p["eta"] * T)
        assert abs(out[19 + i].mean() - ex) < (p["eta"] * dt) ** 4 * T
        assert np.ptp(out[19 + i]) == 0.0
    np.testing.assert_array_equal(out[7], data[0][7])


def test_enforcement_restores_unit_determinant_and_trace_free():
    """After a stage write: det g~ = 1, g~^ij A~_ij = 0, floors applied."""
    mesh = periodic(8, 4)
    rng = np.random.default_rng(2)
    data = zi.flat(mesh)
    data[0] += 0.05 * rng.standard_normal(data[0].shape)
    data[0][0] = np.abs(data[0][0]) * 0.5
    data[0][0][0, 0, 0] = 1e-5
    data[0][18][1, 1, 1] = 1e-6
    p = zi.params_default(4)
    p["chi_floor"] = 1e-2
    p["alpha_floor"] = 1e-2
    om = oracle.OracleMesh(mesh)
    regs = oracle.Registers(om, data)
    oracle.rk4_stage(regs, p, 1, 1e-9)
    s1 = om.interiors(regs.S1)[0]
    g = np.stack([np.stack([s1[1 + zi.SYM[i][j]] for j in range(3)]) for i in range(3)])
    A = np.stack([np.stack([s1[8 + zi.SYM[i][j]] for j in range(3)]) for i in range(3)])
    gm = np.moveaxis(g, (0, 1), (-2, -1))
    np.testing.assert_allclose(np.linalg.det(gm), 1.0, rtol=0, atol=1e-14)
    tr = np.einsum("...ij,...ij->...", np.linalg.inv(gm), np.moveaxis(A, (0, 1), (-2, -1)))
    assert np.abs(tr).max() < 1e-14
    assert s1[0].min() >= 1e-2 and s1[18].min() >= 1e-2
    assert s1[0][0, 0, 0] == 1e-2
