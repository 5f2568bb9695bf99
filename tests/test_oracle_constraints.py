"""Pins of the oracle's constraint monitors (P9, P14) and refinement
criteria (P15)."""
import numpy as np
import pytest

import oracle
import z4c_inputs as zi
from z4c_inputs import analytic as an


def cons_on(fn, lo, hi, n, order):
    mesh = zi.uniform_mesh((1, 1, 1), n, order // 2 + 1, (lo,) * 3, (hi,) * 3, zi.BC_USER)
    data = an.ghosted_data(mesh, lambda X, Y, Z: an.adm_to_z4c(fn, 0.0, X, Y, Z))
    om = oracle.OracleMesh(mesh)
    c, norms = oracle.constraints(om, zi.params_default(order), om.scatter_ghosted(data), fill=False)
    return mesh, c[0], norms, data[0]


def bl_fn(M=1.0):
    """Brill-Lindquist (time symmetric) as ADM data."""
    def fn(t, X, Y, Z):
        r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
        psi = 1.0 + M / (2 * r)
        gamma = np.zeros((3, 3) + np.shape(r), dtype=r.dtype)
        for i in range(3):
            gamma[i, i] = psi ** 4
        return gamma, np.zeros_like(gamma), psi ** -2, [0 * r, 0 * r, 0 * r]
    return fn


@pytest.mark.parametrize("order", [4, 6])
def test_brill_lindquist_hamiltonian_converges(order):
    """P9: BL data satisfy H = 0 (psi is harmonic); the discrete H vanishes
    at the differencing order away from the puncture."""
    errs = []
    for n in (8, 16, 32):
        _, c, _, _ = cons_on(bl_fn(), 2.0, 4.0, n, order)
        errs.append(np.abs(c[0]).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > order - 0.6, (errs, rates)


@pytest.mark.parametrize("order", [4, 6])
def test_kerr_schild_constraints_converge(order):
    """Kerr-Schild data satisfy H = M^i = 0 and Gamma~^i = Gamma~_d^i; all
    three discrete monitors vanish at the differencing order."""
    errs = []
    for n in (8, 16, 32):
        _, c, _, _ = cons_on(an.kerr_schild(1.0), 2.0, 4.0, n, order)
        errs.append([np.abs(c[0]).max(), np.abs(c[1:4]).max(), np.abs(c[5:8]).max()])
    errs = np.array(errs)
    for q in range(3):
        rate = np.log2(errs[-2, q] / errs[-1, q])
        assert rate > order - 0.7, (q, errs[:, q], rate)


def test_momentum_constraint_zero_for_vanishing_curvature():
    """P14: with A~ = 0, Khat = Theta = 0 every term of M^i vanishes: exactly 0."""
    _, c, _, data = cons_on(bl_fn(), 1.0, 3.0, 8, 6)
    assert np.all(c[1:4] == 0.0)
    np.testing.assert_array_equal(c[4], data[17][4:-4, 4:-4, 4:-4])


def test_norm_definitions():
    """L2 = sqrt(sum H^2 dV / sum dV) and Linf over the kept zones."""
    mesh = zi.uniform_mesh((2, 2, 2), 8, 4, (-4,) * 3, (4,) * 3, zi.BC_OUTFLOW)
    data = zi.brill_lindquist(mesh, [(1.0, (0.0, 0.0, 0.0))])
    om = oracle.OracleMesh(mesh)
    u = om.scatter(data)
    c, norms = oracle.constraints(om, zi.params_default(6), u, exclude=[(0.0, 0.0, 0.0)], r_exc=1.0)
    H, keep = [], []
    for b in range(mesh.nb):
        X, Y, Z = mesh.grid(b)
        k = np.sqrt(X ** 2 + Y ** 2 + Z ** 2) >= 1.0
        H.append(c[b][0][k])
    H = np.concatenate(H)
    np.testing.assert_allclose(norms[0], np.sqrt(np.mean(H ** 2)), rtol=1e-12)
    assert norms[1] == np.abs(H).max()


def test_refinement_flags_match_analytic():
    """P15: chi-min flags equal those from the analytic chi at the cell
    centres; dchi-max flags agree with the analytic gradient except inside a
    narrow band around the threshold; radius flags follow the geometry;
    level limits are respected."""
    mesh = zi.uniform_mesh((4, 4, 4), 8, 4, (-8,) * 3, (8,) * 3, zi.BC_OUTFLOW)
    data = zi.brill_lindquist(mesh, [(1.0, (0.5, 0.0, 0.0))])
    om = oracle.OracleMesh(mesh)
    u = om.scatter(data)
    p = zi.params_default(6)
    f = oracle.refine_flags(om, p, u, oracle.CRIT_CHI_MIN, chi_thr=0.3, level_max=5)
    for b in range(mesh.nb):
        cm = data[b][0].min()
        want = 1 if cm < 0.3 else (-1 if cm > 0.45 else 0)
        want = 0 if want < 0 else want   # level 0 cannot derefine
        assert f[b] == want
    f = oracle.refine_flags(om, p, u, oracle.CRIT_CHI_MIN, chi_thr=0.3, level_max=0)
    assert np.all(f == 0)
    thr = 0.05
    f = oracle.refine_flags(om, p, u, oracle.CRIT_DCHI_MAX, dchi_thr=thr, level_max=5)
    for b in range(mesh.nb):
        X, Y, Z = mesh.grid(b)
        x = X - 0.5
        r = np.sqrt(x ** 2 + Y ** 2 + Z ** 2)
        psi = 1 + 0.5 / r
        dchi = 4 * psi ** -5 * 0.5 / r ** 2   # |grad chi| = 4 psi^-5 |grad psi|
        g = dchi.max()
        if g > 1.05 * thr:
            assert f[b] == 1
        elif g < 0.95 * thr:
            assert f[b] == 0
    f = oracle.refine_flags(om, p, u, oracle.CRIT_RADIUS, radius=3.0, centre=(0, 0, 0),
                            radius_level=1, level_max=5)
    for b in range(mesh.nb):
        X, Y, Z = mesh.grid(b)
        near = np.sqrt(X ** 2 + Y ** 2 + Z ** 2).min() < 3.0
        assert f[b] == (1 if near else 0)


@pytest.mark.slow
def test_brill_lindquist_evolved_hamiltonian_converges():
    """P9 after evolution: Brill-Lindquist data (M = 1, pre-collapsed lapse)
    on [-8, 8]^3 evolved by the full method (6th order, Sec. 4.3 parameters)
    to the same time T = 1/8 with dt = 0.25 dx at dx = 1/2, 1/4, 1/8; the
    volume-weighted L2 norm of H over 2 <= r <= 6 converges at second order
    or better (measured: 6.2 and 6.0)."""
    T = 0.125
    errs = []
    for dx, nb in ((0.5, 1), (0.25, 2), (0.125, 4)):
        mesh = zi.uniform_mesh((nb,) * 3, 32, 4, (-8.0,) * 3, (8.0,) * 3, zi.BC_OUTFLOW)
        data = zi.brill_lindquist(mesh, [(1.0, (0.0, 0.0, 0.0))])
        p = zi.params_default(6)
        om = oracle.OracleMesh(mesh)
        regs = oracle.Registers(om, data)
        dt = 0.25 * dx
        oracle.rk4_steps(regs, p, dt, int(round(T / dt)), threads=8)
        c, _ = oracle.constraints(om, p, regs.U)
        num = den = 0.0
        for b in range(mesh.nb):
            X, Y, Z = mesh.grid(b)
            r = np.sqrt(X * X + Y * Y + Z * Z)
            m = (r >= 2.0) & (r <= 6.0)
            num += float((c[b][0][m] ** 2).sum())
            den += float(m.sum())
        errs.append(np.sqrt(num / den))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates >= 2.0), (errs, rates)


def test_threaded_oracle_step_equals_serial():
    """The host-threaded RK4 driver splits each stage's blocks over threads;
    it runs the same per-zone arithmetic, so the state is bitwise the serial
    one."""
    mesh = zi.uniform_mesh((2, 2, 1), 8, 4, (-4.0, -4.0, -2.0), (4.0, 4.0, 2.0), zi.BC_OUTFLOW)
    data = zi.add_perturbation(mesh, zi.brill_lindquist(mesh, [(1.0, (0.0, 0.0, 0.0))]), seed=5,
                               amp=1e-4)
    p = zi.params_default(6)
    om = oracle.OracleMesh(mesh)
    a = oracle.Registers(om, data)
    b = oracle.Registers(om, data)
    oracle.rk4_steps(a, p, 0.125, 1)
    oracle.rk4_steps(b, p, 0.125, 1, threads=3)
    assert all(np.array_equal(x, y) for x, y in zip(om.interiors(a.U), om.interiors(b.U)))
    assert all(np.array_equal(x, y) for x, y in zip(om.interiors(a.A), om.interiors(b.A)))
