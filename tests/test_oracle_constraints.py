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
