"""Pins of the oracle's Z4c right-hand side (P2, P7, P8, P10, P11 and exact
solutions).  Each case compares the discrete RHS with something the
mathematics fixes independently of the oracle's formulas."""
import numpy as np
import pytest

import oracle
import z4c_inputs as zi
from z4c_inputs import analytic as an

PHYS, GAUGE, ADVECT, DISSIP = 1, 2, 4, 8


def rhs_on(fn, lo, hi, n, order, terms, t0=0.0):
    mesh = zi.uniform_mesh((1, 1, 1), n, order // 2 + 1, (lo,) * 3, (hi,) * 3, zi.BC_USER)
    data = an.ghosted_data(mesh, lambda X, Y, Z: an.adm_to_z4c(fn, t0, X, Y, Z))
    om = oracle.OracleMesh(mesh)
    p = zi.params_default(order)
    p["terms"] = terms
    r = oracle.rhs(om, p, om.scatter_ghosted(data), fill=False)[0]
    return mesh, r


def orders(errs):
    errs = np.asarray(errs)
    return np.log2(errs[:-1] / errs[1:])


@pytest.mark.parametrize("order", [4, 6, 8])
def test_flat_space_rhs_is_zero(order):
    """P2: Minkowski data give an RHS of exactly 0.0 in every field."""
    mesh = zi.uniform_mesh((2, 1, 1), 8, order // 2 + 1, (0, 0, 0), (2, 1, 1), zi.BC_OUTFLOW)
    om = oracle.OracleMesh(mesh)
    r = oracle.rhs(om, zi.params_default(order), om.scatter(zi.flat(mesh)))
    for b in r:
        assert np.all(b == 0.0)


def test_kasner_rhs_is_exact_time_derivative():
    """Rotated Kasner (homogeneous vacuum, geodesic slicing, gauge frozen):
    every spatial derivative vanishes, so the algebraic terms of the chi, g~,
    Khat, A~ and Theta equations must reproduce the exact time derivative of
    the solution, to rounding."""
    th, ph = 0.7, 0.4
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, np.cos(ph), -np.sin(ph)], [0, np.sin(ph), np.cos(ph)]])
    fn = an.kasner(2.0, Rz @ Rx)
    for t0 in (0.6, 1.7):
        mesh, r = rhs_on(fn, 0.0, 1.0, 8, 6, PHYS, t0)
        ex = an.z4c_time_derivative(fn, t0, *mesh.grid(0))
        for f in range(18):
            np.testing.assert_allclose(r[f], ex[f], rtol=0, atol=2e-15 * max(1, np.abs(ex).max()))


@pytest.mark.parametrize("order,lo_order,ns", [(4, 3.4, (8, 16, 32)), (6, 5.3, (8, 16, 32)),
                                               (8, 6.5, (12, 16, 20))])
def test_kerr_schild_stationary(order, lo_order, ns):
    """Kerr-Schild Schwarzschild is stationary in its own lapse and shift:
    with the gauge frozen, every Z4c RHS must vanish at the order of the
    differencing (non-zero K_ij, shift and curvature exercise nearly every
    term, the advection stencils included)."""
    fn = an.kerr_schild(1.0)
    errs = []
    for n in ns:
        _, r = rhs_on(fn, 2.0, 4.0, n, order, PHYS | ADVECT)
        errs.append([np.abs(r[f]).max() for f in range(18)])
    errs = np.array(errs)
    for f in range(18):
        o = np.log(errs[:-1, f] / errs[1:, f]) / np.log(np.array(ns[1:]) / np.array(ns[:-1]))
        assert o[-1] > lo_order, (zi.FIELDS[f], errs[:, f], o)


@pytest.mark.parametrize("order", [4, 6])
def test_isotropic_schwarzschild_static(order):
    """P8: static Schwarzschild in isotropic coordinates with its static
    lapse; the full method (gauge, advection, dissipation on) gives an RHS
    that vanishes at the differencing order.  Pins the Ricci tensor, D_iD_j
    alpha and the trace-free projection (alpha R_ij = D_i D_j alpha)."""
    fn = an.schwarzschild_isotropic(1.0)
    errs = []
    for n in (8, 16, 32):
        _, r = rhs_on(fn, 2.0, 4.0, n, order, PHYS | GAUGE | ADVECT | DISSIP)
        errs.append([np.abs(r[f]).max() for f in range(22)])
    errs = np.array(errs)
    for f in (0, 7, 8, 9, 17, 18):
        assert orders(errs[:, f])[-1] > order - 0.6, (zi.FIELDS[f], errs[:, f])
    for f in (1, 2, 3, 4, 5, 6, 14, 15, 16, 19, 20, 21):
        assert errs[:, f].max() < 1e-13


def test_linear_wave_time_derivative():
    """P10: the linearised TT wave (Sec. 4.1 test problem) along x: the RHS
    matches the analytic time derivative at order 2N (amplitude small
    enough for the quadratic error to be negligible)."""
    fn = an.linear_wave(1e-7, 1.0)
    errs = []
    ns = (8, 12, 16)
    for n in ns:
        mesh, r = rhs_on(fn, 0.0, 1.0, n, 6, PHYS | GAUGE | ADVECT)
        ex = an.z4c_time_derivative(fn, 0.0, *mesh.grid(0))
        errs.append(max(np.abs(r[f] - ex[f]).max() for f in (4, 6, 11, 13)))
    for a in range(2):
        rate = np.log(errs[a] / errs[a + 1]) / np.log(ns[a + 1] / ns[a])
        assert rate > 5.5, errs


def test_axis_permutation_covariance():
    """P11: cyclically permuting the axes (and tensor indices) of the data
    permutes the RHS the same way (smooth non-symmetric data, full method)."""
    mesh = zi.uniform_mesh((1, 1, 1), 12, 4, (0,) * 3, (1,) * 3, zi.BC_PERIODIC)
    data = zi.add_perturbation(mesh, zi.flat(mesh), seed=7, amp=1e-3, periodic_box=1.0)
    for b in data:   # a non-zero shift of both signs
        b[19:22] += 0.05
    om = oracle.OracleMesh(mesh)
    p = zi.params_default(6)
    r = oracle.rhs(om, p, om.scatter(data))[0]

    # cyclic permutation x->y->z->x of the coordinates: new(x,y,z) = old(z,x,y)
    def perm(u):
        v = np.empty_like(u)
        # scalar map: new(X,Y,Z) = old(Z,X,Y) -> array new[k,j,i] = old[j,i,k]
        def sc(a):
            return np.transpose(a, (1, 2, 0))
        # vector component: new^x = old^z, new^y = old^x, new^z = old^y
        vmap = {0: 2, 1: 0, 2: 1}
        for s in (0, 7, 17, 18):
            v[s] = sc(u[s])
        for i in range(3):
            v[14 + i] = sc(u[14 + vmap[i]])
            v[19 + i] = sc(u[19 + vmap[i]])
            for j in range(i, 3):
                a, bb = vmap[i], vmap[j]
                v[1 + zi.SYM[i][j]] = sc(u[1 + zi.SYM[a][bb]])
                v[8 + zi.SYM[i][j]] = sc(u[8 + zi.SYM[a][bb]])
        return v
    rp = oracle.rhs(om, p, om.scatter([perm(data[0])]))[0]
    np.testing.assert_allclose(rp, perm(r), rtol=0, atol=1e-12 * np.abs(r).max())


@pytest.mark.parametrize("bc", [zi.BC_PERIODIC, zi.BC_OUTFLOW])
def test_multiblock_equals_single_block(bc):
    """Splitting a uniform grid into MeshBlocks must not change the RHS:
    same-level ghosts are exact copies, so the result is bitwise equal."""
    g = 4
    big = zi.uniform_mesh((1, 1, 1), 16, g, (-1,) * 3, (1,) * 3, bc)
    split = zi.uniform_mesh((2, 2, 2), 8, g, (-1,) * 3, (1,) * 3, bc)
    rng = np.random.default_rng(5)
    field = zi.flat(big)[0] + 1e-3 * rng.standard_normal((22, 16, 16, 16))
    field[19:22] += 0.01 * rng.standard_normal((3, 16, 16, 16))
    p = zi.params_default(6)
    ob = oracle.OracleMesh(big)
    r_big = oracle.rhs(ob, p, ob.scatter([field]))[0]
    osp = oracle.OracleMesh(split)
    parts = []
    for b in range(split.nb):
        i0, j0, k0 = split.ilo[b]
        parts.append(field[:, k0:k0 + 8, j0:j0 + 8, i0:i0 + 8].copy())
    r_sp = oracle.rhs(osp, p, osp.scatter(parts))
    for b in range(split.nb):
        i0, j0, k0 = split.ilo[b]
        np.testing.assert_array_equal(r_sp[b], r_big[:, k0:k0 + 8, j0:j0 + 8, i0:i0 + 8])
