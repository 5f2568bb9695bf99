"""Pins of the oracle's ghost fill: same-level copies and boundary
conditions against numpy's own padding, and the cross-level Lagrange
restriction/prolongation (Sec. 3.1, Eqs. 1-2) against polynomial exactness
and its convergence order (P13)."""
import numpy as np
import pytest

import oracle
import z4c_inputs as zi


@pytest.mark.parametrize("bc,mode", [(zi.BC_PERIODIC, "wrap"), (zi.BC_OUTFLOW, "edge")])
def test_same_level_fill_matches_numpy_pad(bc, mode):
    g, n = 4, 8
    mesh = zi.uniform_mesh((2, 3, 2), n, g, (0, 0, 0), (2, 3, 2), bc)
    rng = np.random.default_rng(0)
    glob = rng.standard_normal((22, 2 * n, 3 * n, 2 * n))  # [f, z, y, x]
    parts = []
    for b in range(mesh.nb):
        i0, j0, k0 = mesh.ilo[b]
        parts.append(glob[:, k0:k0 + n, j0:j0 + n, i0:i0 + n].copy())
    om = oracle.OracleMesh(mesh)
    u = om.scatter(parts)
    oracle.fill_ghosts(om, u)
    padded = np.pad(glob, ((0, 0), (g, g), (g, g), (g, g)), mode=mode)
    for b in range(mesh.nb):
        i0, j0, k0 = mesh.ilo[b]
        want = padded[:, k0:k0 + n + 2 * g, j0:j0 + n + 2 * g, i0:i0 + n + 2 * g]
        np.testing.assert_array_equal(om.block_view(u, b), want)


def two_level(n=8, g=4, bc=zi.BC_OUTFLOW):
    base = zi.uniform_mesh((4, 4, 4), n, g, (0.0,) * 3, (32.0,) * 3, bc)
    centre = zi.blocks_in_box(base, (8.0,) * 3, (24.0,) * 3)
    return zi.refine_blocks(base, centre)


def _ghost_check(mesh, u_fn, deg_ok):
    """Fill ghosts of polynomial data; compare ghost cells inside the domain."""
    from z4c_inputs import analytic as an
    om = oracle.OracleMesh(mesh)
    inter = [u_fn(*mesh.grid(b)) for b in range(mesh.nb)]
    u = om.scatter(inter)
    oracle.fill_ghosts(om, u)
    worst = 0.0
    scale = 0.0
    for b in range(mesh.nb):
        X, Y, Z = an.ghosted_grid(mesh, b)
        inside = ((X > 0) & (X < 32) & (Y > 0) & (Y < 32) & (Z > 0) & (Z < 32))
        got = om.block_view(u, b)
        want = u_fn(X, Y, Z)
        worst = max(worst, np.abs(got - want)[:, inside].max())
        scale = max(scale, np.abs(want).max())
    return worst, scale


@pytest.mark.parametrize("g", [2, 4, 5])
def test_cross_level_exact_for_polynomials(g):
    """n = g+1 point Lagrange interpolation is exact for per-axis degree g
    (Sec. 3.1 chooses n = N_g + 1); one degree more is not reproduced."""
    mesh = two_level(8, g)
    rng = np.random.default_rng(g)
    c = rng.uniform(-1, 1, size=(g + 2, g + 2, g + 2))

    def poly(deg):
        cc = np.zeros_like(c)
        cc[:deg + 1, :deg + 1, :deg + 1] = c[:deg + 1, :deg + 1, :deg + 1]
        def fn(X, Y, Z):
            v = np.polynomial.polynomial.polyval3d(X / 32, Y / 32, Z / 32, cc)
            return np.broadcast_to(v, (22,) + v.shape) * 1.0
        return fn
    worst, scale = _ghost_check(mesh, poly(g), True)
    assert worst < 1e-12 * scale, (worst, scale)
    worst, scale = _ghost_check(mesh, poly(g + 1), False)
    assert worst > 1e-10 * scale


@pytest.mark.parametrize("g", [2, 4])
def test_cross_level_convergence_order(g):
    """P13: interpolation error of smooth data falls at order g+1
    (3rd order with 2 ghosts, 5th with 4, as the paper states)."""
    errs = []
    for n in (8, 16):
        mesh = two_level(n, g)

        def fn(X, Y, Z):
            v = np.sin(0.3 * X + 0.2 * Y) * np.cos(0.25 * Z)
            return np.broadcast_to(v, (22,) + v.shape) * 1.0
        worst, _ = _ghost_check(mesh, fn, True)
        errs.append(worst)
    rate = np.log2(errs[0] / errs[1])
    assert rate > g + 1 - 0.5, (errs, rate)


def test_cross_level_rhs_smooth():
    """With two levels the RHS of smooth data stays close to the analytic one
    on both sides of the refinement boundary (no spurious jumps)."""
    from z4c_inputs import analytic as an
    mesh = two_level(8, 4)
    fn = an.kerr_schild(1.0, centre=(16.0, 16.0, 16.0))
    inter = [an.adm_to_z4c(fn, 0.0, *mesh.grid(b)) for b in range(mesh.nb)]
    om = oracle.OracleMesh(mesh)
    p = zi.params_default(6)
    p["terms"] = 5
    r = oracle.rhs(om, p, om.scatter(inter))
    worst = 0.0
    for b in range(mesh.nb):
        X, Y, Z = mesh.grid(b)
        rr = np.sqrt((X - 16) ** 2 + (Y - 16) ** 2 + (Z - 16) ** 2)
        far = (rr > 5) & (X > 6) & (X < 26) & (Y > 6) & (Y < 26) & (Z > 6) & (Z < 26)
        if far.any():
            worst = max(worst, np.abs(r[b][:18][:, far]).max())
    assert worst < 5e-4, worst


def test_threaded_fill_equals_serial():
    """Filling disjoint block sets in host threads from one copy of the
    register gives bitwise the serial fill (values depend on active zones
    only), on a two-level mesh with restriction and prolongation."""
    base = zi.uniform_mesh((4, 4, 4), 8, 4, (0.0,) * 3, (32.0,) * 3, zi.BC_OUTFLOW)
    mesh = zi.refine_blocks(base, zi.blocks_in_box(base, (8.0,) * 3, (24.0,) * 3))
    rng = np.random.default_rng(3)
    data = [rng.standard_normal((22, int(n), int(n), int(n))) for n in mesh.n]
    om = oracle.OracleMesh(mesh)
    a = om.scatter(data)
    b = a.copy()
    oracle.fill_ghosts(om, a)
    oracle.fill_ghosts(om, b, threads=5)
    assert np.array_equal(a, b)
