"""Pins of the reference regrid (oracle/regrid.py) against what the method
fixes: the plan's rules (identity, round trip, 2:1 spreading and merge
cancellation checked on the raster), polynomial exactness of the transfer
operators (per-axis degree g exact, g+1 not: Lagrange interpolation with
g+1 nodes, Sec. 3.1), and agreement with the oracle's own cross-level ghost
fill (C code): a refined block's fine cells that coincide with a fine
neighbour's prolongated ghosts, and a merged block's coarse cells that
coincide with a coarse neighbour's restricted ghosts, must hold the same
values -- both are the same operator on the same coarse/fine data."""
import numpy as np
import pytest

import oracle
import z4c_inputs as zi
from oracle import regrid as rg

N8 = 8


def base(g=4, bc=zi.BC_OUTFLOW):
    """2 x 2 x 2 blocks of 8^3 on [0, 2]^3 (dx0 = 1/8)."""
    return zi.uniform_mesh((2, 2, 2), N8, g, (0.0,) * 3, (2.0,) * 3, bc)


def same_mesh(a, b):
    return (np.array_equal(a.level, b.level) and np.array_equal(a.n, b.n)
            and np.array_equal(a.ilo, b.ilo))


def volume_ok(m):
    F = int(m.level.max())
    vol = sum((int(m.n[b]) << (F - int(m.level[b]))) ** 3 for b in range(m.nb))
    return vol == np.prod([int(v) << F for v in m.nroot])


# ------------------------------------------------------------------ plan

def test_plan_identity_without_flags():
    m = zi.refine_blocks(base(), [0])
    assert same_mesh(rg.plan(m, np.zeros(m.nb), 3), m)


def test_plan_refine_all_then_merge_all_round_trip():
    m0 = base()
    m1 = rg.plan(m0, np.ones(m0.nb), 3)
    assert m1.nb == 64 and np.all(m1.level == 1) and volume_ok(m1)
    assert same_mesh(m1, zi.refine_blocks(m0, range(8)))
    m2 = rg.plan(m1, -np.ones(m1.nb), 3)
    assert same_mesh(m2, m0)


def test_plan_level_max_caps_refinement():
    m0 = base()
    assert same_mesh(rg.plan(m0, np.ones(m0.nb), 0), m0)


def test_plan_refinement_spreads_to_coarser_neighbours():
    m = zi.refine_blocks(base(), [0])          # levels 0 (7 blocks) and 1 (8 blocks)
    flags = np.zeros(m.nb)
    flags[7] = 1                               # the level-1 child at the far corner (1,1,1)
    out = rg.plan(m, flags, 3)
    assert rg.two_to_one_ok(out) and volume_ok(out)
    assert int(out.level.max()) == 2
    # every coarse block touching the refined child's region was refined
    assert np.sum(out.level == 0) < 7
    assert rg.two_to_one_ok(m)


def test_plan_merges_only_where_the_rule_allows():
    m = zi.refine_blocks(base(), range(8))     # uniform level 1, 64 blocks
    m = zi.refine_blocks(m, [7])               # one level-2 corner inside parent 0's region
    assert rg.two_to_one_ok(m)
    flags = -np.ones(m.nb)
    out = rg.plan(m, flags, 3)
    assert rg.two_to_one_ok(out) and volume_ok(out)
    # groups far from the level-2 blocks merged, the one holding them did not
    assert np.sum(out.level == 0) >= 1 and np.sum(out.level == 2) == 0
    # seven leaves of a parent (the eighth is refined) are no sibling group
    flags2 = np.zeros(m.nb)
    flags2[:7] = -1
    assert same_mesh(rg.plan(m, flags2, 3), m)
    # the children of M0's block 1 (indices 15..22 after the level-2 split)
    # would merge into a level-0 block touching the level-2 corner: cancelled
    assert np.all(m.level[15:23] == 1) and tuple(m.ilo[15]) == (16, 0, 0)
    flags3 = np.zeros(m.nb)
    flags3[15:23] = -1
    assert same_mesh(rg.plan(m, flags3, 3), m)
    # the same group merges once the level-2 blocks merge as well
    flags3[7:15] = -1
    out3 = rg.plan(m, flags3, 3)
    assert rg.two_to_one_ok(out3) and np.sum(out3.level == 0) == 1 and np.sum(out3.level == 2) == 0


# -------------------------------------------------------------- transfer

def poly_fields(X, Y, Z, deg, seed=0):
    """22 fields, each a random polynomial of per-axis degree <= deg."""
    rng = np.random.default_rng(seed)
    out = np.empty((22,) + X.shape)
    for f in range(22):
        c = rng.standard_normal((deg + 1, deg + 1, deg + 1))
        out[f] = np.polynomial.polynomial.polyval3d(X, Y, Z, c)
    return out


def user_ghosted(mesh, deg):
    from z4c_inputs import analytic as an
    return [poly_fields(*an.ghosted_grid(mesh, b), deg) for b in range(mesh.nb)]


@pytest.mark.parametrize("g", [3, 4, 5])
def test_transfer_polynomial_exactness(g):
    m = zi.refine_blocks(base(g=g, bc=zi.BC_USER), [0])
    om = oracle.OracleMesh(m)
    refined = zi.refine_blocks(m, [8])         # M0's block 1 -> eight children
    merged = base(g=g, bc=zi.BC_USER)          # block 0's children merged back
    for deg, exact in ((g, True), (g + 1, False)):
        u = om.scatter_ghosted(user_ghosted(m, deg))
        for new in (refined, merged):
            got = rg.transfer(m, u, new, fill=False)
            err = 0.0
            for b in range(new.nb):
                want = poly_fields(*new.grid(b), deg)
                err = max(err, np.max(np.abs(got[b] - want)) / np.max(np.abs(want)))
            if exact:
                assert err < 1e-12, (g, deg, err)
            else:
                assert err > 1e-8, (g, deg, err)


@pytest.mark.parametrize("g", [3, 4])
def test_transfer_matches_cross_level_ghost_fill(g):
    m0 = base(g=g)
    m = zi.refine_blocks(m0, [0])              # children of M0's block 0 are blocks 0..7
    om = oracle.OracleMesh(m)
    rng = np.random.default_rng(5)
    u = om.scatter([rng.standard_normal((22, N8, N8, N8)) for _ in range(m.nb)])
    filled = u.copy()
    oracle.fill_ghosts(om, filled)
    n = N8
    # restriction: merging block 0's children; M0's block 1 (index 8 here)
    # has its -x ghosts inside the merged block, filled by restriction
    merged = rg.transfer(m, u, m0)
    ghost = om.block_view(filled, 8)[:, g:g + n, g:g + n, 0:g]
    np.testing.assert_allclose(merged[0][:, :, :, n - g:n], ghost, rtol=0, atol=1e-13)
    # prolongation: refining block 8; the +x ghosts of block 0's children
    # with cx = 1 lie in the new children with cx = 0, filled by prolongation
    refined = zi.refine_blocks(m, [8])
    new = rg.transfer(m, u, refined)
    first_new = 8                              # the children replace block 8 in the order
    for cz in range(2):
        for cy in range(2):
            old = cz * 4 + cy * 2 + 1
            kid = first_new + cz * 4 + cy * 2 + 0
            assert refined.level[kid] == 1 and tuple(refined.ilo[kid]) == (16, 8 * cy, 8 * cz)
            ghost = om.block_view(filled, old)[:, g:g + n, g:g + n, g + n:g + n + g]
            np.testing.assert_allclose(new[kid][:, :, :, 0:g], ghost, rtol=0, atol=1e-13)


def test_prolongating_chi_through_a_puncture_overshoots_below_zero():
    """Refining the block that holds a Brill-Lindquist puncture prolongates
    chi = psi^-4 through its near-zero minimum: the (g+1)-point Lagrange
    interpolant (g = 4) of the coarse values, all positive, is negative at
    the fine cells next to the puncture, while the exact chi there is
    positive.  This is why initial refinement around punctures sets the
    data on the refined mesh instead of prolongating them."""
    m0 = zi.uniform_mesh((2, 2, 2), N8, 4, (-1.0,) * 3, (1.0,) * 3, zi.BC_OUTFLOW)
    p0 = (-0.5, -0.5, -0.5)                      # a cell corner of both levels, inside block 0
    data = zi.brill_lindquist(m0, [(0.5, p0)])
    assert min(float(b[0].min()) for b in data) > 0.0
    flags = np.zeros(m0.nb)
    flags[0] = 1
    m1 = rg.plan(m0, flags, 1)
    om = oracle.OracleMesh(m0)
    new = rg.transfer(m0, om.scatter(data), m1)
    exact = zi.brill_lindquist(m1, [(0.5, p0)])
    fine = [b for b in range(m1.nb) if m1.level[b] == 1]
    got_min = min(float(new[b][0].min()) for b in fine)
    exact_min = min(float(exact[b][0].min()) for b in fine)
    assert exact_min > 0.0 and got_min < 0.0, (got_min, exact_min)


def test_refinement_interface_rhs_error_is_third_order():
    """Reading R22 (Sec. 4.1's refined corner): the cross-level ghost values
    (n = N_g + 1 = 5 point Lagrange interpolation, Sec. 3.1) err at O(H^5),
    and the right-hand side takes second differences of them, so next to the
    refinement interface it errs at O(H^5 / h^2) = O(H^3) on both sides
    (prolongated fine ghosts and restricted coarse ghosts).  Measured as the
    RHS with the oracle's fill minus the RHS with exact (analytic) ghosts, on
    the linear wave with one octant refined."""
    from z4c_inputs import analytic as an

    def refined_corner(n, bc):
        base = zi.uniform_mesh((2, 2, 2), n // 2, 4, (0.0,) * 3, (1.0,) * 3, bc)
        return zi.refine_blocks(base, [0])
    fn = an.linear_wave_diagonal(1e-3, 1.0)

    def f(X, Y, Z):
        return an.adm_to_z4c(fn, 0.0, X, Y, Z)
    p = zi.params_default(6)
    errs = []
    for n in (16, 32):
        m1, m0 = refined_corner(n, zi.BC_PERIODIC), refined_corner(n, zi.BC_USER)
        o1, o0 = oracle.OracleMesh(m1), oracle.OracleMesh(m0)
        r1 = oracle.rhs(o1, p, o1.scatter([f(*m1.grid(b)) for b in range(m1.nb)]))
        r0 = oracle.rhs(o0, p, o0.scatter_ghosted(an.ghosted_data(m0, f)), fill=False)
        errs.append([max(np.abs(r1[b] - r0[b]).max() for b in range(m1.nb) if m1.level[b] == lev)
                     for lev in (1, 0)])
    rates = np.log2(np.array(errs[0]) / np.array(errs[1]))
    assert np.all((rates > 2.6) & (rates < 3.4)), (errs, rates)   # measured 2.98, 2.81
