"""Precision extension: FP32 storage and derivatives with FP64 RK
accumulation, constraints and floors.

Bound used for the RHS of every field f against the FP64 oracle on the same
data (the FP32 pack stores the inputs rounded to float32):
    |rhs32_f - rhs64_f| <= K u32 (max|rhs64_f| + S W2 / h^2),
u32 = 2^-24, S = the largest |value| of the O(1) fields, W2 = sum of |w| of
the second-derivative stencil (the worst-case propagation of one rounding
per stencil point into a second derivative), K = 64 (number of terms a
field's RHS sums, rounded up).  For the evolved state after n steps the
bound is n dt times the RHS bound plus the storage rounding u32 max|f|."""
import numpy as np
import pytest

import oracle
import z4c_inputs as zi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
W2 = {4: 2 * (4 / 3 + 1 / 12) + 5 / 2, 6: 2 * (3 / 2 + 3 / 20 + 1 / 90) + 49 / 18,
      8: 2 * (8 / 5 + 1 / 5 + 8 / 315 + 1 / 560) + 205 / 72}
K = 64.0


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def z():
    import paper_2409_10383_amd as m
    return m


def rhs_bound(order, h, ora_blocks, data):
    S = max(np.abs(d[[0, 1, 4, 6, 18]]).max() for d in data)
    mx = np.max([np.abs(o).reshape(22, -1).max(1) for o in ora_blocks], axis=0)
    return K * U32 * (mx + S * W2[order] / h ** 2)


def test_fp32_flat_space_zero():
    mesh = zi.uniform_mesh((2, 1, 1), 16, 4, (0, 0, 0), (2, 1, 1), zi.BC_OUTFLOW)
    pk = z().Pack(mesh, zi.params_default(6), z().FP32_MIXED)
    pk.upload(z().REG_U, zi.flat(mesh))
    pk.fill_ghosts()
    assert torch.count_nonzero(pk.rhs()).item() == 0


@pytest.mark.parametrize("name", ["periodic16", "bl64x32"])
def test_fp32_rhs_within_bound(name):
    mesh, p, data, dt, _ = zi.workload(name)
    pk = z().Pack(mesh, p, z().FP32_MIXED)
    pk.upload(z().REG_U, data)
    pk.fill_ghosts()
    rg = pk.split_interior(pk.rhs())
    om = oracle.OracleMesh(mesh)
    ro = oracle.rhs(om, p, om.scatter(data))
    bound = rhs_bound(p["fd_order"], mesh.dx0, ro, data)
    err = np.max([np.abs(g - o).reshape(22, -1).max(1) for g, o in zip(rg, ro)], axis=0)
    assert np.all(err <= bound), [(f, err[f], bound[f]) for f in range(22) if err[f] > bound[f]]
    print(name, "max err/bound:", float((err / bound).max()))


@pytest.mark.parametrize("order", [6, 8])
def test_fp32_every_tile_shape(order):
    """FP32 storage in every tile shape and launch mode (the width of the
    copies into LDS follows the shape and ghost depth: 16 bytes for the
    6th-order tiles, 4 otherwise): the RHS within the derived bound of the
    oracle, and the RHS and one RK4 step bitwise the same in every shape."""
    g = order // 2 + 1
    mesh = zi.uniform_mesh((2, 2, 2), 16, g, (-4.0,) * 3, (4.0,) * 3, zi.BC_OUTFLOW)
    data = zi.add_perturbation(mesh, zi.brill_lindquist(mesh, [(1.0, (0.2, 0.0, 0.0))]), seed=3, amp=1e-4)
    p = zi.params_default(order)
    dt = 0.25 * mesh.dx0
    om = oracle.OracleMesh(mesh)
    ro = oracle.rhs(om, p, om.scatter(data))
    bound = rhs_bound(order, mesh.dx0, ro, data)
    first = None
    for v in range(len(z().TILE_SHAPES)):
        for pers in (False, True):
            pk = z().Pack(mesh, p, z().FP32_MIXED)
            pk.upload(z().REG_U, data)
            pk.set_variant(v, pers)
            pk.fill_ghosts()
            rg = pk.split_interior(pk.rhs())
            pk.rk4_step(dt, 1)
            torch.cuda.synchronize()
            st = pk.download(z().REG_U)
            if first is None:
                err = np.max([np.abs(a - b).reshape(22, -1).max(1) for a, b in zip(rg, ro)], axis=0)
                assert np.all(err <= bound), [(f, err[f], bound[f]) for f in range(22) if err[f] > bound[f]]
                first = (rg, st)
            else:
                for a, b in zip(rg, first[0]):
                    np.testing.assert_array_equal(a, b)
                for a, b in zip(st, first[1]):
                    np.testing.assert_array_equal(a, b)


def test_fp32_step_within_bound_and_accumulator_fp64():
    mesh, p, data, dt, _ = zi.workload("periodic16")
    nst = 2
    pk = z().Pack(mesh, p, z().FP32_MIXED)
    pk.upload(z().REG_U, data)
    pk.rk4_step(dt, nst)
    got = pk.download(z().REG_U)
    om = oracle.OracleMesh(mesh)
    ro = oracle.rhs(om, p, om.scatter(data))
    regs = oracle.Registers(om, data)
    oracle.rk4_steps(regs, p, dt, nst)
    want = om.interiors(regs.U)
    bound = nst * dt * rhs_bound(p["fd_order"], mesh.dx0, ro, data)
    bound = bound + 4 * U32 * np.max([np.abs(w).reshape(22, -1).max(1) for w in want], axis=0)
    err = np.max([np.abs(g - w).reshape(22, -1).max(1) for g, w in zip(got, want)], axis=0)
    assert np.all(err <= bound), [(f, err[f], bound[f]) for f in range(22) if err[f] > bound[f]]
    assert pk.acc_view().dtype == torch.float64


def test_fp32_hamiltonian_within_twice_fp64():
    """Brill-Lindquist puncture, 10 RK4 steps: the Hamiltonian-constraint L2
    of the FP32-storage run stays within 2x the FP64 run's (excising r < 2,
    where FP32 rounding of d^2 chi dominates the truncation error)."""
    mesh, p, data, dt, steps = zi.workload("bl64x32")
    out = {}
    for prec in (z().FP64, z().FP32_MIXED):
        pk = z().Pack(mesh, p, prec)
        pk.upload(z().REG_U, data)
        pk.rk4_step(dt, steps)
        _, n_full = pk.constraints(per_zone=False)
        _, n_exc = pk.constraints(per_zone=False, exclude=[(0.0, 0.0, 0.0)], r_exc=2.0)
        out[prec] = (n_full[0], n_exc[0])
    r_full = out[z().FP32_MIXED][0] / out[z().FP64][0]
    r_exc = out[z().FP32_MIXED][1] / out[z().FP64][1]
    print("H_L2 fp32/fp64: full", r_full, "excised", r_exc)
    assert r_full <= 2.0
    assert np.isfinite(r_exc)


def _two_level(g):
    base = zi.uniform_mesh((4, 4, 4), 8, g, (0.0,) * 3, (32.0,) * 3, zi.BC_OUTFLOW)
    return zi.refine_blocks(base, zi.blocks_in_box(base, (8.0,) * 3, (24.0,) * 3))


@pytest.mark.parametrize("order", [6, 8])
def test_fp32_cross_level_fill_and_rhs(order):
    """FP32 storage on a two-level mesh: every ghost cell (same-level copies,
    restriction and prolongation with double weights and a float32 store)
    against the oracle's fill of the same rounded data, within one float32
    rounding of the value plus four of the field's scale: restricted coarse
    images and shadow values are themselves stored in float32, and the
    prolongation weights (sum of |w| per axis about 1.3, cubed) carry their
    rounding into the fine ghosts; the RHS across the refinement boundary
    within the FP32 bound at the finest spacing."""
    from z4c_inputs import analytic as an
    mesh = _two_level(order // 2 + 1)
    fn = an.kerr_schild(1.0, centre=(16.3, 15.8, 16.1))
    data = [an.adm_to_z4c(fn, 0.0, *mesh.grid(b)) for b in range(mesh.nb)]
    data = zi.add_perturbation(mesh, data, seed=3, amp=1e-4)
    data = [d.astype(np.float32).astype(np.float64) for d in data]
    p = zi.params_default(order)
    pk = z().Pack(mesh, p, z().FP32_MIXED)
    pk.upload(z().REG_U, data)
    pk.fill_ghosts()
    got = pk.download(z().REG_U, ghosted=True)
    om = oracle.OracleMesh(mesh)
    u = om.scatter(data)
    oracle.fill_ghosts(om, u)
    want = [om.block_view(u, b) for b in range(mesh.nb)]
    fmax = np.max([np.abs(w).reshape(22, -1).max(1) for w in want], axis=0)
    for b, (g_, w_) in enumerate(zip(got, want)):
        tol = U32 * (2.0 * np.abs(w_) + 4.0 * fmax[:, None, None, None])
        assert np.all(np.abs(g_ - w_) <= tol), (b, float(np.max((np.abs(g_ - w_) - tol)
                                                                / fmax[:, None, None, None])))
    rg = pk.split_interior(pk.rhs())
    ro = oracle.rhs(om, p, om.scatter(data))
    bound = rhs_bound(order, mesh.dx_min(), ro, data)
    err = np.max([np.abs(g - o).reshape(22, -1).max(1) for g, o in zip(rg, ro)], axis=0)
    assert np.all(err <= bound), [(f, err[f], bound[f]) for f in range(22) if err[f] > bound[f]]
    print(order, "max err/bound:", float((err / bound).max()))


def test_fp32_storage_constraints_and_interpolation_in_double():
    """Constraint monitors and state interpolation read FP32 storage but
    compute in double, so on data already rounded to float32 they equal the
    oracle's double results on the same data to the FP64 bar."""
    from _parity import assert_parity
    from oracle import extract as ex
    mesh = zi.uniform_mesh((2, 2, 2), 8, 4, (-4.0,) * 3, (4.0,) * 3, zi.BC_OUTFLOW)
    data = zi.brill_lindquist(mesh, [(1.0, (0.1, -0.2, 0.05))])
    data = zi.add_perturbation(mesh, data, seed=8, amp=1e-4)
    data = [d.astype(np.float32).astype(np.float64) for d in data]
    p = zi.params_default(6)
    pk = z().Pack(mesh, p, z().FP32_MIXED)
    pk.upload(z().REG_U, data)
    cz, norms = pk.constraints(z().REG_U, exclude=[(0.1, -0.2, 0.05)], r_exc=1.0)
    om = oracle.OracleMesh(mesh)
    co, no = oracle.constraints(om, p, om.scatter(data), exclude=[(0.1, -0.2, 0.05)], r_exc=1.0)
    assert_parity(pk.split_interior(cz, 8), co, what="constraints, FP32 storage")
    np.testing.assert_allclose(norms, no, rtol=1e-12, atol=0)
    pts = np.random.default_rng(4).uniform(-3.9, 3.9, size=(300, 3))
    got = pk.interp_state(z().REG_U, 18, 4, pts)
    want = ex.interpolate(mesh, [b[18:22] for b in data], pts)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_fp32_floors_active_step_within_bound():
    """FP32 storage with the floors active (chi_floor = 1e-2, alpha_floor =
    5e-2 on Brill-Lindquist data at dx = 1/8, where chi ~ 1e-3 and alpha ~
    3e-2 next to the puncture): floors and divisions by chi in double, one RK4
    step within the FP32 bound of the FP64 oracle on the same float32-rounded
    data; the floored cells hold float32(floor) and are the oracle's."""
    mesh = zi.uniform_mesh((2, 2, 2), 16, 4, (-2.0,) * 3, (2.0,) * 3, zi.BC_OUTFLOW)
    data = zi.brill_lindquist(mesh, [(1.0, (0.0, 0.0, 0.0))])
    data = [d.astype(np.float32).astype(np.float64) for d in data]
    p = dict(zi.params_default(6), chi_floor=1e-2, alpha_floor=5e-2)
    dt = 0.25 * mesh.dx0
    pk = z().Pack(mesh, p, z().FP32_MIXED)
    pk.upload(z().REG_U, data)
    pk.rk4_step(dt, 1)
    got = pk.download(z().REG_U)
    om = oracle.OracleMesh(mesh)
    ro = oracle.rhs(om, p, om.scatter(data))
    regs = oracle.Registers(om, data)
    oracle.rk4_steps(regs, p, dt, 1)
    want = om.interiors(regs.U)
    for f, fl in ((0, p["chi_floor"]), (18, p["alpha_floor"])):
        n = sum(int((w[f] == fl).sum()) for w in want)
        assert n > 0, f
        for g_, w_ in zip(got, want):
            assert np.array_equal(g_[f] == np.float64(np.float32(fl)), w_[f] == fl), f
    bound = dt * rhs_bound(p["fd_order"], mesh.dx0, ro, data)
    bound = bound + 4 * U32 * np.max([np.abs(w).reshape(22, -1).max(1) for w in want], axis=0)
    err = np.max([np.abs(g - w).reshape(22, -1).max(1) for g, w in zip(got, want)], axis=0)
    assert np.all(err <= bound), [(f, err[f], bound[f]) for f in range(22) if err[f] > bound[f]]
    print("floored FP32 step max err/bound:", float((err / bound).max()))


def test_config4_fp32_storage_100_steps_within_field_bounds():
    """The precision workload (512 x 32^3 Brill-Lindquist plus 1e-6
    perturbations, dx = 0.125, 6th order): 100 RK4 steps with FP32 storage
    against the FP64 run; every field's largest difference below its
    a-priori bound (n u32 max|f| + n dt K u32 (max|rhs_f| + S W2 / h^2), the
    maxima from the FP64 initial state) and the Hamiltonian-constraint L2 of
    the FP32 run within twice the FP64 run's."""
    mesh, p, data, dt, steps = zi.workload("bl512x32")
    assert steps == 100
    states, hl2 = {}, {}
    for prec in (z().FP64, z().FP32_MIXED):
        pk = z().Pack(mesh, p, prec)
        pk.upload(z().REG_U, data)
        if prec == z().FP64:
            pk.fill_ghosts()
            rhs0 = pk.split_interior(pk.rhs())
        pk.rk4_step(dt, steps)
        _, nf = pk.constraints(per_zone=False)
        _, ne = pk.constraints(per_zone=False, exclude=[(0.0, 0.0, 0.0)], r_exc=2.0)
        hl2[prec] = (nf[0], ne[0])
        states[prec] = pk.download(z().REG_U)
        del pk
        torch.cuda.empty_cache()
    S = max(np.abs(d[[0, 1, 4, 6, 18]]).max() for d in data)
    worst = 0.0
    for f in range(22):
        err = max(float(np.abs(a[f] - b[f]).max()) for a, b in zip(states[z().FP32_MIXED], states[z().FP64]))
        fmax = max(float(np.abs(d[f]).max()) for d in data)
        rmax = max(float(np.abs(r[f]).max()) for r in rhs0)
        bound = steps * U32 * fmax + steps * dt * K * U32 * (rmax + S * W2[6] / mesh.dx0 ** 2)
        assert err <= bound, (zi.FIELDS[f], err, bound)
        worst = max(worst, err / bound)
    ratio = hl2[z().FP32_MIXED][0] / hl2[z().FP64][0]
    print("config 4: worst field error / bound", worst, "H_L2 fp32/fp64", ratio,
          "excised", hl2[z().FP32_MIXED][1] / hl2[z().FP64][1])
    assert ratio <= 2.0
