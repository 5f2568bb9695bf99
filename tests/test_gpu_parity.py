"""GPU parity: every C-ABI call of libz4c against the oracle on the same
seeded inputs (relative L-infinity per field <= 1e-12 in FP64; integer
outputs exact)."""
import numpy as np
import pytest

import oracle
import z4c_inputs as zi
from _parity import assert_parity, field_errors, oracle_steps, ulp_perturbed, K_ROUND

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def z():
    import paper_2409_10383_amd as m
    return m


def small_bl(order, nblk=2, n=8, bc=zi.BC_OUTFLOW, perturb=True):
    g = order // 2 + 1
    mesh = zi.uniform_mesh((nblk,) * 3, n, g, (-4.0,) * 3, (4.0,) * 3, bc)
    data = zi.brill_lindquist(mesh, [(1.0, (0.0, 0.0, 0.0))])
    if perturb:
        data = zi.add_perturbation(mesh, data, seed=9, amp=1e-4)
        for b in data:
            b[19:22] += 0.05   # shift of both signs after perturbation
            b[19] -= 0.08
    return mesh, zi.params_default(order), data


def gpu_rhs(mesh, p, data, precision=0):
    pk = z().Pack(mesh, p, precision)
    pk.upload(z().REG_U, data)
    pk.fill_ghosts(z().REG_U)
    r = pk.rhs(z().REG_U)
    torch.cuda.synchronize()
    return pk, pk.split_interior(r)


def ora_rhs(mesh, p, data):
    om = oracle.OracleMesh(mesh)
    return oracle.rhs(om, p, om.scatter(data))


def test_flat_space_rhs_is_exactly_zero():
    mesh = zi.uniform_mesh((2, 1, 1), 16, 4, (0, 0, 0), (2, 1, 1), zi.BC_OUTFLOW)
    _, r = gpu_rhs(mesh, zi.params_default(6), zi.flat(mesh))
    for b in r:
        assert np.all(b == 0.0)


def test_ghost_fill_bitwise_equal():
    for bc in (zi.BC_PERIODIC, zi.BC_OUTFLOW):
        mesh = zi.uniform_mesh((2, 3, 2), 8, 4, (0, 0, 0), (2, 3, 2), bc)
        rng = np.random.default_rng(1)
        data = [rng.standard_normal((22, 8, 8, 8)) for _ in range(mesh.nb)]
        pk = z().Pack(mesh, zi.params_default(6))
        pk.upload(z().REG_U, data)
        pk.fill_ghosts(z().REG_U)
        got = pk.download(z().REG_U, ghosted=True)
        om = oracle.OracleMesh(mesh)
        u = om.scatter(data)
        oracle.fill_ghosts(om, u)
        for b in range(mesh.nb):
            np.testing.assert_array_equal(got[b], om.block_view(u, b))


def test_rhs_parity_periodic16():
    """The 16^3 periodic block, 4th order, seeded sinusoids (one RK4 step)."""
    mesh, p, data, dt, _ = zi.workload("periodic16")
    _, rg = gpu_rhs(mesh, p, data)
    assert_parity(rg, ora_rhs(mesh, p, data), what="rhs periodic16")


@pytest.mark.parametrize("order", [4, 6, 8])
def test_rhs_parity_multiblock_outflow(order):
    mesh, p, data = small_bl(order)
    _, rg = gpu_rhs(mesh, p, data)
    assert_parity(rg, ora_rhs(mesh, p, data), what=f"rhs order {order}")


@pytest.mark.parametrize("terms", [1, 2, 4, 8, 5, 15])
def test_rhs_parity_term_masks(terms):
    mesh, p, data = small_bl(6)
    p["terms"] = terms
    _, rg = gpu_rhs(mesh, p, data)
    assert_parity(rg, ora_rhs(mesh, p, data), what=f"terms {terms}")


def test_rk4_stages_parity_periodic16():
    """Each stage's output register and the FP64 accumulator, stage by stage
    (evolved-state bar: the oracle runs the same stages from inputs moved by
    one ulp beside it for the per-field rounding floor)."""
    mesh, p, data, dt, _ = zi.workload("periodic16")
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    om = oracle.OracleMesh(mesh)
    regs = oracle.Registers(om, data)
    alt = oracle.Registers(om, ulp_perturbed(data))
    for stage in (1, 2, 3, 4):
        pk.rk4_stage(stage, dt)
        oracle.rk4_stage(regs, p, stage, dt)
        oracle.rk4_stage(alt, p, stage, dt)
        torch.cuda.synchronize()
        reg = {1: 1, 2: 2, 3: 1, 4: 0}[stage]
        name = {0: "U", 1: "S1", 2: "S2"}[reg]
        ora, oalt = om.interiors(getattr(regs, name)), om.interiors(getattr(alt, name))
        floor = K_ROUND * field_errors(oalt, ora)[1]
        assert_parity(pk.download(reg), ora, what=f"stage {stage}", floor=floor)
        if stage < 4:
            acc = pk.split_interior(pk.acc_view())
            oa, oaa = om.interiors(regs.A), om.interiors(alt.A)
            assert_parity(acc, oa, what=f"accumulator stage {stage}",
                          floor=K_ROUND * field_errors(oaa, oa)[1])


def test_rk4_steps_parity_bl():
    """Two full RK4 steps of a Brill-Lindquist pack, 6th order, outflow."""
    mesh = zi.uniform_mesh((2, 2, 2), 16, 4, (-8.0,) * 3, (8.0,) * 3, zi.BC_OUTFLOW)
    data = zi.brill_lindquist(mesh, [(1.0, (0.0, 0.0, 0.0))])
    p = zi.params_default(6)
    dt = 0.25 * mesh.dx0
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    pk.rk4_step(dt, 2)
    want, floor = oracle_steps(mesh, p, data, dt, 2)
    torch.cuda.synchronize()
    assert_parity(pk.download(0), want, what="2 steps BL", floor=floor)


@pytest.mark.parametrize("order,g", [(6, 5), (4, 4)])
def test_rk4_step_parity_odd_ghost_offset(order, g):
    """Ghost depths that differ from the staged halo (order/2 + 1) by an odd
    count, so that FP64 tiles go to LDS in 4-byte halves (a kernel of its
    own): one RK4 step in every tile shape and launch mode, bitwise equal
    across them and at the evolved-state bar against the oracle."""
    mesh = zi.uniform_mesh((2, 2, 2), 16, g, (-8.0,) * 3, (8.0,) * 3, zi.BC_OUTFLOW)
    data = zi.add_perturbation(mesh, zi.brill_lindquist(mesh, [(1.0, (0.3, 0.0, 0.0))]),
                               seed=5, amp=1e-4)
    p = zi.params_default(order)
    dt = 0.25 * mesh.dx0
    want, floor = oracle_steps(mesh, p, data, dt, 1)
    first = None
    for v in range(len(z().TILE_SHAPES)):
        for pers in (False, True):
            pk = z().Pack(mesh, p)
            pk.upload(z().REG_U, data)
            pk.set_variant(v, pers)
            pk.rk4_step(dt, 1)
            torch.cuda.synchronize()
            got = pk.download(0)
            if first is None:
                first = got
                assert_parity(got, want, what=f"order {order} g {g}", floor=floor)
            else:
                for a, b in zip(got, first):
                    np.testing.assert_array_equal(a, b)


def test_constraints_parity():
    mesh, p, data = small_bl(6)
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    cz, norms = pk.constraints(z().REG_U, exclude=[(0.0, 0.0, 0.0)], r_exc=1.0)
    om = oracle.OracleMesh(mesh)
    co, no = oracle.constraints(om, p, om.scatter(data), exclude=[(0.0, 0.0, 0.0)], r_exc=1.0)
    assert_parity(pk.split_interior(cz, 8), co, what="constraints")
    np.testing.assert_allclose(norms, no, rtol=1e-12, atol=0)


@pytest.mark.parametrize("crit", [0, 1, 2])
def test_refine_flags_exact(crit):
    mesh = zi.uniform_mesh((4, 4, 4), 8, 4, (-8,) * 3, (8,) * 3, zi.BC_OUTFLOW)
    data = zi.brill_lindquist(mesh, [(1.0, (0.5, 0.0, 0.0))])
    p = zi.params_default(6)
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    kw = dict(chi_thr=0.3, dchi_thr=0.05, level_max=5, radius=3.0, centre=(0.0, 0.0, 0.0),
              radius_level=1)
    fg = pk.refine_flags(z().REG_U, crit, **kw)
    om = oracle.OracleMesh(mesh)
    fo = oracle.refine_flags(om, p, om.scatter(data), crit, **kw)
    np.testing.assert_array_equal(fg, fo)
    assert (fg != 0).any()


def test_bl64x32_full_size_rhs_parity():
    """The 64 x 32^3 Brill-Lindquist pack at full size (the benchmarked
    configuration): RHS of the initial data against the oracle."""
    mesh, p, data, dt, _ = zi.workload("bl64x32")
    _, rg = gpu_rhs(mesh, p, data)
    assert_parity(rg, ora_rhs(mesh, p, data), what="rhs bl64x32")


def test_bl64x32_full_size_step_in_bench_launch_configuration():
    """One RK4 step of the full 64 x 32^3 pack exactly as the benchmark runs
    it (tile shape and launch mode from the autotuner, same dt) against one
    oracle step of the whole mesh: every zone of every field."""
    mesh, p, data, dt, _ = zi.workload("bl64x32")
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    chosen, _ = pk.autotune(reps=1)
    pk.rk4_step(dt, 1)
    torch.cuda.synchronize()
    got = pk.download(z().REG_U)
    want, floor = oracle_steps(mesh, p, data, dt, 1)
    assert_parity(got, want, what=f"step bl64x32 (variant {chosen})", floor=floor)


@pytest.mark.parametrize("n", [64, 128])
def test_large_block_parity(n):
    """One periodic block of 64^3 (Table 1's MeshBlock size) or 128^3
    holding the linear wave plus perturbations of every field: RHS against
    the oracle, and for 64^3 one RK4 step in the autotuner's launch."""
    mesh, data = zi.linear_wave_pack(1, n)
    data = zi.add_perturbation(mesh, data, seed=6, amp=1e-6, periodic_box=1.0)
    p = zi.params_default(6)
    _, rg = gpu_rhs(mesh, p, data)
    assert_parity(rg, ora_rhs(mesh, p, data), what=f"rhs {n}^3")
    if n == 64:
        dt = 0.25 * mesh.dx0
        pk = z().Pack(mesh, p)
        pk.upload(z().REG_U, data)
        chosen, _ = pk.autotune(reps=1)
        pk.rk4_step(dt, 1)
        torch.cuda.synchronize()
        want, floor = oracle_steps(mesh, p, data, dt, 1)
        assert_parity(pk.download(z().REG_U), want, what=f"step 64^3 (variant {chosen})", floor=floor)


# tile counts that are not a multiple of 8 (the XCD-interleaved slot map has
# a short last slice): one 24^3 block = 54 tiles, 3x3x1 blocks of 8^3 = 18
RAGGED = {"one24": ((1, 1, 1), 24, (6.0, 6.0, 6.0)), "three_by_three8": ((3, 3, 1), 8, (6.0, 6.0, 2.0))}


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("shape", sorted(RAGGED))
def test_ragged_tile_count_parity(shape, persistent):
    nblk, n, half = RAGGED[shape]
    mesh = zi.uniform_mesh(nblk, n, 4, tuple(-x for x in half), half, zi.BC_OUTFLOW)
    data = zi.brill_lindquist(mesh, [(1.0, (0.0, 0.0, 0.0))])
    data = zi.add_perturbation(mesh, data, seed=5, amp=1e-4)
    p = zi.params_default(6)
    pk = z().Pack(mesh, p)
    assert pk.nwork % 8 != 0 and pk.nwork > 8
    pk.set_variant(0, persistent)
    pk.upload(z().REG_U, data)
    pk.fill_ghosts(z().REG_U)
    rg = pk.split_interior(pk.rhs(z().REG_U))
    torch.cuda.synchronize()
    assert_parity(rg, ora_rhs(mesh, p, data), what=f"rhs {shape}")
    dt = 0.25 * mesh.dx0
    pk.upload(z().REG_U, data)
    pk.rk4_step(dt, 1)
    want, floor = oracle_steps(mesh, p, data, dt, 1)
    torch.cuda.synchronize()
    assert_parity(pk.download(0), want, what=f"step {shape}", floor=floor)


@pytest.mark.parametrize("graph", [False, True])
def test_check_finite_flag(graph):
    """Z4C_FLAG_CHECK_FINITE: a NaN in one active cell of the input makes
    z4c_rk4_step return Z4C_ENONFINITE; finite data passes, and without the
    flag the same NaN goes unreported."""
    mesh, p, data = small_bl(6)
    dt = 0.25 * mesh.dx0
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pk = z().Pack(mesh, dict(p, check_finite=1, graph=int(graph)))
        pk.upload(z().REG_U, data)
        pk.rk4_step(dt, 2, stream=s)
        bad = [b.copy() for b in data]
        bad[3][7, 2, 5, 1] = np.nan
        pk.upload(z().REG_U, bad)
        with pytest.raises(z().Z4cError) as err:
            pk.rk4_step(dt, 1, stream=s)
        assert err.value.code == -5
        quiet = z().Pack(mesh, p)
        quiet.upload(z().REG_U, bad)
        quiet.rk4_step(dt, 1, stream=s)
        torch.cuda.synchronize()
        assert not np.isfinite(quiet.download(z().REG_U)[3]).all()


def floored_bl():
    """Brill-Lindquist M = 1 on [-2, 2]^3 at dx = 1/8 with chi_floor = 1e-2
    and alpha_floor = 5e-2: next to the puncture chi = psi^-4 ~ 1e-3 and
    alpha = psi^-2 ~ 3e-2, so both floors act at every stage write and chi is
    floored wherever it divides."""
    mesh = zi.uniform_mesh((2, 2, 2), 16, 4, (-2.0,) * 3, (2.0,) * 3, zi.BC_OUTFLOW)
    data = zi.brill_lindquist(mesh, [(1.0, (0.0, 0.0, 0.0))])
    p = dict(zi.params_default(6), chi_floor=1e-2, alpha_floor=5e-2)
    return mesh, p, data, 0.25 * mesh.dx0


def test_floors_active_step_parity_fp64():
    """R8 floors in action (moving-puncture data, Sec. 2): two RK4 steps with
    both floors active against the oracle; the floored cells are the same and
    hold the floor values exactly."""
    mesh, p, data, dt = floored_bl()
    assert min(d[0].min() for d in data) < p["chi_floor"]
    assert min(d[18].min() for d in data) < p["alpha_floor"]
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    pk.rk4_step(dt, 2)
    torch.cuda.synchronize()
    got = pk.download(z().REG_U)
    want, floor = oracle_steps(mesh, p, data, dt, 2)
    nchi = sum(int((w[0] == p["chi_floor"]).sum()) for w in want)
    nal = sum(int((w[18] == p["alpha_floor"]).sum()) for w in want)
    assert nchi > 0 and nal > 0, (nchi, nal)
    for g_, w_ in zip(got, want):
        assert np.array_equal(g_[0] == p["chi_floor"], w_[0] == p["chi_floor"])
        assert np.array_equal(g_[18] == p["alpha_floor"], w_[18] == p["alpha_floor"])
    assert_parity(got, want, what="floored step", floor=floor)
