"""GPU regrid (z4c_regrid_transfer) against the reference transfer on the
same inputs, and one adaptive cycle (flags on the GPU, plan, transfer,
RK4 step on the new pack) against the oracle doing the same steps."""
import numpy as np
import pytest

import oracle
import z4c_inputs as zi
from _parity import assert_parity, oracle_steps
from oracle import regrid as rg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def z():
    import paper_2409_10383_amd as m
    return m


def two_level(order, bc):
    g = order // 2 + 1
    m0 = zi.uniform_mesh((2, 2, 2), 8, g, (-4.0,) * 3, (4.0,) * 3, bc)
    return zi.refine_blocks(zi.refine_blocks(m0, range(8)), [7])   # levels 1 and 2


def data_for(mesh, seed):
    if mesh.bc == zi.BC_PERIODIC:
        return zi.add_perturbation(mesh, zi.flat(mesh), seed=seed, amp=1e-3, periodic_box=8.0)
    d = zi.brill_lindquist(mesh, [(0.5, (-1.0, 0.0, 0.0)), (0.5, (1.0, 0.0, 0.0))])
    return zi.add_perturbation(mesh, d, seed=seed, amp=1e-4)


CASES = [("spread-outflow", 6, zi.BC_OUTFLOW, "spread"), ("merge-periodic", 8, zi.BC_PERIODIC, "merge"),
         ("mixed-outflow", 4, zi.BC_OUTFLOW, "mixed")]


def flags_for(mesh, kind):
    f = np.zeros(mesh.nb, np.int8)
    if kind == "spread":
        f[7] = 1                     # a level-2 block at the corner of the level-2 region
    elif kind == "merge":
        f[:] = -1
    else:
        f[15:23] = -1                # a mergeable level-1 group ...
        f[40] = 1                    # ... and a refinement elsewhere
    return f


@pytest.mark.parametrize("name,order,bc,kind", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [0, 1])
def test_transfer_parity(name, order, bc, kind, precision):
    mesh = two_level(order, bc)
    data = data_for(mesh, 3)
    flags = flags_for(mesh, kind)
    pk = z().Pack(mesh, zi.params_default(order), precision)
    pk.upload(z().REG_U, data)
    new = pk.regrid(flags, 3)
    torch.cuda.synchronize()
    want_mesh = rg.plan(mesh, flags, 3)
    assert np.array_equal(new.mesh.ilo, want_mesh.ilo) and np.array_equal(new.mesh.level, want_mesh.level)
    got = new.download(z().REG_U)
    om = oracle.OracleMesh(mesh)
    src = om.scatter(data)
    if precision:
        # the FP32 pack holds float-rounded data: the reference starts from it
        src = om.scatter([np.asarray(b, np.float32).astype(np.float64) for b in data])
    want = rg.transfer(mesh, src, want_mesh)
    if precision == 0:
        assert_parity(got, want, what=f"regrid {name}")
    else:
        for b in range(len(want)):
            scale = np.max(np.abs(want[b]), axis=(1, 2, 3), keepdims=True) + 1e-300
            assert np.max(np.abs(got[b] - want[b]) / scale) < 4e-6, (name, b)


def test_adaptive_cycle_matches_oracle():
    """chi-min flags -> plan -> transfer -> one RK4 step, GPU vs oracle."""
    order = 6
    mesh = two_level(order, zi.BC_OUTFLOW)
    data = zi.brill_lindquist(mesh, [(0.5, (-1.0, 0.0, 0.0)), (0.5, (1.0, 0.0, 0.0))])
    p = zi.params_default(order)
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    flags = pk.refine_flags(z().REG_U, z().CRIT_CHI_MIN, chi_thr=0.45, level_max=3)
    om = oracle.OracleMesh(mesh)
    u = om.scatter(data)
    oflags = oracle.refine_flags(om, p, u.copy(), 0, chi_thr=0.45, level_max=3)
    assert np.array_equal(flags, oflags)
    assert flags.max() == 1
    new = pk.regrid(flags, 3)
    dt = 0.25 * new.mesh.dx_min()
    new.rk4_step(dt, 1)
    torch.cuda.synchronize()
    omesh = rg.plan(mesh, oflags, 3)
    odata = rg.transfer(mesh, u, omesh)
    want, floor = oracle_steps(omesh, p, odata, dt, 1)
    assert_parity(new.download(z().REG_U), want, what="adaptive cycle", floor=floor)
