"""GPU parity on multi-level packs: the cross-level Lagrange ghost fill
(restriction / prolongation, Sec. 3.1) and the RHS / RK4 across
refinement boundaries, against the oracle."""
import numpy as np
import pytest

import oracle
import z4c_inputs as zi
from _parity import assert_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def z():
    import paper_2409_10383_amd as m
    return m


def two_level(n=8, g=4, bc=zi.BC_OUTFLOW):
    base = zi.uniform_mesh((4, 4, 4), n, g, (0.0,) * 3, (32.0,) * 3, bc)
    return zi.refine_blocks(base, zi.blocks_in_box(base, (8.0,) * 3, (24.0,) * 3))


def smooth_data(mesh, seed=3):
    from z4c_inputs import analytic as an
    fn = an.kerr_schild(1.0, centre=(16.3, 15.8, 16.1))
    data = [an.adm_to_z4c(fn, 0.0, *mesh.grid(b)) for b in range(mesh.nb)]
    return zi.add_perturbation(mesh, data, seed=seed, amp=1e-4)


@pytest.mark.parametrize("order", [6, 8])
@pytest.mark.parametrize("bc", [zi.BC_OUTFLOW, zi.BC_PERIODIC])
def test_cross_level_ghost_fill(order, bc):
    g = order // 2 + 1
    mesh = two_level(8, g, bc)
    data = smooth_data(mesh)
    pk = z().Pack(mesh, zi.params_default(order))
    pk.upload(z().REG_U, data)
    pk.fill_ghosts(z().REG_U)
    got = pk.download(z().REG_U, ghosted=True)
    om = oracle.OracleMesh(mesh)
    u = om.scatter(data)
    oracle.fill_ghosts(om, u)
    want = [om.block_view(u, b) for b in range(mesh.nb)]
    assert_parity(got, want, what=f"ghosts order {order} bc {bc}")


@pytest.mark.parametrize("order", [6, 8])
def test_cross_level_rhs_and_step(order):
    g = order // 2 + 1
    mesh = two_level(8, g)
    data = smooth_data(mesh)
    p = zi.params_default(order)
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    pk.fill_ghosts(z().REG_U)
    rg = pk.split_interior(pk.rhs(z().REG_U))
    om = oracle.OracleMesh(mesh)
    ro = oracle.rhs(om, p, om.scatter(data))
    assert_parity(rg, ro, what="rhs")
    dt = 0.25 * mesh.dx_min()
    pk.rk4_step(dt, 1)
    regs = oracle.Registers(om, data)
    oracle.rk4_steps(regs, p, dt, 1)
    torch.cuda.synchronize()
    assert_parity(pk.download(z().REG_U), om.interiors(regs.U), what="step", mode="state")


def test_bbh512mixed_full_size():
    """The 512-block, 4-level, 16^3/32^3 two-puncture pack at full size
    (8th order, 5 ghosts): every ghost cell against the oracle, and the RHS
    on a sample of blocks at every level and size."""
    mesh, p, data, dt, _ = zi.workload("bbh512mixed")
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    pk.fill_ghosts(z().REG_U)
    rg = pk.split_interior(pk.rhs(z().REG_U))
    got = pk.download(z().REG_U, ghosted=True)
    om = oracle.OracleMesh(mesh)
    u = om.scatter(data)
    oracle.fill_ghosts(om, u)
    want = [om.block_view(u, b) for b in range(mesh.nb)]
    assert_parity(got, want, what="ghosts bbh512mixed")
    rng = np.random.default_rng(0)
    sample = []
    for lev in range(4):
        for n in (16, 32):
            cand = np.where((mesh.level == lev) & (mesh.n == n))[0]
            if cand.size:
                sample += list(rng.choice(cand, size=min(3, cand.size), replace=False))
    # include the blocks holding the punctures, where the RHS is largest
    for xp in (5.0, -5.0):
        for b in range(mesh.nb):
            hb = mesh.dx(b)
            x0 = [mesh.lo[a] + mesh.ilo[b, a] * hb for a in range(3)]
            if all(x0[a] <= (xp, 0.0, 0.0)[a] <= x0[a] + mesh.n[b] * hb for a in range(3)):
                sample.append(b)
    sample = sorted(set(int(b) for b in sample))
    ro = oracle.rhs(om, p, u, fill=False, blocks=sample)
    S = max(np.abs(data[b][[0, 1, 4, 6, 18]]).max() for b in sample)
    hmin = mesh.dx_min()
    assert_parity([rg[b] for b in sample], [ro[b] for b in sample], what="rhs bbh512mixed sample",
                  mode="rounding", S=S, order=8, h=hmin)


def test_fill_is_ordered_on_the_callers_stream():
    """Multi-level fills run their same-level copies on the pack's side stream
    and join back: work enqueued on the caller's stream right after the fill
    sees every ghost (the ghosts are NaN before each fill)."""
    mesh = two_level(8, 4)
    data = smooth_data(mesh)
    pk = z().Pack(mesh, zi.params_default(6))
    pk.upload(z().REG_U, data)
    pk.fill_ghosts(z().REG_U)
    torch.cuda.synchronize()
    ref = pk.state_view(z().REG_U).cpu().numpy()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(4):
            pk.upload(z().REG_U, data)           # interiors, NaN ghosts
            pk.fill_ghosts(z().REG_U, stream=s)
            snap = pk.state_view(z().REG_U).clone()
            s.synchronize()
            # slab padding stays NaN in both: NaN-aware bitwise comparison
            assert np.array_equal(snap.cpu().numpy(), ref, equal_nan=True), f"fill {rep}"
