"""Ghost cells the stage kernel writes itself: the x-face ghosts of the
same-level neighbours (FP32 storage, odd FP64 ghost depths) and the ghost
columns beyond outflow x faces (the nearest active cell, Sec. 3.1's boundary
fill), which the next stage's fill then leaves alone.  Within one multi-step
call, a step's first stage also takes them from the previous step's last
stage.  Checked here: every step count per call gives bitwise the same
state, and the written ghost columns equal what a full fill writes."""
import numpy as np
import pytest

import z4c_inputs as zi
from _parity import assert_parity, oracle_steps

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def z():
    import paper_2409_10383_amd as m
    return m


def mesh_of(kind, g, bc=zi.BC_OUTFLOW):
    base = zi.uniform_mesh((4, 4, 4), 8, g, (-8.0,) * 3, (8.0,) * 3, bc)
    if kind == "uniform":
        return base
    if kind == "central":      # refined box away from the domain faces
        return zi.refine_blocks(base, zi.blocks_in_box(base, (-4.0,) * 3, (4.0,) * 3))
    # refined box on the low x face: x-face blocks with a finer neighbour
    # across y or z, and refined x-face blocks among themselves
    return zi.refine_blocks(base, zi.blocks_in_box(base, (-8.0, -4.0, -4.0), (-4.0, 0.0, 4.0)))


def data_of(mesh):
    data = zi.brill_lindquist(mesh, [(1.0, (0.4, -0.3, 0.2))])
    return zi.add_perturbation(mesh, data, seed=13, amp=1e-4)


CASES = [  # (mesh, precision, order, ghosts)
    ("uniform", 0, 6, 4),     # every direction read in place
    ("uniform", 0, 8, 5),     # odd ghost depth: x-face ghosts pushed
    ("uniform", 1, 6, 4),     # FP32 storage: x-face ghosts pushed
    ("uniform", 1, 8, 5),
    ("central", 0, 6, 4),
    ("xface", 0, 8, 5),
    ("xface", 1, 6, 4),
    ("xface", 0, 6, 4),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{m}-{'fp32' if p else 'fp64'}-o{o}-g{g}" for m, p, o, g in CASES])
def test_steps_in_one_call_equal_steps_in_separate_calls(case):
    kind, prec, order, g = case
    mesh = mesh_of(kind, g)
    data = data_of(mesh)
    p = zi.params_default(order)
    dt = 0.25 * mesh.dx_min()
    outs = []
    for split in (False, True):
        pk = z().Pack(mesh, p, prec)
        pk.upload(z().REG_U, data)
        if split:
            for _ in range(3):
                pk.rk4_step(dt, 1)
        else:
            pk.rk4_step(dt, 3)
        torch.cuda.synchronize()
        outs.append(pk.download(0))
        del pk
    for b, (a1, a2) in enumerate(zip(*outs)):
        assert np.all(np.isfinite(a1)), f"block {b}"
        np.testing.assert_array_equal(a1, a2, err_msg=f"block {b}")


@pytest.mark.parametrize("prec,order,g", [(0, 6, 4), (0, 8, 5), (1, 6, 4)])
def test_outflow_x_face_ghosts_written_by_the_last_stage(prec, order, g):
    """After a step, the ghost columns beyond the outflow x faces of U hold
    what a full fill writes: the last stage wrote them.  Edges and corners
    included where x directions are read in place (FP64, even ghost depth);
    with the x halos read from the block's own ghosts (FP32 storage, odd
    ghost depth) a staged cell beyond a y or z face takes its x ghosts from
    the block across that face or from the clamped row, so only the block's
    own rows are read and written."""
    mesh = mesh_of("uniform", g)
    pk = z().Pack(mesh, zi.params_default(order), prec)
    pk.upload(z().REG_U, data_of(mesh))
    pk.rk4_step(0.25 * mesh.dx0, 2)
    torch.cuda.synchronize()
    before = pk.download(0, ghosted=True)
    pk.fill_ghosts(z().REG_U)
    torch.cuda.synchronize()
    after = pk.download(0, ghosted=True)
    nface = 0
    for b in range(mesh.nb):
        n = int(mesh.n[b])
        ilo = int(mesh.ilo[b, 0])
        nx = int(mesh.nroot[0]) << int(mesh.level[b])
        cols = []
        if ilo == 0:
            cols.append(slice(0, g))
        if ilo + n == nx:
            cols.append(slice(n + g, n + 2 * g))
        rows = slice(None) if (prec == 0 and g % 2 == 0) else slice(g, g + n)
        for c in cols:
            nface += 1
            np.testing.assert_array_equal(before[b][:, rows, rows, c], after[b][:, rows, rows, c],
                                          err_msg=f"block {b}")
    assert nface == 32


@pytest.mark.parametrize("case", [("xface", 0, 8, 5), ("uniform", 1, 6, 4), ("uniform", 0, 6, 4)],
                         ids=["xface-fp64-o8-g5", "uniform-fp32-o6-g4", "uniform-fp64-o6-g4"])
def test_graph_replayed_steps_equal_eager_steps(case):
    """Graph-replayed steps: a call's first step replays the captured step
    whose stage 1 fills every ghost, later steps the one whose stage 1 finds
    the ghosts of U the previous step's stage 4 wrote.  Two calls (3 + 2
    steps, the second without capturing) equal five eager steps bitwise."""
    kind, prec, order, g = case
    mesh = mesh_of(kind, g)
    data = data_of(mesh)
    p = zi.params_default(order)
    dt = 0.25 * mesh.dx_min()
    eager = z().Pack(mesh, p, prec)
    eager.upload(z().REG_U, data)
    eager.rk4_step(dt, 5)
    torch.cuda.synchronize()
    want = eager.download(0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        graph = z().Pack(mesh, dict(p, graph=1), prec)
        graph.upload(z().REG_U, data)
        torch.cuda.synchronize()
        graph.rk4_step(dt, 3, stream=s)
        graph.rk4_step(dt, 2, stream=s)
        s.synchronize()
        got = graph.download(0)
    for b, (a1, a2) in enumerate(zip(got, want)):
        np.testing.assert_array_equal(a1, a2, err_msg=f"block {b}")


@pytest.mark.parametrize("kind,order,g,bc", [("xface", 8, 5, zi.BC_OUTFLOW), ("xface", 6, 4, zi.BC_OUTFLOW),
                                             ("central", 8, 5, zi.BC_PERIODIC), ("central", 6, 4, zi.BC_PERIODIC)],
                         ids=["xface-o8-g5", "xface-o6-g4", "central-periodic-o8-g5", "central-periodic-o6-g4"])
def test_multilevel_steps_against_the_oracle(kind, order, g, bc):
    """Two steps in one call on two-level packs (refinement touching an
    outflow x face, or periodic), x halos read in place (even ghost depth) or
    from the block's own ghosts (odd): the stage path's fill leaves out what
    the stage kernel reads in place, never reads or wrote itself, and the
    state still matches the oracle's two steps at the evolved-state bar."""
    mesh = mesh_of(kind, g, bc)
    data = data_of(mesh)
    p = zi.params_default(order)
    dt = 0.25 * mesh.dx_min()
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    pk.rk4_step(dt, 2)
    want, floor = oracle_steps(mesh, p, data, dt, 2)
    torch.cuda.synchronize()
    assert_parity(pk.download(0), want, what=f"{kind} order {order}", floor=floor)
