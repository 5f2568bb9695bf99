"""GPU wave extraction and puncture tracking against the reference:
z4c_psi4 (FP64 on a two-level mesh, FP32 storage on one level), z4c_interp
and z4c_interp_state at random points, z4c_swsh_project, the RK4 tracker on
perturbed two-puncture data and in flat space with a uniform shift (exact
RK4 polynomial, eager and graph replay), and the sphere chain
(interpolate -> project) on a synthetic mode field."""
import math

import numpy as np
import pytest

import oracle
import z4c_inputs as zi
from _parity import assert_parity, oracle_steps
from oracle import extract as ex

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def z():
    import paper_2409_10383_amd as m
    return m


def bbh(levels=2, n=8, order=6):
    g = order // 2 + 1
    m = zi.uniform_mesh((2, 2, 2), n, g, (-4.0,) * 3, (4.0,) * 3, zi.BC_OUTFLOW)
    if levels > 1:
        m = zi.refine_blocks(m, [0, 7])
    d = zi.brill_lindquist(m, [(0.5, (-1.1, 0.13, 0.07)), (0.5, (1.2, -0.1, 0.05))])
    return m, zi.add_perturbation(m, d, seed=4, amp=1e-4)


ORIGIN = (0.11, -0.07, 0.05)


@pytest.mark.parametrize("precision,levels", [(0, 2), (1, 1)])
def test_psi4_parity(precision, levels):
    mesh, data = bbh(levels)
    if precision:
        data = [np.asarray(b, np.float32).astype(np.float64) for b in data]
    p = zi.params_default(6)
    pk = z().Pack(mesh, p, precision)
    pk.upload(z().REG_U, data)
    got = pk.split_interior(pk.psi4(z().REG_U, ORIGIN), 2)
    om = oracle.OracleMesh(mesh)
    want = oracle.psi4(om, p, om.scatter(data), ORIGIN)
    assert_parity(got, want, what=f"psi4 prec {precision}")


def test_interp_parity():
    mesh, data = bbh(2)
    p = zi.params_default(6)
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    ps = pk.psi4(z().REG_U, ORIGIN)
    rng = np.random.default_rng(2)
    pts = rng.uniform(-3.9, 3.9, size=(500, 3))
    got = pk.interp(ps, 2, pts)
    om = oracle.OracleMesh(mesh)
    want = ex.interpolate(mesh, pk.split_interior(ps, 2), pts)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    gb = pk.interp_state(z().REG_U, 19, 3, pts)
    wb = ex.interpolate(mesh, [b[19:22] for b in data], pts)
    assert np.max(np.abs(gb - wb)) <= 1e-12 * np.max(np.abs(wb))
    assert np.all(np.isnan(pk.interp_state(z().REG_U, 0, 1, [[9.0, 0.0, 0.0]])))


def test_swsh_projection_parity():
    P, w = zi.geodesic_sphere(4, 2.5, ORIGIN)
    rng = np.random.default_rng(9)
    vals = rng.standard_normal(len(P)) + 1j * rng.standard_normal(len(P))
    got = z().swsh_project(vals, P, w, ORIGIN, 8)
    want = ex.project(vals, P, w, ORIGIN, 8)
    scale = max(abs(v) for v in want.values())
    for key, v in want.items():
        assert abs(got[key] - v) <= 1e-12 * scale, key


def test_sphere_chain_recovers_modes():
    """Zone values f(r) sum a_lm -2Y_lm on a mesh -> interpolation onto a
    geodesic sphere -> projection: the GPU chain equals the reference chain
    and recovers f(R) a_lm to interpolation accuracy."""
    mesh = zi.uniform_mesh((4, 4, 4), 16, 4, (-4.0,) * 3, (4.0,) * 3, zi.BC_OUTFLOW)
    rng = np.random.default_rng(5)
    coef = {(l, m): complex(*rng.standard_normal(2)) for l in range(2, 4) for m in range(-l, l + 1)}
    inter = []
    for b in range(mesh.nb):
        X, Y, Z = mesh.grid(b)
        th, ph = ex.angles(np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1), ORIGIN)
        r = np.sqrt((X - ORIGIN[0]) ** 2 + (Y - ORIGIN[1]) ** 2 + (Z - ORIGIN[2]) ** 2).ravel()
        v = sum(c * ex.swsh(-2, l, m, th, ph) for (l, m), c in coef.items()) * np.exp(-0.1 * r)
        inter.append(np.stack([v.real, v.imag]).reshape(2, 16, 16, 16))
    flat = torch.as_tensor(np.concatenate([a.reshape(-1) for a in inter]), device="cuda")
    pk = z().Pack(mesh, zi.params_default(6))
    R = 2.7
    P, w = zi.geodesic_sphere(4, R, ORIGIN)
    vals = pk.interp(flat, 2, P)
    wv = ex.interpolate(mesh, inter, P)
    assert np.max(np.abs(vals - wv)) <= 1e-12 * np.max(np.abs(wv))
    got = z().swsh_project(vals[:, 0] + 1j * vals[:, 1], P, w, ORIGIN, 4)
    for (l, m), c in coef.items():
        assert abs(got[(l, m)] - c * math.exp(-0.1 * R)) < 2e-3 * abs(c) + 1e-3, (l, m)


def test_tracker_parity_two_punctures():
    mesh, data = bbh(2)
    for blk in data:                                 # a nonzero shift to follow
        blk[19] += 0.05
        blk[20] -= 0.03
    p = zi.params_default(6)
    dt = 0.25 * mesh.dx(1)
    x0 = np.array([[-1.1, 0.13, 0.07], [1.2, -0.1, 0.05]])
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    pk.tracker_set(x0)
    pk.rk4_step(dt, 3)
    got = pk.tracker_get()
    om = oracle.OracleMesh(mesh)
    regs = oracle.Registers(om, data)
    x = x0.copy()
    for _ in range(3):
        x = ex.rk4_step_with_tracker(regs, p, dt, x)
    assert np.max(np.abs(got - x)) <= 1e-12 * np.max(np.abs(x)), (got, x)
    want, floor = oracle_steps(mesh, p, data, dt, 3)
    assert np.array_equal(np.concatenate([a.ravel() for a in want]),
                          np.concatenate([a.ravel() for a in om.interiors(regs.U)]))
    assert_parity(pk.download(0), want, what="state with tracker", floor=floor)


@pytest.mark.parametrize("graph", [False, True])
def test_tracker_uniform_shift_is_exact_rk4(graph):
    mesh = zi.uniform_mesh((2, 2, 2), 8, 4, (0.0,) * 3, (2.0,) * 3, zi.BC_PERIODIC)
    p = zi.params_default(6, eta=2.0)
    beta0 = np.array([0.3, -0.2, 0.1])
    data = zi.flat(mesh)
    for blk in data:
        for a in range(3):
            blk[19 + a] = beta0[a]
    x0 = np.array([[0.7, 1.1, 0.9], [1.5, 0.4, 1.2]])
    dt, nsteps = 0.05, 6
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pk = z().Pack(mesh, dict(p, graph=1) if graph else p)
        pk.upload(z().REG_U, data)
        pk.tracker_set(x0, stream=s)
        pk.rk4_step(dt, nsteps, stream=s)
        x = pk.tracker_get(stream=s)
    A = np.array([[-p["eta"], 0.0], [-1.0, 0.0]]) * dt
    Rn = np.linalg.matrix_power(np.eye(2) + A + A @ A / 2 + A @ A @ A / 6 + A @ A @ A @ A / 24, nsteps)
    for q in range(2):
        for a in range(3):
            assert abs(x[q, a] - (Rn @ np.array([beta0[a], x0[q, a]]))[1]) < 1e-14


def test_empty_and_invalid_point_sets():
    """Zero points: interpolation returns an empty result without a launch;
    trackers: n = 0 stops tracking (a step still runs), more than
    Z4C_MAXTRACK or a harmonic degree above 12 is rejected."""
    mesh, data = bbh(1)
    p = zi.params_default(6)
    pk = z().Pack(mesh, p)
    pk.upload(z().REG_U, data)
    ps = pk.psi4(z().REG_U, ORIGIN)
    assert pk.interp(ps, 2, np.zeros((0, 3))).shape == (0, 2)
    assert pk.interp_state(z().REG_U, 0, 3, np.zeros((0, 3))).shape == (0, 3)
    pk.tracker_set(np.array([[0.5, 0.5, 0.5]]))
    pk.tracker_set(np.zeros((0, 3)))
    pk.rk4_step(0.1 * mesh.dx0, 1)
    assert pk.tracker_get().shape == (0, 3)
    with pytest.raises(z().Z4cError):
        pk.tracker_set(np.zeros((9, 3)))
    P, w = zi.geodesic_sphere(2, 2.0, ORIGIN)
    with pytest.raises(z().Z4cError):
        z().swsh_project(np.ones(len(P), complex), P, w, ORIGIN, 13)
