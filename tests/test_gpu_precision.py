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
