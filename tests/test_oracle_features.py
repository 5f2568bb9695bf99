"""Pin of the oracle's sixteen per-block features of the learned refinement
indicator (the chi-based quantities of Sec. 3.3 widened to the other
fields): on fields of per-axis degree <= 2 every centred first and second
difference of order 2N >= 4 is exact, so each feature equals the closed form
of its definition, evaluated here directly from the polynomial's analytic
derivatives at the zone centres.

The fields are chosen so that a plausible slip fails a feature: the largest
second derivative of the conformal metric is a mixed one of one off-diagonal
component (a wrong mixed pair reads 0), |d chi| varies over the block (max
and mean differ), d alpha has an x-dependent part, and the constant tensors
have distinct entries (off-diagonal ones count twice in sqrt(A~_ij A~_ij))."""
import numpy as np
import pytest

import oracle
import z4c_inputs as zi
from z4c_inputs import analytic as an

I = zi.IDX


def fields(X, Y, Z):
    u = np.zeros((22,) + X.shape)
    u[I["chi"]] = 0.6 + 0.1 * X + 0.05 * Y * Y
    for c in ("gxx", "gyy", "gzz"):
        u[I[c]] = 1.0
    u[I["gxx"]] += 0.02 * Z * Z           # d_zz = 0.04
    u[I["gxy"]] = 0.03 * X * Y            # d_xy = 0.03
    u[I["gyz"]] = 0.07 * Y * Z            # d_yz = 0.07: the largest
    u[I["gzz"]] += 0.01 * X * X           # d_xx = 0.02
    u[I["Khat"]] = 0.3 * X - 0.4 * Y + 0.2
    A = {"Axx": 0.1, "Axy": -0.2, "Axz": 0.05, "Ayy": 0.3, "Ayz": 0.01, "Azz": -0.4}
    for k, v in A.items():
        u[I[k]] = v
    u[I["Gamx"]], u[I["Gamy"]], u[I["Gamz"]] = 0.1, -0.2, 0.2
    u[I["Theta"]] = -0.25
    u[I["alpha"]] = 0.5 + 0.2 * Z + 0.1 * X * X
    u[I["betax"]], u[I["betaz"]] = 0.3, -0.4
    return u


@pytest.mark.parametrize("order", [4, 6, 8])
def test_features_closed_form(order):
    g = order // 2 + 1
    mesh = zi.uniform_mesh((2, 1, 1), 8, g, (-1.0, -0.5, -0.25), (1.0, 0.5, 0.75), zi.BC_USER)
    om = oracle.OracleMesh(mesh)
    u = om.scatter_ghosted(an.ghosted_data(mesh, fields))
    got = oracle.block_features(om, zi.params_default(order), u, fill=False)
    for b in range(mesh.nb):
        X, Y, Z = mesh.grid(b)
        nchi = np.sqrt(0.1 ** 2 + (0.1 * Y) ** 2)
        nal = np.sqrt((0.2 * X) ** 2 + 0.2 ** 2)
        al = 0.5 + 0.2 * Z + 0.1 * X * X
        chi = 0.6 + 0.1 * X + 0.05 * Y * Y
        A2 = 0.1 ** 2 + 0.3 ** 2 + 0.4 ** 2 + 2 * (0.2 ** 2 + 0.05 ** 2 + 0.01 ** 2)
        want = np.array([
            nchi.max(), nchi.mean(), nal.max(), nal.mean(),
            0.07, 0.07,                              # max |dd g~| everywhere
            al.min(), chi.min(),
            np.abs(0.3 * X - 0.4 * Y + 0.2).max(), np.sqrt(A2), 0.25,
            np.sqrt(0.1 ** 2 + 0.2 ** 2 + 0.2 ** 2), 0.5,
            0.1,                                     # d_yy chi
            0.5,                                     # |d Khat|
            np.log2(mesh.dx(b))])
        np.testing.assert_allclose(got[b], want, rtol=1e-12, atol=1e-13, err_msg=f"block {b}")


def test_features_reduce_over_active_zones_only():
    """Only active zones are reduced over (Sec. 3.3): garbage in the outermost
    ghost layer, which no centred stencil of half-width N < g reaches, leaves
    every feature unchanged."""
    order = 6
    g = order // 2 + 1
    N = order // 2
    mesh = zi.uniform_mesh((1, 1, 1), 8, g, (-1.0,) * 3, (1.0,) * 3, zi.BC_USER)
    om = oracle.OracleMesh(mesh)
    arr = an.ghosted_data(mesh, fields)[0]
    u = om.scatter_ghosted([arr])
    ref = oracle.block_features(om, zi.params_default(order), u, fill=False)
    # the outermost ghost layer (beyond the stencil's half-width N) is unread
    assert g > N
    bad = arr.copy()
    for a in (1, 2, 3):
        sl = [slice(None)] * 4
        sl[a] = 0
        bad[tuple(sl)] = 1e30
        sl[a] = -1
        bad[tuple(sl)] = -1e30
    got = oracle.block_features(om, zi.params_default(order), om.scatter_ghosted([bad]), fill=False)
    assert np.array_equal(got, ref)
