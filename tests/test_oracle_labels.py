"""Pin of the h-vs-2h truncation-error labels (P17): on polynomial data of
per-axis degree 2N every operator is exact at both spacings, so the RHS at
coinciding points agrees to rounding and the label is at the rounding floor;
on a single Fourier mode the difference shrinks by ~2^(2N) per halving."""
import numpy as np

import oracle
import z4c_inputs as zi
from z4c_inputs import analytic as an


def label_pair(fn, n, order, lo=-1.0, hi=1.0):
    g = order // 2 + 1
    mh = zi.uniform_mesh((1, 1, 1), n, g, (lo,) * 3, (hi,) * 3, zi.BC_USER)
    m2 = zi.coarse_2h_mesh(mh)
    p = zi.params_default(order)
    oh, o2 = oracle.OracleMesh(mh), oracle.OracleMesh(m2)
    rh = oracle.rhs(oh, p, oh.scatter_ghosted(an.ghosted_data(mh, fn)), fill=False)[0]
    r2 = oracle.rhs(o2, p, o2.scatter_ghosted(an.ghosted_data(m2, fn)), fill=False)[0]
    d = rh[:, ::2, ::2, ::2] - r2
    return np.log10(np.sqrt(np.mean(d * d)) + 1e-30), np.abs(rh).max()


def test_polynomial_data_labels_vanish():
    rng = np.random.default_rng(4)
    N = 3
    coef = rng.uniform(-1, 1, size=(22, 2 * N + 1, 2 * N + 1, 2 * N + 1)) * 1e-3 / (2 * N + 1) ** 3

    def fn(X, Y, Z):
        u = np.zeros((22,) + X.shape)
        for f in range(22):
            u[f] = np.polynomial.polynomial.polyval3d(X, Y, Z, coef[f])
        for f in (0, 1, 4, 6, 18):
            u[f] += 1.0
        return u
    lab, scale = label_pair(fn, 16, 2 * N)
    assert lab < np.log10(scale) - 10.0, (lab, scale)   # rounding floor, not truncation


def test_fourier_mode_labels_converge():
    def make(k):
        def fn(X, Y, Z):
            u = np.zeros((22,) + X.shape)
            s = 1e-3 * np.sin(k * X + 0.3) * np.cos(0.7 * k * Y)
            for f in range(22):
                u[f] = s * (1 + 0.05 * f)
            for f in (0, 1, 4, 6, 18):
                u[f] += 1.0
            return u
        return fn
    l1, _ = label_pair(make(3.0), 16, 6)
    l2, _ = label_pair(make(3.0), 32, 6)
    assert 1.5 < l1 - l2 < 2.3, (l1, l2)   # 6th order: log10(2^6) = 1.8
