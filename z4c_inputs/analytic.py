"""Closed-form spacetimes written as Z4c initial data, with ghost zones.

Used to pin the oracle against known solutions.  Each solution is an ADM
data set (gamma_ij, K_ij, alpha, beta^i) at time t; `adm_to_z4c` turns it
into the Z4c variables:
  chi = det(gamma)^(-1/3), g~_ij = chi gamma_ij, Khat = K (Theta = 0),
  A~_ij = chi (K_ij - gamma_ij K / 3), Gamma~^i = -d_j g~^ij (det g~ = 1).
Spatial and time derivatives of the analytic fields are taken by the
complex-step method (Im f(x + i e)/e), which is exact to rounding.

All functions accept complex coordinates so that the complex step works.
"""
from __future__ import annotations

import numpy as np

from . import NF, IDX, SYM, Mesh

EPS_CS = 1e-30


def _sym_to_full(a6):
    return np.stack([np.stack([a6[SYM[i][j]] for j in range(3)]) for i in range(3)])


def _inv3(g):
    """Inverse of a (3,3,...) array of matrices."""
    a, b, c = g[0, 0], g[0, 1], g[0, 2]
    d, e, f = g[1, 0], g[1, 1], g[1, 2]
    gg, h, i = g[2, 0], g[2, 1], g[2, 2]
    det = a * (e * i - f * h) - b * (d * i - f * gg) + c * (d * h - e * gg)
    inv = np.empty_like(g)
    inv[0, 0] = (e * i - f * h) / det
    inv[0, 1] = (c * h - b * i) / det
    inv[0, 2] = (b * f - c * e) / det
    inv[1, 0] = (f * gg - d * i) / det
    inv[1, 1] = (a * i - c * gg) / det
    inv[1, 2] = (c * d - a * f) / det
    inv[2, 0] = (d * h - e * gg) / det
    inv[2, 1] = (b * gg - a * h) / det
    inv[2, 2] = (a * e - b * d) / det
    return inv, det


def _z4c_algebraic(gamma, K, alpha, beta):
    """Z4c variables except Gamma~ (complex-safe)."""
    ginv, det = _inv3(gamma)
    chi = det ** (-1.0 / 3.0)
    trK = np.einsum("ij...,ij...->...", ginv, K)
    gt = chi * gamma
    At = chi * (K - gamma * trK / 3.0)
    return chi, gt, trK, At


def _conf_inverse(fn, t, X, Y, Z):
    gamma, K, alpha, beta = fn(t, X, Y, Z)
    chi, gt, _, _ = _z4c_algebraic(gamma, K, alpha, beta)
    gtu, _ = _inv3(gt)
    return gtu


def adm_to_z4c(fn, t, X, Y, Z) -> np.ndarray:
    """Z4c fields (22, ...) of the ADM solution fn(t, X, Y, Z) at real points."""
    gamma, K, alpha, beta = fn(t, X, Y, Z)
    chi, gt, trK, At = _z4c_algebraic(gamma, K, alpha, beta)
    out = np.zeros((NF,) + np.shape(X))
    out[IDX["chi"]] = np.real(chi)
    for i in range(3):
        for j in range(i, 3):
            out[IDX["gxx"] + SYM[i][j]] = np.real(gt[i, j])
            out[IDX["Axx"] + SYM[i][j]] = np.real(At[i, j])
    out[IDX["Khat"]] = np.real(trK)
    out[IDX["alpha"]] = np.real(alpha) * np.ones(np.shape(X))
    for i in range(3):
        out[IDX["betax"] + i] = np.real(beta[i]) * np.ones(np.shape(X))
    # Gamma~^i = -d_j g~^{ij}
    Xc = [np.asarray(X, complex), np.asarray(Y, complex), np.asarray(Z, complex)]
    gam = np.zeros((3,) + np.shape(X))
    for j in range(3):
        P = list(Xc)
        P[j] = P[j] + 1j * EPS_CS
        gtu = _conf_inverse(fn, t, *P)
        for i in range(3):
            gam[i] -= np.imag(gtu[i, j]) / EPS_CS
    for i in range(3):
        out[IDX["Gamx"] + i] = gam[i]
    return out


def z4c_time_derivative(fn, t, X, Y, Z) -> np.ndarray:
    """d/dt of the Z4c fields (except Gamma~, Theta, lapse and shift, which
    are left 0) by a complex step in t."""
    gamma, K, alpha, beta = fn(t + 1j * EPS_CS, np.asarray(X, complex), np.asarray(Y, complex),
                               np.asarray(Z, complex))
    chi, gt, trK, At = _z4c_algebraic(gamma, K, alpha, beta)
    out = np.zeros((NF,) + np.shape(X))
    out[IDX["chi"]] = np.imag(chi) / EPS_CS
    for i in range(3):
        for j in range(i, 3):
            out[IDX["gxx"] + SYM[i][j]] = np.imag(gt[i, j]) / EPS_CS
            out[IDX["Axx"] + SYM[i][j]] = np.imag(At[i, j]) / EPS_CS
    out[IDX["Khat"]] = np.imag(trK) / EPS_CS
    return out


# ------------------------------------------------------------- solutions

def _ones(X):
    return np.ones(np.shape(X), dtype=np.result_type(X, float))


def kasner(u: float = 2.0, rot=None):
    """Kasner vacuum cosmology ds^2 = -dt^2 + sum t^(2 p_a) dx_a^2 in geodesic
    slicing (alpha = 1, beta = 0), with the exponents of the one-parameter
    family p = (-u, 1+u, u(1+u))/(1+u+u^2), optionally rotated by a constant
    orthogonal matrix.  Spatially homogeneous."""
    s = 1.0 + u + u * u
    p = np.array([-u / s, (1.0 + u) / s, u * (1.0 + u) / s])
    R = np.eye(3) if rot is None else np.asarray(rot)

    def fn(t, X, Y, Z):
        one = _ones(X) * (1.0 + 0 * t)
        D = [t ** (2 * p[a]) for a in range(3)]
        dD = [2 * p[a] * t ** (2 * p[a] - 1) for a in range(3)]
        gamma = np.zeros((3, 3) + np.shape(one), dtype=one.dtype)
        K = np.zeros_like(gamma)
        for i in range(3):
            for j in range(3):
                gamma[i, j] = sum(R[i, a] * R[j, a] * D[a] for a in range(3)) * one
                K[i, j] = -0.5 * sum(R[i, a] * R[j, a] * dD[a] for a in range(3)) * one
        return gamma, K, one, [0 * one, 0 * one, 0 * one]
    fn.exponents = p
    return fn


def kerr_schild(M: float = 1.0, centre=(0.0, 0.0, 0.0)):
    """Schwarzschild in Kerr-Schild coordinates (stationary, K_ij != 0):
    gamma_ij = delta_ij + 2H l_i l_j, H = M/r, l = x/r, alpha = (1+2H)^(-1/2),
    beta^i = 2H l^i/(1+2H), K_ij = 2 H alpha/r (delta_ij - (2+H) l_i l_j)."""
    def fn(t, X, Y, Z):
        x = [X - centre[0], Y - centre[1], Z - centre[2]]
        r = np.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)
        H = M / r
        l = [x[a] / r for a in range(3)]
        alpha = (1.0 + 2.0 * H) ** -0.5
        gamma = np.zeros((3, 3) + np.shape(r), dtype=r.dtype)
        K = np.zeros_like(gamma)
        for i in range(3):
            for j in range(3):
                d = 1.0 if i == j else 0.0
                gamma[i, j] = d + 2.0 * H * l[i] * l[j]
                K[i, j] = 2.0 * H * alpha / r * (d - (2.0 + H) * l[i] * l[j])
        beta = [2.0 * H * l[a] / (1.0 + 2.0 * H) for a in range(3)]
        return gamma, K, alpha, beta
    return fn


def schwarzschild_isotropic(M: float = 1.0):
    """Static Schwarzschild, isotropic coordinates: gamma = psi^4 delta,
    psi = 1 + M/(2r), K_ij = 0, alpha = (1 - M/2r)/(1 + M/2r), beta = 0."""
    def fn(t, X, Y, Z):
        r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
        psi = 1.0 + M / (2.0 * r)
        gamma = np.zeros((3, 3) + np.shape(r), dtype=r.dtype)
        for i in range(3):
            gamma[i, i] = psi ** 4
        K = np.zeros_like(gamma)
        alpha = (1.0 - M / (2.0 * r)) / (1.0 + M / (2.0 * r))
        return gamma, K, alpha, [0 * r, 0 * r, 0 * r]
    return fn


def linear_wave(A: float = 1e-8, d: float = 1.0):
    """Linearised TT gravitational wave travelling along +x:
    h_yy = -h_zz = A sin(2 pi (x - t)/d), alpha = 1, beta = 0,
    K_ij = -d_t h_ij / 2 (the linear-wave test of Sec. 4.1)."""
    w = 2.0 * np.pi / d

    def fn(t, X, Y, Z):
        ph = w * (X - t)
        one = _ones(X) * (1.0 + 0 * t) * (1.0 + 0 * ph)
        h = A * np.sin(ph)
        ht = -A * w * np.cos(ph)
        gamma = np.zeros((3, 3) + np.shape(one), dtype=one.dtype)
        K = np.zeros_like(gamma)
        gamma[0, 0] = one
        gamma[1, 1] = one + h
        gamma[2, 2] = one - h
        K[1, 1] = -0.5 * ht
        K[2, 2] = 0.5 * ht
        return gamma, K, one, [0 * one, 0 * one, 0 * one]
    return fn


def linear_wave_diagonal(A: float = 1e-8, L: float = 1.0):
    """Linearised TT wave travelling along the diagonal of a periodic cube
    of side L (one wavelength across the cube in each direction):
    h_ab = A e_ab sin(k.x - w t), k = (2 pi / L)(1, 1, 1), w = |k|,
    e = u u - v v with u, v orthonormal and orthogonal to k; alpha = 1,
    beta = 0, K_ab = -d_t h_ab / 2.  Period 2 pi / w = L / sqrt(3)."""
    kv = 2.0 * np.pi / L * np.ones(3)
    w = float(np.linalg.norm(kv))
    n = kv / w
    u = np.array([1.0, -1.0, 0.0]) / np.sqrt(2.0)
    v = np.cross(n, u)
    e = np.outer(u, u) - np.outer(v, v)

    def fn(t, X, Y, Z):
        ph = kv[0] * X + kv[1] * Y + kv[2] * Z - w * t
        one = _ones(X) * (1.0 + 0 * t) * (1.0 + 0 * ph)
        s = A * np.sin(ph)
        st = -A * w * np.cos(ph)
        gamma = np.zeros((3, 3) + np.shape(one), dtype=one.dtype)
        K = np.zeros_like(gamma)
        for a in range(3):
            for b in range(3):
                gamma[a, b] = (1.0 if a == b else 0.0) * one + e[a, b] * s
                K[a, b] = -0.5 * e[a, b] * st
        return gamma, K, one, [0 * one, 0 * one, 0 * one]
    fn.period = 2.0 * np.pi / w
    return fn


# ------------------------------------------------------- ghosted blocks

def ghosted_grid(mesh: Mesh, b: int):
    """Cell-centre coordinates of block b including its ghost layers."""
    g = mesh.g
    n = int(mesh.n[b])
    h = mesh.dx(b)
    ax = [mesh.lo[a] + (mesh.ilo[b, a] + np.arange(-g, n + g) + 0.5) * h for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


def ghosted_data(mesh: Mesh, fields_fn):
    """Per-block (22, E, E, E) arrays (ghosts included) of fields_fn(X, Y, Z)."""
    return [fields_fn(*ghosted_grid(mesh, b)) for b in range(mesh.nb)]
