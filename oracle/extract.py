"""Reference wave extraction and puncture tracking -- TEST INFRASTRUCTURE ONLY.

Sec. 3.4 (other diagnostics): Psi4 is interpolated onto spheres and
decomposed into spin-weighted spherical harmonics; punctures are advected
with the shift.

* Interpolation: a point belongs to the finest block whose active cells
  contain it; along each axis the value is the Lagrange cubic through the
  four cell centres nearest the point inside that block (window shifted
  inward at the block's faces), tensor product over the three axes.
* Spin-weighted harmonics sY_lm: Goldberg et al.'s explicit sum.
* Projection: C_lm = sum_p w_p psi(p) conj(sY_lm(theta_p, phi_p)) with the
  sphere's quadrature weights.
* Tracker: dx/dt = -beta(x), integrated by the classic RK4 of the evolution
  itself: stage s reads beta from that stage's input state at
  x_n + c_s dt k_(s-1), c = (0, 1/2, 1/2, 1), weights (1, 2, 2, 1)/6.
"""
from __future__ import annotations

import math

import numpy as np

import oracle


# --------------------------------------------------------- interpolation

def locate(mesh, p):
    """Index of the finest block whose active cells contain point p."""
    for lev in range(int(mesh.level.max()), -1, -1):
        h = mesh.dx0 / (1 << lev)
        cell = [math.floor((p[a] - mesh.lo[a]) / h) for a in range(3)]
        for b in range(mesh.nb):
            if int(mesh.level[b]) != lev:
                continue
            n = int(mesh.n[b])
            if all(int(mesh.ilo[b, a]) <= cell[a] < int(mesh.ilo[b, a]) + n for a in range(3)):
                return b
    raise ValueError(f"point {p} outside the mesh")


def _cubic(xt, n):
    """Nodes (4 local cell indices) and Lagrange weights at local index xt."""
    i0 = min(max(math.floor(xt) - 1, 0), n - 4)
    nodes = np.arange(i0, i0 + 4)
    w = np.ones(4)
    for i in range(4):
        for j in range(4):
            if i != j:
                w[i] *= (xt - nodes[j]) / (nodes[i] - nodes[j])
    return nodes, w


def interpolate(mesh, interiors, points):
    """Values (npts, ncomp) of per-block interior data (ncomp, n, n, n) at
    the points (npts, 3)."""
    pts = np.atleast_2d(np.asarray(points, dtype=float))
    ncomp = interiors[0].shape[0]
    out = np.empty((len(pts), ncomp))
    for q, p in enumerate(pts):
        b = locate(mesh, p)
        h = mesh.dx(b)
        n = int(mesh.n[b])
        W = []
        for a in range(3):
            xt = (p[a] - mesh.lo[a]) / h - 0.5 - int(mesh.ilo[b, a])
            W.append(_cubic(xt, n))
        (ix, wx), (iy, wy), (iz, wz) = W
        blk = interiors[b][:, iz[0]:iz[0] + 4, iy[0]:iy[0] + 4, ix[0]:ix[0] + 4]
        out[q] = np.einsum("i,j,k,fkji->f", wx, wy, wz, blk)
    return out


# ------------------------------------------------ spin-weighted harmonics

def swsh(s, l, m, theta, phi):
    """sY_lm(theta, phi), Goldberg et al. (1967) explicit sum."""
    theta = np.asarray(theta, dtype=float)
    phi = np.asarray(phi, dtype=float)
    f = math.factorial
    pref = (-1.0) ** m * math.sqrt(f(l + m) * f(l - m) * (2 * l + 1) / (4.0 * math.pi * f(l + s) * f(l - s)))
    half = theta / 2.0
    tot = np.zeros(np.shape(theta), dtype=complex)
    for r in range(0, l - s + 1):
        k2 = r + s - m
        if k2 < 0 or k2 > l + s:
            continue
        c = math.comb(l - s, r) * math.comb(l + s, k2) * (-1.0) ** (l - r - s)
        # sin^(2l)(t/2) cot^(2r+s-m)(t/2) = sin^(2l-2r-s+m) cos^(2r+s-m)
        tot = tot + c * np.sin(half) ** (2 * l - 2 * r - s + m) * np.cos(half) ** (2 * r + s - m)
    return pref * tot * np.exp(1j * m * phi)


def angles(points, centre):
    d = np.asarray(points, dtype=float) - np.asarray(centre, dtype=float)
    r = np.linalg.norm(d, axis=1)
    return np.arccos(np.clip(d[:, 2] / r, -1.0, 1.0)), np.arctan2(d[:, 1], d[:, 0])


def project(values, points, weights, centre, lmax, s=-2):
    """{(l, m): C_lm} of complex values on a sphere, l = |s| .. lmax."""
    th, ph = angles(points, centre)
    vals = np.asarray(values)
    out = {}
    for l in range(abs(s), lmax + 1):
        for m in range(-l, l + 1):
            out[(l, m)] = complex(np.sum(np.asarray(weights) * vals * np.conj(swsh(s, l, m, th, ph))))
    return out


# ---------------------------------------------------------------- tracker

def rk4_step_with_tracker(regs, params, dt, positions):
    """One RK4 step of the registers (oracle.Registers) and of the puncture
    positions (P, 3); returns the new positions."""
    om = regs.om
    mesh = om.mesh
    x = np.atleast_2d(np.asarray(positions, dtype=float)).copy()
    c = (0.0, 0.5, 0.5, 1.0)
    wts = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)
    src = {1: "U", 2: "S1", 3: "S2", 4: "S1"}
    kprev = np.zeros_like(x)
    acc = np.zeros_like(x)
    for s in (1, 2, 3, 4):
        xs = x + c[s - 1] * dt * kprev
        beta = interpolate(mesh, [blk[19:22] for blk in om.interiors(getattr(regs, src[s]))], xs)
        k = -beta
        acc += wts[s - 1] * k
        kprev = k
        oracle.rk4_stage(regs, params, s, dt)
    return x + dt * acc
