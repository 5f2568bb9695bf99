"""Seeded synthetic inputs for the Z4c hot path: mesh layouts and initial data.

This module holds no arithmetic of the evolution method itself.  It describes
MeshBlock layouts (block lists of level, size and integer corner) and writes
initial data at cell centres, x_i = lo + (ilo + i + 1/2) dx (cell-centred
nodes, Sec. 3.2 of the paper).  The oracle and the GPU library both receive
exactly these arrays.

Per-block interior arrays have shape (22, n, n, n), indexed [field, z, y, x].
Field order:
  chi, gxx, gxy, gxz, gyy, gyz, gzz, Khat, Axx, Axy, Axz, Ayy, Ayz, Azz,
  Gamx, Gamy, Gamz, Theta, alpha, betax, betay, betaz
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

NF = 22
FIELDS = ["chi", "gxx", "gxy", "gxz", "gyy", "gyz", "gzz", "Khat",
          "Axx", "Axy", "Axz", "Ayy", "Ayz", "Azz", "Gamx", "Gamy", "Gamz",
          "Theta", "alpha", "betax", "betay", "betaz"]
IDX = {n: i for i, n in enumerate(FIELDS)}
SYM = ((0, 1, 2), (1, 3, 4), (2, 4, 5))

BC_PERIODIC, BC_OUTFLOW, BC_USER = 0, 1, 2


@dataclasses.dataclass
class Mesh:
    """A Mesh of cubic MeshBlocks (interior n^3 each) with g ghost layers."""
    level: np.ndarray          # [nb] int32
    n: np.ndarray              # [nb] int32
    ilo: np.ndarray            # [nb, 3] int32, interior corner in cells of its level
    g: int
    nroot: tuple               # root cells per axis over the domain
    bc: int
    lo: tuple                  # domain lower corner
    dx0: float                 # root cell size

    @property
    def nb(self) -> int:
        return int(self.level.shape[0])

    def dx(self, b: int) -> float:
        """Cell size of block b."""
        return self.dx0 / (1 << int(self.level[b]))

    def dx_min(self) -> float:
        """Cell size of the finest level present."""
        return self.dx0 / (1 << int(self.level.max()))

    def centres(self, b: int):
        """1D cell-centre coordinates of block b along x, y, z."""
        h = self.dx(b)
        return [self.lo[a] + (self.ilo[b, a] + np.arange(self.n[b]) + 0.5) * h for a in range(3)]

    def grid(self, b: int):
        x, y, z = self.centres(b)
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return X, Y, Z

    def zones(self) -> int:
        return int(np.sum(self.n.astype(np.int64) ** 3))


def uniform_mesh(nblk: Sequence[int], n: int, g: int, lo, hi, bc: int) -> Mesh:
    """Single-level mesh: nblk[a] blocks of n^3 per axis over [lo, hi]."""
    nroot = tuple(int(nblk[a] * n) for a in range(3))
    dx0 = (hi[0] - lo[0]) / nroot[0]
    ilo = []
    for k in range(nblk[2]):
        for j in range(nblk[1]):
            for i in range(nblk[0]):
                ilo.append((i * n, j * n, k * n))
    nb = len(ilo)
    return Mesh(level=np.zeros(nb, np.int32), n=np.full(nb, n, np.int32),
                ilo=np.array(ilo, np.int32).reshape(nb, 3), g=g, nroot=nroot, bc=bc,
                lo=tuple(float(v) for v in lo), dx0=float(dx0))


def refine_blocks(mesh: Mesh, which) -> Mesh:
    """Replace each listed block by its 8 children (same n, level + 1)."""
    which = set(int(b) for b in which)
    lev, ns, ilo = [], [], []
    for b in range(mesh.nb):
        if b not in which:
            lev.append(int(mesh.level[b]))
            ns.append(int(mesh.n[b]))
            ilo.append(tuple(int(v) for v in mesh.ilo[b]))
            continue
        n = int(mesh.n[b])
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    lev.append(int(mesh.level[b]) + 1)
                    ns.append(n)
                    ilo.append((2 * int(mesh.ilo[b, 0]) + dx * n, 2 * int(mesh.ilo[b, 1]) + dy * n,
                                2 * int(mesh.ilo[b, 2]) + dz * n))
    nb = len(lev)
    return Mesh(level=np.array(lev, np.int32), n=np.array(ns, np.int32),
                ilo=np.array(ilo, np.int32).reshape(nb, 3), g=mesh.g, nroot=mesh.nroot,
                bc=mesh.bc, lo=mesh.lo, dx0=mesh.dx0)


def split_blocks(mesh: Mesh, which) -> Mesh:
    """Replace each listed block of n^3 by 8 blocks of (n/2)^3 at the same level."""
    which = set(int(b) for b in which)
    lev, ns, ilo = [], [], []
    for b in range(mesh.nb):
        n = int(mesh.n[b])
        if b not in which:
            lev.append(int(mesh.level[b]))
            ns.append(n)
            ilo.append(tuple(int(v) for v in mesh.ilo[b]))
            continue
        h = n // 2
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    lev.append(int(mesh.level[b]))
                    ns.append(h)
                    ilo.append((int(mesh.ilo[b, 0]) + dx * h, int(mesh.ilo[b, 1]) + dy * h,
                                int(mesh.ilo[b, 2]) + dz * h))
    nb = len(lev)
    return Mesh(level=np.array(lev, np.int32), n=np.array(ns, np.int32),
                ilo=np.array(ilo, np.int32).reshape(nb, 3), g=mesh.g, nroot=mesh.nroot,
                bc=mesh.bc, lo=mesh.lo, dx0=mesh.dx0)


def nested_bbh_mesh(g: int = 5) -> Mesh:
    """512 MeshBlocks over four levels around two punctures at x = +-5:
    root 4^3 blocks of 32^3 (dx = 1) on [-64, 64]^3; level 1 (dx = 1/2) on
    [-32, 32]^3, level 2 (dx = 1/4) on [-16, 16]^3, both in 32^3 blocks;
    level 3 (dx = 1/8) on [-8, 8]^3 in 4-unit blocks of which five of the
    eight (inner/outer per axis) classes are split into 16^3 blocks:
    56 + 56 + 56 + 24 x 32^3 + 320 x 16^3 = 512 blocks, 7,602,176 zones."""
    m = uniform_mesh((4, 4, 4), 32, g, (-64.0,) * 3, (64.0,) * 3, BC_OUTFLOW)
    m = refine_blocks(m, blocks_in_box(m, (-32.0,) * 3, (32.0,) * 3))
    m = refine_blocks(m, blocks_in_box(m, (-16.0,) * 3, (16.0,) * 3))
    m = refine_blocks(m, blocks_in_box(m, (-8.0,) * 3, (8.0,) * 3))
    split_classes = {("o", "i", "i"), ("o", "o", "i"), ("o", "i", "o"), ("i", "i", "i"), ("o", "o", "o")}
    which = []
    for b in range(m.nb):
        if m.level[b] != 3:
            continue
        h = m.dx(b)
        cls = []
        for a in range(3):
            x0 = m.lo[a] + m.ilo[b, a] * h          # block spans [x0, x0 + 4]
            cls.append("i" if -4.0 <= x0 < 4.0 else "o")
        if tuple(cls) in split_classes:
            which.append(b)
    return split_blocks(m, which)


def coarse_2h_mesh(mesh: Mesh) -> Mesh:
    """The even-sublattice (2h) mesh of a single-level mesh: the same blocks
    with n/2 cells and corner ilo/2, cell size 2h, domain shifted by -h/2 so
    that its cell centres are the even fine cell centres."""
    assert int(mesh.level.max()) == 0, "2h meshes are defined for single-level meshes"
    h = mesh.dx0
    return Mesh(level=mesh.level.copy(), n=(mesh.n // 2).astype(np.int32),
                ilo=(mesh.ilo // 2).astype(np.int32), g=mesh.g,
                nroot=tuple(int(v) // 2 for v in mesh.nroot), bc=mesh.bc,
                lo=tuple(v - 0.5 * h for v in mesh.lo), dx0=2.0 * h)


def blocks_in_box(mesh: Mesh, lo, hi):
    """Indices of blocks whose interior lies inside the physical box [lo, hi]."""
    out = []
    for b in range(mesh.nb):
        h = mesh.dx(b)
        x0 = [mesh.lo[a] + mesh.ilo[b, a] * h for a in range(3)]
        x1 = [x0[a] + mesh.n[b] * h for a in range(3)]
        if all(x0[a] >= lo[a] - 1e-12 and x1[a] <= hi[a] + 1e-12 for a in range(3)):
            out.append(b)
    return out


def analytic_interiors(mesh: Mesh, fn):
    """Per-block (22, n, n, n) arrays of fn(X, Y, Z) -> (22, ...) at cell centres."""
    return [fn(*mesh.grid(b)) for b in range(mesh.nb)]


# ------------------------------------------------------------ initial data

def flat(mesh: Mesh) -> List[np.ndarray]:
    """Minkowski space: chi = alpha = 1, g~ = delta, all else 0."""
    out = []
    for b in range(mesh.nb):
        n = int(mesh.n[b])
        u = np.zeros((NF, n, n, n))
        u[IDX["chi"]] = 1.0
        u[IDX["alpha"]] = 1.0
        for c in ("gxx", "gyy", "gzz"):
            u[IDX[c]] = 1.0
        out.append(u)
    return out


def brill_lindquist(mesh: Mesh, punctures) -> List[np.ndarray]:
    """Conformally flat Brill-Lindquist punctures, psi = 1 + sum m/(2|x-x_p|);
    chi = psi^-4, g~ = delta, K = A~ = Theta = Gamma~ = beta = 0, and the
    pre-collapsed lapse alpha = psi^-2."""
    out = flat(mesh)
    for b in range(mesh.nb):
        X, Y, Z = mesh.grid(b)
        psi = np.ones_like(X)
        for (m, xp) in punctures:
            r = np.sqrt((X - xp[0]) ** 2 + (Y - xp[1]) ** 2 + (Z - xp[2]) ** 2)
            psi += m / (2.0 * r)
        out[b][IDX["chi"]] = psi ** -4
        out[b][IDX["alpha"]] = psi ** -2
    return out


def perturbation_modes(seed: int, nmodes: int = 8, periodic_box: float | None = None,
                       kmin: float = math.pi / 4, kmax: float = math.pi):
    """Wavevectors and phases for every field (PCG64 draws in a fixed order:
    field by field, mode by mode).  With periodic_box = L, k = 2 pi n / L with
    integer n_i in -2..2 (not all zero); otherwise |k| ~ U[kmin, kmax] in a
    uniformly random direction.  Returns k[NF, nmodes, 3], phase[NF, nmodes]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.zeros((NF, nmodes, 3))
    ph = np.zeros((NF, nmodes))
    for f in range(NF):
        for m in range(nmodes):
            if periodic_box is not None:
                while True:
                    nvec = rng.integers(-2, 3, size=3)
                    if np.any(nvec != 0):
                        break
                k[f, m] = 2.0 * math.pi * nvec / periodic_box
            else:
                kk = rng.uniform(kmin, kmax)
                v = rng.normal(size=3)
                k[f, m] = kk * v / np.linalg.norm(v)
            ph[f, m] = rng.uniform(0.0, 2.0 * math.pi)
    return k, ph


def add_perturbation(mesh: Mesh, data: List[np.ndarray], seed: int, amp: float = 1e-6,
                     nmodes: int = 8, periodic_box: float | None = None) -> List[np.ndarray]:
    """Add sum_m amp sin(k_m . x + phi_m) to every field (amplitude per term)."""
    k, ph = perturbation_modes(seed, nmodes, periodic_box)
    for b in range(mesh.nb):
        X, Y, Z = mesh.grid(b)
        for f in range(NF):
            s = np.zeros_like(X)
            for m in range(nmodes):
                s += np.sin(k[f, m, 0] * X + k[f, m, 1] * Y + k[f, m, 2] * Z + ph[f, m])
            data[b][f] += amp * s
    return data


# ---------------------------------------------- learned indicator weights

MLP_SIZES = [("W1", (64, 16)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (1, 64)),
             ("b3", (1,))]


def mlp_init(seed: int = 0) -> np.ndarray:
    """Seeded initial weights of the 16-64-64-1 network, packed W1, b1, W2,
    b2, W3, b3: He-uniform weights, zero biases, float32-representable."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, shp in MLP_SIZES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            parts.append(rng.uniform(-lim, lim, size=shp).reshape(-1))
        else:
            parts.append(np.zeros(int(np.prod(shp))))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


# ------------------------------------------------------ standard workloads

def params_default(fd_order: int, eta: float = 2.0) -> dict:
    """Sec. 4.3: K.O. dissipation 0.5, kappa1 = 0.02, kappa2 = 0, CFL 0.25."""
    return dict(fd_order=fd_order, ko_sigma=0.5, kappa1=0.02, kappa2=0.0, eta=eta,
                mu_S=1.0, chi_floor=1e-12, alpha_floor=1e-12, terms=0xF, enforce=1)


def workload(name: str):
    """Named workloads: returns (mesh, params, initial interiors, dt, steps).

    periodic16  one periodic 16^3 block on [0,1]^3, 4th order, flat space plus
                8 sinusoids of amplitude 1e-6 per field (seed 1), dt = 1/64.
    bl64x32     64 blocks of 32^3 on [-16,16]^3 (dx = 0.25), 6th order,
                Brill-Lindquist M = 1 at the origin, outflow, dt = 0.0625.
    bl512x32    512 blocks of 32^3 on [-16,16]^3 (dx = 0.125), 6th order,
                BL M = 1 plus 8 sinusoids of 1e-6 per field (seed 4).
    bbh512mixed 512 blocks of 16^3 and 32^3 over 4 levels (nested_bbh_mesh),
                8th order, 5 ghosts, two BL punctures m = 0.5 at x = +-5.
    bbh4096x16  4096 blocks of 16^3 on [-16,16]^3 (dx = 0.125), 6th order,
                two BL punctures m = 0.5 at x = +-5.
    wave64x64   the linear gravitational wave of Sec. 4.1 (amplitude 1e-8,
                along the diagonal of the periodic unit cube) on 64 blocks of
                64^3 (256^3 zones), 6th order: Table 1's MeshBlock size.
    """
    cfl = 0.25
    if name == "periodic16":
        mesh = uniform_mesh((1, 1, 1), 16, 4, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), BC_PERIODIC)
        data = add_perturbation(mesh, flat(mesh), seed=1, periodic_box=1.0)
        return mesh, params_default(4), data, cfl * mesh.dx0, 1
    if name == "bl64x32":
        mesh = uniform_mesh((4, 4, 4), 32, 4, (-16.0,) * 3, (16.0,) * 3, BC_OUTFLOW)
        data = brill_lindquist(mesh, [(1.0, (0.0, 0.0, 0.0))])
        return mesh, params_default(6, eta=2.0), data, cfl * mesh.dx0, 10
    if name == "bl512x32":
        mesh = uniform_mesh((8, 8, 8), 32, 4, (-16.0,) * 3, (16.0,) * 3, BC_OUTFLOW)
        data = add_perturbation(mesh, brill_lindquist(mesh, [(1.0, (0.0, 0.0, 0.0))]), seed=4)
        return mesh, params_default(6, eta=2.0), data, cfl * mesh.dx0, 100
    if name == "bbh512mixed":
        mesh = nested_bbh_mesh()
        data = brill_lindquist(mesh, [(0.5, (5.0, 0.0, 0.0)), (0.5, (-5.0, 0.0, 0.0))])
        return mesh, params_default(8, eta=2.0), data, cfl * mesh.dx_min(), 1
    if name == "wave64x64":
        mesh, data = linear_wave_pack(4, 64)
        return mesh, params_default(6), data, cfl * mesh.dx0, 1
    if name == "bbh4096x16":
        mesh = uniform_mesh((16, 16, 16), 16, 4, (-16.0,) * 3, (16.0,) * 3, BC_OUTFLOW)
        data = brill_lindquist(mesh, [(0.5, (5.0, 0.0, 0.0)), (0.5, (-5.0, 0.0, 0.0))])
        return mesh, params_default(6, eta=2.0), data, cfl * mesh.dx0, 1
    raise KeyError(name)


def linear_wave_pack(nblk: int, n: int, amplitude: float = 1e-8):
    """nblk^3 blocks of n^3 on the periodic unit cube holding the linear wave
    travelling along the diagonal (analytic.linear_wave_diagonal) at t = 0.
    The wave depends on the position only through x + y + z, so the fields
    are evaluated once per value of the global index sum i + j + k (on the
    diagonal point with that coordinate sum) and gathered into the blocks."""
    from z4c_inputs import analytic
    mesh = uniform_mesh((nblk,) * 3, n, 4, (0.0,) * 3, (1.0,) * 3, BC_PERIODIC)
    fn = analytic.linear_wave_diagonal(amplitude, 1.0)
    h = mesh.dx0
    m = np.arange(3 * nblk * n - 2)
    d = (m + 1.5) * h / 3.0                       # x = y = z with x + y + z = (m + 3/2) h
    line = analytic.adm_to_z4c(fn, 0.0, d, d, d)  # (22, len(m))
    out = []
    for b in range(mesh.nb):
        i = mesh.ilo[b, 0] + np.arange(n)
        j = mesh.ilo[b, 1] + np.arange(n)
        k = mesh.ilo[b, 2] + np.arange(n)
        idx = k[:, None, None] + j[None, :, None] + i[None, None, :]
        out.append(line[:, idx])
    return mesh, out


# ------------------------------------------------------- geodesic spheres

def geodesic_sphere(level: int, radius: float = 1.0, centre=(0.0, 0.0, 0.0)):
    """Points (N, 3) and quadrature weights (N,) of a geodesic sphere: the
    icosahedron with every triangle split into four `level` times, vertices
    projected onto the sphere.  Each vertex carries a third of the solid
    angle of every triangle it belongs to (weights sum to 4 pi)."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    V = [np.array(v, float) / np.linalg.norm(v) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                v = V[a] + V[b]
                V.append(v / np.linalg.norm(v))
                cache[key] = len(V) - 1
            return cache[key]
        G = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            G += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = G
    P = np.array(V)
    w = np.zeros(len(P))
    for a, b, c in F:
        A, B, C = P[a], P[b], P[c]
        # solid angle of the spherical triangle (Van Oosterom and Strackee)
        num = abs(np.dot(A, np.cross(B, C)))
        den = 1.0 + np.dot(A, B) + np.dot(B, C) + np.dot(C, A)
        om = 2.0 * np.arctan2(num, den)
        w[[a, b, c]] += om / 3.0
    return P * radius + np.asarray(centre, float), w
