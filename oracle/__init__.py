"""Z4c reference oracle (plain single-threaded FP64 C, driven through ctypes).

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does.  It shares no code with the GPU library.

Layout: one flat float64 array per register; block b holds 22 fields of
(n_b + 2g)^3 cells, x fastest, blocks back to back (no padding).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

NF = 22
_lib = None


class _Mesh(C.Structure):
    _fields_ = [("nb", C.c_int32), ("level", C.POINTER(C.c_int32)), ("n", C.POINTER(C.c_int32)),
                ("ilo", C.POINTER(C.c_int32)), ("g", C.c_int32), ("nroot", C.c_int32 * 3),
                ("bc", C.c_int32), ("pad", C.c_int32), ("lo", C.c_double * 3), ("dx0", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("fd_order", C.c_int32), ("terms", C.c_uint32), ("enforce", C.c_int32),
                ("pad", C.c_int32), ("ko_sigma", C.c_double), ("kappa1", C.c_double),
                ("kappa2", C.c_double), ("eta", C.c_double), ("mu_S", C.c_double),
                ("chi_floor", C.c_double), ("alpha_floor", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.or_fd_weights.argtypes = [C.c_int, C.c_int, dp, dp]
        L.or_fill_ghosts.argtypes = [C.POINTER(_Mesh), dp]
        L.or_fill_ghosts_from.argtypes = [C.POINTER(_Mesh), dp, dp, C.POINTER(C.c_int8)]
        L.or_rhs.argtypes = [C.POINTER(_Mesh), C.POINTER(_Params), dp, dp]
        L.or_rhs_blocks.argtypes = [C.POINTER(_Mesh), C.POINTER(_Params), dp, dp,
                                    C.POINTER(C.c_int8)]
        L.or_rk4_stage.argtypes = [C.POINTER(_Mesh), C.POINTER(_Params), C.c_int, C.c_double,
                                   dp, dp, dp, dp]
        L.or_constraints.argtypes = [C.POINTER(_Mesh), C.POINTER(_Params), dp, dp, C.c_int, dp,
                                     C.c_double, dp]
        L.or_refine_flags.argtypes = [C.POINTER(_Mesh), C.POINTER(_Params), dp, C.c_int,
                                      C.c_double, C.c_double, C.c_int, C.c_double, dp, C.c_int,
                                      C.POINTER(C.c_int8)]
        L.or_psi4.argtypes = [C.POINTER(_Mesh), C.POINTER(_Params), dp, dp, dp]
        L.or_rk4_update.argtypes = [C.POINTER(_Mesh), C.POINTER(_Params), C.c_int, C.c_double,
                                    dp, dp, dp, dp, dp, C.POINTER(C.c_int8)]
        if hasattr(L, "or_block_features"):
            L.or_block_features.argtypes = [C.POINTER(_Mesh), C.POINTER(_Params), dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleMesh:
    """Holds the ctypes mesh description (keeps the index arrays alive)."""

    def __init__(self, mesh):
        self.mesh = mesh
        self._level = np.ascontiguousarray(mesh.level, dtype=np.int32)
        self._n = np.ascontiguousarray(mesh.n, dtype=np.int32)
        self._ilo = np.ascontiguousarray(mesh.ilo, dtype=np.int32).reshape(-1)
        m = _Mesh()
        m.nb = mesh.nb
        m.level = self._level.ctypes.data_as(C.POINTER(C.c_int32))
        m.n = self._n.ctypes.data_as(C.POINTER(C.c_int32))
        m.ilo = self._ilo.ctypes.data_as(C.POINTER(C.c_int32))
        m.g = mesh.g
        m.nroot = (C.c_int32 * 3)(*mesh.nroot)
        m.bc = mesh.bc
        m.lo = (C.c_double * 3)(*mesh.lo)
        m.dx0 = mesh.dx0
        self.c = m
        g = mesh.g
        self.E = [int(n) + 2 * g for n in mesh.n]
        self.off = np.concatenate([[0], np.cumsum([NF * E ** 3 for E in self.E])]).astype(np.int64)
        self.ioff = np.concatenate([[0], np.cumsum([NF * int(n) ** 3 for n in mesh.n])]).astype(np.int64)

    @property
    def size(self) -> int:
        return int(self.off[-1])

    def block_view(self, u: np.ndarray, b: int) -> np.ndarray:
        E = self.E[b]
        return u[self.off[b]:self.off[b + 1]].reshape(NF, E, E, E)

    def scatter(self, interiors) -> np.ndarray:
        """Register from per-block interior arrays; ghosts set to NaN."""
        u = np.full(self.size, np.nan)
        g = self.mesh.g
        for b, a in enumerate(interiors):
            n = int(self.mesh.n[b])
            self.block_view(u, b)[:, g:g + n, g:g + n, g:g + n] = a
        return u

    def scatter_ghosted(self, blocks) -> np.ndarray:
        """Register from per-block arrays that include the ghost layers."""
        u = np.empty(self.size)
        for b, a in enumerate(blocks):
            self.block_view(u, b)[...] = a
        return u

    def interiors(self, u: np.ndarray):
        g = self.mesh.g
        out = []
        for b in range(self.mesh.nb):
            n = int(self.mesh.n[b])
            out.append(self.block_view(u, b)[:, g:g + n, g:g + n, g:g + n].copy())
        return out

    def split_interior(self, r: np.ndarray, ncomp: int = NF):
        out = []
        o = 0
        for b in range(self.mesh.nb):
            n = int(self.mesh.n[b])
            out.append(r[o:o + ncomp * n ** 3].reshape(ncomp, n, n, n))
            o += ncomp * n ** 3
        return out


def make_params(p: dict) -> _Params:
    q = _Params()
    q.fd_order = int(p["fd_order"])
    q.terms = int(p.get("terms", 0xF))
    q.enforce = int(p.get("enforce", 1))
    for k in ("ko_sigma", "kappa1", "kappa2", "eta", "mu_S", "chi_floor", "alpha_floor"):
        setattr(q, k, float(p[k]))
    return q


def fd_weights(deriv: int, pts) -> np.ndarray:
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    w = np.zeros(len(pts))
    rc = lib().or_fd_weights(deriv, len(pts), _dp(pts), _dp(w))
    if rc:
        raise ValueError("bad stencil request")
    return w


def fill_ghosts(om: OracleMesh, u: np.ndarray, threads: int = 1) -> None:
    """Ghost fill of every block of u; with threads > 1 disjoint block sets
    are filled in host threads from one copy of u (same values)."""
    if threads <= 1:
        rc = lib().or_fill_ghosts(C.byref(om.c), _dp(u))
        if rc:
            raise RuntimeError(f"oracle ghost fill failed ({rc})")
        return
    import concurrent.futures as cf
    src = u.copy()
    # ghost-heavy blocks are the small ones: balance by ghost count
    nb, g = om.mesh.nb, om.mesh.g
    load = [0] * threads
    masks = [np.zeros(nb, np.int8) for _ in range(threads)]
    ghosts = [(int(n) + 2 * g) ** 3 - int(n) ** 3 for n in om.mesh.n]
    for b in sorted(range(nb), key=lambda b: -ghosts[b]):
        t = int(np.argmin(load))
        masks[t][b] = 1
        load[t] += ghosts[b]

    def work(mask):
        return lib().or_fill_ghosts_from(C.byref(om.c), _dp(src), _dp(u),
                                         mask.ctypes.data_as(C.POINTER(C.c_int8)))
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        rcs = list(ex.map(work, [m for m in masks if m.any()]))
    if any(rcs):
        raise RuntimeError(f"oracle ghost fill failed ({rcs})")


def _thread_masks(om: OracleMesh, blocks, threads: int):
    """Block masks for `threads` host threads, balanced by zones."""
    nb = om.mesh.nb
    sel = range(nb) if blocks is None else sorted(set(int(b) for b in blocks))
    load = [0] * threads
    masks = [np.zeros(nb, np.int8) for _ in range(threads)]
    for b in sorted(sel, key=lambda b: -int(om.mesh.n[b])):
        t = int(np.argmin(load))
        masks[t][b] = 1
        load[t] += int(om.mesh.n[b]) ** 3
    return [m for m in masks if m.any()]


def rhs(om: OracleMesh, params: dict, u: np.ndarray, fill: bool = True, blocks=None,
        threads: int = 1):
    """Per-block RHS interiors (22, n, n, n); fills ghosts of u first.  With
    `blocks`, only those blocks are computed (the others stay zero); with
    threads > 1 disjoint block sets run in host threads (same arithmetic)."""
    import concurrent.futures as cf
    if fill:
        fill_ghosts(om, u, threads)
    r = np.zeros(int(om.ioff[-1]))
    prm = make_params(params)
    if threads <= 1 and blocks is None:
        masks = [None]
    else:
        masks = _thread_masks(om, blocks, max(1, threads))

    def work(mask):
        only = None if mask is None else mask.ctypes.data_as(C.POINTER(C.c_int8))
        return lib().or_rhs_blocks(C.byref(om.c), C.byref(prm), _dp(u), _dp(r), only)
    with cf.ThreadPoolExecutor(max_workers=max(1, len(masks))) as ex:
        rcs = list(ex.map(work, masks))
    if any(rcs):
        raise RuntimeError(f"oracle rhs failed ({rcs})")
    return om.split_interior(r)


class Registers:
    """U, S1, S2, A registers for the RK4 stages."""

    def __init__(self, om: OracleMesh, interiors):
        self.om = om
        self.U = om.scatter(interiors)
        self.S1 = np.full(om.size, np.nan)
        self.S2 = np.full(om.size, np.nan)
        self.A = np.full(om.size, np.nan)


def rk4_stage(regs: Registers, params: dict, stage: int, dt: float) -> None:
    rc = lib().or_rk4_stage(C.byref(regs.om.c), C.byref(make_params(params)), stage, dt,
                            _dp(regs.U), _dp(regs.S1), _dp(regs.S2), _dp(regs.A))
    if rc:
        raise RuntimeError(f"oracle rk4 stage failed ({rc})")


def rk4_steps(regs: Registers, params: dict, dt: float, nsteps: int, threads: int = 1) -> None:
    """nsteps classic RK4 steps.  With threads > 1 each stage's RHS and
    register update run on disjoint block sets in host threads (the same
    per-zone arithmetic; the ghost fill stays serial)."""
    for _ in range(nsteps):
        for s in (1, 2, 3, 4):
            if threads > 1:
                rk4_stage_threaded(regs, params, s, dt, threads)
            else:
                rk4_stage(regs, params, s, dt)


def rk4_stage_threaded(regs: Registers, params: dict, stage: int, dt: float, threads: int) -> None:
    import concurrent.futures as cf
    om = regs.om
    src = {1: regs.U, 2: regs.S1, 3: regs.S2, 4: regs.S1}[stage]
    fill_ghosts(om, src, threads)
    k = np.zeros(int(om.ioff[-1]))
    prm = make_params(params)
    masks = _thread_masks(om, None, threads)

    def work(mask):
        mp = mask.ctypes.data_as(C.POINTER(C.c_int8))
        rc = lib().or_rhs_blocks(C.byref(om.c), C.byref(prm), _dp(src), _dp(k), mp)
        if rc == 0:
            rc = lib().or_rk4_update(C.byref(om.c), C.byref(prm), stage, dt, _dp(k), _dp(regs.U),
                                     _dp(regs.S1), _dp(regs.S2), _dp(regs.A), mp)
        return rc

    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        rcs = list(ex.map(work, masks))
    if any(rcs):
        raise RuntimeError(f"oracle rk4 stage failed ({rcs})")


def constraints(om: OracleMesh, params: dict, u: np.ndarray, exclude=(), r_exc: float = 0.0,
                fill: bool = True, per_zone: bool = True):
    """Returns (per-block (8, n, n, n) arrays of H, M^i, Theta, G^i; norms[6])."""
    if fill:
        fill_ghosts(om, u)
    out = np.zeros(int(om.ioff[-1]) // NF * 8) if per_zone else None
    exc = np.ascontiguousarray(np.array(exclude, dtype=np.float64).reshape(-1))
    if exc.size == 0:
        exc = np.zeros(3)
    norms = np.zeros(6)
    rc = lib().or_constraints(C.byref(om.c), C.byref(make_params(params)), _dp(u),
                              _dp(out) if per_zone else None, len(exclude), _dp(exc), r_exc,
                              _dp(norms))
    if rc:
        raise RuntimeError(f"oracle constraints failed ({rc})")
    return (om.split_interior(out, 8) if per_zone else None), norms


CRIT_CHI_MIN, CRIT_DCHI_MAX, CRIT_RADIUS = 0, 1, 2


def psi4(om: OracleMesh, params: dict, u: np.ndarray, origin=(0.0, 0.0, 0.0), fill: bool = True):
    """Per-block (2, n, n, n) Re/Im Psi4 in the coordinate tetrad about
    `origin` (ghosts of u filled first unless fill is False)."""
    if fill:
        fill_ghosts(om, u)
    nz = sum(int(n) ** 3 for n in om.mesh.n)
    out = np.zeros(2 * nz)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    rc = lib().or_psi4(C.byref(om.c), C.byref(make_params(params)), _dp(u), _dp(o), _dp(out))
    if rc:
        raise RuntimeError(f"oracle psi4 failed ({rc})")
    return om.split_interior(out, 2)


def block_features(om: OracleMesh, params: dict, u: np.ndarray, fill: bool = True) -> np.ndarray:
    """(nb, 16) raw per-block features (see features.c)."""
    if fill:
        fill_ghosts(om, u)
    out = np.zeros((om.mesh.nb, 16))
    rc = lib().or_block_features(C.byref(om.c), C.byref(make_params(params)), _dp(u), _dp(out))
    if rc:
        raise RuntimeError(f"oracle features failed ({rc})")
    return out


def refine_flags(om: OracleMesh, params: dict, u: np.ndarray, criterion: int, chi_thr=0.3,
                 dchi_thr=0.1, level_max=10, radius=0.0, centre=(0.0, 0.0, 0.0),
                 radius_level=0, fill: bool = True) -> np.ndarray:
    if fill:
        fill_ghosts(om, u)
    flags = np.zeros(om.mesh.nb, np.int8)
    c = np.ascontiguousarray(centre, dtype=np.float64)
    rc = lib().or_refine_flags(C.byref(om.c), C.byref(make_params(params)), _dp(u), criterion,
                               chi_thr, dchi_thr, level_max, radius, _dp(c), radius_level,
                               flags.ctypes.data_as(C.POINTER(C.c_int8)))
    if rc:
        raise RuntimeError(f"oracle flags failed ({rc})")
    return flags
