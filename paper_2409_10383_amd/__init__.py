"""Z4c numerical-relativity hot path for MI355X (gfx950).

Thin Python binding of libz4c.so (include/z4c.h): argument marshalling only.
Every step of the method runs in the library's HIP kernels; PyTorch provides
device memory and streams.  Importing the package does not load the library;
the first call does, and raises if it is missing (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libz4c.so")

NF = 22
NREG = 4
REG_U, REG_S1, REG_S2, REG_A = 0, 1, 2, 3
BC_PERIODIC, BC_OUTFLOW, BC_USER = 0, 1, 2
FP64, FP32_MIXED = 0, 1
TERM_PHYS, TERM_GAUGE, TERM_ADVECT, TERM_DISSIP, TERM_ALL = 1, 2, 4, 8, 15
FLAG_ENFORCE, FLAG_CHECK_FINITE = 1, 2
CRIT_CHI_MIN, CRIT_DCHI_MAX, CRIT_RADIUS = 0, 1, 2
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "ENONFINITE",
          -6: "EUNSUPPORTED"}


class Z4cError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"z4c error {code} ({STATUS.get(code, '?')}): {msg}")
        self.code = code


class Block(C.Structure):
    _fields_ = [("level", C.c_int32), ("n", C.c_int32), ("ilo", C.c_int32 * 3)]


class Params(C.Structure):
    _fields_ = [("fd_order", C.c_int32), ("nghost", C.c_int32), ("precision", C.c_int32),
                ("bc", C.c_int32), ("nroot", C.c_int32 * 3), ("pad0", C.c_int32),
                ("lo", C.c_double * 3), ("dx0", C.c_double), ("ko_sigma", C.c_double),
                ("kappa1", C.c_double), ("kappa2", C.c_double), ("eta", C.c_double),
                ("mu_S", C.c_double), ("chi_floor", C.c_double), ("alpha_floor", C.c_double),
                ("terms", C.c_uint32), ("flags", C.c_uint32)]


class Layout(C.Structure):
    _fields_ = [("reg_bytes", C.c_size_t * 4), ("workspace_bytes", C.c_size_t),
                ("nblocks", C.c_int64), ("zones", C.c_int64), ("state_elem_bytes", C.c_int32),
                ("nwork", C.c_int32)]


class NormRegion(C.Structure):
    _fields_ = [("ncentres", C.c_int32), ("pad", C.c_int32), ("centres", (C.c_double * 3) * 8),
                ("r_exc", C.c_double)]


class RefineParams(C.Structure):
    _fields_ = [("criterion", C.c_int32), ("level_max", C.c_int32), ("chi_thr", C.c_double),
                ("dchi_thr", C.c_double), ("radius", C.c_double), ("centre", C.c_double * 3),
                ("radius_level", C.c_int32), ("pad", C.c_int32)]


EXPORTS = ["z4c_pack_create", "z4c_pack_query", "z4c_block_offset", "z4c_pack_bind",
           "z4c_pack_destroy", "z4c_last_error", "z4c_fill_ghosts", "z4c_rhs", "z4c_rk4_stage",
           "z4c_rk4_step", "z4c_constraints", "z4c_refine_flags", "z4c_stencil_weights",
           "z4c_profile", "z4c_profile_read"]

_lib = None


def lib():
    """Load libz4c.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} missing: run __graft_entry__.build() "
                              "(python paper_2409_10383_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.z4c_pack_create.argtypes = [C.POINTER(Params), C.POINTER(Block), C.c_int32,
                                      C.POINTER(vp)]
        L.z4c_pack_query.argtypes = [vp, C.POINTER(Layout)]
        L.z4c_block_offset.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.z4c_pack_bind.argtypes = [vp, C.POINTER(vp), vp, C.c_size_t, vp]
        L.z4c_pack_destroy.argtypes = [vp]
        L.z4c_pack_destroy.restype = None
        L.z4c_last_error.argtypes = [vp]
        L.z4c_last_error.restype = C.c_char_p
        L.z4c_fill_ghosts.argtypes = [vp, C.c_int32, vp]
        L.z4c_rhs.argtypes = [vp, C.c_int32, vp, vp]
        L.z4c_rk4_stage.argtypes = [vp, C.c_int32, C.c_double, vp]
        L.z4c_rk4_step.argtypes = [vp, C.c_double, C.c_int32, vp]
        L.z4c_constraints.argtypes = [vp, C.c_int32, vp, C.POINTER(NormRegion),
                                      C.POINTER(C.c_double), vp]
        L.z4c_refine_flags.argtypes = [vp, C.c_int32, C.POINTER(RefineParams),
                                       C.POINTER(C.c_int8), vp]
        L.z4c_stencil_weights.argtypes = [C.c_int32, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.z4c_profile.argtypes = [vp, C.c_int32]
        L.z4c_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.c_int32]
        _lib = L
    return _lib


def make_params(mesh, p: dict, precision: int = FP64) -> Params:
    q = Params()
    q.fd_order = int(p["fd_order"])
    q.nghost = int(mesh.g)
    q.precision = int(precision)
    q.bc = int(mesh.bc)
    q.nroot = (C.c_int32 * 3)(*[int(v) for v in mesh.nroot])
    q.lo = (C.c_double * 3)(*[float(v) for v in mesh.lo])
    q.dx0 = float(mesh.dx0)
    for k in ("ko_sigma", "kappa1", "kappa2", "eta", "mu_S", "chi_floor", "alpha_floor"):
        setattr(q, k, float(p[k]))
    q.terms = int(p.get("terms", TERM_ALL))
    q.flags = FLAG_ENFORCE if int(p.get("enforce", 1)) else 0
    return q


def make_blocks(mesh):
    arr = (Block * mesh.nb)()
    for b in range(mesh.nb):
        arr[b].level = int(mesh.level[b])
        arr[b].n = int(mesh.n[b])
        arr[b].ilo = (C.c_int32 * 3)(*[int(v) for v in mesh.ilo[b]])
    return arr


def stencil_weights(fd_order: int):
    N = fd_order // 2
    d1 = (C.c_double * (N + 1))()
    d2 = (C.c_double * (N + 1))()
    lop = (C.c_double * (2 * N + 1))()
    rc = lib().z4c_stencil_weights(fd_order, d1, d2, lop)
    if rc:
        raise Z4cError(rc, "stencil weights")
    return np.array(d1[:]), np.array(d2[:]), np.array(lop[:])


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Pack:
    """A MeshBlockPack bound to torch-owned device registers and workspace."""

    def __init__(self, mesh, params: dict, precision: int = FP64, device: str = "cuda"):
        import torch
        self.mesh = mesh
        self.params = dict(params)
        self.precision = precision
        self._blocks = make_blocks(mesh)
        self._p = make_params(mesh, params, precision)
        h = C.c_void_p()
        rc = lib().z4c_pack_create(C.byref(self._p), self._blocks, mesh.nb, C.byref(h))
        if rc:
            raise Z4cError(rc, "z4c_pack_create rejected the pack description")
        self.h = h
        lay = Layout()
        self._check(lib().z4c_pack_query(self.h, C.byref(lay)))
        self.layout = lay
        self.zones = int(lay.zones)
        self.nwork = int(lay.nwork)
        self.sdtype = torch.float64 if precision == FP64 else torch.float32
        self.regs = []
        for r in range(NREG):
            nbytes = int(lay.reg_bytes[r])
            self.regs.append(torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device))
        self.workspace = torch.zeros(max(int(lay.workspace_bytes), 256), dtype=torch.uint8,
                                     device=device)
        ptrs = (C.c_void_p * NREG)(*[t.data_ptr() for t in self.regs])
        self._check(lib().z4c_pack_bind(self.h, ptrs, C.c_void_p(self.workspace.data_ptr()),
                                        self.workspace.numel(), _stream_ptr(None)))
        # per-block offsets
        self.soff, self.ioff = [], []
        for b in range(mesh.nb):
            so, io = C.c_int64(), C.c_int64()
            self._check(lib().z4c_block_offset(self.h, b, C.byref(so), C.byref(io)))
            self.soff.append(int(so.value))
            self.ioff.append(int(io.value))
        esz = 8 if precision == FP64 else 4
        self.slab = []
        for b in range(mesh.nb):
            E = int(mesh.n[b]) + 2 * mesh.g
            per = 256 // esz
            self.slab.append((E ** 3 + per - 1) // per * per)

    # ------------------------------------------------------------ helpers
    def _check(self, rc):
        if rc:
            msg = lib().z4c_last_error(self.h).decode() if getattr(self, "h", None) else ""
            raise Z4cError(rc, msg)

    def close(self):
        if getattr(self, "h", None):
            lib().z4c_pack_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state_view(self, reg: int):
        """Register `reg` (U, S1, S2) as a flat torch tensor of the state dtype."""
        return self.regs[reg].view(self.sdtype)

    def acc_view(self):
        import torch
        return self.regs[REG_A].view(torch.float64)

    def block_state(self, reg: int, b: int):
        """(22, E, E, E) view of block b in a state register (ghosts included)."""
        E = int(self.mesh.n[b]) + 2 * self.mesh.g
        t = self.state_view(reg)[self.soff[b]:self.soff[b] + NF * self.slab[b]]
        return t.view(NF, self.slab[b])[:, :E ** 3].view(NF, E, E, E)

    def upload(self, reg: int, interiors, ghosted: bool = False, fill_nan: bool = True):
        """Write per-block (22, n, n, n) interiors (or ghosted arrays)."""
        import torch
        g = self.mesh.g
        host = torch.full((self.state_view(reg).numel(),), float("nan") if fill_nan else 0.0,
                          dtype=self.sdtype)
        for b, a in enumerate(interiors):
            n = int(self.mesh.n[b])
            E = n + 2 * g
            blk = host[self.soff[b]:self.soff[b] + NF * self.slab[b]].view(NF, self.slab[b])
            blk = blk[:, :E ** 3].view(NF, E, E, E)
            src = torch.from_numpy(np.ascontiguousarray(a)).to(self.sdtype)
            if ghosted:
                blk[...] = src
            else:
                blk[:, g:g + n, g:g + n, g:g + n] = src
        self.state_view(reg).copy_(host.to(self.state_view(reg).device))

    def download(self, reg: int, ghosted: bool = False):
        """Per-block numpy float64 arrays of a state register."""
        g = self.mesh.g
        host = self.state_view(reg).cpu().double()
        out = []
        for b in range(self.mesh.nb):
            n = int(self.mesh.n[b])
            E = n + 2 * g
            blk = host[self.soff[b]:self.soff[b] + NF * self.slab[b]].view(NF, self.slab[b])
            blk = blk[:, :E ** 3].view(NF, E, E, E)
            out.append((blk if ghosted else blk[:, g:g + n, g:g + n, g:g + n]).numpy().copy())
        return out

    def split_interior(self, flat, ncomp: int = NF):
        """Per-block (ncomp, n, n, n) numpy arrays of an interior-layout tensor."""
        host = flat.cpu().numpy()
        out, o = [], 0
        for b in range(self.mesh.nb):
            n = int(self.mesh.n[b])
            out.append(host[o:o + ncomp * n ** 3].reshape(ncomp, n, n, n).copy())
            o += ncomp * n ** 3
        return out

    # ------------------------------------------------------------ ABI calls
    def fill_ghosts(self, reg: int = REG_U, stream=None):
        self._check(lib().z4c_fill_ghosts(self.h, reg, _stream_ptr(stream)))

    def rhs(self, src_reg: int = REG_U, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(NF * self.zones, dtype=torch.float64, device=self.regs[0].device)
        self._check(lib().z4c_rhs(self.h, src_reg, C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def profile(self, enable: bool = True):
        self._check(lib().z4c_profile(self.h, 1 if enable else 0))

    def profile_read(self, reset: bool = True):
        """(stage ms, stage launches, fill ms, fill launches) since the last reset."""
        out = (C.c_double * 4)()
        self._check(lib().z4c_profile_read(self.h, out, 1 if reset else 0))
        return tuple(out[:])

    def rk4_stage(self, stage: int, dt: float, stream=None):
        self._check(lib().z4c_rk4_stage(self.h, stage, dt, _stream_ptr(stream)))

    def rk4_step(self, dt: float, nsteps: int = 1, stream=None):
        self._check(lib().z4c_rk4_step(self.h, dt, nsteps, _stream_ptr(stream)))

    def constraints(self, reg: int = REG_U, per_zone: bool = True, exclude=(), r_exc=0.0,
                    stream=None):
        import torch
        out = None
        if per_zone:
            out = torch.empty(8 * self.zones, dtype=torch.float64, device=self.regs[0].device)
        region = NormRegion()
        region.ncentres = len(exclude)
        for e, c in enumerate(exclude):
            for d in range(3):
                region.centres[e][d] = float(c[d])
        region.r_exc = float(r_exc)
        norms = (C.c_double * 6)()
        self._check(lib().z4c_constraints(self.h, reg, C.c_void_p(out.data_ptr() if out is not None else 0),
                                          C.byref(region), norms, _stream_ptr(stream)))
        return out, np.array(norms[:])

    def refine_flags(self, reg: int = REG_U, criterion: int = CRIT_CHI_MIN, chi_thr=0.3,
                     dchi_thr=0.1, level_max=10, radius=0.0, centre=(0.0, 0.0, 0.0),
                     radius_level=0, stream=None):
        rp = RefineParams()
        rp.criterion = criterion
        rp.level_max = level_max
        rp.chi_thr = chi_thr
        rp.dchi_thr = dchi_thr
        rp.radius = radius
        rp.centre = (C.c_double * 3)(*centre)
        rp.radius_level = radius_level
        flags = (C.c_int8 * self.mesh.nb)()
        self._check(lib().z4c_refine_flags(self.h, reg, C.byref(rp), flags, _stream_ptr(stream)))
        return np.array(flags[:], dtype=np.int8)
