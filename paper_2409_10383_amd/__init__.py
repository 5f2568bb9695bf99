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
# Z4C_LIB: load the library from another path (e.g. a variant build)
LIB_PATH = os.environ.get("Z4C_LIB", os.path.join(HERE, "libz4c.so"))

NF = 22
NREG = 4
REG_U, REG_S1, REG_S2, REG_A = 0, 1, 2, 3
BC_PERIODIC, BC_OUTFLOW, BC_USER = 0, 1, 2
FP64, FP32_MIXED = 0, 1
TERM_PHYS, TERM_GAUGE, TERM_ADVECT, TERM_DISSIP, TERM_ALL = 1, 2, 4, 8, 15
FLAG_ENFORCE, FLAG_CHECK_FINITE, FLAG_GRAPH = 1, 2, 4
CRIT_CHI_MIN, CRIT_DCHI_MAX, CRIT_RADIUS = 0, 1, 2
# tile shapes of the stage-kernel variants (x, y, z active cells per workgroup)
TILE_SHAPES = [(8, 8, 4), (16, 4, 4), (8, 4, 8), (16, 8, 2)]
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
                ("nwork", C.c_int32), ("nxfer", C.c_int64), ("nprolong", C.c_int64)]


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
           "z4c_profile", "z4c_profile_read", "z4c_features", "z4c_pack_inject_2h", "z4c_labels",
           "z4c_feature_stats", "z4c_mlp_normalize", "z4c_mlp_forward", "z4c_mlp_backward",
           "z4c_mlp_adam", "z4c_refine_flags_learned", "z4c_set_variant", "z4c_autotune",
           "z4c_regrid_plan", "z4c_regrid_transfer", "z4c_psi4", "z4c_interp", "z4c_interp_state",
           "z4c_swsh_project", "z4c_tracker_set", "z4c_tracker_get", "z4c_mlp_backward_noalloc", "z4c_autotune_cached"]
MLP_NPARAM = 5313


class MlpModel(C.Structure):
    _fields_ = [("params", C.c_void_p), ("stats", C.c_void_p), ("range", C.POINTER(C.c_double)),
                ("tau_ref", C.c_double), ("tau_deref", C.c_double), ("chi_thr", C.c_double),
                ("dchi_thr", C.c_double), ("level_max", C.c_int32), ("pad", C.c_int32)]

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
        L.z4c_features.argtypes = [vp, C.c_int32, vp, C.POINTER(C.c_double), vp]
        L.z4c_pack_inject_2h.argtypes = [vp, C.c_int32, vp, C.c_int32, vp]
        L.z4c_labels.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_double), vp]
        L.z4c_feature_stats.argtypes = [vp, C.c_int32, vp, vp]
        L.z4c_mlp_normalize.argtypes = [vp, C.c_int32, vp, vp, vp]
        L.z4c_mlp_forward.argtypes = [vp, vp, C.c_int32, vp, vp, vp]
        L.z4c_mlp_backward.argtypes = [vp, vp, vp, vp, vp, C.c_int32, vp, vp, vp, vp]
        L.z4c_mlp_backward_noalloc.argtypes = [vp, vp, vp, vp, vp, C.c_int32, vp, vp, vp]
        L.z4c_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float, C.c_float, C.c_float,
                                   C.c_float, vp]
        L.z4c_refine_flags_learned.argtypes = [vp, C.c_int32, C.POINTER(MlpModel),
                                               C.POINTER(C.c_int8), C.POINTER(C.c_int8), vp]
        L.z4c_set_variant.argtypes = [vp, C.c_int32, C.c_int32, vp]
        L.z4c_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32), vp]
        L.z4c_autotune_cached.argtypes = [vp, C.c_char_p, C.c_int32, C.POINTER(C.c_double),
                                          C.POINTER(C.c_int32), C.POINTER(C.c_int32), vp]
        L.z4c_regrid_plan.argtypes = [vp, C.POINTER(C.c_int8), C.c_int32, C.POINTER(Block), C.c_int32,
                                      C.POINTER(C.c_int32)]
        L.z4c_regrid_transfer.argtypes = [vp, C.c_int32, vp, C.c_int32, vp]
        dp = C.POINTER(C.c_double)
        L.z4c_psi4.argtypes = [vp, C.c_int32, dp, vp, vp]
        L.z4c_interp.argtypes = [vp, vp, C.c_int32, vp, C.c_int32, vp, vp]
        L.z4c_interp_state.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp, C.c_int32, vp, vp]
        L.z4c_swsh_project.argtypes = [vp, vp, vp, C.c_int32, dp, C.c_int32, vp, vp]
        L.z4c_tracker_set.argtypes = [vp, C.c_int32, dp, vp]
        L.z4c_tracker_get.argtypes = [vp, dp, vp]
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
    q.flags = ((FLAG_ENFORCE if int(p.get("enforce", 1)) else 0) | (FLAG_GRAPH if p.get("graph") else 0)
               | (FLAG_CHECK_FINITE if p.get("check_finite") else 0))
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

    def rebind(self, stream=None):
        """Move the pack to freshly allocated registers and workspace (their
        contents copied over) through z4c_pack_bind."""
        import torch
        self.regs = [t.clone() for t in self.regs]
        self.workspace = self.workspace.clone()
        torch.cuda.synchronize()
        ptrs = (C.c_void_p * NREG)(*[t.data_ptr() for t in self.regs])
        self._check(lib().z4c_pack_bind(self.h, ptrs, C.c_void_p(self.workspace.data_ptr()),
                                        self.workspace.numel(), _stream_ptr(stream)))

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

    def psi4(self, reg: int = REG_U, origin=(0.0, 0.0, 0.0), out=None, stream=None):
        """z4c_psi4: device tensor, interior layout with 2 components (Re, Im)."""
        import torch
        if out is None:
            out = torch.empty(2 * self.zones, dtype=torch.float64, device=self.regs[0].device)
        o = (C.c_double * 3)(*origin)
        self._check(lib().z4c_psi4(self.h, reg, o, C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def _points(self, points):
        import torch
        p = torch.as_tensor(np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3),
                            device=self.regs[0].device)
        return p, int(p.shape[0])

    def interp(self, src, ncomp: int, points, stream=None):
        """z4c_interp of an interior-layout device tensor at points -> (npts, ncomp)."""
        import torch
        p, npts = self._points(points)
        out = torch.empty(npts * ncomp, dtype=torch.float64, device=p.device)
        self._check(lib().z4c_interp(self.h, C.c_void_p(src.data_ptr()), ncomp, C.c_void_p(p.data_ptr()),
                                     npts, C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out.cpu().numpy().reshape(npts, ncomp)

    def interp_state(self, reg: int, first: int, nfield: int, points, stream=None):
        """z4c_interp_state: fields first..first+nfield-1 of `reg` at points."""
        import torch
        p, npts = self._points(points)
        out = torch.empty(npts * nfield, dtype=torch.float64, device=p.device)
        self._check(lib().z4c_interp_state(self.h, reg, first, nfield, C.c_void_p(p.data_ptr()), npts,
                                           C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out.cpu().numpy().reshape(npts, nfield)

    def tracker_set(self, positions, stream=None):
        pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
        self._check(lib().z4c_tracker_set(self.h, pos.shape[0], pos.ctypes.data_as(C.POINTER(C.c_double)),
                                          _stream_ptr(stream)))
        self._ntrack = pos.shape[0]

    def tracker_get(self, stream=None):
        n = getattr(self, "_ntrack", 0)
        pos = np.zeros((max(n, 1), 3))
        self._check(lib().z4c_tracker_get(self.h, pos.ctypes.data_as(C.POINTER(C.c_double)), _stream_ptr(stream)))
        return pos[:n]

    def set_variant(self, variant: int, persistent: bool = False, stream=None):
        self._check(lib().z4c_set_variant(self.h, variant, 1 if persistent else 0, _stream_ptr(stream)))

    def autotune(self, reps: int = 3, stream=None, cache: str | None = None):
        """Time every tile shape / launch mode; keep the fastest.  Returns
        (chosen index, times in ms per RHS launch indexed 2*variant+persistent).
        With `cache` (a file path) a stored winner for this configuration is
        applied without timing (times then all -1) and new winners stored."""
        t = (C.c_double * 8)()
        ch = C.c_int32()
        if cache is None:
            self._check(lib().z4c_autotune(self.h, reps, t, C.byref(ch), _stream_ptr(stream)))
        else:
            hit = C.c_int32()
            self._check(lib().z4c_autotune_cached(self.h, os.fsencode(cache), reps, t, C.byref(ch),
                                                  C.byref(hit), _stream_ptr(stream)))
            self.tuned_from_cache = bool(hit.value)
        return int(ch.value), np.array(t[:])

    def regrid_plan(self, flags, level_max: int):
        """The mesh z4c_regrid_plan makes from per-block flags (+1 refine,
        -1 derefine, 0 keep): a z4c_inputs.Mesh on the same domain."""
        return _plan(self.h, self.mesh, flags, level_max)

    def regrid(self, flags, level_max: int, reg: int = REG_U, stream=None) -> "Pack":
        """A new pack on the regridded mesh whose U holds register `reg` of
        this one, carried over by z4c_regrid_transfer (fills this pack's
        ghosts of `reg` first)."""
        new = Pack(self.regrid_plan(flags, level_max), self.params, self.precision)
        self._check(lib().z4c_regrid_transfer(self.h, reg, new.h, REG_U, _stream_ptr(stream)))
        return new

    def profile(self, enable: bool = True):
        self._check(lib().z4c_profile(self.h, 1 if enable else 0))

    def profile_read(self, reset: bool = True):
        """(stage ms, stage launches, fill ms, fill launches, graph ms, graph
        launches) since the last reset."""
        out = (C.c_double * 6)()
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


# ---------------------------------------------------------------- regrid
def _plan(h, mesh, flags, level_max):
    import dataclasses
    f = np.ascontiguousarray(flags, dtype=np.int8)
    if f.shape != (mesh.nb,):
        raise ValueError("one flag per block")
    fp = f.ctypes.data_as(C.POINTER(C.c_int8))
    n = C.c_int32()
    rc = lib().z4c_regrid_plan(h, fp, level_max, None, 0, C.byref(n))
    if rc not in (0, -2):
        raise Z4cError(rc, "z4c_regrid_plan rejected its arguments")
    out = (Block * max(n.value, 1))()
    rc = lib().z4c_regrid_plan(h, fp, level_max, out, n.value, C.byref(n))
    if rc:
        raise Z4cError(rc, "z4c_regrid_plan")
    nb = n.value
    return dataclasses.replace(
        mesh,
        level=np.array([out[b].level for b in range(nb)], dtype=np.int32),
        n=np.array([out[b].n for b in range(nb)], dtype=np.int32),
        ilo=np.array([list(out[b].ilo) for b in range(nb)], dtype=np.int32).reshape(nb, 3))


def regrid_plan(mesh, params: dict, flags, level_max: int):
    """z4c_regrid_plan on a host-only pack of `mesh` (no device memory)."""
    P = make_params(mesh, params)
    h = C.c_void_p()
    rc = lib().z4c_pack_create(C.byref(P), make_blocks(mesh), mesh.nb, C.byref(h))
    if rc:
        raise Z4cError(rc, "z4c_pack_create rejected the pack description")
    try:
        return _plan(h, mesh, flags, level_max)
    finally:
        lib().z4c_pack_destroy(h)


def swsh_project(values, points, weights, centre, lmax: int, device: str = "cuda"):
    """z4c_swsh_project of complex values on a quadrature sphere:
    {(l, m): C_lm} for l = 2..lmax."""
    import torch
    v = np.asarray(values, dtype=complex)
    vals = torch.as_tensor(np.stack([v.real, v.imag], 1).reshape(-1).copy(), device=device)
    p = torch.as_tensor(np.ascontiguousarray(points, dtype=np.float64).reshape(-1), device=device)
    w = torch.as_tensor(np.ascontiguousarray(weights, dtype=np.float64), device=device)
    nm = (lmax + 1) ** 2 - 4
    out = torch.empty(2 * nm, dtype=torch.float64, device=device)
    c = (C.c_double * 3)(*centre)
    rc = lib().z4c_swsh_project(C.c_void_p(vals.data_ptr()), C.c_void_p(p.data_ptr()),
                                C.c_void_p(w.data_ptr()), int(w.shape[0]), c, lmax,
                                C.c_void_p(out.data_ptr()), None)
    if rc:
        raise Z4cError(rc, "z4c_swsh_project")
    o = out.cpu().numpy()
    res, q = {}, 0
    for l in range(2, lmax + 1):
        for m in range(-l, l + 1):
            res[(l, m)] = complex(o[2 * q], o[2 * q + 1])
            q += 1
    return res


# ---------------------------------------------------------------- learned part
def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _ok(rc, what):
    if rc:
        raise Z4cError(rc, what)


def features(pack: "Pack", reg: int = REG_U, device_out=None, stream=None):
    """(nb, 16) float64 features (numpy); optionally also into a device tensor."""
    out = np.zeros(pack.mesh.nb * 16)
    pack._check(lib().z4c_features(pack.h, reg, _ptr(device_out) if device_out is not None else None,
                                   out.ctypes.data_as(C.POINTER(C.c_double)), _stream_ptr(stream)))
    return out.reshape(pack.mesh.nb, 16)


def inject_2h(pack_h: "Pack", pack_2h: "Pack", reg_h: int = REG_U, reg_2h: int = REG_U, stream=None):
    pack_h._check(lib().z4c_pack_inject_2h(pack_h.h, reg_h, pack_2h.h, reg_2h, _stream_ptr(stream)))


def labels(pack_h: "Pack", rhs_h, pack_2h: "Pack", rhs_2h, stream=None):
    out = np.zeros(pack_h.mesh.nb)
    pack_h._check(lib().z4c_labels(pack_h.h, _ptr(rhs_h), pack_2h.h, _ptr(rhs_2h),
                                   out.ctypes.data_as(C.POINTER(C.c_double)), _stream_ptr(stream)))
    return out


MLP_SLICE = 64


def mlp_work_floats(B: int) -> int:
    """Floats of the backward pass's work buffer (Z4C_MLP_WORK)."""
    return B * 129 + (B + MLP_SLICE - 1) // MLP_SLICE * MLP_NPARAM


class Mlp:
    """Device state of the 16-64-64-1 indicator network (float32 master
    weights, Adam moments, feature statistics); all arithmetic in libz4c."""

    def __init__(self, init_params: np.ndarray, device: str = "cuda"):
        import torch
        self.device = device
        self.params = torch.tensor(np.asarray(init_params, np.float32), device=device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.stats = torch.zeros(64, dtype=torch.float64, device=device)
        self.step = 0

    def fit_stats(self, raw):
        """Feature statistics (mean, std, min, max of phi) from a device
        float64 tensor of raw features (B, 16)."""
        _ok(lib().z4c_feature_stats(_ptr(raw), raw.shape[0], _ptr(self.stats), _stream_ptr(None)),
            "feature stats")

    def normalize(self, raw):
        import torch
        X = torch.empty((raw.shape[0], 16), dtype=torch.float32, device=self.device)
        _ok(lib().z4c_mlp_normalize(_ptr(raw), raw.shape[0], _ptr(self.stats), _ptr(X),
                                    _stream_ptr(None)), "normalize")
        return X

    def forward(self, X, cache=None):
        import torch
        Y = torch.empty(X.shape[0], dtype=torch.float32, device=self.device)
        _ok(lib().z4c_mlp_forward(_ptr(self.params), _ptr(X), X.shape[0], _ptr(Y),
                                  _ptr(cache) if cache is not None else None, _stream_ptr(None)),
            "mlp forward")
        return Y

    def loss_grad(self, X, T):
        """Forward + backward: returns (Y, grad tensor, loss tensor)."""
        import torch
        B = X.shape[0]
        cache = torch.empty(B * 128, dtype=torch.float32, device=self.device)
        work = torch.empty(mlp_work_floats(B), dtype=torch.float32, device=self.device)
        Y = self.forward(X, cache)
        _ok(lib().z4c_mlp_backward(_ptr(self.params), _ptr(X), _ptr(Y), _ptr(T), _ptr(cache), B,
                                   _ptr(self.grad), _ptr(self.loss), _ptr(work), _stream_ptr(None)),
            "mlp backward")
        return Y, self.grad, self.loss

    def loss_grad_noalloc(self, X, T):
        """loss_grad through z4c_mlp_backward_noalloc (no work buffer)."""
        import torch
        B = X.shape[0]
        cache = torch.empty(B * 128, dtype=torch.float32, device=self.device)
        Y = self.forward(X, cache)
        _ok(lib().z4c_mlp_backward_noalloc(_ptr(self.params), _ptr(X), _ptr(Y), _ptr(T), _ptr(cache), B,
                                           _ptr(self.grad), _ptr(self.loss), _stream_ptr(None)),
            "mlp backward (no allocation)")
        return Y, self.grad, self.loss

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        _ok(lib().z4c_mlp_adam(_ptr(self.params), _ptr(self.grad), _ptr(self.m), _ptr(self.v),
                               self.step, lr, b1, b2, eps, _stream_ptr(None)), "adam")

    def train(self, X, T, epochs: int, lr=1e-3, batch: int = 0, seed: int = 0):
        """Full-batch (batch=0) or fixed mini-batch Adam; returns the final loss."""
        import torch
        B = X.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        for _ in range(epochs):
            if batch and batch < B:
                perm = torch.randperm(B, generator=g).to(X.device)
                for s in range(0, B - batch + 1, batch):
                    idx = perm[s:s + batch]
                    self.loss_grad(X[idx].contiguous(), T[idx].contiguous())
                    self.adam_step(lr)
            else:
                self.loss_grad(X, T)
                self.adam_step(lr)
        _, _, loss = self.loss_grad(X, T)
        return float(loss.item())


def refine_flags_learned(pack: "Pack", mlp: Mlp, phi_range: np.ndarray, tau_ref: float,
                         tau_deref: float, chi_thr=0.3, dchi_thr=0.1, level_max=10,
                         reg: int = REG_U, stream=None):
    md = MlpModel()
    md.params = mlp.params.data_ptr()
    md.stats = mlp.stats.data_ptr()
    rng = np.ascontiguousarray(phi_range, dtype=np.float64)
    md.range = rng.ctypes.data_as(C.POINTER(C.c_double))
    md.tau_ref, md.tau_deref, md.chi_thr, md.dchi_thr = tau_ref, tau_deref, chi_thr, dchi_thr
    md.level_max = level_max
    flags = (C.c_int8 * pack.mesh.nb)()
    fb = (C.c_int8 * pack.mesh.nb)()
    pack._check(lib().z4c_refine_flags_learned(pack.h, reg, C.byref(md), flags, fb, _stream_ptr(stream)))
    return np.array(flags[:], np.int8), np.array(fb[:], np.int8)
