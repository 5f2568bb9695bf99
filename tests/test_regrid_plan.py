"""The library's regrid plan (z4c_regrid_plan, host code) against the
reference plan, exact block lists, on meshes and flag patterns that
exercise plain refinement, 2:1 spreading, merges and cancelled merges with
outflow and periodic boundaries.  Host only: no device memory is used."""
import numpy as np
import pytest

import z4c_inputs as zi
from oracle import regrid as rg


def lib_plan(mesh, flags, level_max, order=6):
    import paper_2409_10383_amd as z4c
    return z4c.regrid_plan(mesh, zi.params_default(order), np.asarray(flags, np.int8), level_max)


def base(bc, g=4):
    return zi.uniform_mesh((2, 2, 2), 8, g, (0.0,) * 3, (2.0,) * 3, bc)


def cases():
    for bc in (zi.BC_OUTFLOW, zi.BC_PERIODIC):
        m0 = base(bc)
        yield f"identity-{bc}", m0, np.zeros(m0.nb), 3
        yield f"refine-all-{bc}", m0, np.ones(m0.nb), 3
        m1 = zi.refine_blocks(m0, [0])
        f = np.zeros(m1.nb)
        f[7] = 1
        yield f"spread-{bc}", m1, f, 3
        m2 = zi.refine_blocks(zi.refine_blocks(m0, range(8)), [7])
        f = np.zeros(m2.nb)
        f[15:23] = -1
        yield f"cancel-{bc}", m2, f, 3
        f = -np.ones(m2.nb)
        yield f"merge-all-{bc}", m2, f, 3
        rng = np.random.default_rng(11 + bc)
        yield f"random-{bc}", m2, rng.integers(-1, 2, m2.nb), 3
        yield f"random-capped-{bc}", m2, rng.integers(-1, 2, m2.nb), 2


@pytest.mark.parametrize("name,mesh,flags,lmax", list(cases()), ids=[c[0] for c in cases()])
def test_plan_matches_reference(name, mesh, flags, lmax):
    got = lib_plan(mesh, flags, lmax)
    want = rg.plan(mesh, flags, lmax)
    assert np.array_equal(got.level, want.level), name
    assert np.array_equal(got.n, want.n), name
    assert np.array_equal(got.ilo, want.ilo), name
    assert rg.two_to_one_ok(got)


def test_plan_rejects_bad_flags_and_reports_size():
    import ctypes as C
    import paper_2409_10383_amd as z4c
    m = base(zi.BC_OUTFLOW)
    P = z4c.make_params(m, zi.params_default(6))
    h = C.c_void_p()
    assert z4c.lib().z4c_pack_create(C.byref(P), z4c.make_blocks(m), m.nb, C.byref(h)) == 0
    try:
        n = C.c_int32()
        bad = np.full(m.nb, 2, np.int8)
        assert z4c.lib().z4c_regrid_plan(h, bad.ctypes.data_as(C.POINTER(C.c_int8)), 3, None, 0,
                                         C.byref(n)) == -1
        ones = np.ones(m.nb, np.int8)
        out = (z4c.Block * 4)()
        rc = z4c.lib().z4c_regrid_plan(h, ones.ctypes.data_as(C.POINTER(C.c_int8)), 3, out, 4, C.byref(n))
        assert rc == -2 and n.value == 64
    finally:
        z4c.lib().z4c_pack_destroy(h)
