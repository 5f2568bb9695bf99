"""Shared comparison helpers for the GPU-vs-oracle parity tests.

The bar is per field f (over every active zone of every block):

    max |g_f - o_f|  <=  1e-12 * max |o_f|  +  floor_f

floor_f = 0 for outputs of identical inputs on smooth data (RHS, ghosts,
constraints): the plain relative bar of 1e-12 per field.

Where a field's own magnitude is far below what feeds it, two correct FP64
codes cannot agree to 1e-12 of that field's scale, and floor_f states by
how much they may differ.  Two cases:
  - evolved states (after RK stages / steps): every stage's update rounds
    each O(1) field (chi, g~_ii, alpha ~ 1) by up to half an ulp, and those
    differences pass through the second-derivative stencils (sum |w| / h^2)
    and dt into every field's next increment, including fields of size
    ~1e-5 (Theta, A~, beta);
  - right-hand sides that are small residuals of large cancelling terms
    (d_t Theta ~ H ~ 0 on constraint-satisfying puncture data).
floor_f is measured, by the oracle alone, as the sensitivity of that field
to rounding-level changes of the input: the same oracle computation is run
on the inputs with every value moved by one ulp up or down at random, and

    floor_f = K * max |o_f(inputs moved by one ulp) - o_f(inputs)|,  K = 16.

Each code returns the exact result of inputs within a few ulps (one rounding
per stage update and per stencil product; differences of neighbouring
values of smooth data are exact), so their difference is a few times this
one-ulp response; K = 16 covers two codes x four stages x two roundings.
No GPU value enters the floor.
"""
import os

import numpy as np

TOL_FP64 = 1e-12
K_ROUND = 16
# host threads for the oracle's RK4 driver (its per-block work split)
ORACLE_THREADS = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                            else (os.cpu_count() or 1)))


def field_errors(gpu_blocks, ora_blocks, nf=None):
    """Per-field max|g - o| and max|o| over all blocks."""
    nf = nf or gpu_blocks[0].shape[0]
    num = np.zeros(nf)
    den = np.zeros(nf)
    for g, o in zip(gpu_blocks, ora_blocks):
        d = np.abs(g - o).reshape(nf, -1).max(axis=1)
        m = np.abs(o).reshape(nf, -1).max(axis=1)
        num = np.maximum(num, d)
        den = np.maximum(den, m)
    return num / np.maximum(den, 1e-300), num, den


def ulp_perturbed(arrays, seed=20240910):
    """Every value moved by one ulp, up or down at random (seeded)."""
    rng = np.random.default_rng(seed)
    out = []
    for a in arrays:
        up = rng.random(a.shape) < 0.5
        out.append(np.where(up, np.nextafter(a, np.inf), np.nextafter(a, -np.inf)))
    return out


def rounding_floor(run, inputs, K=K_ROUND):
    """(run(inputs), per-field floor): K times the largest change of each
    output field when every input value moves by one ulp."""
    ref = run(inputs)
    print("[parity] oracle reference done; run on inputs moved by one ulp", flush=True)
    alt = run(ulp_perturbed(inputs))
    _, num, _ = field_errors(alt, ref)
    return ref, K * num


def assert_parity(gpu_blocks, ora_blocks, tol=TOL_FP64, what="", floor=None):
    """Per-field bar above; returns the per-field ratio of the error to the
    bar (<= 1 passes) and prints its largest value."""
    _, num, den = field_errors(gpu_blocks, ora_blocks)
    bound = tol * den + (0.0 if floor is None else np.asarray(floor))
    ratio = num / np.maximum(bound, 1e-300)
    bad = np.where(~(num <= bound))[0]
    print(f"[parity] {what}: worst field {int(np.argmax(ratio))} at {ratio.max():.3g} of the bar"
          + ("" if floor is None else f" (floors used on {int((np.asarray(floor) > tol * den).sum())} fields)"))
    assert bad.size == 0, (f"{what}: fields {bad.tolist()} err {num[bad]} > bar {bound[bad]} "
                           f"(scale {den[bad]})")
    return ratio


def oracle_steps(mesh, p, data, dt, nsteps, floor=True):
    """The oracle's U interiors after nsteps RK4 steps from `data`, and (with
    floor) the per-field rounding floor of that evolution."""
    import oracle

    def run(d):
        om = oracle.OracleMesh(mesh)
        regs = oracle.Registers(om, d)
        oracle.rk4_steps(regs, p, dt, nsteps, threads=ORACLE_THREADS)
        return om.interiors(regs.U)
    if not floor:
        return run(data), None
    return rounding_floor(run, data)


def oracle_rhs(mesh, p, data, blocks=None, floor=False):
    """The oracle's RHS interiors of `data` (ghosts filled by the oracle),
    optionally only on `blocks` (returned in that order), and (with floor)
    the per-field rounding floor of those values."""
    import oracle

    def run(d):
        om = oracle.OracleMesh(mesh)
        r = oracle.rhs(om, p, om.scatter(d), blocks=blocks)
        return r if blocks is None else [r[b] for b in blocks]
    if not floor:
        return run(data), None
    return rounding_floor(run, data)
