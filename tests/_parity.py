"""Shared comparison helpers for the GPU-vs-oracle parity tests.

Two bars, both at 1e-12 in FP64:
  field: outputs computed from identical inputs (RHS, constraints): the
         error of every field relative to that field's own max |value|.
  state: evolved states (after RK stages/steps, whose inputs already differ
         by rounding): the relative L-infinity error of the whole state
         vector, max_f max|g_f - o_f| / max_f max|o_f|.  Rounding of the O(1)
         fields (2^-53) passes through second-derivative stencils
         (sum|w|/h^2) and dt into every field's increment, so a field whose
         values are far below the state scale (e.g. Theta ~ 1e-5) cannot be
         held to 1e-12 of its own magnitude by two different FP64 codes.
"""
import numpy as np

TOL_FP64 = 1e-12


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


def assert_parity(gpu_blocks, ora_blocks, tol=TOL_FP64, what="", mode="field"):
    rel, num, den = field_errors(gpu_blocks, ora_blocks)
    if mode == "state":
        rel = num / max(den.max(), 1e-300)
    bad = np.where(~(rel <= tol))[0]
    assert bad.size == 0, f"{what}: fields {bad.tolist()} rel err {rel[bad]} (abs {num[bad]}, scale {den[bad]})"
    return rel
