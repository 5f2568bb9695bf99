"""Shared comparison helpers for the GPU-vs-oracle parity tests.

Two bars, both at 1e-12 in FP64:
  field: outputs computed from identical inputs (RHS, constraints): the
         error of every field relative to that field's own max |value|.
  rounding: RHS values that are small residuals of large cancelling terms
         (constraint-satisfying puncture data at t = 0, where d_t Theta is
         proportional to H ~ 0): |g - o| <= 1e-12 max|o| + K u64 S W2 / h^2,
         the FP64 rounding floor of a second derivative of O(1) fields
         (u64 = 2^-53, S = largest |value| of the O(1) fields, W2 = sum of
         |w| of the second-derivative stencil, h the finest spacing, K = 64).
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


W2 = {4: 2 * (4 / 3 + 1 / 12) + 5 / 2, 6: 2 * (3 / 2 + 3 / 20 + 1 / 90) + 49 / 18,
      8: 2 * (8 / 5 + 1 / 5 + 8 / 315 + 1 / 560) + 205 / 72}


def assert_parity(gpu_blocks, ora_blocks, tol=TOL_FP64, what="", mode="field", S=1.0, order=6,
                  h=1.0):
    rel, num, den = field_errors(gpu_blocks, ora_blocks)
    if mode == "state":
        rel = num / max(den.max(), 1e-300)
    if mode == "rounding":
        floor = 64 * 2.0 ** -53 * S * W2[order] / h ** 2
        rel = num / (den + floor / tol)
    bad = np.where(~(rel <= tol))[0]
    assert bad.size == 0, f"{what}: fields {bad.tolist()} rel err {rel[bad]} (abs {num[bad]}, scale {den[bad]})"
    return rel
