"""Error metrics used by the tests (test-side only).

J is symmetric positive semi-definite, so |J_ij| <= sqrt(J_ii J_jj); the
normalised error  e_J = max_ij |dJ_ij| / sqrt(J_ii J_jj)  is well defined even
for zero or sign-changing entries (p-type products), where a plain entrywise
relative error is not.
"""
import numpy as np


def e_J(J, J_ref):
    """Normalised error.  Entries whose reference diagonals vanish (a
    function that is zero on the whole grid) must match exactly."""
    J = np.asarray(J, dtype=np.float64)
    J_ref = np.asarray(J_ref, dtype=np.float64)
    d = np.sqrt(np.abs(np.diag(J_ref)))
    scale = np.outer(d, d)
    diff = np.abs(J - J_ref)
    zero = scale == 0
    err = np.where(zero, np.where(diff == 0, 0.0, np.inf), diff / np.where(zero, 1.0, scale))
    return float(np.max(err))


def e_J_block(Jblock, Jref_block, diag_rows, diag_cols):
    scale = np.sqrt(np.outer(np.abs(diag_rows), np.abs(diag_cols)))
    return float(np.max(np.abs(np.asarray(Jblock) - np.asarray(Jref_block)) / scale))


def entrywise_rel(J, J_ref, floor=1e-3):
    """Relative error over entries with |J_ij| >= floor * sqrt(J_ii J_jj)."""
    J = np.asarray(J)
    J_ref = np.asarray(J_ref)
    d = np.sqrt(np.abs(np.diag(J_ref)))
    mask = np.abs(J_ref) >= floor * np.outer(d, d)
    return float(np.max(np.abs(J - J_ref)[mask] / np.abs(J_ref[mask])))


def rel_fro(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
