"""Comparison rules of the GPU parity tests (no test functions here).

Every parity check compares column by column, in two norms:
  - the relative 2-norm  ||g - r||_2 / ||r||_2  over all columns, and
  - the elementwise bound  max_i |g_i - r_i| / max_i |r_i|  per column,
so that one wrong block, level or interface segment cannot hide inside a
norm ratio.  A column whose reference is exactly zero must come back exactly
zero.
"""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_rel_cols(a, b):
    """max_i |a_i - b_i| / max_i |b_i| for each column (1-D input: one column)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.ndim == 1:
        a, b = a[:, None], b[:, None]
    out = []
    for j in range(b.shape[1]):
        scale = np.abs(b[:, j]).max() if b.shape[0] else 0.0
        err = np.abs(a[:, j] - b[:, j]).max() if b.shape[0] else 0.0
        out.append(0.0 if err == 0.0 else (np.inf if scale == 0.0 else float(err / scale)))
    return out


def assert_close(got, ref, tol, what="", elem_tol=None):
    """Both rules above, at the same tolerance unless elem_tol is given."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    r2 = rel(got, ref)
    cols = max_rel_cols(got, ref)
    assert r2 <= tol, f"{what}: relative 2-norm difference {r2:.3e} > {tol:.1e}"
    worst = int(np.argmax(cols))
    et = tol if elem_tol is None else elem_tol
    assert cols[worst] <= et, f"{what}: column {worst} elementwise difference {cols[worst]:.3e} > {et:.1e}"


def assert_converged_close(got, ref, tol, what=""):
    """Two solutions of the same system, each from a Krylov run stopped at
    ||r|| <= 1e-6 ||b|| (possibly one step apart).  They are not the same
    computation: they differ by the runs' final errors, A^{-1} r, which are
    bounded in norm by the stopping rule but can concentrate near strong
    coefficient jumps.  The 2-norm rule keeps `tol`; the elementwise rule
    allows ten times it."""
    assert_close(got, ref, tol, what, elem_tol=10 * tol)
