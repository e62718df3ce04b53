"""Adjoint of x(A) = A^{-1} b for a loss L(x) (test infrastructure only).

For A x = b and a scalar loss L(x): solve A^T lambda = dL/dx, then
dL/dA_ij = -lambda_i x_j and dL/db = lambda. The chain to coefficient parameters theta
runs through the sparse Jacobian dA_e/dtheta_p of the problem's assembly. GaBP solves
A^T lambda = g on the transposed graph (A_ij and A_ji swapped), the same iteration as the
forward solve (Sec. 2.3 rules applied to A^T).
"""
from __future__ import annotations

import numpy as np

from . import gabp as _g


def nnz_gradient(rows, cols, lam, x):
    """G_e = dL/dA_e = -lambda_row(e) x_col(e) for every stored entry e."""
    return -np.asarray(lam)[rows] * np.asarray(x)[cols]


def reduce_to_params(G, jptr, jnnz, jw):
    """dL/dtheta_p = sum_k jw[k] G[jnnz[k]] over k in jptr[p]:jptr[p+1]."""
    jptr = np.asarray(jptr, dtype=np.int64)
    owner = np.repeat(np.arange(len(jptr) - 1), np.diff(jptr))
    return np.bincount(owner, weights=np.asarray(jw) * G[np.asarray(jnnz)],
                       minlength=len(jptr) - 1)


def dense_reference(a_dense, b, x_target, rows, cols, jac=None):
    """Dense-LU forward and adjoint for L = 0.5 ||x - x_target||^2."""
    x = np.linalg.solve(a_dense, b)
    gx = x - x_target
    lam = np.linalg.solve(a_dense.T, gx)
    G = nnz_gradient(rows, cols, lam, x)
    out = {"x": x, "lam": lam, "G": G, "loss": 0.5 * float(gx @ gx)}
    if jac is not None:
        out["dtheta"] = reduce_to_params(G, *jac)
    return out


def gabp_adjoint(g: _g.Graph, b, x_target, tol, max_sweeps, jac=None, check_every=1):
    """Forward GaBP solve, transposed GaBP solve, scatter to entries and parameters."""
    x, info_f, _, _ = _g.solve(g, b, tol, max_sweeps, check_every)
    gx = x - x_target
    gt = g.transposed()
    lam, info_b, _, _ = _g.solve(gt, gx, tol, max_sweeps, check_every)
    G = nnz_gradient(g.rows, g.cols, lam, x)
    out = {"x": x, "lam": lam, "G": G, "info": (info_f, info_b)}
    if jac is not None:
        out["dtheta"] = reduce_to_params(G, *jac)
    return out
