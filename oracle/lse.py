"""Two-pass log-sum-exp over an implicit squared-Euclidean cost, FP64.

Test infrastructure only (see the package docstring).

The LSE operator of Algorithm 1 reduces over the columns of its matrix
argument, [LSE(M)]_p = log sum_q exp(M_pq); the column update applies the same
operator to the transposed cost (Sec. 3.5, "Algorithm and Log-Domain
Execution").  Here each output is computed the plain way the stable
evaluation of Algorithm 2 does it: first the maximum of the log weights, then
the sum of exp(weight - max), then max + log(sum).  Costs are recomputed from
the points, C_ij = s * ||x_i - y_j||^2, in FP64 from the FP32 coordinates
(upcast exactly), a block of rows at a time so memory stays linear.
"""
from __future__ import annotations

import numpy as np

TILE = 256


def cost_block(xb: np.ndarray, y: np.ndarray, s: float) -> np.ndarray:
    """C_ij = s * sum_d (x_id - y_jd)^2 for a block of rows, FP64 (Eq. 1 cost)."""
    xb = np.asarray(xb, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    acc = np.zeros((xb.shape[0], y.shape[0]))
    for d in range(xb.shape[1]):
        diff = xb[:, d, None] - y[None, :, d]
        acc += diff * diff
    return s * acc


def cost_matrix(x: np.ndarray, y: np.ndarray, s: float) -> np.ndarray:
    """Dense cost matrix (small problems only)."""
    return cost_block(x, y, s)


def lse_rows_of(W: np.ndarray) -> np.ndarray:
    """[LSE(W)]_p = log sum_q exp(W_pq), max first, then the shifted sum.

    A row whose weights are all -inf has LSE -inf (an empty sum).
    """
    M = W.max(axis=1)
    fin = np.isfinite(M)
    Ms = np.where(fin, M, 0.0)
    S = np.exp(W - Ms[:, None]).sum(axis=1)
    with np.errstate(divide="ignore"):
        out = Ms + np.log(S)
    return np.where(fin, out, M)


def implicit_lse(x: np.ndarray, y: np.ndarray, s: float, eps: float,
                 w: np.ndarray, rows: np.ndarray | None = None) -> np.ndarray:
    """out_i = LSE_j( w_j - C_ij / eps ) for every row i (or the listed rows).

    With (x, y, w) = (source points, target points, log t) this is the
    reduction of the row update of Algorithm 1; with the roles of the point
    sets swapped and w = log A it is the column update.
    """
    w = np.asarray(w, dtype=np.float64)
    idx = np.arange(x.shape[0]) if rows is None else np.asarray(rows)
    out = np.empty(idx.shape[0])
    for a in range(0, idx.shape[0], TILE):
        sel = idx[a:a + TILE]
        C = cost_block(x[sel], y, s)
        out[a:a + TILE] = lse_rows_of(w[None, :] - C / eps)
    return out
