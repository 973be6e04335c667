"""The state plan of Dual (O-)BDRS and what the experiments read from it, FP64.

Test infrastructure only (see the package docstring).

After k finished iterations the scalings alpha^{k-1}, beta^{k-1} of Algorithm 1
define the state plan X^k = diag(alpha^{k-1}) K^{.lambda k} diag(beta^{k-1})
(the O-BDRS state of Prop. 2; Lemma 1 for lambda = 1), i.e. the entrywise
kernel power lambda k of K = exp(-C / eta), a Gibbs kernel at temperature
eta / (lambda k).  It is never formed: its row and column sums are
log-sum-exp reductions, and the colour-transfer experiments read from it

* the marginal errors of their accuracy tables (l1, largest absolute and
  largest relative error of X 1 against r and of X^T 1 against c), and
* the barycentric projection y^_i = sum_j X_ij y_j / sum_j X_ij of the
  source points onto the target points (the "implicit implementation and
  output" paragraph), in which alpha cancels.
"""
from __future__ import annotations

import numpy as np

from .lse import TILE, cost_block, implicit_lse, lse_rows_of


def plan_temperature(eta: float, lam: float, k_done: int) -> float:
    """Temperature of K^{.lambda k}: exp(-lambda k C / eta) = exp(-C / (eta / (lambda k)))."""
    return eta / (lam * k_done)


def row_marginal(x, y, s, eps, la, lb):
    """(X 1)_i = alpha_i sum_j K_ij beta_j = exp(log alpha_i + LSE_j(log beta_j - C_ij / eps))."""
    return np.exp(np.asarray(la, dtype=np.float64) + implicit_lse(x, y, s, eps, lb))


def col_marginal(x, y, s, eps, la, lb):
    """(X^T 1)_j = beta_j sum_i K_ij alpha_i (the same reduction over the rows)."""
    return np.exp(np.asarray(lb, dtype=np.float64) + implicit_lse(y, x, s, eps, la))


def barycentric(x, y, s, eps, lb, rows=None):
    """y^_i = sum_j X_ij y_j / sum_j X_ij with X_ij proportional to beta_j K_ij.

    Per block of rows the normalised weights of each row are formed from the
    log weights log beta_j - C_ij / eps (max first, as in the LSE), and the
    weighted mean of the target points is one matrix product.
    """
    lb = np.asarray(lb, dtype=np.float64)
    yd = np.asarray(y, dtype=np.float64)
    idx = np.arange(x.shape[0]) if rows is None else np.asarray(rows)
    out = np.empty((idx.shape[0], yd.shape[1]))
    for a in range(0, idx.shape[0], TILE):
        sel = idx[a:a + TILE]
        W = lb[None, :] - cost_block(x[sel], y, s) / eps
        W = np.exp(W - lse_rows_of(W)[:, None])      # each row sums to 1
        out[a:a + TILE] = W @ yd
    return out


def marginal_stats(row, col, r, c) -> dict:
    """The marginal-error statistics of the colour-transfer accuracy tables."""
    er = np.abs(np.asarray(row) - np.asarray(r))
    ec = np.abs(np.asarray(col) - np.asarray(c))
    return dict(row_l1=float(er.sum()), col_l1=float(ec.sum()),
                row_max_abs=float(er.max()), col_max_abs=float(ec.max()),
                row_max_rel=float((er / np.asarray(r)).max()),
                col_max_rel=float((ec / np.asarray(c)).max()),
                mass=float(np.sum(row)))
