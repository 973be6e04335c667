"""Feasible repair of the intermediate plan (proof of Prop. 3, "Feasible primal repair"). FP64.

Test infrastructure only (see the package docstring).

Z = diag(A) K_eps diag(t) has row marginal r and column marginal s.  The
one-sided rounding clips over-full columns, e_j = min(1, c_j / s_j),
Z~ = Z diag(e), then spreads the deficits p = r - Z~ 1 and q = c - Z~^T 1 =
(c - s)_+ as Z^ = Z~ + p q^T / delta, which lies in Pi(r, c) and costs at
most <C, Z> + osc(C) delta.
"""
from __future__ import annotations

import numpy as np

from .lse import cost_block, cost_matrix, implicit_lse


def intermediate_plan(x, y, s, lah, lt, eps):
    """Dense Z_ij = A_i exp(-C_ij / eps) t_j (Sec. 3.4, the plan after the row update)."""
    C = cost_matrix(x, y, s)
    return np.exp(np.asarray(lah)[:, None] - C / eps + np.asarray(lt)[None, :]), C


def dense_repair(x, y, s, r, c, lah, lt, eps):
    """Returns dict(Z, Zhat, C, p, q, e, delta, cost_Z, cost_Zhat), dense (small n)."""
    Z, C = intermediate_plan(x, y, s, lah, lt, eps)
    s_col = Z.sum(axis=0)
    delta = 0.5 * float(np.abs(s_col - c).sum())
    e = np.minimum(1.0, c / s_col)
    Zt = Z * e[None, :]
    p = r - Zt.sum(axis=1)
    q = c - Zt.sum(axis=0)
    Zhat = Zt + (np.outer(p, q) / delta if delta > 0 else 0.0)
    return dict(Z=Z, Zhat=Zhat, C=C, p=p, q=q, e=e, delta=delta, s=s_col,
                cost_Z=float((C * Z).sum()), cost_Zhat=float((C * Zhat).sum()))


def implicit_repair(x, y, s, r, c, lah, lt, eps, s_col, mu):
    """Repaired cost <C, Z^> without forming any m x n matrix.

    <C, Z~> = sum_j e_j s_j mu_j (the clipped columns keep their mean cost);
    p_i = sum_j Z_ij (1 - e_j) = A_i sum_j K_ij t_j (1 - e_j), i.e. one more
    row reduction with log weights log t_j + log(1 - e_j); q_j = (c_j - s_j)_+;
    the correction costs p^T C q / delta, evaluated here by its plain
    definition over blocks of rows.
    """
    s_col = np.asarray(s_col, dtype=np.float64)
    e = np.minimum(1.0, c / s_col)
    q = np.maximum(c - s_col, 0.0)
    delta = 0.5 * float(np.abs(s_col - c).sum())
    one_minus_e = 1.0 - e
    with np.errstate(divide="ignore"):
        lw = np.asarray(lt, dtype=np.float64) + np.log(one_minus_e)
    p = np.exp(np.asarray(lah) + implicit_lse(x, y, s, eps, lw))
    pCq = 0.0
    for a in range(0, x.shape[0], 256):
        pCq += float(p[a:a + 256] @ (cost_block(x[a:a + 256], y, s) @ q))
    cost_clip = float(np.dot(e * s_col, mu))
    cost_hat = cost_clip + (pCq / delta if delta > 0 else 0.0)
    return dict(p=p, q=q, e=e, delta=delta, pCq=pCq, cost_clip=cost_clip,
                cost_Zhat=cost_hat)
