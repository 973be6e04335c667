"""Primal-dual certificate of Proposition 3, evaluated as in Algorithm 2. FP64.

Test infrastructure only (see the package docstring).

Inputs are the scalings of the table in Sec. 3.4 ("Scalings shared by both
methods"): A = alpha-hat^k (a^k for BDRS), B = beta-hat^k (b^k), t =
beta-tilde^{k-1}, eps = eta / (lambda k + 1), all in natural-log form here.

* dual potentials f = eps log A, g = eps log(B / c)   (Prop. 3, Eq. for f, g)
* lower bound     L = <r, f> + <c, g>                  (Prop. 3)
* per column j (Algorithm 2): l_ij = log A_i - C_ij / eps, M_j = max_i l_ij,
  D_j = sum_i exp(l_ij - M_j), N_j = sum_i C_ij exp(l_ij - M_j),
  mu_j = N_j / D_j, d_j = M_j + log D_j, s_j = exp(log t_j + d_j)
* delta = 1/2 ||s - c||_1, U = sum_j s_j mu_j + Omega delta (Algorithm 2)
* relative gap (U - L) / U (experiments, "relative duality gap").

The upper bound only needs a plan Z = diag(A) K_eps diag(t) whose row sums
are r, i.e. A = r / (K_eps t) (the proof of Prop. 3 uses nothing else), and
the lower bound only a dual feasible pair: g is the soft c-transform of f at
the temperature of the column update.  The ablation variants, whose row and
column updates use different temperatures (or whose column update reads a
debiased row scaling), therefore take U from the row update (A, t, eps) and
L from the column update (its row scaling ``colw`` and temperature
``eps_col``); for Algorithm 1 both coincide.
"""
from __future__ import annotations

import numpy as np

from .lse import cost_block

TILE = 256


def column_statistics(x, y, s, eps, lah, cols=None):
    """(M_j, D_j, N_j) of Algorithm 2 for every column j (or the listed ones).

    Columns of the implicit cost are rows of the transposed cost, so the loop
    runs over blocks of target points y_j against all source points x_i.
    """
    lah = np.asarray(lah, dtype=np.float64)
    idx = np.arange(y.shape[0]) if cols is None else np.asarray(cols)
    M = np.empty(idx.shape[0])
    D = np.empty(idx.shape[0])
    N = np.empty(idx.shape[0])
    for a in range(0, idx.shape[0], TILE):
        sel = idx[a:a + TILE]
        Ct = cost_block(y[sel], x, s)            # (cols, m): C_ij transposed
        ell = lah[None, :] - Ct / eps            # l_ij for this block of columns
        Mj = ell.max(axis=1)
        E = np.exp(ell - Mj[:, None])
        M[a:a + TILE] = Mj
        D[a:a + TILE] = E.sum(axis=1)
        N[a:a + TILE] = (Ct * E).sum(axis=1)
    return M, D, N


def lower_bound(r, c, lah, lbh, eps):
    """L = <r, f> + <c, g> with f = eps log A and g = eps log(B / c) (Prop. 3)."""
    f = eps * np.asarray(lah, dtype=np.float64)
    g = eps * (np.asarray(lbh, dtype=np.float64) - np.log(c))
    return float(np.dot(r, f) + np.dot(c, g)), f, g


def certificate(x, y, s, r, c, lah, lbh, lt, eps, omega=1.0, colw=None, eps_col=None):
    """All quantities of Proposition 3 / Algorithm 2 for one iteration."""
    L, f, g = lower_bound(r, c, lah if colw is None else colw, lbh, eps if eps_col is None else eps_col)
    M, D, N = column_statistics(x, y, s, eps, lah)
    mu = N / D
    d = M + np.log(D)
    log_s = np.asarray(lt, dtype=np.float64) + d
    s_col = np.exp(log_s)
    delta = 0.5 * float(np.abs(s_col - c).sum())
    cost_Z = float(np.dot(s_col, mu))
    U = cost_Z + omega * delta
    gap = U - L
    rel = gap / U if U > 1e-300 else gap
    return dict(L=L, U=U, gap=gap, rel=rel, delta=delta, cost_Z=cost_Z,
                f=f, g=g, M=M, D=D, N=N, mu=mu, log_s=log_s, s=s_col, eps=eps)
