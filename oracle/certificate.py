"""Primal-dual certificate of Proposition 3, evaluated as in Algorithm 2. FP64.

Test infrastructure only (see the package docstring).

Inputs are the scalings the iteration has at hand (table of Sec. 3.4): the
unrelaxed row scaling A, the unrelaxed column scaling B, the column scaling t
the row update read, and that update's temperature eps, all in natural-log
form here.  They satisfy the two normalisations A = r / (K t) and
B = c / (K^T A) with K = exp(-C / eps).

* Lower bound: the potentials f = eps log A and g = eps log(B / c) form a
  feasible pair of the Kantorovich dual (g is the soft c-transform of f), so
  L = <r, f> + <c, g> <= p*.
* Upper bound: the plan Z = diag(A) K diag(t) has row sums r by the first
  normalisation; its column sums are s = c t / B.  Its cost plus Omega
  times the column mass that must move, delta = 1/2 ||s - c||_1, bounds the
  cost of a feasible repair of Z, hence p*: U = <C, Z> + Omega delta.
* Evaluation column by column (Algorithm 2): with the log terms
  l_ij = log A_i - C_ij / eps of column j, shifted by the column's largest
  one so that no exponential overflows or underflows to zero for the
  leading terms (App. E), the shifted mass D_j and shifted cost-weighted
  mass N_j give the mean cost mu_j = N_j / D_j of Z's column and the log of
  its mass, log s_j = log t_j + max_i l_ij + log D_j; then <C, Z> =
  sum_j s_j mu_j.
* Relative gap (U - L) / U (experiments, "relative duality gap").

The upper bound only needs a plan whose row sums are r, i.e. A = r / (K t)
(the proof of Prop. 3 uses nothing else), and the lower bound only a dual
feasible pair.  The ablation variants, whose row and column updates use
different temperatures (or whose column update reads a debiased row
scaling), therefore take U from the row update (A, t, eps) and L from the
column update (its row scaling ``colw`` and temperature ``eps_col``); for
Algorithm 1 both coincide.
"""
from __future__ import annotations

import numpy as np

from .lse import cost_block

TILE = 256


def column_statistics(x, y, s, eps, lah, cols=None, workers: int = 1):
    """(M_j, D_j, N_j) of Algorithm 2 for every column j (or the listed ones).

    Columns of the implicit cost are rows of the transposed cost, so the loop
    runs over blocks of target points y_j against all source points x_i.
    With workers > 1 the columns are split into chunks (multiples of the
    block size) evaluated by that many threads (NumPy releases the
    interpreter lock inside its array operations); every column's
    arithmetic is the same, so the result is identical.
    """
    lah = np.asarray(lah, dtype=np.float64)
    idx = np.arange(y.shape[0]) if cols is None else np.asarray(cols)
    if workers > 1 and idx.shape[0] > TILE:
        from concurrent.futures import ThreadPoolExecutor
        per = -(-idx.shape[0] // workers)
        per = -(-per // TILE) * TILE
        chunks = [idx[a:a + per] for a in range(0, idx.shape[0], per)]
        with ThreadPoolExecutor(len(chunks)) as ex:
            parts = list(ex.map(lambda c: column_statistics(x, y, s, eps, lah, c), chunks))
        return tuple(np.concatenate([p[i] for p in parts]) for i in range(3))
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


def certificate(x, y, s, r, c, lah, lbh, lt, eps, omega=1.0, colw=None, eps_col=None, workers: int = 1):
    """All quantities of Proposition 3 / Algorithm 2 for one iteration."""
    L, f, g = lower_bound(r, c, lah if colw is None else colw, lbh, eps if eps_col is None else eps_col)
    M, D, N = column_statistics(x, y, s, eps, lah, workers=workers)
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
