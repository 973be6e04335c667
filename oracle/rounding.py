"""Two-sided rounding of a positive plan onto Pi(r, c), FP64.

Test infrastructure only (see the package docstring).

The momentum / kernel ablation evaluates every method by the cost of a
feasible plan obtained with the rounding of Altschuler, Weed and Rigollet
(2017, "Near-linear time approximation algorithms for optimal transport via
Sinkhorn iteration", Algorithm 2), which for a positive matrix F is:

1. scale the rows down to r:   F' = diag(x) F,    x_i = min(1, r_i / (F 1)_i);
2. scale the columns down to c: F'' = F' diag(y), y_j = min(1, c_j / (F'^T 1)_j);
3. add the missing mass:        G = F'' + e_r e_c^T / ||e_r||_1,
   e_r = r - F'' 1 >= 0, e_c = c - F''^T 1 >= 0 (both of mass ||e_r||_1).

G lies in Pi(r, c), and ||G - F||_1 <= 2 (||F 1 - r||_1 + ||F^T 1 - c||_1)
(their Lemma 7).  Here F is the state plan X^k of Dual (O-)BDRS
(``plan.py``), so every step is an LSE reduction over the implicit cost, and
e_r^T C e_c has a closed form for the squared Euclidean cost.
"""
from __future__ import annotations

import numpy as np

from .lse import TILE, cost_block, implicit_lse


def dense_round(F, r, c):
    """Algorithm 2 of Altschuler et al. on a dense positive matrix; returns dict."""
    F = np.asarray(F, dtype=np.float64)
    x = np.minimum(1.0, r / F.sum(axis=1))
    F1 = x[:, None] * F
    y = np.minimum(1.0, c / F1.sum(axis=0))
    F2 = F1 * y[None, :]
    er = r - F2.sum(axis=1)
    ec = c - F2.sum(axis=0)
    mass = float(er.sum())
    G = F2 + (np.outer(er, ec) / mass if mass > 0 else 0.0)
    return dict(G=G, F2=F2, x=x, y=y, er=er, ec=ec, mass=mass)


def implicit_round(xp, yp, s, eps, la, lb, r, c):
    """<C, G> for F = diag(e^la) exp(-C / eps) diag(e^lb), without forming F.

    Returns dict(cost, cost_clipped = <C, F''>, mass = ||e_r||_1, x, y, er, ec).
    """
    la = np.asarray(la, dtype=np.float64)
    lb = np.asarray(lb, dtype=np.float64)
    # step 1: row sums of F and the row factors
    row = np.exp(la + implicit_lse(xp, yp, s, eps, lb))
    lx = np.log(np.minimum(1.0, r / row))
    # step 2: column sums of diag(x) F and the column factors
    col1 = np.exp(lb + implicit_lse(yp, xp, s, eps, la + lx))
    ly = np.log(np.minimum(1.0, c / col1))
    # step 3: row sums and cost of F'' = diag(x) F diag(y), one block of rows at a time
    wa = la + lx
    wb = lb + ly
    row2 = np.empty(xp.shape[0])
    cost2 = 0.0
    for a in range(0, xp.shape[0], TILE):
        C = cost_block(xp[a:a + TILE], yp, s)
        E = np.exp(wa[a:a + TILE, None] + wb[None, :] - C / eps)
        row2[a:a + TILE] = E.sum(axis=1)
        cost2 += float((E * C).sum())
    er = r - row2
    ec = c - np.exp(ly) * col1
    mass = float(er.sum())
    cross = 0.0
    if mass > 0:
        for a in range(0, xp.shape[0], TILE):
            C = cost_block(xp[a:a + TILE], yp, s)
            cross += float(er[a:a + TILE] @ C @ ec)
        cross /= mass
    return dict(cost=cost2 + cross, cost_clipped=cost2, mass=mass, x=np.exp(lx), y=np.exp(ly), er=er, ec=ec)
