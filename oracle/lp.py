"""Exact optima p* of the unregularised problem (Eq. 1), for bracketing tests.

Test infrastructure only (see the package docstring).

* ``brute_force_uniform``: r = c = 1/n, the optimum is attained at a vertex
  of the Birkhoff polytope (a permutation matrix / n); enumerate n! of them.
* ``linprog_ot``: the transportation LP solved by scipy's HiGHS.
* ``sorted_1d``: for d = 1 and a convex cost of x - y, the monotone
  (north-west corner on sorted supports) coupling is optimal.
"""
from __future__ import annotations

import itertools

import numpy as np


def brute_force_uniform(C):
    n = C.shape[0]
    assert C.shape == (n, n) and n <= 8
    best = np.inf
    rows = np.arange(n)
    for perm in itertools.permutations(range(n)):
        best = min(best, C[rows, list(perm)].sum() / n)
    return float(best)


def linprog_ot(C, r, c):
    from scipy.optimize import linprog
    from scipy.sparse import coo_matrix, vstack
    m, n = C.shape
    ii = np.repeat(np.arange(m), n)
    jj = np.tile(np.arange(n), m)
    rows = coo_matrix((np.ones(m * n), (ii, np.arange(m * n))), shape=(m, m * n))
    cols = coo_matrix((np.ones(m * n), (jj, np.arange(m * n))), shape=(n, m * n))
    A = vstack([rows, cols]).tocsr()
    b = np.concatenate([r, c])
    res = linprog(C.ravel(), A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    assert res.status == 0, res.message
    return float(res.fun)


def sorted_1d(x, y, r, c, s):
    """Exact p* for 1-D supports with cost s (x - y)^2 (monotone rearrangement)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    y = np.asarray(y, dtype=np.float64).ravel()
    ox, oy = np.argsort(x, kind="stable"), np.argsort(y, kind="stable")
    xs, ys = x[ox], y[oy]
    rr, cc = np.array(r, dtype=np.float64)[ox], np.array(c, dtype=np.float64)[oy]
    i = j = 0
    total = 0.0
    ri, cj = rr[0], cc[0]
    while i < len(xs) and j < len(ys):
        if ri <= cj:          # row i is exhausted first: ship all of it to column j
            total += ri * s * (xs[i] - ys[j]) ** 2
            cj -= ri
            i += 1
            ri = rr[i] if i < len(xs) else 0.0
        else:                 # column j is filled first
            total += cj * s * (xs[i] - ys[j]) ** 2
            ri -= cj
            j += 1
            cj = cc[j] if j < len(ys) else 0.0
    return total
