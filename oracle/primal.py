"""Primal-plan forms, linear domain, dense, FP64 (small problems, short runs).

Test infrastructure only (see the package docstring).  These pin the dual
recursion of ``alg1`` from outside it:

* ``bdrs_primal``   -- primal-dual BDRS (Eq. 3a-c): u^k = r / ((X^k . K) v^{k-1}),
  v^k = c / ((X^k . K)^T u^k), X^{k+1} = diag(u^k) (X^k . K) diag(v^k),
  X^0 = 1, v^{-1} = 1, K = exp(-C / eta).
* ``obdrs_primal``  -- O-BDRS (Sec. 3.3): the same u, v, but
  X^{k+1} = X^k . (K . u^k v^kT)^lambda.
* ``ipot``          -- IPOT of Xie et al. (2020, Algorithm 1) with L inner
  Sinkhorn steps on Q = G . Gamma, warm-started b, Gamma^1 = 1, b = 1/n;
  with L = 1 it coincides with BDRS (App. B mapping mu, nu, G, Gamma <-> r, c, K, X).
"""
from __future__ import annotations

import numpy as np


def bdrs_primal(C, r, c, eta, iters):
    """Returns lists X[k] (X^k, k = 0..iters), u[k], v[k]."""
    K = np.exp(-C / eta)
    X = np.ones_like(C)
    v = np.ones(C.shape[1])
    Xs, us, vs = [X], [], []
    for _ in range(iters):
        Q = X * K
        u = r / (Q @ v)
        v = c / (Q.T @ u)
        X = u[:, None] * Q * v[None, :]
        Xs.append(X)
        us.append(u)
        vs.append(v)
    return Xs, us, vs


def obdrs_primal(C, r, c, eta, lam, iters):
    """O-BDRS primal update X^{k+1} = X^k . (K . u v^T)^lambda (Sec. 3.3)."""
    K = np.exp(-C / eta)
    X = np.ones_like(C)
    v = np.ones(C.shape[1])
    Xs, us, vs = [X], [], []
    for _ in range(iters):
        Q = X * K
        u = r / (Q @ v)
        v = c / (Q.T @ u)
        X = X * (K * np.outer(u, v)) ** lam
        Xs.append(X)
        us.append(u)
        vs.append(v)
    return Xs, us, vs


def ipot(C, mu, nu, beta, outer, inner=1):
    """IPOT with ``inner`` Sinkhorn steps per proximal step; returns the Gammas."""
    n = C.shape[1]
    G = np.exp(-C / beta)
    Gamma = np.ones_like(C)
    b = np.ones(n) / n
    out = [Gamma]
    for _ in range(outer):
        Q = G * Gamma
        for _ in range(inner):
            a = mu / (Q @ b)
            b = nu / (Q.T @ a)
        Gamma = a[:, None] * Q * b[None, :]
        out.append(Gamma)
    return out
