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
* ``annealed_scalings`` -- the scaling recursions of the momentum / kernel
  ablation (Cor. 1 and the ablation appendix) in the linear domain:
  a^k = [(a^{k-1})^theta_k] r / (K^{.k or .(k+1)} t), t = b^{k-1} or
  (b^{k-1})^2 / b^{k-2}, and the shared column update b^k = c / (K^{.(k+1)})^T a^k.
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


def annealed_scalings(C, r, c, eta, iters, old_kernel, momentum, debiased):
    """Row / column scalings a^k, b^k (k = 0..iters-1) of the ablation family.

    b^{-1} = b^{-2} = 1 and a^{-1} = 1; K^{.j} = exp(-j C / eta) (K^{.0} = 1);
    theta_k = 0 for k <= 1 and 1 / k afterwards (debiased row update).
    """
    m, n = C.shape
    a_prev = np.ones(m)
    b1 = np.ones(n)
    b2 = np.ones(n)
    As, Bs = [], []
    for k in range(iters):
        Kr = np.exp(-(k if old_kernel else k + 1) * C / eta)
        t = b1 * b1 / b2 if momentum else b1
        a = r / (Kr @ t)
        if debiased:
            theta = 0.0 if k <= 1 else 1.0 / k
            a = a_prev ** theta * a
        Kc = np.exp(-(k + 1) * C / eta)
        b = c / (Kc.T @ a)
        As.append(a)
        Bs.append(b)
        a_prev, b2, b1 = a, b1, b
    return As, Bs
