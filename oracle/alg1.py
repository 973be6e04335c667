"""Algorithm 1 (Dual O-BDRS, log domain), step by step in FP64.

Test infrastructure only (see the package docstring).

Notation follows Algorithm 1 and Proposition 2 in natural-log form:
``la`` = log alpha^k, ``lah`` = log alpha-hat^k, ``lb`` = log beta^k,
``lbh`` = log beta-hat^k, ``lt`` = log beta-tilde^{k-1}.  lambda = 1 is Dual
BDRS (Prop. 1; alpha = alpha-hat = a, beta = beta-hat = b).

Initialisation: log alpha^{-1} = log beta^{-2} = log beta^{-1} = 0.
Iteration k:
  eps_k   = eta / (lambda k + 1)
  lt      = lb1 + (lb1 - lb2) / lambda          (lb1 = log beta^{k-1}, lb2 = log beta^{k-2})
  lah     = log r - LSE_j(lt_j - C_ij / eps_k)
  la      = (1 - lambda) la_prev + lambda lah
  lbh     = log c - LSE_i(lah_i - C_ij / eps_k)  (the column update uses alpha-hat)
  lb      = (1 - lambda) lb1 + lambda lbh
then, when requested, the certificate of Prop. 3 from (lah, lbh, lt, eps_k).

The state also keeps log beta^{k-1}: the next extrapolation needs both
beta^k and beta^{k-1}, and the tuple Algorithm 1 returns lacks it.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .lse import implicit_lse
from .certificate import certificate


def schedule(eta: float, lam: float, k: int) -> float:
    """Effective temperature eta_k = eta / (lambda k + 1) (Algorithm 1)."""
    return eta / (lam * k + 1.0)


@dataclasses.dataclass
class State:
    la: np.ndarray      # log alpha^{k-1}
    lb1: np.ndarray     # log beta^{k-1}
    lb2: np.ndarray     # log beta^{k-2}
    lah: np.ndarray     # log alpha-hat of the last finished iteration
    lbh: np.ndarray     # log beta-hat of the last finished iteration
    lt: np.ndarray      # log beta-tilde used by the last finished iteration
    k: int              # index of the next iteration

    @staticmethod
    def initial(m: int, n: int) -> "State":
        z = np.zeros
        return State(la=z(m), lb1=z(n), lb2=z(n), lah=z(m), lbh=z(n), lt=z(n), k=0)

    def copy(self) -> "State":
        return State(*(v.copy() if isinstance(v, np.ndarray) else v
                       for v in dataclasses.astuple(self)))


def momentum(lb1, lb2, lam):
    """log beta-tilde^{k-1} = log beta^{k-1} + (log beta^{k-1} - log beta^{k-2}) / lambda."""
    return lb1 + (lb1 - lb2) / lam


def row_update(prob, lt, eps):
    """log alpha-hat^k = log r - LSE_j(log beta-tilde_j - C_ij / eps_k)."""
    return np.log(prob.r) - implicit_lse(prob.x, prob.y, prob.cost_scale, eps, lt)


def col_update(prob, lah, eps):
    """log beta-hat^k = log c - LSE_i(log alpha-hat_i - C_ij / eps_k)."""
    return np.log(prob.c) - implicit_lse(prob.y, prob.x, prob.cost_scale, eps, lah)


def iterate(prob, st: State, eta: float, lam: float) -> State:
    """One iteration of Algorithm 1; returns the new state (input untouched)."""
    k = st.k
    eps = schedule(eta, lam, k)
    lt = momentum(st.lb1, st.lb2, lam)
    lah = row_update(prob, lt, eps)
    la = (1.0 - lam) * st.la + lam * lah
    lbh = col_update(prob, lah, eps)
    lb = (1.0 - lam) * st.lb1 + lam * lbh
    return State(la=la, lb1=lb, lb2=st.lb1.copy(), lah=lah, lbh=lbh, lt=lt, k=k + 1)


def cert_due(k: int, cert_every: int, last: int) -> bool:
    """Certificate after iteration k when (k+1) is a multiple of cert_every, and at the last."""
    return cert_every > 0 and ((k + 1) % cert_every == 0 or k == last)


def run(prob, eta: float, lam: float, iters: int, cert_every: int = 0,
        omega: float = 1.0, tau_rel: float | None = None, state: State | None = None,
        keep_states: bool = False):
    """Run Algorithm 1 for up to ``iters`` iterations.

    Returns (state, certs, states): certs is a list of dicts (iteration k, the
    Prop. 3 quantities, and best-so-far bounds U_best = min U, L_best = max L);
    with ``tau_rel`` the loop stops at the first certificate whose best
    relative gap (U_best - L_best) / U_best is at most tau_rel.
    """
    st = State.initial(prob.m, prob.n) if state is None else state.copy()
    certs, states = [], []
    U_best, L_best = np.inf, -np.inf
    k_end = st.k + iters - 1
    for _ in range(iters):
        k = st.k
        st = iterate(prob, st, eta, lam)
        if keep_states:
            states.append(st.copy())
        if cert_due(k, cert_every, k_end):
            eps = schedule(eta, lam, k)
            ce = certificate(prob.x, prob.y, prob.cost_scale, prob.r, prob.c,
                             st.lah, st.lbh, st.lt, eps, omega)
            U_best = min(U_best, ce["U"])
            L_best = max(L_best, ce["L"])
            ce.update(k=k, U_best=U_best, L_best=L_best,
                      rel_best=(U_best - L_best) / U_best if U_best > 1e-300
                      else U_best - L_best)
            certs.append(ce)
            if tau_rel is not None and ce["rel_best"] <= tau_rel:
                break
    return st, certs, states
