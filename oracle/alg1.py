"""Dual O-BDRS (Algorithm 1) in the log domain, in FP64.

Test infrastructure only (see the package docstring).

What the method computes, in terms of Prop. 2: two scaling vectors, alpha
for the rows and beta for the columns, kept as natural logarithms.  Each
iteration k works at the temperature eta_k = eta / (lambda k + 1), i.e. with
the kernel exp(-C / eta_k).  It first extrapolates the column scaling along
its last change (momentum: beta^{k-1} moved on by 1/lambda of its step from
beta^{k-2}); then it makes the row scaling exact for the row marginal r
against that extrapolated column scaling, and the column scaling exact for
the column marginal c against the new (unrelaxed) row scaling.  The
overrelaxation mixes each unrelaxed scaling with the previous relaxed one,
weight lambda on the new one (a geometric mix in the linear domain); the
unrelaxed ones carry a hat.  With lambda = 1 there is no mixing and no hat:
Dual BDRS (Prop. 1).  All three scalings start at one (zero in the log).

Names: ``la`` = log alpha^k, ``lah`` = log alpha-hat^k, ``lb`` = log beta^k,
``lbh`` = log beta-hat^k, ``lt`` = log beta-tilde^{k-1} (the extrapolated
column scaling the row update of iteration k reads).  The state also keeps
log beta^{k-1}: the next extrapolation needs both beta^k and beta^{k-1},
which the tuple the algorithm returns does not hold.

Ablation variants (lambda = 1; the controlled ablation of the appendix and
Cor. 1, which names the two changes that turn annealed Sinkhorn into Dual
BDRS).  All share the column update at eta_k = eta / (k + 1), the schedule
and the initialisation, and differ in the row update:

  log a^k = [theta_k log a^{k-1}] + log r - LSE_j(log t_j - C_ij / eps_row)

with OLD_KERNEL: eps_row = eta / k (the kernel K^{.k}; K^{.0} is all ones,
eps_row = inf) instead of eta_k; NO_MOMENTUM: t = b^{k-1} instead of the
extrapolated b~^{k-1}; DEBIASED (with both of the former, the debiased
annealed Sinkhorn): the bracketed factor with theta_k = 0 for k <= 1 and
1 / k for k >= 2 (the first iteration that has a previous row scaling uses
theta = 0, as the ablation's formula does for its first index).  The
column update reads the row scaling a^k itself (for DEBIASED the factor
included).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .lse import implicit_lse
from .certificate import certificate


OLD_KERNEL, NO_MOMENTUM, DEBIASED = 1, 2, 4


def schedule(eta: float, lam: float, k: int) -> float:
    """Effective temperature eta_k = eta / (lambda k + 1) (Algorithm 1)."""
    return eta / (lam * k + 1.0)


def row_temperature(eta: float, lam: float, k: int, variant: int = 0) -> float:
    """Temperature of the row update: eps_k, or for OLD_KERNEL that of K^{.k}."""
    if variant & OLD_KERNEL:
        return eta / k if k >= 1 else np.inf
    return schedule(eta, lam, k)


def debias_theta(k: int) -> float:
    """theta_k of the debiased row update: 0 for k <= 1, 1 / k afterwards."""
    return 0.0 if k <= 1 else 1.0 / k


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


def row_update(prob, lt, eps, perturb=None):
    """log alpha-hat^k = log r - LSE_j(log beta-tilde_j - C_ij / eps_k)."""
    out = implicit_lse(prob.x, prob.y, prob.cost_scale, eps, lt)
    return np.log(prob.r) - (out if perturb is None else perturb(out))


def col_update(prob, lah, eps, perturb=None):
    """log beta-hat^k = log c - LSE_i(log alpha-hat_i - C_ij / eps_k)."""
    out = implicit_lse(prob.y, prob.x, prob.cost_scale, eps, lah)
    return np.log(prob.c) - (out if perturb is None else perturb(out))


def column_weights(st: "State", variant: int = 0):
    """The row scaling the column update of the last iteration read."""
    return st.la if variant & DEBIASED else st.lah


def iterate(prob, st: State, eta: float, lam: float, variant: int = 0, perturb=None) -> State:
    """One iteration of Algorithm 1 (or of an ablation variant); returns the new state.

    perturb (tests only): a map applied to every LSE result, e.g. rounding to
    float32, to measure how far a given rounding of the sweeps moves the
    trajectory; None leaves the FP64 arithmetic untouched."""
    k = st.k
    eps = schedule(eta, lam, k)
    eps_row = row_temperature(eta, lam, k, variant)
    lt = st.lb1.copy() if variant & NO_MOMENTUM else momentum(st.lb1, st.lb2, lam)
    lah = row_update(prob, lt, eps_row, perturb)
    if variant & DEBIASED:
        la = debias_theta(k) * st.la + lah
        colw = la
    else:
        la = (1.0 - lam) * st.la + lam * lah
        colw = lah
    lbh = col_update(prob, colw, eps, perturb)
    lb = (1.0 - lam) * st.lb1 + lam * lbh
    return State(la=la, lb1=lb, lb2=st.lb1.copy(), lah=lah, lbh=lbh, lt=lt, k=k + 1)


def cert_due(k: int, cert_every: int, last: int) -> bool:
    """Certificate after iteration k when (k+1) is a multiple of cert_every, and at the last."""
    return cert_every > 0 and ((k + 1) % cert_every == 0 or k == last)


def run(prob, eta: float, lam: float, iters: int, cert_every: int = 0,
        omega: float = 1.0, tau_rel: float | None = None, state: State | None = None,
        keep_states: bool = False, variant: int = 0, perturb=None):
    """Run Algorithm 1 for up to ``iters`` iterations.

    Returns (state, certs, states): certs is a list of dicts (iteration k, the
    Prop. 3 quantities, and best-so-far bounds U_best = min U, L_best = max L);
    with ``tau_rel`` the loop stops at the first certificate whose best
    relative gap (U_best - L_best) / U_best is at most tau_rel.

    For an ablation variant the certificate's plan Z uses the row update's
    temperature and weights t, and its lower bound the column update's
    temperature and row scaling (see ``certificate``).
    """
    if variant and lam != 1.0:
        raise ValueError("the ablation variants are defined for lambda = 1")
    st = State.initial(prob.m, prob.n) if state is None else state.copy()
    certs, states = [], []
    U_best, L_best = np.inf, -np.inf
    k_end = st.k + iters - 1
    for _ in range(iters):
        k = st.k
        st = iterate(prob, st, eta, lam, variant, perturb)
        if keep_states:
            states.append(st.copy())
        if cert_due(k, cert_every, k_end):
            eps = schedule(eta, lam, k)
            if variant:
                ce = certificate(prob.x, prob.y, prob.cost_scale, prob.r, prob.c,
                                 st.lah, st.lbh, st.lt, row_temperature(eta, lam, k, variant), omega,
                                 colw=column_weights(st, variant), eps_col=eps)
            else:
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
