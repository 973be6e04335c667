"""ctypes binding of libbdrs.so (include/bdrs.h): argument marshalling only.

Every step of the solver runs in the library's HIP kernels; PyTorch only
supplies device memory (the workspace and the input/output tensors) and the
stream.  There is no fallback: if the library is missing, loading fails.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbdrs.so")
# Split-count table written by `python -m paper_2609_33814_amd.autotune`; it is
# loaded into the library when the library is first loaded.  BDRS_TUNING
# names another file, or "none" to keep the built-in heuristic.
TUNING_PATH = os.path.join(PKG, "tuning_gfx950.json")

OK, NOT_CONVERGED = 0, 1
E_INVALID, E_NOMEM, E_DEVICE, E_STATE, E_NUMERIC = -1, -2, -3, -4, -5
F_REPAIR = 1
F_OLD_KERNEL, F_NO_MOMENTUM, F_DEBIASED = 2, 4, 8
F_NO_GRAPH = 16
F_KEEP_BEST_STATE = 32
# Row-update variants of the momentum / kernel ablation (lambda = 1).
VARIANTS = {
    "dual_bdrs": 0,
    "annealed_sinkhorn": F_OLD_KERNEL | F_NO_MOMENTUM,
    "as_momentum": F_OLD_KERNEL,
    "as_current_kernel": F_NO_MOMENTUM,
    "debiased_as": F_OLD_KERNEL | F_NO_MOMENTUM | F_DEBIASED,
}

EXPORTS = [
    "bdrs_workspace_size", "bdrs_create", "bdrs_step", "bdrs_certificate", "bdrs_solve",
    "bdrs_get_state", "bdrs_set_state", "bdrs_lse", "bdrs_destroy", "bdrs_last_error",
    "bdrs_version", "bdrs_profile", "bdrs_profile_read", "bdrs_batch_workspace_size",
    "bdrs_batch_solve", "bdrs_server_create", "bdrs_server_submit", "bdrs_server_poll",
    "bdrs_server_wait", "bdrs_server_stats", "bdrs_server_now", "bdrs_server_destroy",
    "bdrs_get_hints", "bdrs_set_hints", "bdrs_autotune_workspace_size", "bdrs_autotune",
    "bdrs_tune_set", "bdrs_tune_get", "bdrs_tune_clear", "bdrs_plan", "bdrs_server_set_policy",
    "bdrs_round", "bdrs_profile_evaluated", "bdrs_restore_best", "bdrs_export_plan",
    "bdrs_plan_entries", "bdrs_batch_solve_static",
]
BATCH_STATIC_BYTES = 16 << 20   # BDRS_BATCH_STATIC_BYTES

PLAN_ROUNDED = 0
PLAN_REPAIRED = 1
PLAN_KINDS = {"rounded": PLAN_ROUNDED, "repaired": PLAN_REPAIRED}


class Params(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("dim", ctypes.c_int32),
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
        ("r", ctypes.c_void_p), ("c", ctypes.c_void_p),
        ("cost_scale", ctypes.c_double), ("eta", ctypes.c_double),
        ("lambda_", ctypes.c_double), ("omega", ctypes.c_double),
        ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p), ("flags", ctypes.c_uint32),
    ]


class Cert(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int64), ("eps", ctypes.c_double), ("L", ctypes.c_double),
        ("U", ctypes.c_double), ("gap", ctypes.c_double), ("rel_gap", ctypes.c_double),
        ("L_best", ctypes.c_double), ("U_best", ctypes.c_double),
        ("rel_gap_best", ctypes.c_double), ("k_L_best", ctypes.c_int64),
        ("k_U_best", ctypes.c_int64), ("delta", ctypes.c_double),
        ("cost_Z", ctypes.c_double), ("repaired_cost", ctypes.c_double),
        ("n_nonfinite", ctypes.c_int64), ("negative_gap", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Request(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("dim", ctypes.c_int32),
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
        ("r", ctypes.c_void_p), ("c", ctypes.c_void_p),
        ("cost_scale", ctypes.c_double), ("eta", ctypes.c_double),
        ("lambda_", ctypes.c_double), ("omega", ctypes.c_double),
        ("tau", ctypes.c_double), ("tau_relative", ctypes.c_int32), ("max_iters", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int32), ("status", ctypes.c_int32), ("cert", Cert),
        ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return dict(state=self.state, status=self.status, cert=self.cert.as_dict(),
                    t_submit=self.t_submit, t_admit=self.t_admit, t_done=self.t_done)


class PlanStats(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int64), ("eps", ctypes.c_double),
        ("row_l1", ctypes.c_double), ("col_l1", ctypes.c_double),
        ("row_max_abs", ctypes.c_double), ("col_max_abs", ctypes.c_double),
        ("row_max_rel", ctypes.c_double), ("col_max_rel", ctypes.c_double),
        ("mass", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class RoundStats(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int64), ("eps", ctypes.c_double), ("cost", ctypes.c_double),
        ("cost_clipped", ctypes.c_double), ("mass_moved", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class PlanExport(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("k", ctypes.c_int64), ("eps", ctypes.c_double),
        ("cost_scale", ctypes.c_double), ("cost", ctypes.c_double), ("mass", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class TuneEntry(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("m", ctypes.c_int32), ("n", ctypes.c_int32),
        ("splits_row", ctypes.c_int32), ("splits_col", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("us_row", ctypes.c_double), ("us_col", ctypes.c_double),
        ("us_row_default", ctypes.c_double), ("us_col_default", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class BdrsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bdrs status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libbdrs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2609_33814_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.bdrs_workspace_size.argtypes = [P(Params), P(ctypes.c_size_t)]
        L.bdrs_create.argtypes = [P(Params), P(vp)]
        L.bdrs_step.argtypes = [vp, ctypes.c_int32]
        L.bdrs_certificate.argtypes = [vp, P(Cert)]
        L.bdrs_solve.argtypes = [vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, P(Cert)]
        L.bdrs_get_state.argtypes = [vp] * 7 + [P(ctypes.c_int64)]
        L.bdrs_set_state.argtypes = [vp] * 7 + [ctypes.c_int64]
        L.bdrs_lse.argtypes = [vp, ctypes.c_int32, ctypes.c_double, vp, vp]
        L.bdrs_get_hints.argtypes = [vp, vp, vp]
        L.bdrs_set_hints.argtypes = [vp, vp, vp]
        L.bdrs_destroy.argtypes = [vp]
        L.bdrs_profile.argtypes = [vp, ctypes.c_int32]
        L.bdrs_batch_workspace_size.argtypes = [P(vp), ctypes.c_int32, P(ctypes.c_size_t)]
        L.bdrs_batch_solve.argtypes = [P(vp), ctypes.c_int32, vp, ctypes.c_size_t, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       P(Cert), P(ctypes.c_int32)]
        L.bdrs_batch_solve_static.argtypes = [P(vp), ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int32, P(Cert), P(ctypes.c_int32)]
        L.bdrs_profile_read.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_double), P(ctypes.c_double)]
        L.bdrs_server_create.argtypes = [vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, P(vp)]
        L.bdrs_server_submit.argtypes = [vp, P(Request), P(ctypes.c_uint64)]
        L.bdrs_server_poll.argtypes = [vp, ctypes.c_uint64, P(Result)]
        L.bdrs_server_wait.argtypes = [vp, ctypes.c_uint64, P(Result)]
        L.bdrs_server_stats.argtypes = [vp, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_size_t)]
        L.bdrs_server_now.argtypes = [vp, P(ctypes.c_double)]
        L.bdrs_server_destroy.argtypes = [vp]
        L.bdrs_autotune_workspace_size.argtypes = [P(Params), P(ctypes.c_size_t)]
        L.bdrs_autotune.argtypes = [P(Params), ctypes.c_int32, P(TuneEntry)]
        L.bdrs_tune_set.argtypes = [P(TuneEntry)]
        L.bdrs_tune_get.argtypes = [ctypes.c_int32, P(TuneEntry), P(ctypes.c_int32)]
        L.bdrs_tune_clear.argtypes = []
        L.bdrs_plan.argtypes = [vp, vp, vp, vp, P(PlanStats)]
        L.bdrs_server_set_policy.argtypes = [vp, ctypes.c_double]
        L.bdrs_round.argtypes = [vp, P(RoundStats)]
        L.bdrs_profile_evaluated.argtypes = [vp, P(ctypes.c_double)]
        L.bdrs_restore_best.argtypes = [vp, P(ctypes.c_int64)]
        L.bdrs_export_plan.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, P(PlanExport)]
        L.bdrs_plan_entries.argtypes = [vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int64,
                                        ctypes.c_int64, vp]
        L.bdrs_last_error.restype = ctypes.c_char_p
        L.bdrs_version.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("bdrs_last_error", "bdrs_version"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
        path = os.environ.get("BDRS_TUNING", TUNING_PATH)
        if path != "none" and os.path.exists(path):
            load_tuning(path)
    return _lib


def last_error() -> str:
    return lib().bdrs_last_error().decode()


def check(status: int, allow=(OK,)) -> int:
    if status not in allow:
        raise BdrsError(status, last_error())
    return status


def make_params(m, n, dim, x=0, y=0, r=0, c=0, cost_scale=1.0, eta=1.0, lam=1.0,
                omega=1.0, workspace=0, workspace_bytes=0, stream=0, flags=0) -> Params:
    return Params(m, n, dim, x, y, r, c, cost_scale, eta, lam, omega, workspace,
                  workspace_bytes, stream, flags)


def workspace_size(m: int, n: int, dim: int, flags: int = 0) -> int:
    out = ctypes.c_size_t()
    p = make_params(m, n, dim, flags=flags)
    check(lib().bdrs_workspace_size(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


class Solver:
    """One OT problem on the current device; inputs are torch tensors on the GPU.

    x (m, d) float32, y (n, d) float32, r (m,) float64, c (n,) float64.
    """

    def __init__(self, x, y, r, c, cost_scale, eta=1.0, lam=1.0, omega=1.0,
                 stream=None, repair=False, variant: str = "dual_bdrs", graph: bool = True,
                 keep_best: bool = False):
        import torch
        self._torch = torch
        m, dim = int(x.shape[0]), int(x.shape[1])
        n = int(y.shape[0])
        self.m, self.n, self.dim = m, n, dim
        flags = ((F_REPAIR if repair else 0) | VARIANTS[variant] | (0 if graph else F_NO_GRAPH) |
                 (F_KEEP_BEST_STATE if keep_best else 0))
        self.bytes = workspace_size(m, n, dim, flags)
        # 256-byte aligned workspace carved out of a torch allocation
        self._ws = torch.empty(self.bytes + 256, dtype=torch.uint8, device=x.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.current_stream(x.device)
        self._inputs = (x.contiguous(), y.contiguous(), r.contiguous(), c.contiguous())
        xx, yy, rr, cc = self._inputs
        self.params = make_params(m, n, dim, _ptr(xx), _ptr(yy), _ptr(rr), _ptr(cc),
                                  float(cost_scale), float(eta), float(lam), float(omega),
                                  self._ws_ptr, self.bytes, int(self._stream.cuda_stream),
                                  flags)
        h = ctypes.c_void_p()
        check(lib().bdrs_create(ctypes.byref(self.params), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def step(self, iters: int) -> None:
        check(lib().bdrs_step(self._h, int(iters)))

    def certificate(self) -> dict:
        ce = Cert()
        check(lib().bdrs_certificate(self._h, ctypes.byref(ce)))
        return ce.as_dict()

    def solve(self, tau: float, max_iters: int, cert_every: int, relative: bool = True):
        ce = Cert()
        st = check(lib().bdrs_solve(self._h, float(tau), 1 if relative else 0, int(max_iters),
                                    int(cert_every), ctypes.byref(ce)), allow=(OK, NOT_CONVERGED))
        return st == OK, ce.as_dict()

    def solve_logged(self, tau: float, max_iters: int, cert_every: int, path: str, relative: bool = True):
        """bdrs_solve one certificate block at a time, appending one JSON line per
        certificate to `path` (k, eps, L, U, gap, rel_gap, the best bounds, delta,
        cost_Z, n_nonfinite, negative_gap and the wall-clock seconds since the
        call).  The first block ends at the next multiple of cert_every, the
        others run cert_every iterations and the last one the remainder, so the
        iterates and certificates are those of solve(tau, max_iters,
        cert_every) from the same state; returns the same (reached,
        certificate)."""
        import json
        import time
        t0 = time.perf_counter()
        k0 = self.iterations()
        done, ok, ce = 0, False, None
        keys = ("k", "eps", "L", "U", "gap", "rel_gap", "L_best", "U_best", "rel_gap_best", "k_L_best",
                "k_U_best", "delta", "cost_Z", "n_nonfinite", "negative_gap")
        with open(path, "a") as log:
            while done < max_iters and not ok:
                to_grid = cert_every - (k0 + done) % cert_every
                block = min(to_grid, max_iters - done)
                ok, ce = self.solve(tau, block, cert_every, relative)
                done = int(ce["k"]) + 1 - k0
                rec = {key: ce[key] for key in keys}
                rec["t_wall"] = round(time.perf_counter() - t0, 6)
                log.write(json.dumps(rec) + "\n")
                log.flush()
        return ok, ce

    def iterations(self) -> int:
        """Finished iterations k of the solver (synchronises its stream)."""
        k = ctypes.c_int64()
        check(lib().bdrs_get_state(self._h, None, None, None, None, None, None, ctypes.byref(k)))
        return k.value

    def restore_best(self) -> int:
        """Makes the retained lowest-gap state current (keep_best=True); returns its iteration count."""
        k = ctypes.c_int64()
        check(lib().bdrs_restore_best(self._h, ctypes.byref(k)))
        return k.value

    def get_state(self) -> dict:
        torch = self._torch
        dev = self._inputs[0].device
        la = torch.empty(self.m, dtype=torch.float64, device=dev)
        lah = torch.empty_like(la)
        lb, lb1, lbh, lt = (torch.empty(self.n, dtype=torch.float64, device=dev) for _ in range(4))
        k = ctypes.c_int64()
        check(lib().bdrs_get_state(self._h, _ptr(la), _ptr(lb), _ptr(lb1), _ptr(lah), _ptr(lbh),
                                   _ptr(lt), ctypes.byref(k)))
        return dict(la=la, lb=lb, lb_prev=lb1, lah=lah, lbh=lbh, lt=lt, k=k.value)

    def set_state(self, st: dict) -> None:
        f = lambda key: None if st.get(key) is None else st[key].to(self._torch.float64).contiguous()
        keep = [f(key) for key in ("la", "lb", "lb_prev", "lah", "lbh", "lt")]
        check(lib().bdrs_set_state(self._h, *[_ptr(t) for t in keep], int(st["k"])))

    def get_hints(self) -> dict:
        torch = self._torch
        dev = self._inputs[0].device
        rh = torch.empty(self.m, dtype=torch.int32, device=dev)
        ch = torch.empty(self.n, dtype=torch.int32, device=dev)
        check(lib().bdrs_get_hints(self._h, _ptr(rh), _ptr(ch)))
        return dict(row=rh, col=ch)

    def set_hints(self, hints: dict) -> None:
        rh, ch = hints["row"].contiguous(), hints["col"].contiguous()
        check(lib().bdrs_set_hints(self._h, _ptr(rh), _ptr(ch)))

    def lse(self, w, eps: float, transpose: bool = False):
        """out_i = LSE_j(w_j - C_ij/eps) (or the transposed reduction); float64 in and out."""
        torch = self._torch
        w = w.to(torch.float64).contiguous()
        out = torch.empty(self.n if transpose else self.m, dtype=torch.float64, device=w.device)
        check(lib().bdrs_lse(self._h, 1 if transpose else 0, float(eps), _ptr(w), _ptr(out)))
        return out

    def plan(self, bary: bool = True, marginals: bool = True) -> dict:
        """State plan of the current iterate: stats, and (optionally) the
        barycentric projection (m, dim) and the row / column sums (float64)."""
        torch = self._torch
        dev = self._inputs[0].device
        b = torch.empty((self.m, self.dim), dtype=torch.float64, device=dev) if bary else None
        rm = torch.empty(self.m, dtype=torch.float64, device=dev) if marginals else None
        cm = torch.empty(self.n, dtype=torch.float64, device=dev) if marginals else None
        st = PlanStats()
        check(lib().bdrs_plan(self._h, _ptr(b), _ptr(rm), _ptr(cm), ctypes.byref(st)))
        return dict(stats=st.as_dict(), bary=b, row=rm, col=cm)

    def round(self) -> dict:
        """Cost of the two-sided rounding of the current state plan onto Pi(r, c)."""
        st = RoundStats()
        check(lib().bdrs_round(self._h, ctypes.byref(st)))
        return st.as_dict()

    def export_plan(self, kind: str = "rounded") -> dict:
        """Factors of a feasible plan of the current iterate (float64, original
        order): P_ij = exp(log_u_i + log_v_j - C_ij / eps) + a_i b_j.  kind
        "rounded" is the two-sided rounding of the state plan, "repaired" the
        repair of the last iteration's intermediate plan."""
        torch = self._torch
        dev = self._inputs[0].device
        u, a = (torch.empty(self.m, dtype=torch.float64, device=dev) for _ in range(2))
        v, b = (torch.empty(self.n, dtype=torch.float64, device=dev) for _ in range(2))
        info = PlanExport()
        check(lib().bdrs_export_plan(self._h, PLAN_KINDS[kind], _ptr(u), _ptr(v), _ptr(a), _ptr(b),
                                     ctypes.byref(info)))
        return dict(info=info.as_dict(), log_u=u, log_v=v, a=a, b=b)

    def plan_entries(self, plan: dict, row_begin: int = 0, row_end=None):
        """Dense rows [row_begin, row_end) of an exported plan, (rows, n) float64."""
        torch = self._torch
        row_end = self.m if row_end is None else int(row_end)
        out = torch.empty((max(row_end - int(row_begin), 0), self.n), dtype=torch.float64,
                          device=self._inputs[0].device)
        f = lambda key: None if plan.get(key) is None else plan[key].to(torch.float64).contiguous()
        u, v, a, b = f("log_u"), f("log_v"), f("a"), f("b")
        check(lib().bdrs_plan_entries(self._h, _ptr(u), _ptr(v), _ptr(a), _ptr(b),
                                      float(plan["info"]["eps"]), int(row_begin), row_end, _ptr(out)))
        return out

    def profile(self, enable: bool) -> None:
        check(lib().bdrs_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        n, ms, ent = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        check(lib().bdrs_profile_read(self._h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(ent)))
        ev = ctypes.c_double()
        check(lib().bdrs_profile_evaluated(self._h, ctypes.byref(ev)))
        return dict(sweeps=n.value, ms=ms.value, entries=ent.value, evaluated=ev.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().bdrs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_solve(solvers, tau: float, max_iters: int, cert_every: int, relative: bool = True,
                use_graph: bool = True):
    """Solves several Solver objects together (bdrs_batch_solve).

    Returns (status, [cert dict per solver], [status per solver]).
    """
    import torch
    n = len(solvers)
    arr = (ctypes.c_void_p * n)(*[s.handle.value for s in solvers])
    size = ctypes.c_size_t()
    check(lib().bdrs_batch_workspace_size(arr, n, ctypes.byref(size)))
    dev = solvers[0]._inputs[0].device
    ws = torch.empty(size.value + 256, dtype=torch.uint8, device=dev)
    ptr = (ws.data_ptr() + 255) // 256 * 256
    outs = (Cert * n)()
    sts = (ctypes.c_int32 * n)()
    st = lib().bdrs_batch_solve(arr, n, ptr, size.value, float(tau), 1 if relative else 0,
                                int(max_iters), int(cert_every), 1 if use_graph else 0, outs, sts)
    check(st, allow=(OK, NOT_CONVERGED))
    del ws
    return st, [o.as_dict() for o in outs], list(sts)


def batch_solve_static(solvers, tau: float, max_iters: int, cert_every: int, relative: bool = True):
    """bdrs_batch_solve_static: the batched solve with the library's static
    device array for its work lists (no workspace, no allocation).

    Returns (status, [cert dict per solver], [status per solver]).
    """
    n = len(solvers)
    arr = (ctypes.c_void_p * n)(*[s.handle.value for s in solvers])
    outs = (Cert * n)()
    sts = (ctypes.c_int32 * n)()
    st = lib().bdrs_batch_solve_static(arr, n, float(tau), 1 if relative else 0, int(max_iters),
                                       int(cert_every), outs, sts)
    check(st, allow=(OK, NOT_CONVERGED))
    return st, [o.as_dict() for o in outs], list(sts)


class Server:
    """Continuous-batching solve server over a device memory pool (bdrs_server_*)."""

    def __init__(self, pool_bytes: int, max_slots: int, block_iters: int = 50, device=None):
        import torch
        dev = device if device is not None else torch.device("cuda:0")
        self._pool = torch.empty(pool_bytes + 256, dtype=torch.uint8, device=dev)
        ptr = (self._pool.data_ptr() + 255) // 256 * 256
        torch.cuda.synchronize(dev)
        h = ctypes.c_void_p()
        check(lib().bdrs_server_create(ptr, pool_bytes, int(max_slots), int(block_iters), ctypes.byref(h)))
        self._h = h
        self.block_iters = block_iters

    def set_policy(self, big_work: float) -> None:
        """Requests with m n > big_work run one at a time (<= 0: arrival order only)."""
        check(lib().bdrs_server_set_policy(self._h, float(big_work)))

    def submit(self, prob, eta=1.0, lam=1.0, omega=1.0, tau=0.01, relative=True, max_iters=20000) -> int:
        """prob: an inputs.Problem (host arrays).  Returns the ticket."""
        import numpy as np
        x = np.ascontiguousarray(prob.x, dtype=np.float32)
        y = np.ascontiguousarray(prob.y, dtype=np.float32)
        r = np.ascontiguousarray(prob.r, dtype=np.float64)
        c = np.ascontiguousarray(prob.c, dtype=np.float64)
        req = Request(x.shape[0], y.shape[0], x.shape[1], x.ctypes.data, y.ctypes.data, r.ctypes.data,
                      c.ctypes.data, float(prob.cost_scale), float(eta), float(lam), float(omega),
                      float(tau), 1 if relative else 0, int(max_iters))
        t = ctypes.c_uint64()
        check(lib().bdrs_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> dict:
        out = Result()
        check(lib().bdrs_server_poll(self._h, ticket, ctypes.byref(out)))
        return out.as_dict()

    def wait(self, ticket: int) -> dict:
        out = Result()
        check(lib().bdrs_server_wait(self._h, ticket, ctypes.byref(out)))
        return out.as_dict()

    def stats(self) -> dict:
        a, q, u = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        check(lib().bdrs_server_stats(self._h, ctypes.byref(a), ctypes.byref(q), ctypes.byref(u)))
        return dict(running=a.value, queued=q.value, pool_used=u.value)

    def now(self) -> float:
        t = ctypes.c_double()
        check(lib().bdrs_server_now(self._h, ctypes.byref(t)))
        return t.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().bdrs_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# tile-shape autotuner (bdrs_autotune / bdrs_tune_*)
# ----------------------------------------------------------------------------
def autotune(x, y, r, c, cost_scale, eta=0.1, lam=1.0, omega=1.0, rounds=20, stream=None) -> dict:
    """Times candidate split counts on this problem (torch tensors on the GPU,
    as for Solver) and enters the fastest into the library's table."""
    import torch
    m, dim = int(x.shape[0]), int(x.shape[1])
    n = int(y.shape[0])
    p = make_params(m, n, dim)
    need = ctypes.c_size_t()
    check(lib().bdrs_autotune_workspace_size(ctypes.byref(p), ctypes.byref(need)))
    ws = torch.empty(need.value + 256, dtype=torch.uint8, device=x.device)
    wp = (ws.data_ptr() + 255) // 256 * 256
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    xx, yy, rr, cc = (t.contiguous() for t in (x, y, r, c))
    p = make_params(m, n, dim, _ptr(xx), _ptr(yy), _ptr(rr), _ptr(cc), float(cost_scale), float(eta),
                    float(lam), float(omega), wp, need.value, int(st.cuda_stream))
    e = TuneEntry()
    check(lib().bdrs_autotune(ctypes.byref(p), int(rounds), ctypes.byref(e)))
    del ws
    return e.as_dict()


def tune_set(entry: dict) -> None:
    e = TuneEntry(**{k: entry.get(k, 0) for k, _ in TuneEntry._fields_})
    check(lib().bdrs_tune_set(ctypes.byref(e)))


def tune_table() -> list[dict]:
    count = ctypes.c_int32()
    check(lib().bdrs_tune_get(0, None, ctypes.byref(count)))
    out = []
    for i in range(count.value):
        e = TuneEntry()
        check(lib().bdrs_tune_get(i, ctypes.byref(e), None))
        out.append(e.as_dict())
    return out


def tune_clear() -> None:
    check(lib().bdrs_tune_clear())


def save_tuning(path: str, device: str = "gfx950") -> None:
    import json
    with open(path, "w") as f:
        json.dump({"device": device, "entries": tune_table()}, f, indent=1)
        f.write("\n")


def load_tuning(path: str) -> int:
    """Enters every entry of a saved table; returns their number."""
    import json
    with open(path) as f:
        doc = json.load(f)
    for e in doc.get("entries", []):
        tune_set(e)
    return len(doc.get("entries", []))
