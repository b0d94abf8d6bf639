"""Python binding of librfm.so (ctypes): argument marshalling only.

Every computation runs in the HIP library; this module allocates device tensors with
PyTorch (the caching allocator is the memory manager, the current torch stream is the
HIP stream) and passes raw pointers through the C ABI declared in include/rfm.h.
Importing it raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "librfm.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"librfm.so not built ({_LIB_PATH}); run python -m paper_2506_17626_amd.build")
_lib = C.CDLL(_LIB_PATH)

RFM_OK, RFM_EINVAL, RFM_EHIP, RFM_ENOTCONV, RFM_EUNSUPPORTED = 0, 1, 3, 4, 5
FORM_Q, FORM_R, FORM_M = 0, 1, 2
RRQR_AUTO, RRQR_DIRECT, RRQR_RFIRST = 0, 1, 2
F64, F32, BF16 = 0, 1, 2

_p = C.c_void_p
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_dp = C.POINTER(C.c_double)


class Layout(C.Structure):
    _fields_ = [("d", C.c_int32), ("J", C.c_int32), ("N", C.c_int64), ("nnz_rows", C.c_int64),
                ("nnz", C.c_int64), ("ncols", C.c_int64), ("nrsq", C.c_int64),
                ("max_rows", C.c_int32), ("max_cols", C.c_int32),
                ("row_off", _p), ("rows", _p), ("inc_blk", _p), ("rinc_off", _p), ("rinc", _p),
                ("feat_off", _p), ("blk_off", _p), ("rsq_off", _p)]


class Problem(C.Structure):
    _fields_ = [("x", _p), ("rowop", _p), ("weight", _p), ("rhs", _p), ("mu", _p), ("hw", _p),
                ("w", _p), ("b", _p), ("kappa", C.c_double), ("ksq", C.c_double), ("activation", C.c_int32),
                ("nopcoef", C.c_int32), ("opcoef", _p), ("ansatz", _p),
                ("depth", C.c_int32), ("hidden", C.c_int32), ("net", _p)]

ACTIVATIONS = {"tanh": 0, "sigmoid": 1, "sin": 2}


class Operator(C.Structure):
    _fields_ = [("form", C.c_int32), ("rank", _p), ("Q", _p), ("M", _p), ("kept", _p), ("R", _p),
                ("Qlow", _p), ("low_dtype", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("rrqr_threads", C.c_int32), ("rrqr_persistent", C.c_int32), ("rrqr_wgs_per_cu", C.c_int32),
                ("adj_tile", C.c_int32), ("rrqr_algo", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelTimes(C.Structure):
    _fields_ = [("ms", C.c_double * 5), ("launches", C.c_int64 * 5)]
    NAMES = ("fwd_local", "gather_beta", "adj_local", "alpha_rotation", "yw_update")

    def as_dict(self):
        return {n: dict(ms=self.ms[k], launches=self.launches[k]) for k, n in enumerate(self.NAMES)}


class LsqrOpts(C.Structure):
    _fields_ = [("atol", C.c_double), ("btol", C.c_double), ("maxit", C.c_int64),
                ("check_every", C.c_int32), ("use_graph", C.c_int32),
                ("times", C.POINTER(KernelTimes)), ("history", _p), ("inner_dtype", C.c_int32),
                ("max_outer", C.c_int32), ("max_inner", C.c_int64), ("inner_tol", C.c_double),
                ("adj_tile", C.c_int32), ("bidiag", _p)]


class LsqrInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("outer", C.c_int64), ("polish", C.c_int64), ("stop", C.c_int32),
                ("warm_rejected", C.c_int32), ("rnorm_est", C.c_double),
                ("artnorm_est", C.c_double), ("anorm", C.c_double), ("hnorm", C.c_double),
                ("ynorm", C.c_double), ("relres", C.c_double), ("eta", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib.rfm_plan.restype = C.c_int
_lib.rfm_plan.argtypes = [C.c_int32, C.c_int32, C.c_int64, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p,
                          _p, _p, _p]
_lib.rfm_assemble_ws_bytes.restype = C.c_size_t
_lib.rfm_assemble_ws_bytes.argtypes = [C.POINTER(Layout)]
_lib.rfm_assemble.restype = C.c_int
_lib.rfm_assemble.argtypes = [C.POINTER(Layout), C.POINTER(Problem), _p, _p, _p, C.c_size_t, _p]
_lib.rfm_rrqr_ws_bytes.restype = C.c_size_t
_lib.rfm_rrqr_ws_bytes.argtypes = [C.POINTER(Layout)]
_lib.rfm_rrqr_filter.restype = C.c_int
_lib.rfm_rrqr_filter.argtypes = [C.POINTER(Layout), _p, C.c_double, _p, _p, _p, _p, _p, _p,
                                 C.c_size_t, _p]
_lib.rfm_lsqr_ws_bytes.restype = C.c_size_t
_lib.rfm_lsqr_ws_bytes.argtypes = [C.POINTER(Layout)]
_lib.rfm_lsqr_solve.restype = C.c_int
_lib.rfm_lsqr_solve.argtypes = [C.POINTER(Layout), C.POINTER(Operator), _p, _p, C.POINTER(LsqrOpts),
                                _p, C.POINTER(LsqrInfo), _p, C.c_size_t, _p]
_lib.rfm_plan_order.restype = C.c_int
_lib.rfm_plan_order.argtypes = [C.c_int32, _p, _p, _p]
_lib.rfm_rrqr_filter_tuned.restype = C.c_int
_lib.rfm_rrqr_filter_tuned.argtypes = [C.POINTER(Layout), _p, C.c_double, _p, _p, _p, _p, _p, _p,
                                       C.POINTER(Tuning), _p, C.c_size_t, _p]
_lib.rfm_autotune.restype = C.c_int
_lib.rfm_autotune.argtypes = [C.POINTER(Layout), _p, C.c_double, _p, _p, _p, _p, _p, _p, _p, C.c_int64,
                              _p, _p, C.c_size_t, C.POINTER(Tuning), _p, _p, _p, _p]
_lib.rfm_pack_q.restype = C.c_int
_lib.rfm_pack_q.argtypes = [C.POINTER(Layout), _p, _p, C.c_int32, _p, _p]
_lib.rfm_coefficients.restype = C.c_int
_lib.rfm_coefficients.argtypes = [C.POINTER(Layout), _p, _p, _p, _p, _p, _p]
_lib.rfm_last_error.restype = C.c_char_p
_lib.rfm_last_error.argtypes = []

EXPORTED = ["rfm_plan", "rfm_assemble_ws_bytes", "rfm_assemble", "rfm_rrqr_ws_bytes",
            "rfm_rrqr_filter", "rfm_lsqr_ws_bytes", "rfm_lsqr_solve", "rfm_coefficients",
            "rfm_pack_q", "rfm_plan_order", "rfm_rrqr_filter_tuned", "rfm_autotune", "rfm_last_error"]


class RfmError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: status {status}: {_lib.rfm_last_error().decode()}")
        self.status = status


def _check(status, where, allow=()):
    if status != RFM_OK and status not in allow:
        raise RfmError(status, where)
    return status


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ws(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


@dataclass
class Plan:
    """Host plan (numpy) plus its device copies and the C layout struct."""
    layout: Layout
    host: dict
    dev: dict

    @property
    def J(self):
        return self.layout.J


def rfm_plan(d, J, x, mu, hw, K, device="cuda") -> Plan:
    """Supports and block layout (host planning; arrays are copied to `device`)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    hw = np.ascontiguousarray(hw, dtype=np.float64)
    K = np.ascontiguousarray(K, dtype=np.int32)
    N = x.shape[0]
    sizes = np.zeros(6, dtype=np.int64)
    nul = [None] * 8
    _check(_lib.rfm_plan(d, J, N, _np_ptr(x), _np_ptr(mu), _np_ptr(hw), _np_ptr(K), _np_ptr(sizes), *nul),
           "rfm_plan")
    nnz_rows, nnz, ncols, nrsq, max_rows, max_cols = (int(v) for v in sizes)
    h = dict(row_off=np.zeros(J + 1, np.int64), rows=np.zeros(max(nnz_rows, 1), np.int32),
             inc_blk=np.zeros(max(nnz_rows, 1), np.int32), rinc_off=np.zeros(N + 1, np.int64),
             rinc=np.zeros(max(nnz_rows, 1), np.int64), feat_off=np.zeros(J + 1, np.int64),
             blk_off=np.zeros(J + 1, np.int64), rsq_off=np.zeros(J + 1, np.int64))
    _check(_lib.rfm_plan(d, J, N, _np_ptr(x), _np_ptr(mu), _np_ptr(hw), _np_ptr(K), _np_ptr(sizes),
                         _np_ptr(h["row_off"]), _np_ptr(h["rows"]), _np_ptr(h["inc_blk"]),
                         _np_ptr(h["rinc_off"]), _np_ptr(h["rinc"]), _np_ptr(h["feat_off"]),
                         _np_ptr(h["blk_off"]), _np_ptr(h["rsq_off"])), "rfm_plan")
    dev = {k: torch.from_numpy(v).to(device) for k, v in h.items()} if device is not None else {}
    L = Layout(d=d, J=J, N=N, nnz_rows=nnz_rows, nnz=nnz, ncols=ncols, nrsq=nrsq, max_rows=max_rows,
               max_cols=max_cols)
    for k in ("row_off", "rows", "inc_blk", "rinc_off", "rinc", "feat_off", "blk_off", "rsq_off"):
        setattr(L, k, dev[k].data_ptr() if dev else 0)
    return Plan(L, h, dev)


def problem_tensors(inst, device="cuda") -> dict:
    """Device copies of an instance's per-row and per-feature arrays (marshalling only)."""
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
    return dict(x=t(inst.x, torch.float64), rowop=t(inst.rowop, torch.int32),
                weight=t(inst.weight, torch.float64), rhs=t(inst.rhs, torch.float64),
                mu=t(inst.mu, torch.float64), hw=t(inst.hw, torch.float64),
                w=t(inst.w, torch.float64), b=t(inst.b, torch.float64),
                kappa=float(inst.kappa), ksq=float(inst.ksq),
                activation=ACTIVATIONS[inst.activation],
                opcoef=None if inst.opcoef is None else t(inst.opcoef, torch.float64),
                ansatz=None if inst.ansatz is None else t(inst.ansatz(inst.x), torch.float64),
                depth=int(inst.depth), hidden=int(inst.hidden),
                net=None if inst.net is None else t(inst.net, torch.float64))


def _problem(prob: dict) -> Problem:
    """C struct of a problem_tensors dict (pointers into its device tensors)."""
    oc = prob.get("opcoef")
    an = prob.get("ansatz")
    return Problem(x=prob["x"].data_ptr(), rowop=prob["rowop"].data_ptr(), weight=prob["weight"].data_ptr(),
                   rhs=prob["rhs"].data_ptr(), mu=prob["mu"].data_ptr(), hw=prob["hw"].data_ptr(),
                   w=prob["w"].data_ptr(), b=prob["b"].data_ptr(), kappa=prob["kappa"], ksq=prob["ksq"],
                   activation=prob.get("activation", 0), nopcoef=0 if oc is None else oc.shape[0],
                   opcoef=_ptr(oc), ansatz=_ptr(an), depth=prob.get("depth", 1), hidden=prob.get("hidden", 0),
                   net=_ptr(prob.get("net")))


def plan_instance(inst, device="cuda") -> Plan:
    return rfm_plan(inst.d, inst.J, inst.x, inst.mu, inst.hw, np.diff(inst.feat_off), device)


def rfm_assemble(plan: Plan, prob: dict, M=None, h=None):
    L = plan.layout
    dev = prob["x"].device
    M = torch.empty(max(L.nnz, 1), dtype=torch.float64, device=dev) if M is None else M
    h = torch.empty(L.N, dtype=torch.float64, device=dev) if h is None else h
    P = _problem(prob)
    nb = _lib.rfm_assemble_ws_bytes(C.byref(L))
    ws = _ws(nb, dev)
    _check(_lib.rfm_assemble(C.byref(L), C.byref(P), _ptr(M), _ptr(h), _ptr(ws), nb, _stream()),
           "rfm_assemble")
    return M, h


_lib.rfm_assemble_low.restype = C.c_int
_lib.rfm_assemble_low.argtypes = [C.POINTER(Layout), C.POINTER(Problem), C.c_int32, _p, _p, _p, C.c_size_t, _p]
EXPORTED += ["rfm_assemble_low"]


def rfm_assemble_low(plan: Plan, prob: dict, dtype=F32, M=None, h=None):
    """Entries evaluated in binary32, stored as float32 (F32) or bfloat16 (BF16)."""
    L = plan.layout
    dev = prob["x"].device
    tdt = {F32: torch.float32, BF16: torch.bfloat16}[dtype]
    M = torch.empty(max(L.nnz, 1), dtype=tdt, device=dev) if M is None else M
    h = torch.empty(L.N, dtype=torch.float64, device=dev) if h is None else h
    P = _problem(prob)
    nb = _lib.rfm_assemble_ws_bytes(C.byref(L))
    ws = _ws(nb, dev)
    _check(_lib.rfm_assemble_low(C.byref(L), C.byref(P), int(dtype), _ptr(M), _ptr(h), _ptr(ws), nb, _stream()),
           "rfm_assemble_low")
    return M, h


_lib.rfm_evaluate_ws_bytes.restype = C.c_size_t
_lib.rfm_evaluate_ws_bytes.argtypes = [C.POINTER(Layout)]
_lib.rfm_evaluate.restype = C.c_int
_lib.rfm_evaluate.argtypes = [C.POINTER(Layout), C.POINTER(Problem), _p, _p, _p, C.POINTER(C.c_double), _p,
                              C.c_size_t, _p]
EXPORTED += ["rfm_evaluate_ws_bytes", "rfm_evaluate"]


def evaluation_points(inst, xt: np.ndarray, device="cuda"):
    """Layout of the test points xt [T, d] over the instance's subdomains, and xt on the
    device (host planning, once per point set)."""
    tplan = rfm_plan(inst.d, inst.J, xt, inst.mu, inst.hw, np.diff(inst.feat_off), device)
    xd = torch.from_numpy(np.ascontiguousarray(xt, dtype=np.float64)).to(device)
    return tplan, xd


def evaluation_ansatz(inst, xt: np.ndarray, device="cuda"):
    """The instance's hard-constraint factor at the test points (device [T*(1+2d)]), or None."""
    if inst.ansatz is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(inst.ansatz(xt), dtype=np.float64)).to(device)


def rfm_evaluate(tplan: Plan, xd, prob: dict, a, u_exact=None, ws=None, ansatz=None):
    """u_hat at the test points for coefficients a (device [ncols]), times the ansatz factor
    (evaluation_ansatz) when given; with u_exact (device [T]) also e_L1.  Returns (uhat,
    e_l1 or None)."""
    L = tplan.layout
    dev = xd.device
    P = Problem(x=xd.data_ptr(), mu=prob["mu"].data_ptr(), hw=prob["hw"].data_ptr(), w=prob["w"].data_ptr(),
                b=prob["b"].data_ptr(), activation=prob.get("activation", 0), ansatz=_ptr(ansatz),
                depth=prob.get("depth", 1), hidden=prob.get("hidden", 0), net=_ptr(prob.get("net")))
    uhat = torch.empty(L.N, dtype=torch.float64, device=dev)
    nb = _lib.rfm_evaluate_ws_bytes(C.byref(L))
    if ws is None or ws.numel() < nb:
        ws = _ws(nb, dev)
    e = C.c_double(0.0)
    _check(_lib.rfm_evaluate(C.byref(L), C.byref(P), _ptr(a), _ptr(uhat), _ptr(u_exact),
                             C.byref(e) if u_exact is not None else None, _ptr(ws), nb, _stream()), "rfm_evaluate")
    return uhat, (e.value if u_exact is not None else None)


def rfm_plan_order(plan: Plan):
    """Block ids by decreasing factorisation cost (host), copied to the device."""
    order = np.zeros(plan.J, dtype=np.int32)
    _check(_lib.rfm_plan_order(plan.J, _np_ptr(plan.host["row_off"]), _np_ptr(plan.host["feat_off"]),
                               _np_ptr(order)), "rfm_plan_order")
    return torch.from_numpy(order).to(plan.dev["row_off"].device) if plan.dev else order


def _rrqr_out(L, dev, with_ratios):
    return dict(rank=torch.empty(L.J, dtype=torch.int32, device=dev),
                kept=torch.empty(max(L.ncols, 1), dtype=torch.int32, device=dev),
                R=torch.zeros(max(L.nrsq, 1), dtype=torch.float64, device=dev),
                Q=torch.empty(max(L.nnz, 1), dtype=torch.float64, device=dev),
                ratios=torch.empty(max(L.ncols, 1), dtype=torch.float64, device=dev) if with_ratios else None)


def rfm_rrqr_filter(plan: Plan, M, tau, with_ratios=True, out=None, order=None, tune=None):
    L = plan.layout
    dev = M.device
    out = _rrqr_out(L, dev, with_ratios) if out is None else out
    nb = _lib.rfm_rrqr_ws_bytes(C.byref(L))
    ws = _ws(nb, dev)
    _check(_lib.rfm_rrqr_filter_tuned(C.byref(L), _ptr(M), float(tau), _ptr(out["rank"]), _ptr(out["kept"]),
                                      _ptr(out["R"]), _ptr(out["Q"]), _ptr(out["ratios"]), _ptr(order),
                                      C.byref(tune) if tune is not None else None, _ptr(ws), nb, _stream()),
           "rfm_rrqr_filter")
    return out


_lib.rfm_rrqr_strong_ws_bytes.restype = C.c_size_t
_lib.rfm_rrqr_strong_ws_bytes.argtypes = [C.POINTER(Layout)]
_lib.rfm_rrqr_strong.restype = C.c_int
_lib.rfm_rrqr_strong.argtypes = [C.POINTER(Layout), _p, C.c_double, C.c_double, C.c_int32, _p, _p, _p, _p, _p,
                                 C.POINTER(C.c_int32), _p, C.c_size_t, _p]
EXPORTED += ["rfm_rrqr_strong_ws_bytes", "rfm_rrqr_strong"]


def rfm_rrqr_strong(plan: Plan, M, tau, f=2.0, max_rounds=32, out=None):
    """Strong RRQR variant of the filter; returns (outputs with rho [J] and pending = blocks
    whose last test still exceeds f^2 when max_rounds stopped the loop, swaps, rounds)."""
    L = plan.layout
    dev = M.device
    out = _rrqr_out(L, dev, False) if out is None else out
    out["rho"] = torch.zeros(max(L.J, 1), dtype=torch.float64, device=dev)
    nb = _lib.rfm_rrqr_strong_ws_bytes(C.byref(L))
    ws = _ws(nb, dev)
    stats = (C.c_int32 * 3)()
    _check(_lib.rfm_rrqr_strong(C.byref(L), _ptr(M), float(tau), float(f), int(max_rounds), _ptr(out["rank"]),
                                _ptr(out["kept"]), _ptr(out["R"]), _ptr(out["Q"]), _ptr(out["rho"]), stats,
                                _ptr(ws), nb, _stream()), "rfm_rrqr_strong")
    out["pending"] = int(stats[2])
    return out, int(stats[0]), int(stats[1])


def rfm_autotune(plan: Plan, M, tau, h, order=None, lsqr_iters=64, out=None):
    """Time the candidate launch shapes (filter, then the LSQR adjoint tile); returns
    (best Tuning, [(Tuning, ms)], filter outputs)."""
    L = plan.layout
    dev = M.device
    out = _rrqr_out(L, dev, True) if out is None else out
    nb = max(_lib.rfm_rrqr_ws_bytes(C.byref(L)), _lib.rfm_lsqr_ws_bytes(C.byref(L)))
    ws = _ws(nb, dev)
    y = torch.empty(max(L.ncols, 1), dtype=torch.float64, device=dev)
    best = Tuning()
    ms = (C.c_double * 32)()
    cands = (Tuning * 32)()
    n = C.c_int32(0)
    _check(_lib.rfm_autotune(C.byref(L), _ptr(M), float(tau), _ptr(out["rank"]), _ptr(out["kept"]), _ptr(out["R"]),
                             _ptr(out["Q"]), _ptr(out["ratios"]), _ptr(order), _ptr(h), int(lsqr_iters), _ptr(y),
                             _ptr(ws), nb, C.byref(best), ms, cands, C.byref(n), _stream()), "rfm_autotune")
    table = [(cands[i].as_dict(), ms[i]) for i in range(min(n.value, 32))]
    return best, table, out


def rfm_pack_q(plan: Plan, fact: dict, dtype, Qlow=None):
    """Narrow copy of Q_hat (binary32 or bfloat16) in the block layout."""
    L = plan.layout
    tdt = {F32: torch.float32, BF16: torch.bfloat16}[dtype]
    Qlow = torch.zeros(max(L.nnz, 1), dtype=tdt, device=fact["Q"].device) if Qlow is None else Qlow
    _check(_lib.rfm_pack_q(C.byref(L), _ptr(fact["rank"]), _ptr(fact["Q"]), dtype, _ptr(Qlow), _stream()),
           "rfm_pack_q")
    return Qlow


def rfm_lsqr_solve(plan: Plan, fact: dict, h, y0=None, atol=1e-8, btol=1e-8, maxit=10000,
                   check_every=16, use_graph=0, form=FORM_Q, y=None, ws=None, times=None,
                   history=None, inner_dtype=F64, max_outer=1, max_inner=None, inner_tol=None,
                   adj_tile=0, bidiag=None):
    """Precision form defaults: one narrow solve to the caller's rule (inner_tol = atol, all
    of maxit), then the binary64 check and finish."""
    L = plan.layout
    if max_inner is None:
        max_inner = maxit
    if inner_tol is None:
        inner_tol = atol if 0.0 < atol < 1.0 else 1e-8
    dev = h.device
    y = torch.empty(max(L.ncols, 1), dtype=torch.float64, device=dev) if y is None else y
    qlow = fact.get("Qlow")
    low_dtype = {torch.float32: F32, torch.bfloat16: BF16}.get(qlow.dtype, F64) if qlow is not None else F64
    ptr = lambda key: fact[key].data_ptr() if fact.get(key) is not None else 0
    op = Operator(form=form, rank=fact["rank"].data_ptr(), Q=ptr("Q"), M=ptr("M"), kept=ptr("kept"), R=ptr("R"),
                  Qlow=qlow.data_ptr() if qlow is not None else 0, low_dtype=low_dtype)
    opts = LsqrOpts(atol=atol, btol=btol, maxit=maxit, check_every=check_every, use_graph=use_graph,
                    times=C.pointer(times) if times is not None else None, history=_ptr(history),
                    inner_dtype=inner_dtype, max_outer=max_outer, max_inner=max_inner, inner_tol=inner_tol,
                    adj_tile=adj_tile, bidiag=_ptr(bidiag))
    info = LsqrInfo()
    nb = _lib.rfm_lsqr_ws_bytes(C.byref(L))
    if ws is None or ws.numel() < nb:
        ws = _ws(nb, dev)
    _check(_lib.rfm_lsqr_solve(C.byref(L), C.byref(op), _ptr(h), _ptr(y0), C.byref(opts), _ptr(y),
                               C.byref(info), _ptr(ws), nb, _stream()), "rfm_lsqr_solve",
           allow=(RFM_ENOTCONV,))
    return y, info


def rfm_coefficients(plan: Plan, fact: dict, y, a=None):
    L = plan.layout
    a = torch.empty(max(L.ncols, 1), dtype=torch.float64, device=y.device) if a is None else a
    _check(_lib.rfm_coefficients(C.byref(L), _ptr(fact["rank"]), _ptr(fact["kept"]), _ptr(fact["R"]),
                                 _ptr(y), _ptr(a), _stream()), "rfm_coefficients")
    return a


# ---------------------------------------------------------------- learned warm start (MLP)
class Mlp(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_hidden", C.c_int32), ("n_out", C.c_int32), ("W1", _p), ("b1", _p),
                ("W2", _p), ("b2", _p), ("W3", _p), ("b3", _p)]


MLP_KEYS = ("W1", "b1", "W2", "b2", "W3", "b3")

_lib.rfm_mlp_ws_bytes.restype = C.c_size_t
_lib.rfm_mlp_ws_bytes.argtypes = [C.POINTER(Mlp), C.c_int32]
_lib.rfm_mlp_forward.restype = C.c_int
_lib.rfm_mlp_forward.argtypes = [C.POINTER(Mlp), _p, C.c_int32, _p, _p, _p, _p]
_lib.rfm_mlp_backward.restype = C.c_int
_lib.rfm_mlp_backward.argtypes = [C.POINTER(Mlp), C.POINTER(Mlp), _p, _p, _p, _p, _p, C.c_int32, _p, _p, _p, _p,
                                  _p, C.c_size_t, _p]
_lib.rfm_adam_step.restype = C.c_int
_lib.rfm_adam_step.argtypes = [C.c_int64, _p, _p, _p, _p, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32, _p]
_lib.rfm_gather_rows.restype = C.c_int
_lib.rfm_gather_rows.argtypes = [C.c_int32, C.c_int32, _p, _p, _p, _p]
EXPORTED += ["rfm_mlp_ws_bytes", "rfm_mlp_forward", "rfm_mlp_backward", "rfm_adam_step", "rfm_gather_rows"]


def mlp_struct(P: dict) -> Mlp:
    n_in, n_hidden = P["W1"].shape
    n_out = P["W3"].shape[1]
    return Mlp(n_in=n_in, n_hidden=n_hidden, n_out=n_out, **{k: P[k].data_ptr() for k in MLP_KEYS})


def rfm_mlp_forward(P: dict, X, H1=None, H2=None, Y=None):
    S = mlp_struct(P)
    B = X.shape[0]
    H1 = torch.empty(B, S.n_hidden, dtype=torch.float32, device=X.device) if H1 is None else H1
    H2 = torch.empty(B, S.n_hidden, dtype=torch.float32, device=X.device) if H2 is None else H2
    Y = torch.empty(B, S.n_out, dtype=torch.float32, device=X.device) if Y is None else Y
    _check(_lib.rfm_mlp_forward(C.byref(S), _ptr(X), B, _ptr(H1), _ptr(H2), _ptr(Y), _stream()), "rfm_mlp_forward")
    return H1, H2, Y


def rfm_mlp_backward(P: dict, G: dict, X, H1, H2, Y, T, scratch=None):
    S, SG = mlp_struct(P), mlp_struct(G)
    B = X.shape[0]
    dev = X.device
    if scratch is None:
        nb = _lib.rfm_mlp_ws_bytes(C.byref(S), B)
        scratch = dict(dY=torch.empty_like(Y), dH1=torch.empty_like(H1), dH2=torch.empty_like(H2),
                       loss=torch.empty(1, dtype=torch.float32, device=dev), ws=_ws(nb, dev))
    ws = scratch["ws"]
    _check(_lib.rfm_mlp_backward(C.byref(S), C.byref(SG), _ptr(X), _ptr(H1), _ptr(H2), _ptr(Y), _ptr(T), B,
                                 _ptr(scratch["dY"]), _ptr(scratch["dH1"]), _ptr(scratch["dH2"]),
                                 _ptr(scratch["loss"]), _ptr(ws), ws.numel(), _stream()), "rfm_mlp_backward")
    return scratch["loss"]


def rfm_adam_step(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(_lib.rfm_adam_step(p.numel(), _ptr(p), _ptr(g), _ptr(m), _ptr(v), lr, beta1, beta2, eps, step,
                              _stream()), "rfm_adam_step")


def rfm_gather_rows(idx, src, out):
    _check(_lib.rfm_gather_rows(idx.numel(), src.shape[1], _ptr(idx), _ptr(src), _ptr(out), _stream()),
           "rfm_gather_rows")
    return out


# ---------------------------------------------------------------- multiple right-hand sides
_lib.rfm_lsqr_multi_ws_bytes.restype = C.c_size_t
_lib.rfm_lsqr_multi_ws_bytes.argtypes = [C.POINTER(Layout), C.c_int32]
_lib.rfm_lsqr_multi.restype = C.c_int
_lib.rfm_lsqr_multi.argtypes = [C.POINTER(Layout), C.POINTER(Operator), _p, C.c_int32, _p, C.POINTER(LsqrOpts), _p,
                                _p, _p, _p, _p, C.c_size_t, _p]
EXPORTED += ["rfm_lsqr_multi_ws_bytes", "rfm_lsqr_multi"]


def rfm_lsqr_multi(plan: Plan, fact: dict, H, Y0=None, atol=1e-8, btol=1e-8, maxit=10000, check_every=64,
                   Y=None, ws=None, rejected=None):
    """H: [N, nrhs] binary64 (right-hand-side-minor); returns Y [ncols, nrhs], iters, stops.
    ``rejected`` (optional int32 numpy array [nrhs]) receives the warm-start guard's flags."""
    L = plan.layout
    B = H.shape[1]
    dev = H.device
    Y = torch.empty(max(L.ncols, 1), B, dtype=torch.float64, device=dev) if Y is None else Y
    op = Operator(form=FORM_Q, rank=fact["rank"].data_ptr(), Q=fact["Q"].data_ptr(), kept=fact["kept"].data_ptr(),
                  R=fact["R"].data_ptr())
    opts = LsqrOpts(atol=atol, btol=btol, maxit=maxit, check_every=check_every)
    nb = _lib.rfm_lsqr_multi_ws_bytes(C.byref(L), B)
    if ws is None or ws.numel() < nb:
        ws = _ws(nb, dev)
    iters = np.zeros(B, dtype=np.int64)
    stops = np.zeros(B, dtype=np.int32)
    _check(_lib.rfm_lsqr_multi(C.byref(L), C.byref(op), _ptr(H), B, _ptr(Y0), C.byref(opts), _ptr(Y),
                               _np_ptr(iters), _np_ptr(stops), _np_ptr(rejected), _ptr(ws), nb, _stream()),
           "rfm_lsqr_multi",
           allow=(RFM_ENOTCONV,))
    return Y, iters, stops


# ---------------------------------------------------------------- learned form: data and training
_lib.rfm_weighted_rhs.restype = C.c_int
_lib.rfm_weighted_rhs.argtypes = [C.c_int64, C.c_int32, _p, _p, _p, _p]
_lib.rfm_solutions_to_rows.restype = C.c_int
_lib.rfm_solutions_to_rows.argtypes = [C.c_int64, C.c_int32, _p, C.c_int64, _p, _p]
_lib.rfm_standardize_columns.restype = C.c_int
_lib.rfm_standardize_columns.argtypes = [C.c_int64, C.c_int64, _p, _p, _p, _p]
_lib.rfm_decode_start.restype = C.c_int
_lib.rfm_decode_start.argtypes = [C.POINTER(Layout), _p, C.c_int32, _p, _p, _p, _p, _p]
_lib.rfm_mlp_train.restype = C.c_int
_lib.rfm_mlp_train.argtypes = [C.POINTER(Mlp), C.POINTER(Mlp), C.POINTER(Mlp), C.POINTER(Mlp), _p, _p, C.c_int64,
                               C.c_int32, C.c_int32, C.c_float, C.c_uint64, _p, _p, C.c_size_t, _p, C.c_size_t, _p, _p]
EXPORTED += ["rfm_weighted_rhs", "rfm_solutions_to_rows", "rfm_standardize_columns", "rfm_decode_start",
             "rfm_mlp_train"]


def rfm_weighted_rhs(weight, rhs_nb):
    """rhs_nb: [N, nrhs] binary64 -> H [N, nrhs] scaled by the row weights."""
    H = torch.empty_like(rhs_nb)
    _check(_lib.rfm_weighted_rhs(rhs_nb.shape[0], rhs_nb.shape[1], _ptr(weight), _ptr(rhs_nb), _ptr(H), _stream()),
           "rfm_weighted_rhs")
    return H


def rfm_solutions_to_rows(Y, row0, out):
    _check(_lib.rfm_solutions_to_rows(Y.shape[0], Y.shape[1], _ptr(Y), row0, _ptr(out), _stream()),
           "rfm_solutions_to_rows")
    return out


def rfm_standardize_columns(T):
    mean = torch.empty(T.shape[1], dtype=torch.float32, device=T.device)
    sd = torch.empty_like(mean)
    _check(_lib.rfm_standardize_columns(T.shape[0], T.shape[1], _ptr(T), _ptr(mean), _ptr(sd), _stream()),
           "rfm_standardize_columns")
    return mean, sd


def rfm_decode_start(plan: Plan, fact: dict, pred, mean, sd):
    """pred [nrhs, ncols] binary32 -> starts [ncols, nrhs] binary64 (a vector for nrhs = 1)."""
    L = plan.layout
    B = pred.shape[0]
    y0 = torch.empty(L.ncols, B, dtype=torch.float64, device=pred.device)
    _check(_lib.rfm_decode_start(C.byref(L), _ptr(fact["rank"]), B, _ptr(pred), _ptr(mean), _ptr(sd), _ptr(y0),
                                 _stream()), "rfm_decode_start")
    return y0[:, 0].contiguous() if B == 1 else y0


def rfm_mlp_train(P: dict, X, T, epochs, batch=256, lr=1e-3, seed=0):
    """Mini-batch Adam on the device; P is updated in place.  Returns the per-epoch mean loss."""
    S = mlp_struct(P)
    dev = X.device
    G = {k: torch.zeros_like(v) for k, v in P.items()}
    Mo = {k: torch.zeros_like(v) for k, v in P.items()}
    Va = {k: torch.zeros_like(v) for k, v in P.items()}
    n = X.shape[0]
    nsc = batch * (S.n_in + 3 * S.n_out + 4 * S.n_hidden) + 65
    scratch = torch.empty(nsc, dtype=torch.float32, device=dev)
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    nb = _lib.rfm_mlp_ws_bytes(C.byref(S), batch)
    ws = _ws(nb, dev)
    hist = np.zeros(epochs, dtype=np.float32)
    _check(_lib.rfm_mlp_train(C.byref(S), C.byref(mlp_struct(G)), C.byref(mlp_struct(Mo)), C.byref(mlp_struct(Va)),
                              _ptr(X), _ptr(T), n, batch, epochs, lr, seed, _ptr(idx), _ptr(scratch), nsc, _ptr(ws),
                              nb, _np_ptr(hist), _stream()), "rfm_mlp_train")
    return hist
