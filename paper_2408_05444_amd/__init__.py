"""Python binding of libmek.so: greedy randomized block Kaczmarz solvers for
A X B = C on AMD MI355X (gfx950).

The functions below carry the names of the C ABI in include/mek.h and only
marshal arguments: torch tensors on the GPU (float64, contiguous, row-major)
become device pointers, the current torch stream becomes the HIP stream,
and results come back as tensors. Every numerical step runs in the library's
HIP kernels; if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import sys
import math
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmek.so")

MEK_BK, MEK_RBK, MEK_GRBK, MEK_RGRBK, MEK_MWRBK = 0, 1, 2, 3, 4
MEK_TWOSIDED = 5
VARIANTS = {"bk": MEK_BK, "rbk": MEK_RBK, "grbk": MEK_GRBK, "rgrbk": MEK_RGRBK, "mwrbk": MEK_MWRBK,
            "twosided": MEK_TWOSIDED}
MEK_STOP_NONE, MEK_STOP_REL_ERR, MEK_STOP_REL_RESID = 0, 1, 2
STOPS = {"none": 0, "rel_err": 1, "rel_resid": 2}
MEK_FP64, MEK_FP32, MEK_MIXED = 0, 1, 2
MEK_UPDATE_DENSE, MEK_UPDATE_SPARSE = 0, 1
UPDATES = {"dense": MEK_UPDATE_DENSE, "sparse": MEK_UPDATE_SPARSE}
PRECISIONS = {"fp64": 0, "fp32": 1, "mixed": 2}
MEK_OK, MEK_MAXITER, MEK_EXACT = 0, 1, 2
MEK_EINVAL, MEK_ENOMEM, MEK_EHIP, MEK_ENONFINITE = -1, -2, -3, -4
MEK_EDIVERGED, MEK_EUNSUPPORTED, MEK_ETIMEOUT = -5, -6, -7


class MekError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {mek_status_string(code)} ({code})")


class mek_plan_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("alpha", ctypes.c_double),
                ("team_wgs", ctypes.c_int), ("r_in_lds", ctypes.c_int),
                ("update", ctypes.c_int)]


class mek_solve_opts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int), ("theta", ctypes.c_double),
                ("alpha", ctypes.c_double), ("stop", ctypes.c_int), ("tol", ctypes.c_double),
                ("X_ref", ctypes.c_void_p), ("max_iters", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("instance", ctypes.c_uint64),
                ("replay_idx", ctypes.c_void_p), ("replay_len", ctypes.c_int64),
                ("diverge", ctypes.c_double),
                ("resid_hist", ctypes.c_void_p), ("err_hist", ctypes.c_void_p),
                ("idx_hist", ctypes.c_void_p), ("set_hist", ctypes.c_void_p),
                ("hist_cap", ctypes.c_int64), ("inner_iters", ctypes.c_int64),
                ("block_rows", ctypes.c_int), ("block_cols", ctypes.c_int),
                ("tau", ctypes.c_double), ("rows_hist", ctypes.c_void_p),
                ("cols_hist", ctypes.c_void_p), ("refresh_period", ctypes.c_int64)]


class mek_report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("status", ctypes.c_int), ("resid2", ctypes.c_double),
                ("rel_err", ctypes.c_double), ("alpha", ctypes.c_double),
                ("team_wgs", ctypes.c_int), ("r_in_lds", ctypes.c_int), ("passes", ctypes.c_int),
                ("kernel_ms", ctypes.c_double)]


_lib_handle = None


def lib() -> ctypes.CDLL:
    """Load libmek.so (building it first only if no build exists)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, u64, d, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
        L.mek_version.argtypes = []
        L.mek_version.restype = ci
        L.mek_status_string.argtypes = [ci]
        L.mek_status_string.restype = ctypes.c_char_p
        L.mek_plan_create.argtypes = [ctypes.POINTER(vp), i64, i64, i64, i64, vp, vp,
                                      ctypes.POINTER(mek_plan_opts), vp]
        L.mek_plan_create.restype = ci
        L.mek_plan_destroy.argtypes = [vp]
        L.mek_plan_destroy.restype = ci
        L.mek_plan_query.argtypes = [vp, vp, vp, vp, ctypes.POINTER(d), vp]
        L.mek_plan_query.restype = ci
        L.mek_plan_sparse_widths.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.mek_plan_sparse_widths.restype = ci
        L.mek_solve.argtypes = [vp, vp, vp, ctypes.POINTER(mek_solve_opts), vp,
                                ctypes.POINTER(mek_report), vp]
        L.mek_solve.restype = ci
        L.mek_solve_batched.argtypes = [vp, i64, vp, vp, ctypes.POINTER(mek_solve_opts), vp,
                                        ctypes.POINTER(mek_report), vp]
        L.mek_solve_batched.restype = ci
        L.mek_solve_multi.argtypes = [i64, vp, vp, vp, vp, ctypes.POINTER(mek_solve_opts), vp,
                                      vp, vp]
        L.mek_solve_multi.restype = ci
        L.mek_solve_async.argtypes = [vp, vp, vp, ctypes.POINTER(mek_solve_opts), vp, vp, vp]
        L.mek_solve_async.restype = ci
        L.mek_solve_multi_async.argtypes = [i64, vp, vp, vp, vp, ctypes.POINTER(mek_solve_opts),
                                            vp, vp, vp]
        L.mek_solve_multi_async.restype = ci
        L.mek_cnn_conv3x3.argtypes = [i64, i64, i64, i64, i64, vp, vp, vp, ci, vp, vp, vp, vp]
        L.mek_cnn_conv3x3.restype = ci
        L.mek_cnn_conv3x3_grad_input.argtypes = [i64, i64, i64, i64, i64, vp, vp, vp, vp, vp]
        L.mek_cnn_conv3x3_grad_input.restype = ci
        L.mek_cnn_conv3x3_grad_weight.argtypes = [i64, i64, i64, i64, i64, vp, vp, vp, vp, vp, vp]
        L.mek_cnn_conv3x3_grad_weight.restype = ci
        L.mek_cnn_mse_grad.argtypes = [i64, vp, vp, vp, ctypes.POINTER(d), vp]
        L.mek_cnn_mse_grad.restype = ci
        L.mek_cnn_adam.argtypes = [i64, vp, vp, vp, vp, vp, d, d, d, d, i64, vp]
        L.mek_cnn_adam.restype = ci
        L.mek_cnn_to_bf16.argtypes = [i64, vp, d, vp, vp]
        L.mek_cnn_to_bf16.restype = ci
        L.mek_cnn_round_bf16.argtypes = [i64, vp, vp, vp]
        L.mek_cnn_round_bf16.restype = ci
        L.mek_philox_uniform.argtypes = [u64, u64, i64, i64, vp, vp]
        L.mek_philox_uniform.restype = ci
        L.mek_select.argtypes = [ci, i64, vp, vp, d, d, u64, u64, i64, i64, vp, vp, vp, vp, vp]
        L.mek_select.restype = ci
        L.mek_residual.argtypes = [i64, i64, i64, i64, vp, vp, vp, vp, vp, vp]
        L.mek_residual.restype = ci
        L.mek_residual_batched.argtypes = [i64, i64, i64, i64, i64, vp, vp, vp, vp, vp, vp]
        L.mek_residual_batched.restype = ci
        L.mek_residual_noalloc.argtypes = [i64, i64, i64, i64, vp, vp, vp, vp, vp, vp]
        L.mek_residual_noalloc.restype = ci
        L.mek_exchange_floor.argtypes = [i64, i64, i64, i64, i64, vp, vp]
        L.mek_exchange_floor.restype = ci
        L.mek_residual_split.argtypes = [ci, i64, i64, i64, i64, i64, vp, vp, vp, vp, vp, vp]
        L.mek_residual_split.restype = ci
        L.mek_gram.argtypes = [i64, i64, vp, ci, vp, vp]
        L.mek_gram.restype = ci
        _lib_handle = L
    return _lib_handle


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: Optional[torch.Tensor], dtype=torch.float64, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _check(code: int, where: str, ok=(MEK_OK,)):
    if code not in ok:
        raise MekError(code, where)
    return code


def mek_version() -> int:
    return int(lib().mek_version())


def mek_status_string(code: int) -> str:
    return lib().mek_status_string(int(code)).decode()


@dataclass
class Plan:
    handle: ctypes.c_void_p
    m: int
    p: int
    q: int
    n: int
    precision: int

    def __del__(self, _finalizing=sys.is_finalizing):
        # A plan dropped during interpreter shutdown is left to the process
        # exit: by then the HIP runtime (and any profiler attached to it) may
        # already be tearing down, and a device synchronise or free issued
        # from a finaliser at that point can crash the exit path. (The check
        # is bound as a default: module globals may already be cleared.)
        if _finalizing():
            return
        try:
            if self.handle:
                lib().mek_plan_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        mek_plan_destroy(self)
        return False


def mek_plan_create(A: torch.Tensor, B: torch.Tensor, precision="fp64", alpha: float = 0.0,
                    team_wgs: int = 0, r_in_lds: int = -1, update="dense") -> Plan:
    """update "sparse": updates touch only the rows that the nonzeros of A,
    B and A A^T reach, one work-group per instance."""
    m, p = A.shape
    q, n = B.shape
    prec = PRECISIONS.get(precision, precision)
    o = mek_plan_opts(int(prec), float(alpha), int(team_wgs), int(r_in_lds),
                      int(UPDATES.get(update, update)))
    h = ctypes.c_void_p()
    code = lib().mek_plan_create(ctypes.byref(h), m, p, q, n, _dev(A, name="A"), _dev(B, name="B"),
                                 ctypes.byref(o), _stream())
    _check(code, "mek_plan_create")
    return Plan(h, m, p, q, n, int(prec))


def mek_plan_destroy(plan: Plan) -> None:
    if plan.handle:
        _check(lib().mek_plan_destroy(plan.handle), "mek_plan_destroy")
        plan.handle = None


def mek_plan_query(plan: Plan):
    """(row_norms (m), A A^T (m x m), B^T B (n x n), alpha)."""
    dev = torch.device("cuda")
    a = torch.empty(plan.m, dtype=torch.float64, device=dev)
    GA = torch.empty(plan.m, plan.m, dtype=torch.float64, device=dev)
    GB = torch.empty(plan.n, plan.n, dtype=torch.float64, device=dev)
    al = ctypes.c_double(0.0)
    _check(lib().mek_plan_query(plan.handle, _dev(a), _dev(GA), _dev(GB), ctypes.byref(al),
                                _stream()), "mek_plan_query")
    return a, GA, GB, al.value


def mek_plan_sparse_widths(plan: Plan):
    """Nonzeros per line of a sparse plan: (rows of A, rows of B, columns of
    B, columns of A A^T)."""
    w = (ctypes.c_int32 * 4)()
    _check(lib().mek_plan_sparse_widths(plan.handle, w), "mek_plan_sparse_widths")
    return tuple(int(x) for x in w)


@dataclass
class SolveResult:
    X: torch.Tensor
    status: int
    iters: int
    resid2: float
    rel_err: float
    alpha: float
    team_wgs: int
    r_in_lds: bool
    passes: int
    kernel_ms: float = 0.0
    resid_hist: Optional[torch.Tensor] = None
    err_hist: Optional[torch.Tensor] = None
    idx_hist: Optional[torch.Tensor] = None
    set_hist: Optional[torch.Tensor] = None
    rows_hist: Optional[list] = None
    cols_hist: Optional[list] = None


def _solve_opts(nb, dev, variant, theta, alpha, stop, tol, X_ref_ptr, max_iters, seed, instance,
                replay_idx, diverge, hist_cap, inner_iters, block_rows=0, block_cols=0, tau=0.0,
                refresh_period=0):
    hists = {}
    twosided = VARIANTS.get(variant, variant) == MEK_TWOSIDED
    if hist_cap > 0:
        hists["resid_hist"] = torch.full((nb, hist_cap), float("nan"), dtype=torch.float64, device=dev)
        hists["err_hist"] = torch.full((nb, hist_cap), float("nan"), dtype=torch.float64, device=dev)
        if twosided:
            hists["rows_hist"] = torch.full((nb, hist_cap, block_rows), -1, dtype=torch.int32,
                                            device=dev)
            hists["cols_hist"] = torch.full((nb, hist_cap, block_cols), -1, dtype=torch.int32,
                                            device=dev)
        else:
            hists["idx_hist"] = torch.full((nb, hist_cap), -1, dtype=torch.int32, device=dev)
            hists["set_hist"] = torch.zeros((nb, hist_cap), dtype=torch.int32, device=dev)
    o = mek_solve_opts()
    o.block_rows = int(block_rows)
    o.block_cols = int(block_cols)
    o.tau = float(tau)
    o.variant = VARIANTS.get(variant, variant)
    o.theta = float(theta)
    o.alpha = float(alpha)
    o.stop = STOPS.get(stop, stop)
    o.tol = float(tol)
    o.X_ref = X_ref_ptr
    o.max_iters = int(max_iters)
    o.seed = int(seed) & (2 ** 64 - 1)
    o.instance = int(instance) & (2 ** 64 - 1)
    if replay_idx is not None:
        o.replay_idx = _dev(replay_idx, dtype=torch.int32, name="replay_idx")
        o.replay_len = replay_idx.numel()
    o.diverge = float(diverge)
    for k, t in hists.items():
        setattr(o, k, _dev(t, dtype=t.dtype, name=k))
    o.hist_cap = int(hist_cap)
    o.inner_iters = int(inner_iters)
    o.refresh_period = int(refresh_period)
    return o, hists


def _result(X, code, rep, hists, b, hist_cap):
    res = SolveResult(X, int(code), int(rep.iters), rep.resid2, rep.rel_err, rep.alpha,
                      int(rep.team_wgs), bool(rep.r_in_lds), int(rep.passes), rep.kernel_ms)
    if hist_cap > 0:
        k = min(int(rep.iters), hist_cap - 1)
        kk = min(int(rep.iters), hist_cap)
        res.resid_hist = hists["resid_hist"][b, :k + 1]
        res.err_hist = hists["err_hist"][b, :k + 1]
        if "rows_hist" in hists:
            rows = hists["rows_hist"][b, :kk].cpu()
            cols = hists["cols_hist"][b, :kk].cpu()
            res.rows_hist = [r[r >= 0].tolist() for r in rows]
            res.cols_hist = [c[c >= 0].tolist() for c in cols]
        else:
            res.idx_hist = hists["idx_hist"][b, :kk]
            res.set_hist = hists["set_hist"][b, :kk]
    return res


def mek_solve(plan: Plan, C: torch.Tensor, X0: Optional[torch.Tensor] = None, variant="grbk",
              theta: float = 0.5, alpha: float = 0.0, stop="none", tol: float = 0.0,
              X_ref: Optional[torch.Tensor] = None, max_iters: int = 100000, seed: int = 0,
              instance: int = 0, replay_idx: Optional[torch.Tensor] = None, diverge: float = 0.0,
              hist_cap: int = 0, inner_iters: int = 0, X_out: Optional[torch.Tensor] = None,
              block_rows: int = 32, block_cols: int = 32, tau: float = 0.0,
              refresh_period: int = 0, raise_on_error: bool = True) -> SolveResult:
    """variant "twosided" takes block_rows / block_cols (1..32) and tau; its
    histories are rows_hist / cols_hist (lists of I and J per step)."""
    m, p, q, n = plan.m, plan.p, plan.q, plan.n
    dev = C.device
    X = X_out if X_out is not None else torch.empty(p, q, dtype=torch.float64, device=dev)
    o, hists = _solve_opts(1, dev, variant, theta, alpha, stop, tol,
                           _dev(X_ref, shape=(p, q), name="X_ref"), max_iters, seed, instance,
                           replay_idx, diverge, hist_cap, inner_iters, block_rows, block_cols, tau,
                           refresh_period)
    rep = mek_report()
    code = lib().mek_solve(plan.handle, _dev(C, shape=(m, n), name="C"),
                           _dev(X0, shape=(p, q), name="X0"), ctypes.byref(o),
                           _dev(X, shape=(p, q), name="X"), ctypes.byref(rep), _stream())
    if raise_on_error and code < 0:
        raise MekError(code, "mek_solve")
    return _result(X, code, rep, hists, 0, hist_cap)


def mek_solve_batched(plan: Plan, C: torch.Tensor, X0: Optional[torch.Tensor] = None,
                      variant="grbk", theta: float = 0.5, alpha: float = 0.0, stop="none",
                      tol: float = 0.0, X_ref: Optional[torch.Tensor] = None,
                      max_iters: int = 100000, seed: int = 0, instance: int = 0,
                      replay_idx: Optional[torch.Tensor] = None, diverge: float = 0.0,
                      hist_cap: int = 0, inner_iters: int = 0, block_rows: int = 32,
                      block_cols: int = 32, tau: float = 0.0, refresh_period: int = 0,
                      raise_on_error: bool = True):
    """Uniform batch: C (nb, m, n) [, X0, X_ref (nb, p, q)] sharing the plan's A
    and B. Returns (status, [SolveResult per instance]); instance b draws
    under Philox key (seed, instance + b)."""
    m, p, q, n = plan.m, plan.p, plan.q, plan.n
    nb = C.shape[0]
    dev = C.device
    X = torch.empty(nb, p, q, dtype=torch.float64, device=dev)
    o, hists = _solve_opts(nb, dev, variant, theta, alpha, stop, tol,
                           _dev(X_ref, shape=(nb, p, q), name="X_ref"), max_iters, seed,
                           instance, replay_idx, diverge, hist_cap, inner_iters, block_rows,
                           block_cols, tau, refresh_period)
    reps = (mek_report * nb)()
    code = lib().mek_solve_batched(plan.handle, nb, _dev(C, shape=(nb, m, n), name="C"),
                                   _dev(X0, shape=(nb, p, q), name="X0"), ctypes.byref(o),
                                   _dev(X, shape=(nb, p, q), name="X"), reps, _stream())
    if raise_on_error and code < 0:
        raise MekError(code, "mek_solve_batched")
    return int(code), [_result(X[b], reps[b].status, reps[b], hists, b, hist_cap)
                       for b in range(nb)]


DEVICE_REPORT_BYTES = 32   # mek_device_report: int64 iters, int32 status, int32 last_set,
                           # double resid2, double rel_err


def mek_solve_async(plan: Plan, C: torch.Tensor, X0: Optional[torch.Tensor] = None,
                    variant="grbk", theta: float = 0.5, alpha: float = 0.0, stop="none",
                    tol: float = 0.0, X_ref: Optional[torch.Tensor] = None,
                    max_iters: int = 100000, seed: int = 0, instance: int = 0,
                    diverge: float = 0.0, X_out: Optional[torch.Tensor] = None,
                    report: Optional[torch.Tensor] = None, hist: Optional[dict] = None):
    """Stream-ordered solve on the current stream; returns (X, report) where
    report is a 32-byte device tensor holding mek_device_report (decode it
    with read_device_report once the stream has passed the call). With
    `hist` (a dict from make_histories) the histories are recorded there."""
    m, p, q, n = plan.m, plan.p, plan.q, plan.n
    dev = C.device
    X = X_out if X_out is not None else torch.empty(p, q, dtype=torch.float64, device=dev)
    rep = report if report is not None else torch.zeros(DEVICE_REPORT_BYTES, dtype=torch.uint8,
                                                        device=dev)
    o, _ = _solve_opts(1, dev, variant, theta, alpha, stop, tol,
                       _dev(X_ref, shape=(p, q), name="X_ref"), max_iters, seed, instance, None,
                       diverge, 0, 0)
    if hist is not None:
        o.hist_cap = hist["cap"]
        o.resid_hist = _dev(hist["resid_hist"])
        o.err_hist = _dev(hist["err_hist"])
        o.idx_hist = _dev(hist["idx_hist"], dtype=torch.int32)
        o.set_hist = _dev(hist["set_hist"], dtype=torch.int32)
    _check(lib().mek_solve_async(plan.handle, _dev(C, shape=(m, n), name="C"),
                                 _dev(X0, shape=(p, q), name="X0"), ctypes.byref(o),
                                 _dev(X, shape=(p, q), name="X"), _dev(rep, dtype=torch.uint8),
                                 _stream()), "mek_solve_async")
    return X, rep


def make_histories(cap: int, device="cuda", nb: Optional[int] = None) -> dict:
    """Device history buffers for the stream-ordered solves: cap entries
    each, or (nb, cap) for a batch."""
    shp = (cap,) if nb is None else (nb, cap)
    return {"cap": cap,
            "resid_hist": torch.full(shp, float("nan"), dtype=torch.float64, device=device),
            "err_hist": torch.full(shp, float("nan"), dtype=torch.float64, device=device),
            "idx_hist": torch.full(shp, -1, dtype=torch.int32, device=device),
            "set_hist": torch.zeros(shp, dtype=torch.int32, device=device)}


def read_device_report(rep: torch.Tensor) -> dict:
    import struct
    it, st, ls, r2, err = struct.unpack("<qiidd", bytes(rep.cpu().tolist()))
    return {"iters": it, "status": st, "last_set": ls, "resid2": r2, "rel_err": err}


def _ptr_array(tensors, shapes, name):
    """Host array of device pointers (NULL for None entries)."""
    arr = (ctypes.c_void_p * len(tensors))()
    for b, (t, shp) in enumerate(zip(tensors, shapes)):
        arr[b] = _dev(t, shape=shp, name=f"{name}[{b}]") if t is not None else None
    return arr


def mek_solve_multi(plans, C, X0=None, X_ref=None, variant="grbk", theta: float = 0.5,
                    alpha: float = 0.0, stop="none", tol: float = 0.0, max_iters: int = 100000,
                    seed: int = 0, instance: int = 0, diverge: float = 0.0, hist_cap: int = 0,
                    raise_on_error: bool = True):
    """Ragged batch: plans[b] with its own A_b, B_b; C, X0, X_ref are lists of
    per-instance tensors (X0 / X_ref entries may be None). One persistent
    launch; instance b draws under Philox key (seed, instance + b). Returns
    (status, [SolveResult per instance])."""
    nb = len(plans)
    if len(C) != nb:
        raise ValueError("one C per plan")
    dev = C[0].device
    pq = [(P.p, P.q) for P in plans]
    X = [torch.empty(p, q, dtype=torch.float64, device=dev) for p, q in pq]
    handles = (ctypes.c_void_p * nb)(*[P.handle for P in plans])
    Cp = _ptr_array(C, [(P.m, P.n) for P in plans], "C")
    X0p = _ptr_array(X0, pq, "X0") if X0 is not None else None
    Xrp = _ptr_array(X_ref, pq, "X_ref") if X_ref is not None else None
    Xp = _ptr_array(X, pq, "X")
    o, hists = _solve_opts(nb, dev, variant, theta, alpha, stop, tol, None, max_iters, seed,
                           instance, None, diverge, hist_cap, 0)
    reps = (mek_report * nb)()
    code = lib().mek_solve_multi(nb, handles, Cp, X0p, Xrp, ctypes.byref(o), Xp, reps, _stream())
    if raise_on_error and code < 0:
        raise MekError(code, "mek_solve_multi")
    return int(code), [_result(X[b], reps[b].status, reps[b], hists, b, hist_cap)
                       for b in range(nb)]


def mek_solve_multi_async(plans, C, X0=None, X_ref=None, variant="grbk", theta: float = 0.5,
                          alpha: float = 0.0, stop="none", tol: float = 0.0,
                          max_iters: int = 100000, seed: int = 0, instance: int = 0,
                          diverge: float = 0.0, X_out=None, reports=None, hist=None):
    """Stream-ordered ragged batch on the current stream; returns (X list,
    reports) where reports is an (nb, 32) uint8 device tensor, row b holding
    instance b's mek_device_report (decode with read_device_report once the
    stream has passed the call). X_out (list) and reports may be given, for
    instance to capture the call into a graph; hist = make_histories(cap,
    nb=nb) records the histories."""
    nb = len(plans)
    if len(C) != nb:
        raise ValueError("one C per plan")
    dev = C[0].device
    pq = [(P.p, P.q) for P in plans]
    X = X_out if X_out is not None else [torch.empty(p, q, dtype=torch.float64, device=dev)
                                         for p, q in pq]
    rep = reports if reports is not None else torch.zeros(nb, DEVICE_REPORT_BYTES,
                                                          dtype=torch.uint8, device=dev)
    handles = (ctypes.c_void_p * nb)(*[P.handle for P in plans])
    Cp = _ptr_array(C, [(P.m, P.n) for P in plans], "C")
    X0p = _ptr_array(X0, pq, "X0") if X0 is not None else None
    Xrp = _ptr_array(X_ref, pq, "X_ref") if X_ref is not None else None
    Xp = _ptr_array(X, pq, "X")
    o, _ = _solve_opts(nb, dev, variant, theta, alpha, stop, tol, None, max_iters, seed,
                       instance, None, diverge, 0, 0)
    if hist is not None:
        o.hist_cap = hist["cap"]
        o.resid_hist = _dev(hist["resid_hist"])
        o.err_hist = _dev(hist["err_hist"])
        o.idx_hist = _dev(hist["idx_hist"], dtype=torch.int32)
        o.set_hist = _dev(hist["set_hist"], dtype=torch.int32)
    _check(lib().mek_solve_multi_async(nb, handles, Cp, X0p, Xrp, ctypes.byref(o), Xp,
                                       _dev(rep, dtype=torch.uint8), _stream()),
           "mek_solve_multi_async")
    return X, rep


def mek_philox_uniform(seed: int, instance: int, k0: int, count: int) -> torch.Tensor:
    out = torch.empty(max(count, 1), dtype=torch.float64, device="cuda")
    _check(lib().mek_philox_uniform(int(seed) & (2 ** 64 - 1), int(instance) & (2 ** 64 - 1),
                                    int(k0), int(count), _dev(out), _stream()),
           "mek_philox_uniform")
    return out[:count]


def mek_select(variant, r: torch.Tensor, a: torch.Tensor, F_A: float, theta: float = 0.5,
               seed: int = 0, instance: int = 0, k0: int = 0, count: int = 1):
    """Returns (idx (count,), in_set (m,) bool, set_list (size,), stats dict)."""
    m = r.numel()
    v = VARIANTS.get(variant, variant)
    idx = torch.empty(max(count, 1), dtype=torch.int32, device="cuda")
    in_set = torch.zeros(m, dtype=torch.uint8, device="cuda")
    set_list = torch.full((m,), -1, dtype=torch.int32, device="cuda")
    stats = torch.zeros(4, dtype=torch.float64, device="cuda")
    _check(lib().mek_select(int(v), m, _dev(r, name="r"), _dev(a, name="a"), float(F_A),
                            float(theta), int(seed) & (2 ** 64 - 1), int(instance) & (2 ** 64 - 1),
                            int(k0), int(count), _dev(idx, dtype=torch.int32),
                            _dev(in_set, dtype=torch.uint8), _dev(set_list, dtype=torch.int32),
                            _dev(stats), _stream()), "mek_select")
    st = stats.cpu().tolist()
    size = int(st[3])
    return idx[:count], in_set.bool(), set_list[:size], {"t": st[0], "T": st[1], "S": st[2],
                                                         "size": size}


def mek_residual(A, X, B, C) -> torch.Tensor:
    m, p = A.shape
    q, n = B.shape
    R = torch.empty(m, n, dtype=torch.float64, device=A.device)
    _check(lib().mek_residual(m, p, q, n, _dev(A, name="A"), _dev(X, shape=(p, q), name="X"),
                              _dev(B, name="B"), _dev(C, shape=(m, n), name="C"), _dev(R),
                              _stream()), "mek_residual")
    return R


def mek_residual_batched(A, X, B, C) -> torch.Tensor:
    """R_b = C_b - A X_b B for X (nb, p, q) and C (nb, m, n) sharing A, B."""
    m, p = A.shape
    q, n = B.shape
    nb = X.shape[0]
    R = torch.empty(nb, m, n, dtype=torch.float64, device=A.device)
    _check(lib().mek_residual_batched(nb, m, p, q, n, _dev(A, name="A"),
                                      _dev(X, shape=(nb, p, q), name="X"), _dev(B, name="B"),
                                      _dev(C, shape=(nb, m, n), name="C"), _dev(R), _stream()),
           "mek_residual_batched")
    return R


def mek_residual_split(A, X, B, C, pieces: int = 3) -> torch.Tensor:
    """R_b = C_b - (A X_b) B on the BF16 matrix cores with FP32 operands
    split into `pieces` bf16 terms: A (m, p), B (q, n) float32; X (nb, p, q)
    float32; C (nb, m, n) float64; returns R (nb, m, n) float32."""
    m, p = A.shape
    q, n = B.shape
    nb = X.shape[0]
    R = torch.empty(nb, m, n, dtype=torch.float32, device=A.device)
    _check(lib().mek_residual_split(int(pieces), nb, m, p, q, n,
                                    _dev(A, torch.float32, name="A"),
                                    _dev(X, torch.float32, shape=(nb, p, q), name="X"),
                                    _dev(B, torch.float32, name="B"),
                                    _dev(C, shape=(nb, m, n), name="C"),
                                    _dev(R, torch.float32), _stream()), "mek_residual_split")
    return R


def mek_exchange_floor(W: int, m: int, n: int, q: int, rounds: int = 20000) -> float:
    """Microseconds per round of the team solver's exchanges alone (W
    work-groups, m rows, n columns of R, q columns of X)."""
    us = ctypes.c_double(0.0)
    _check(lib().mek_exchange_floor(int(W), int(m), int(n), int(q), int(rounds),
                                    ctypes.byref(us), _stream()), "mek_exchange_floor")
    return us.value


def mek_gram(M: torch.Tensor, transpose_first: bool) -> torch.Tensor:
    rows, cols = M.shape
    g = cols if transpose_first else rows
    G = torch.empty(g, g, dtype=torch.float64, device=M.device)
    _check(lib().mek_gram(rows, cols, _dev(M, name="M"), 1 if transpose_first else 0, _dev(G),
                          _stream()), "mek_gram")
    return G


def solve(A, B, C, X0=None, variant="grbk", relaxation=0.5, tol=1e-6, seed=0, X_ref=None,
          max_iters=10_000_000, precision="fp64", update="dense", **kw) -> SolveResult:
    """One-shot solve(A, B, C, X0, variant, relaxation, tol, seed).

    With X_ref the rule is ||X - X_ref||_F <= tol ||X_ref||_F, otherwise
    ||C - A X B||_F <= tol ||C||_F. update "sparse" for banded / sparse A
    and B.
    """
    plan = mek_plan_create(A, B, precision=precision, update=update)
    try:
        return mek_solve(plan, C, X0=X0, variant=variant, theta=relaxation,
                         stop="rel_err" if X_ref is not None else "rel_resid", tol=tol,
                         X_ref=X_ref, max_iters=max_iters, seed=seed, **kw)
    finally:
        mek_plan_destroy(plan)
