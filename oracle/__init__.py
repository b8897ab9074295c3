"""Python access to the plain FP64 CPU oracle (mek_oracle.c) plus the
pseudoinverse references the paper's theorems name.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library and
its Python binding never do. Nothing here shares code with the GPU path.

Functions that are not thin wrappers of the C oracle:
  least_norm(A, C, B)      X* = A^+ C B^+, the least-norm solution (Sec. 2).
  bk_limit(A, B, C, X0)    A^+ C B^+ + X0 - A^+ A X0 B B^+, the ME-BK limit
                           (Theorem 3.3).
  spectral_alpha(B)        1 / ||B||_2^2, the step used in Sec. 5.
Each uses numpy's SVD-based pinv / norm as the library primitive.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mek_oracle.c")
_SRC_BLOCK = os.path.join(_HERE, "mek_oracle_block.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BK, RBK, GRBK, RGRBK, MWRBK = 0, 1, 2, 3, 4
VARIANTS = {"bk": BK, "rbk": RBK, "grbk": GRBK, "rgrbk": RGRBK, "mwrbk": MWRBK}
STOP_NONE, STOP_REL_ERR, STOP_REL_RESID = 0, 1, 2
OK, MAXITER, EXACT, EINVAL, ENOMEM, EDIVERGED = 0, 1, 2, -1, -2, -5


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA
    contraction), once single-threaded and once with OpenMP (the same source:
    its row loops split over threads, every sum in the same order, so both
    builds give identical results)."""
    for lib_path, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib_path):
            tmp = lib_path + ".tmp"
            subprocess.check_call(["gcc"] + _CFLAGS + extra + ["-o", tmp, _SRC, _SRC_BLOCK, "-lm"])
            os.replace(tmp, lib_path)
    return _LIB


_libs = {}


def lib(omp: bool = False):
    """The single-threaded build, or with omp=True the OpenMP build (threads
    from OMP_NUM_THREADS, else every core)."""
    if omp not in _libs:
        path = _LIB_OMP if omp else _LIB
        if not os.path.exists(path):
            build(force=False)
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        d, i64, u64 = ctypes.c_double, ctypes.c_int64, ctypes.c_uint64
        dp, lp, bp = P(d), P(i64), P(ctypes.c_ubyte)
        L.mo_philox4x64_10.argtypes = [P(u64), P(u64), P(u64)]
        L.mo_philox4x64_10.restype = None
        L.mo_threads.argtypes = []
        L.mo_threads.restype = ctypes.c_int
        L.mo_uniform.argtypes = [u64, u64, i64]
        L.mo_uniform.restype = d
        L.mo_select.argtypes = [ctypes.c_int, i64, dp, dp, d, d, u64, u64, i64, bp, dp, dp]
        L.mo_select.restype = i64
        L.mo_residual.argtypes = [i64, i64, i64, i64, dp, dp, dp, dp, dp]
        L.mo_residual.restype = None
        L.mo_gram_rows.argtypes = [i64, i64, dp, dp]
        L.mo_gram_rows.restype = None
        L.mo_gram_cols.argtypes = [i64, i64, dp, dp]
        L.mo_gram_cols.restype = None
        L.mo_solve.argtypes = [i64, i64, i64, i64, dp, dp, dp, dp, ctypes.c_int, d, d,
                               ctypes.c_int, d, dp, i64, u64, u64, lp, i64, ctypes.c_int, d,
                               dp, lp, P(ctypes.c_int), dp, dp, lp, lp, i64]
        L.mo_solve.restype = ctypes.c_int
        L.mo_select_2s.argtypes = [i64, i64, dp, dp, dp, d, d, d, i64, i64, dp, dp, d, lp,
                                   P(i64), lp, P(i64), P(d), P(d)]
        L.mo_select_2s.restype = ctypes.c_int
        L.mo_solve_2s.argtypes = [i64, i64, i64, i64, dp, dp, dp, dp, d, i64, i64, d,
                                  ctypes.c_int, d, dp, i64, d, dp, lp, P(ctypes.c_int), dp, dp,
                                  lp, lp, lp, lp, i64]
        L.mo_solve_2s.restype = ctypes.c_int
        _libs[omp] = L
    return _libs[omp]


def _dp(x: Optional[np.ndarray]):
    if x is None:
        return None
    assert x.dtype == np.float64 and x.flags.c_contiguous
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(x):
    return None if x is None else np.ascontiguousarray(x, dtype=np.float64)


def philox4x64_10(counter: Sequence[int], key: Sequence[int]) -> list:
    """The four 64-bit output words of Philox4x64-10 for one counter block."""
    u64 = ctypes.c_uint64
    c = (u64 * 4)(*[int(x) & (2 ** 64 - 1) for x in counter])
    k = (u64 * 2)(*[int(x) & (2 ** 64 - 1) for x in key])
    o = (u64 * 4)()
    lib().mo_philox4x64_10(c, k, o)
    return [int(x) for x in o]


def uniform(seed: int, inst: int, k: int) -> float:
    return float(lib().mo_uniform(seed, inst, k))


def select(variant, r, a, theta=0.5, seed=0, inst=0, k=0):
    """Run the selection rule once. Returns (i, in_set (bool m), t, T)."""
    variant = VARIANTS.get(variant, variant)
    r = _f64(r)
    a = _f64(a)
    m = r.shape[0]
    F_A = float(np.sum(a)) if m else 0.0
    # F_A must be the ascending sum the solver uses.
    s = 0.0
    for x in a:
        s += float(x)
    F_A = s
    in_set = np.zeros(m, dtype=np.uint8)
    t = ctypes.c_double(0.0)
    T = ctypes.c_double(0.0)
    i = lib().mo_select(int(variant), m, _dp(r), _dp(a), F_A, float(theta), seed, inst, k,
                        in_set.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)),
                        ctypes.byref(t), ctypes.byref(T))
    return int(i), in_set.astype(bool), t.value, T.value


def residual(A, X, B, C):
    A, X, B, C = map(_f64, (A, X, B, C))
    m, p = A.shape
    q, n = B.shape
    R = np.empty((m, n))
    lib().mo_residual(m, p, q, n, _dp(A), _dp(X), _dp(B), _dp(C), _dp(R))
    return R


def gram_rows(M):
    M = _f64(M)
    G = np.empty((M.shape[0], M.shape[0]))
    lib().mo_gram_rows(M.shape[0], M.shape[1], _dp(M), _dp(G))
    return G


def gram_cols(M):
    M = _f64(M)
    G = np.empty((M.shape[1], M.shape[1]))
    lib().mo_gram_cols(M.shape[0], M.shape[1], _dp(M), _dp(G))
    return G


class Result:
    def __init__(self, X, iters, status, s_hist, e_hist, idx_hist, set_hist):
        self.X = X
        self.iters = iters
        self.status = status
        self.s_hist = s_hist
        self.e_hist = e_hist
        self.idx = idx_hist
        self.set_sizes = set_hist


def threads(omp: bool = False) -> int:
    """Threads the oracle's row loops run on (1 for the plain build)."""
    return int(lib(omp).mo_threads())


def solve(A, B, C, X0=None, variant="grbk", theta=0.5, alpha=None, stop=STOP_NONE, tol=0.0,
          Xref=None, max_iters=1000, seed=0, inst=0, forced=None, literal=False,
          diverge=0.0, hist_cap=None, omp=False) -> Result:
    """Run the oracle iteration. See mo_solve in mek_oracle.c for semantics.
    omp=True runs the OpenMP build (same results, row loops over threads)."""
    variant = VARIANTS.get(variant, variant)
    A, B, C, X0, Xref = map(_f64, (A, B, C, X0, Xref))
    m, p = A.shape
    q, n = B.shape
    assert C.shape == (m, n)
    if alpha is None:
        alpha = spectral_alpha(B)
    X = np.empty((p, q))
    if hist_cap is None:
        hist_cap = max_iters + 1
    s_hist = np.full(hist_cap, np.nan)
    e_hist = np.full(hist_cap, np.nan)
    idx_hist = np.full(hist_cap, -1, dtype=np.int64)
    set_hist = np.zeros(hist_cap, dtype=np.int64)
    it = ctypes.c_int64(0)
    st = ctypes.c_int(0)
    if forced is not None:
        forced = np.ascontiguousarray(forced, dtype=np.int64)
        fp = forced.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        nf = forced.shape[0]
    else:
        fp, nf = None, 0
    LP = ctypes.POINTER(ctypes.c_int64)
    rc = lib(omp).mo_solve(m, p, q, n, _dp(A), _dp(B), _dp(C), _dp(X0), int(variant), float(theta),
                        float(alpha), int(stop), float(tol), _dp(Xref), int(max_iters), int(seed),
                        int(inst), fp, nf, 1 if literal else 0, float(diverge), _dp(X),
                        ctypes.byref(it), ctypes.byref(st), _dp(s_hist), _dp(e_hist),
                        idx_hist.ctypes.data_as(LP), set_hist.ctypes.data_as(LP), hist_cap)
    if rc in (EINVAL, ENOMEM) and it.value == 0 and rc != st.value:
        raise ValueError(f"oracle rejected the arguments (code {rc})")
    k = it.value
    return Result(X, k, st.value, s_hist[:k + 1], e_hist[:k + 1], idx_hist[:k], set_hist[:k])


# ----------------------------------------------------------------------------
# Two-sided block projection (mek_oracle_block.c).
# ----------------------------------------------------------------------------

TAU_DEFAULT = 1e-10


def select_2s(R, a, b, F_A, F_B, GA, GB, theta=0.5, s_max=32, t_max=32, tau=TAU_DEFAULT):
    """One selection: returns (I, J, eps, Omega), I and J in the order taken."""
    R, a, b, GA, GB = map(_f64, (R, a, b, GA, GB))
    m, n = R.shape
    I = np.full(s_max, -1, dtype=np.int64)
    J = np.full(t_max, -1, dtype=np.int64)
    nI, nJ = ctypes.c_int64(0), ctypes.c_int64(0)
    eps, Om = ctypes.c_double(0.0), ctypes.c_double(0.0)
    LP = ctypes.POINTER(ctypes.c_int64)
    rc = lib().mo_select_2s(m, n, _dp(R), _dp(a), _dp(b), float(F_A), float(F_B), float(theta),
                            int(s_max), int(t_max), _dp(GA), _dp(GB), float(tau),
                            I.ctypes.data_as(LP), ctypes.byref(nI), J.ctypes.data_as(LP),
                            ctypes.byref(nJ), ctypes.byref(eps), ctypes.byref(Om))
    if rc != 0:
        raise ValueError("no entry with a_i > 0 and b_j > 0")
    return I[:nI.value], J[:nJ.value], eps.value, Om.value


class Result2s:
    def __init__(self, X, iters, status, s_hist, e_hist, I_hist, J_hist, nI, nJ):
        self.X = X
        self.iters = iters
        self.status = status
        self.s_hist = s_hist
        self.e_hist = e_hist
        self.I = [I_hist[k, :nI[k]] for k in range(iters)]
        self.J = [J_hist[k, :nJ[k]] for k in range(iters)]


def solve_2s(A, B, C, X0=None, theta=0.5, s_max=32, t_max=32, tau=TAU_DEFAULT, stop=STOP_NONE,
             tol=0.0, Xref=None, max_iters=100, diverge=0.0, hist_cap=None) -> Result2s:
    """Run the two-sided block iteration. See mo_solve_2s in mek_oracle_block.c."""
    A, B, C, X0, Xref = map(_f64, (A, B, C, X0, Xref))
    m, p = A.shape
    q, n = B.shape
    assert C.shape == (m, n)
    X = np.empty((p, q))
    if hist_cap is None:
        hist_cap = max_iters + 1
    s_hist = np.full(hist_cap, np.nan)
    e_hist = np.full(hist_cap, np.nan)
    I_hist = np.full((hist_cap, s_max), -1, dtype=np.int64)
    J_hist = np.full((hist_cap, t_max), -1, dtype=np.int64)
    nI = np.zeros(hist_cap, dtype=np.int64)
    nJ = np.zeros(hist_cap, dtype=np.int64)
    it = ctypes.c_int64(0)
    st = ctypes.c_int(0)
    LP = ctypes.POINTER(ctypes.c_int64)
    rc = lib().mo_solve_2s(m, p, q, n, _dp(A), _dp(B), _dp(C), _dp(X0), float(theta),
                           int(s_max), int(t_max), float(tau), int(stop), float(tol), _dp(Xref),
                           int(max_iters), float(diverge), _dp(X), ctypes.byref(it),
                           ctypes.byref(st), _dp(s_hist), _dp(e_hist), I_hist.ctypes.data_as(LP),
                           J_hist.ctypes.data_as(LP), nI.ctypes.data_as(LP),
                           nJ.ctypes.data_as(LP), hist_cap)
    if rc in (EINVAL, ENOMEM) and it.value == 0:
        raise ValueError(f"oracle rejected the arguments (code {rc})")
    k = it.value
    kk = min(k, hist_cap)
    return Result2s(X, kk, st.value, s_hist[:k + 1], e_hist[:k + 1], I_hist, J_hist, nI, nJ)


# ----------------------------------------------------------------------------
# Closed forms from the paper, computed with numpy's SVD-based pinv.
# ----------------------------------------------------------------------------

def least_norm(A, C, B):
    """X* = A^+ C B^+ (the unique least-norm solution, Sec. 2)."""
    return np.linalg.pinv(A) @ C @ np.linalg.pinv(B)


def bk_limit(A, B, C, X0):
    """A^+ C B^+ + X0 - A^+ A X0 B B^+ (Theorem 3.3)."""
    Ap = np.linalg.pinv(A)
    Bp = np.linalg.pinv(B)
    return Ap @ C @ Bp + X0 - Ap @ A @ X0 @ B @ Bp


def spectral_alpha(B):
    """alpha = 1 / ||B||_2^2 (Sec. 5)."""
    return 1.0 / np.linalg.norm(B, 2) ** 2
