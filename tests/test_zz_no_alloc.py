"""The residual engine that allocates nothing (mek_residual_noalloc), called
through the C ABI, against the allocating entry point mek_residual on the
same inputs: two calls in a row, the second with a smaller input (the
shared per-device scratch keeps the first call's contents), then a size
beyond the scratch, which must be refused. Same kernels on both sides, so
the results must agree bit for bit; both are also held to the FP64 GEMM
bound against the oracle's residual (K <= 600 terms of size O(1):
|R_gpu - R| <= 1e-12 max|R| with a margin for the sum's growth)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2408_05444_amd as mek

pytestmark = pytest.mark.gpu

SCRATCH_DOUBLES = 1 << 21


def _call_noalloc(A, X, B, C):
    L = mek.lib()
    L.mek_residual_noalloc.argtypes = [ctypes.c_int64] * 4 + [ctypes.c_void_p] * 6
    L.mek_residual_noalloc.restype = ctypes.c_int
    m, p = A.shape
    q, n = B.shape
    R = torch.full((m, n), float("nan"), dtype=torch.float64, device=A.device)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    st = L.mek_residual_noalloc(m, p, q, n, vp(A), vp(X), vp(B), vp(C), vp(R),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st, R


def _inputs(seed, m, p, q, n):
    rng = np.random.default_rng(seed)
    A, X, B = rng.standard_normal((m, p)), rng.standard_normal((p, q)), rng.standard_normal((q, n))
    C = A @ X @ B + rng.standard_normal((m, n))
    d = torch.device("cuda:0")
    return [torch.from_numpy(v).to(d) for v in (A, X, B, C)], (A, X, B, C)


def test_noalloc_residual_matches_the_allocating_entry_point():
    # The first call fills most of the scratch (2000 x 500 of 2^21), the
    # second uses a smaller, ragged part of it.
    for seed, shape in [(1, (2000, 500, 500, 2000)), (2, (77, 45, 37, 130))]:
        (A, X, B, C), host = _inputs(seed, *shape)
        st, R = _call_noalloc(A, X, B, C)
        assert st == mek.MEK_OK
        R_ref = mek.mek_residual(A, X, B, C)
        assert torch.equal(R, R_ref), float((R - R_ref).abs().max())
        m = shape[0]
        rows = np.unique(np.r_[0, m - 1, np.random.default_rng(seed).choice(m, 16)])
        Ro = oracle.residual(host[0][rows], host[1], host[2], host[3][rows])
        err = np.abs(R.cpu().numpy()[rows] - Ro)
        assert err.max() <= 1e-12 * max(1.0, np.abs(Ro).max()) * 4


def test_noalloc_refuses_a_temporary_beyond_the_scratch():
    m, q = 4097, 512                       # m q = 2^21 + 512 doubles
    assert m * q > SCRATCH_DOUBLES
    (A, X, B, C), _ = _inputs(3, m, 8, q, 8)
    st, R = _call_noalloc(A, X, B, C)
    assert st == mek.MEK_EINVAL
    assert torch.isnan(R).all()            # nothing written
