"""GPU parity of the FP32 residual engine on the BF16 matrix cores
(mek_residual_split): R_b = C_b - (A X_b) B with FP32 operands split into
1, 2 or 3 bf16 terms, against the oracle's FP64 residual (the start of
Alg. 3) on the same FP32-representable inputs.

Error bound, element by element, with u = 2^-24 and H = |A| |X| |B|:
  * splitting: with round-to-nearest terms, each operand value x = sum of
    its P terms plus a rest of at most 2^(-8P) |x|, and term t is at most
    2^(-8t) (1 + 2^-8) |x|; the products of terms of combined order P or
    more that the kernel leaves out, plus the two rests, are at most
    c_P |a| |b| with c_P = (P + 1) 2^(-8P) (1 + 2^-7), in each product;
  * FP32 accumulation of K k-steps of n_P = P (P + 1) / 2 term products:
    at most gamma = (K n_P + 1) u times the sum of |products|;
  * T = A X rounded to FP32 (u |T|), and C - T B formed in FP64 and
    rounded once to FP32 (u |R|).
So |R_gpu - R| <= (2 c_P + (p n_P + q n_P + 3) u) (1 + 2^-6) H + u |R|.
Beyond the bound, the split must pay off: the Frobenius error falls with
every term added (the left-out terms shrink by 2^-8 per order; measured
ratios between orders must exceed 50 and 4, well inside what the split
orders give)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2408_05444_amd as mek

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _bound(P, p, q, H, R):
    nP = P * (P + 1) // 2
    cP = (P + 1) * 2.0 ** (-8 * P) * (1 + 2.0 ** -7)
    return (2 * cP + (p * nP + q * nP + 3) * U) * (1 + 2.0 ** -6) * H + U * np.abs(R)


def _inputs(seed, nb, m, p, q, n, noise=1e-3):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, p)).astype(np.float32)
    B = rng.standard_normal((q, n)).astype(np.float32)
    X = rng.standard_normal((nb, p, q)).astype(np.float32)
    C = np.stack([A.astype(np.float64) @ X[b].astype(np.float64) @ B.astype(np.float64)
                  for b in range(nb)]) + noise * rng.standard_normal((nb, m, n))
    return A, X, B, C


def _run(A, X, B, C, P):
    d = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(d)
    return mek.mek_residual_split(t(A), t(X), t(B), t(C), pieces=P).cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("shape", [(1, 77, 45, 37, 130), (1, 300, 200, 150, 260),
                                   (2, 129, 64, 96, 257), (3, 64, 32, 33, 65)])
@pytest.mark.parametrize("P", [1, 2, 3])
def test_split_residual_within_bound(shape, P):
    nb, m, p, q, n = shape
    A, X, B, C = _inputs(11 + P, nb, m, p, q, n)
    Rg = _run(A, X, B, C, P)
    for b in range(nb):
        R = oracle.residual(A, X[b], B, C[b])
        H = np.abs(A).astype(np.float64) @ np.abs(X[b]).astype(np.float64) @ np.abs(B).astype(np.float64)
        err = np.abs(Rg[b] - R)
        assert np.all(err <= _bound(P, p, q, H, R)), (b, float((err / H).max()))


def test_more_terms_give_smaller_errors():
    nb, m, p, q, n = 1, 256, 160, 128, 288
    A, X, B, C = _inputs(5, nb, m, p, q, n)
    R = oracle.residual(A, X[0], B, C[0])
    errs = [np.linalg.norm(_run(A, X, B, C, P)[0] - R) for P in (1, 2, 3)]
    H = np.abs(A).astype(np.float64) @ np.abs(X[0]).astype(np.float64) @ np.abs(B).astype(np.float64)
    assert errs[0] > 50 * errs[1] and errs[1] > 4 * errs[2], errs
    # Three terms: FP32-grade, a few units of u relative to H.
    assert errs[2] <= 16 * U * np.linalg.norm(H), errs


def test_k_tail_and_single_rows():
    # K below one tile, a single output row and column, K not a multiple of 8.
    for (m, p, q, n) in [(1, 3, 5, 1), (2, 1, 1, 2), (17, 9, 13, 3)]:
        A, X, B, C = _inputs(7, 1, m, p, q, n)
        Rg = _run(A, X, B, C, 3)[0]
        R = oracle.residual(A, X[0], B, C[0])
        H = np.abs(A).astype(np.float64) @ np.abs(X[0]).astype(np.float64) @ np.abs(B).astype(np.float64)
        assert np.all(np.abs(Rg - R) <= _bound(3, p, q, H, R))


@pytest.mark.parametrize("shape", [(1, 2000, 500, 500, 2000), (3, 512, 512, 512, 512)])
def test_full_size_sampled_rows(shape):
    """The two residual workloads at full size (2000 x 500 / 500 x 2000 and
    three 512 x 512 channels), checked on 24 sampled rows per instance that
    the oracle computes on its own (R restricted to rows S is C_S - A_S X B)."""
    nb, m, p, q, n = shape
    A, X, B, C = _inputs(9, nb, m, p, q, n)
    Rg = _run(A, X, B, C, 3)
    rows = np.random.default_rng(1).choice(m, 24, replace=False)
    rows[0], rows[1] = 0, m - 1
    for b in range(nb):
        R = oracle.residual(A[rows], X[b], B, C[b][rows])
        H = (np.abs(A[rows]).astype(np.float64) @ np.abs(X[b]).astype(np.float64)
             @ np.abs(B).astype(np.float64))
        assert np.all(np.abs(Rg[b][rows] - R) <= _bound(3, p, q, H, R))


def test_rejects_bad_arguments():
    d = torch.device("cuda:0")
    A = torch.zeros(4, 3, dtype=torch.float32, device=d)
    X = torch.zeros(1, 3, 2, dtype=torch.float32, device=d)
    B = torch.zeros(2, 5, dtype=torch.float32, device=d)
    C = torch.zeros(1, 4, 5, dtype=torch.float64, device=d)
    for P in (0, 4):
        with pytest.raises(mek.MekError):
            mek.mek_residual_split(A, X, B, C, pieces=P)
