"""Pins for the two-sided block projection in the CPU oracle
(mek_oracle_block.c), each against something other than the oracle itself:

  * the selection against a brute-force evaluation of its definition in
    exact rational arithmetic (entry weights, threshold, ranking, caps);
  * the independence test against exact rank (duplicated / parallel rows);
  * each step against numpy's pseudoinverse form X += A_I^+ R_IJ B_J^+ of the
    projection onto {X : A_I X B_J = C_IJ}, and the block of the new residual
    being zero;
  * Pythagoras for an orthogonal projection onto an affine set holding every
    solution, and the Lemma 3.2-type invariant (every step lies in the span
    of A^T (.) B^T);
  * the limit A^+ C B^+ (SVD pseudoinverses) for full-rank, rank-deficient
    and wide/tall shapes;
  * the single-entry case s = t = 1 against the closed-form projection onto
    one equation A_i X B_j = C_ij;
  * the maintained residual against C - A X B recomputed by numpy.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads


def grams(A, B):
    return A @ A.T, B.T @ B


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def exact_selection(R, a, b, theta, s_max, t_max):
    """The selection's definition in exact arithmetic, assuming every ranked
    candidate is independent of the ones before it (generic data)."""
    m, n = R.shape
    Rf = [[Fraction(float(R[i, j])) for j in range(n)] for i in range(m)]
    af = [Fraction(float(x)) for x in a]
    bf = [Fraction(float(x)) for x in b]
    S = sum(Rf[i][j] ** 2 for i in range(m) for j in range(n))
    FA, FB = sum(af), sum(bf)
    w = {(i, j): Rf[i][j] ** 2 / (af[i] * bf[j]) for i in range(m) for j in range(n)
         if af[i] > 0 and bf[j] > 0}
    Om = max(w.values())
    th = Fraction(float(theta))
    eps = min(Om, th * Om + (1 - th) * S / (FA * FB))
    h = {i: max(w[(i, j)] for j in range(n) if (i, j) in w) for i in range(m) if af[i] > 0}
    g = {j: max(w[(i, j)] for i in range(m) if (i, j) in w) for j in range(n) if bf[j] > 0}
    rows = sorted([i for i in h if h[i] >= eps], key=lambda i: (-h[i], i))[:s_max]
    cols = sorted([j for j in g if g[j] >= eps], key=lambda j: (-g[j], j))[:t_max]
    return rows, cols, eps, Om


@pytest.mark.parametrize("theta", [0.0, 0.3, 0.5, 1.0])
@pytest.mark.parametrize("seed", range(4))
def test_selection_matches_exact_definition(theta, seed):
    rng = np.random.default_rng(300 + seed)
    m, p, q, n = 14, 20, 18, 11
    A = rng.standard_normal((m, p))
    B = rng.standard_normal((q, n))
    A[3] = 0.0                                    # a void row: never taken
    R = rng.standard_normal((m, n)) * rng.exponential(1.0, (m, 1))
    a = (A * A).sum(1)
    b = (B * B).sum(0)
    GA, GB = grams(A, B)
    for s_max, t_max in [(1, 1), (3, 5), (8, 8), (20, 20)]:
        I, J, eps, Om = oracle.select_2s(R, a, b, a.sum(), b.sum(), GA, GB, theta=theta,
                                         s_max=s_max, t_max=t_max)
        rows, cols, e_ex, O_ex = exact_selection(R, a, b, theta, s_max, t_max)
        assert I.tolist() == rows and J.tolist() == cols
        assert 3 not in I.tolist()
        assert Om == pytest.approx(float(O_ex), rel=1e-14)
        assert eps == pytest.approx(float(e_ex), rel=1e-13)


def test_argmax_entry_always_selected():
    # The analogue of Remark 4.1: the row and column of the largest weight
    # are taken first, for every theta, also when rounding makes all weights
    # nearly equal.
    rng = np.random.default_rng(5)
    for trial in range(200):
        m, n = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        A = rng.standard_normal((m, 12))
        B = rng.standard_normal((12, n))
        a, b = (A * A).sum(1), (B * B).sum(0)
        if trial % 2:
            R = np.sqrt(np.outer(a, b)) * rng.choice([-1.0, 1.0], (m, n))   # equal weights
        else:
            R = rng.standard_normal((m, n))
        GA, GB = grams(A, B)
        w = R ** 2 / np.outer(a, b)
        i0, j0 = np.unravel_index(np.argmax(w), w.shape)
        for theta in (0.0, 0.5, 1.0):
            I, J, eps, Om = oracle.select_2s(R, a, b, a.sum(), b.sum(), GA, GB, theta=theta,
                                             s_max=4, t_max=4)
            assert len(I) >= 1 and len(J) >= 1
            assert eps <= Om
            if trial % 2 == 0:
                assert I[0] == i0 and J[0] == j0


def test_dependent_rows_and_columns_are_skipped():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((6, 10))
    A[4] = -2.0 * A[1]                            # parallel rows
    A[5] = A[0] + A[2]                            # a combination of two rows
    B = rng.standard_normal((7, 5))
    B[:, 3] = 3.0 * B[:, 0]                       # parallel columns
    a, b = (A * A).sum(1), (B * B).sum(0)
    GA, GB = grams(A, B)
    R = np.ones((6, 5))
    R[4] *= 1e3                                   # row 4 first, then 1 (parallel) must go
    R[:, 3] *= 1e2
    I, J, _, _ = oracle.select_2s(R, a, b, a.sum(), b.sum(), GA, GB, theta=0.0, s_max=6,
                                  t_max=5)
    taken = set(I.tolist())
    assert 4 in taken and 1 not in taken
    assert not {0, 2, 5} <= taken                 # never all three
    assert np.linalg.matrix_rank(A[I]) == len(I)
    assert 3 in J.tolist() and 0 not in J.tolist()
    assert np.linalg.matrix_rank(B[:, J]) == len(J)


def _ranked_independent(score, M, cap, by_rows):
    """Rank by score (descending, lower index first); of the first cap ranked
    indices keep those that raise the exact rank of the rows (columns) kept
    before them."""
    order = sorted(range(len(score)), key=lambda i: (-score[i], i))[:cap]
    kept = []
    for i in order:
        trial = kept + [i]
        sub = M[trial] if by_rows else M[:, trial]
        if np.linalg.matrix_rank(sub) == len(trial):
            kept = trial
    return kept


def test_selection_with_dependent_rows_matches_rank_definition():
    # Every row and column is a candidate (each holds one dominant entry),
    # A has exactly dependent rows and B exactly dependent columns.
    rng = np.random.default_rng(17)
    m = n = 7
    A = rng.standard_normal((m, 5))
    A[3] = 2.0 * A[0]
    A[5] = A[1] - A[2]
    B = rng.standard_normal((4, n))
    B[:, 6] = -0.5 * B[:, 2]
    a, b = (A * A).sum(1), (B * B).sum(0)
    perm = rng.permutation(n)
    rho = rng.uniform(-0.3, 0.3, (m, n))
    for i in range(m):
        rho[i, perm[i]] = 3.0 * (1.0 + 0.01 * rng.uniform(0.0, 1.0))
    R = np.sqrt(np.outer(a, b)) * rho
    w = R ** 2 / np.outer(a, b)
    GA, GB = grams(A, B)
    for cap in (2, 4, 6, 7):
        I, J, _, _ = oracle.select_2s(R, a, b, a.sum(), b.sum(), GA, GB, theta=0.0,
                                      s_max=cap, t_max=cap)
        assert I.tolist() == _ranked_independent(w.max(1), A, cap, True)
        assert J.tolist() == _ranked_independent(w.max(0), B, cap, False)
    assert len(I) == 5 and len(J) == 4           # rank(A) = 5, rank(B) = 4
    # Dropped rows are not replaced by lower-ranked ones.
    hr = sorted(range(m), key=lambda i: (-w.max(1)[i], i))
    first6 = hr[:6]
    I6, _, _, _ = oracle.select_2s(R, a, b, a.sum(), b.sum(), GA, GB, theta=0.0, s_max=6,
                                   t_max=6)
    assert set(I6.tolist()) <= set(first6)


def test_ties_take_the_lower_index():
    # Small-integer A and B, so equal norms and equal weights are exact.
    rng = np.random.default_rng(23)
    A = rng.integers(-3, 4, (6, 8)).astype(float)
    A[4] = A[1][::-1]                             # same norm, independent
    B = rng.integers(-3, 4, (5, 6)).astype(float)
    B[:, 5] = B[::-1, 2]                          # same norm, independent
    a, b = (A * A).sum(1), (B * B).sum(0)
    assert a[1] == a[4] and b[2] == b[5]
    R = rng.integers(-2, 3, (6, 6)).astype(float)
    R[1] = R[4] = 9.0                             # rows 1 and 4 tie
    R[:, 2] = R[:, 5] = 9.0                       # columns 2 and 5 tie
    R[1, 2] = R[1, 5] = R[4, 2] = R[4, 5] = 30.0  # the top entries
    GA, GB = grams(A, B)
    w = R ** 2 / np.outer(a, b)
    assert np.linalg.matrix_rank(A[[1, 4]]) == 2 and np.linalg.matrix_rank(B[:, [2, 5]]) == 2
    assert w[1].max() == w[4].max() == w.max() and w[:, 2].max() == w[:, 5].max() == w.max()
    for cap in (1, 2):
        I, J, _, _ = oracle.select_2s(R, a, b, a.sum(), b.sum(), GA, GB, theta=1.0,
                                      s_max=cap, t_max=cap)
        assert I.tolist() == [1, 4][:cap] and J.tolist() == [2, 5][:cap]


@pytest.mark.parametrize("s_max,t_max", [(1, 1), (3, 2), (8, 8), (40, 40)])
def test_step_is_the_pseudoinverse_projection(s_max, t_max):
    inst = workloads.small(seed=3)
    A, B, C = inst.A, inst.B, inst.C
    X0 = np.random.default_rng(1).standard_normal((40, 40))
    r = oracle.solve_2s(A, B, C, X0=X0, theta=0.5, s_max=s_max, t_max=t_max, max_iters=1)
    I, J = r.I[0], r.J[0]
    R0 = C - A @ X0 @ B
    dX = np.linalg.pinv(A[I]) @ R0[np.ix_(I, J)] @ np.linalg.pinv(B[:, J])
    assert rel(r.X - X0, dX) <= 1e-10
    R1 = C - A @ r.X @ B
    assert np.abs(R1[np.ix_(I, J)]).max() <= 1e-10 * np.abs(R0).max()


def test_single_entry_closed_form():
    # s = t = 1: the projection onto the one equation A_i X B_j = C_ij,
    # X += R_ij / (||A_i||^2 ||B_j||^2) A_i^T B_j^T, at the largest weight.
    rng = np.random.default_rng(21)
    A = rng.standard_normal((9, 6))
    B = rng.standard_normal((5, 8))
    C = rng.standard_normal((9, 8))               # inconsistent is fine for one step
    X = np.zeros((6, 5))
    for _ in range(12):
        R = C - A @ X @ B
        a, b = (A * A).sum(1), (B * B).sum(0)
        w = R ** 2 / np.outer(a, b)
        i, j = np.unravel_index(np.argmax(w), w.shape)
        X = X + R[i, j] / (a[i] * b[j]) * np.outer(A[i], B[:, j])
    r = oracle.solve_2s(A, B, C, s_max=1, t_max=1, max_iters=12)
    assert rel(r.X, X) <= 1e-12


def test_pythagoras_and_invariant():
    inst = workloads.stacked_rank_deficient(12, 9, 7, 10, seed=4)
    A, B, C = inst.A, inst.B, inst.C
    Xhat = oracle.least_norm(A, C, B)
    X0 = np.random.default_rng(6).standard_normal((A.shape[1], B.shape[0]))
    Ap, Bp = np.linalg.pinv(A), np.linalg.pinv(B)
    inv0 = X0 - Ap @ A @ X0 @ B @ Bp
    Xk = X0
    # Any solution works for Pythagoras: shift Xhat by a null-space part.
    Xsol = Xhat + (X0 - Ap @ A @ X0 @ B @ Bp)
    assert rel(A @ Xsol @ B, C) <= 1e-10
    for k in range(1, 25):
        r = oracle.solve_2s(A, B, C, X0=X0, s_max=3, t_max=2, max_iters=k)
        Xn = r.X
        d_before = np.linalg.norm(Xk - Xsol) ** 2
        d_after = np.linalg.norm(Xn - Xsol) ** 2
        assert d_before - d_after == pytest.approx(np.linalg.norm(Xn - Xk) ** 2,
                                                   rel=1e-7, abs=1e-12 * d_before)
        assert rel(Xn - Ap @ A @ Xn @ B @ Bp, inv0) <= 1e-10
        Xk = Xn


@pytest.mark.parametrize("case", ["full", "rankdef", "wide"])
def test_limit_is_least_norm(case):
    if case == "full":
        inst = workloads.small(seed=5)
    elif case == "rankdef":
        inst = workloads.rank_deficient_left(40, 20, 15, 30, 8, seed=6)
    else:
        inst = workloads.gaussian_consistent(12, 30, 25, 10, seed=7)   # m < p, n < q
    A, B, C = inst.A, inst.B, inst.C
    Xln = oracle.least_norm(A, C, B)
    r = oracle.solve_2s(A, B, C, theta=0.5, s_max=6, t_max=6, stop=oracle.STOP_REL_ERR,
                        tol=1e-9, Xref=Xln, max_iters=200000)
    assert r.status == oracle.OK
    assert rel(r.X, Xln) <= 1e-9


def test_maintained_residual_and_histories():
    inst = workloads.ragged(seed=3)
    A, B, C = inst.A, inst.B, inst.C
    r = oracle.solve_2s(A, B, C, theta=0.7, s_max=5, t_max=7, max_iters=60, Xref=inst.X_star)
    Rtrue = C - A @ r.X @ B
    assert r.s_hist[-1] == pytest.approx(float((Rtrue ** 2).sum()), rel=1e-8)
    assert r.e_hist[-1] == pytest.approx(rel(r.X, inst.X_star), rel=1e-12)
    assert np.all(np.diff(r.e_hist) <= 1e-12)     # error never grows (projections)
    assert all(len(I) == 5 and len(J) == 7 for I, J in zip(r.I, r.J))


def test_invalid_arguments():
    A = np.ones((3, 2))
    B = np.ones((2, 3))
    C = np.ones((3, 3))
    for kw in [dict(s_max=0), dict(t_max=0), dict(theta=1.5), dict(tau=-1.0)]:
        with pytest.raises(ValueError):
            oracle.solve_2s(A, B, C, max_iters=1, **kw)
    with pytest.raises(ValueError):
        oracle.select_2s(np.ones((2, 2)), np.zeros(2), np.ones(2), 0.0, 2.0, np.zeros((2, 2)),
                         np.eye(2))
