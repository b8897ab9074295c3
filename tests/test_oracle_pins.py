"""Pins for the CPU oracle: each test checks the oracle against something the
paper or mathematics fixes, never against a retyped copy of its own code.

  * Philox4x64-10 stream vs numpy's Philox bit generator (library routine).
  * Index sets vs the paper's literal set definitions (Algs. 3/4/5) evaluated
    in exact rational arithmetic.
  * Sampling laws (Algs. 1, 3, 4) vs their stated probabilities.
  * Update arithmetic vs an exact-rational replay of the update written in
    the form of Algs. 1/2/5 (X += alpha/||A_i||^2 A_i^T (C_i - A_i X B) B^T).
  * Limits vs the closed forms: Theorem 3.3 (ME-BK), Theorems 4.2/4.5/4.7
    (least-norm solution A^+ C B^+), via SVD pseudoinverses.
  * Lemma 3.2's invariant and the one-step identity behind (3.7).
  * The special case q = n = 1, B = [1], alpha = 1, which is the classical
    Kaczmarz method (1.2).
  * The paper's printed iteration counts (Tables 2 and 4), in distribution.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


# ---------------------------------------------------------------------------
# Philox4x64-10 (the counter-based generator behind every random draw)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("key", [(0, 0), (12345, 7), (2 ** 64 - 1, 3), (2408054440, 0)])
@pytest.mark.parametrize("k", [0, 1, 2, 1000, 2 ** 40 + 17])
def test_philox_matches_numpy(key, k):
    # numpy's Philox(counter=c).random_raw() increments c first, then emits
    # the block, so the block at counter k+1 is numpy's first block for c=k.
    g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                         counter=np.array([k, 0, 0, 0], dtype=np.uint64))
    expect = [int(x) for x in g.random_raw(4)]
    assert oracle.philox4x64_10([k + 1, 0, 0, 0], key) == expect


def test_philox_full_counter_words():
    ctr = [5, 0xFFFFFFFF00000000, 123456789, 2 ** 63]
    g = np.random.Philox(key=np.array([9, 11], dtype=np.uint64),
                         counter=np.array(ctr, dtype=np.uint64))
    expect = [int(x) for x in g.random_raw(4)]
    assert oracle.philox4x64_10([ctr[0] + 1] + ctr[1:], [9, 11]) == expect


@pytest.mark.parametrize("k", [0, 3, 999])
def test_uniform_matches_numpy_generator(k):
    # numpy turns a 64-bit word into a double as (w >> 11) * 2^-53.
    g = np.random.Generator(np.random.Philox(key=np.array([77, 2], dtype=np.uint64),
                                             counter=np.array([k, 0, 0, 0], dtype=np.uint64)))
    assert oracle.uniform(77, 2, k) == g.random()


# ---------------------------------------------------------------------------
# Index sets and sampling laws
# ---------------------------------------------------------------------------

def _exact_set_relaxed(r, a, theta):
    """Alg. 4's set {i : ||R_i||^2 >= xi ||A_i||^2 ||R||_F^2} in exact arithmetic,
    with xi = theta/||R||^2 max_i(||R_i||^2/||A_i||^2) + (1-theta)/||A||_F^2."""
    R = [Fraction(float(x)) for x in r]
    A = [Fraction(float(x)) for x in a]
    S = sum(R)
    F = sum(A)
    M = max(R[i] / A[i] for i in range(len(r)) if A[i] > 0)
    th = Fraction(float(theta))
    xi = th / S * M + (1 - th) / F
    out, margin = [], []
    for i in range(len(r)):
        if A[i] == 0:
            out.append(False)
            margin.append(None)
            continue
        lhs, rhs = R[i], xi * A[i] * S
        out.append(lhs >= rhs)
        margin.append(abs(float(lhs - rhs)) / max(float(lhs), 1e-300))
    return np.array(out), margin


@pytest.mark.parametrize("theta", [0.0, 0.25, 0.5, 0.8, 1.0])
@pytest.mark.parametrize("seed", range(6))
def test_index_set_matches_paper_definition(theta, seed):
    rng = np.random.default_rng(seed)
    m = 40
    a = rng.uniform(0.5, 3.0, m)
    a[rng.integers(0, m, 3)] = 0.0          # void rows: never in the set
    r = rng.exponential(1.0, m) * a
    # Void rows of an inconsistent system keep their residual; it still
    # counts in ||R||_F^2 (the paper's S is over all rows).
    r[a == 0] = rng.uniform(0, 20.0, (a == 0).sum())
    variant = "grbk" if theta == 0.5 and seed % 2 == 0 else "rgrbk"
    i, in_set, t, T = oracle.select(variant, r, a, theta=theta, seed=seed, k=seed)
    exact, margin = _exact_set_relaxed(r, a, theta)
    for j in range(m):
        if margin[j] is not None and margin[j] < 1e-12:
            continue  # within rounding of the boundary: either answer is valid
        assert in_set[j] == exact[j], (j, theta)
    assert in_set[i]
    assert np.isclose(T, r[in_set].sum(), rtol=1e-14)


def test_grbk_threshold_is_alg3_zeta():
    # Alg. 3: zeta_k = 1/2 (max_i rho_i / ||R||^2 + 1/||A||^2); the set is
    # {i: ||R_i||^2 >= zeta ||A_i||^2 ||R||^2}. Check via exact arithmetic.
    rng = np.random.default_rng(42)
    for trial in range(20):
        m = 25
        a = rng.uniform(0.1, 2.0, m)
        r = rng.exponential(1.0, m)
        R = [Fraction(float(x)) for x in r]
        A = [Fraction(float(x)) for x in a]
        S, F = sum(R), sum(A)
        M = max(R[i] / A[i] for i in range(m))
        zeta = Fraction(1, 2) * (M / S + 1 / F)
        exact = np.array([R[i] >= zeta * A[i] * S for i in range(m)])
        _, in_set, _, _ = oracle.select("grbk", r, a, seed=trial, k=trial)
        assert (in_set == exact).all()


@pytest.mark.parametrize("theta", [0.0, 0.3, 0.5, 0.9, 1.0])
def test_remark_4_1_set_nonempty_and_holds_argmax(theta):
    rng = np.random.default_rng(7)
    cases = [(np.array([3.0]), np.array([1.7]))]                       # m = 1
    cases.append((np.full(9, 2.0), np.full(9, 0.5)))                     # all ratios equal
    cases.append((np.array([1e-300, 4.0, 4.0, 0.0]), np.array([1.0, 2.0, 2.0, 1.0])))
    for _ in range(50):
        m = int(rng.integers(1, 60))
        a = rng.uniform(0.01, 5, m)
        cases.append((rng.exponential(1, m) * rng.choice([1e-8, 1.0, 1e8]), a))
    for r, a in cases:
        ratio = r / a
        amax = int(np.argmax(ratio))
        for k in range(3):
            i, in_set, t, T = oracle.select("rgrbk", r, a, theta=theta, seed=1, k=k)
            assert in_set.any() and in_set[amax] and in_set[i]


def test_remark_4_1_under_rounding_of_equal_ratios():
    # Remark 4.1: the set is never empty. With ||R_i||^2 = c ||A_i||^2 every
    # ratio equals ||R||_F^2/||A||_F^2 in exact arithmetic, but the rounded
    # sums can put the threshold one ulp above every rounded ratio; the set
    # must still hold the maximiser.
    rng = np.random.default_rng(0)
    hit = 0
    for trial in range(400):
        m = int(rng.integers(2, 9))
        a = rng.uniform(0.1, 3.0, m)
        r = a * rng.uniform(0.5, 2.0)
        ratio = r / a
        S, F = 0.0, 0.0
        for x in r:
            S += x
        for x in a:
            F += x
        hit += (S / F) > ratio.max()
        for theta in (0.0, 0.5):
            i, in_set, t, T = oracle.select("rgrbk", r, a, theta=theta, seed=3, k=trial)
            assert in_set.any() and in_set[i] and in_set[int(np.argmax(ratio))]
            assert t <= ratio.max()
    assert hit > 20   # the adversarial rounding case does occur in this sample


def test_theta_one_is_mwrbk_when_argmax_unique():
    rng = np.random.default_rng(3)
    for k in range(100):
        m = 30
        a = rng.uniform(0.5, 2, m)
        r = rng.exponential(1, m)
        i1, s1, _, _ = oracle.select("rgrbk", r, a, theta=1.0, seed=5, k=k)
        i2, _, _, _ = oracle.select("mwrbk", r, a)
        assert s1.sum() == 1 and i1 == i2 == int(np.argmax(r / a))


def test_mwrbk_ties_take_lowest_index():
    a = np.array([1.0, 2.0, 1.0, 4.0, 0.0])
    r = np.array([1.0, 4.0, 2.0, 8.0, 100.0])   # ratios 1, 2, 2, 2 (+ a void row)
    i, in_set, t, T = oracle.select("mwrbk", r, a)
    assert i == 1 and t == 2.0


def _frequencies(variant, r, a, theta, N):
    counts = np.zeros(len(r))
    for k in range(N):
        i, _, _, _ = oracle.select(variant, r, a, theta=theta, seed=2024, inst=3, k=k)
        counts[i] += 1
    return counts / N


def test_greedy_sampling_law():
    # Alg. 3/4: inside the set, Pr(i) = ||R_i||^2 / sum_set ||R_j||^2
    # (weights are residual norms, not the ratios used for the threshold).
    a = np.array([1.0, 0.5, 2.0, 1.0, 0.25, 3.0, 1.0, 1.5])
    r = np.array([4.0, 1.9, 7.0, 0.2, 0.9, 9.0, 3.5, 0.1])
    _, in_set, _, _ = oracle.select("rgrbk", r, a, theta=0.3)
    p = np.where(in_set, r, 0.0) / r[in_set].sum()
    N = 30000
    f = _frequencies("rgrbk", r, a, 0.3, N)
    assert (f[~in_set] == 0).all()
    sd = np.sqrt(p * (1 - p) / N)
    assert (np.abs(f - p) <= 5 * sd + 1e-12).all(), (f, p)


def test_rbk_sampling_law():
    # Alg. 1: Pr(i) = ||A_i||^2 / ||A||_F^2; void rows are never drawn.
    a = np.array([1.0, 0.0, 2.0, 0.5, 4.0, 0.5])
    r = np.ones(6)
    p = a / a.sum()
    N = 30000
    f = _frequencies("rbk", r, a, 0.5, N)
    sd = np.sqrt(p * (1 - p) / N)
    assert f[1] == 0 and (np.abs(f - p) <= 5 * sd + 1e-12).all()


def test_bk_cycles_over_nonvoid_rows():
    a = np.array([1.0, 0.0, 2.0, 3.0, 0.0, 1.0])
    seq = [oracle.select("bk", np.ones(6), a, k=k)[0] for k in range(9)]
    assert seq == [0, 2, 3, 5, 0, 2, 3, 5, 0]


# ---------------------------------------------------------------------------
# Update arithmetic: exact-rational replay of the literal update.
# ---------------------------------------------------------------------------

def _frac_mat(M):
    return [[Fraction(float(x)) for x in row] for row in M]


def _mm(X, Y):
    return [[sum(X[i][l] * Y[l][j] for l in range(len(Y))) for j in range(len(Y[0]))]
            for i in range(len(X))]


def test_exact_rational_replay_of_update():
    rng = np.random.default_rng(11)
    m, p, q, n = 6, 4, 3, 5
    A = rng.integers(-3, 4, (m, p)).astype(float)
    A[A.sum(axis=1) == 0, 0] = 1.0
    B = rng.integers(-2, 3, (q, n)).astype(float)
    C = rng.integers(-5, 6, (m, n)).astype(float)          # need not be consistent
    X0 = rng.integers(-1, 2, (p, q)).astype(float)
    alpha = 1.0 / 64.0
    seq = [int(x) for x in rng.integers(0, m, 15)]
    seq = [i if np.any(A[i]) else 0 for i in seq]
    res = oracle.solve(A, B, C, X0=X0, variant="bk", alpha=alpha, max_iters=len(seq),
                       forced=seq)
    Af, Bf, Cf, X = _frac_mat(A), _frac_mat(B), _frac_mat(C), _frac_mat(X0)
    BT = [list(col) for col in zip(*Bf)]
    al = Fraction(1, 64)
    for i in seq:
        ai = sum(x * x for x in Af[i])
        XB = _mm(X, Bf)
        Ri = [Cf[i][j] - sum(Af[i][s] * XB[s][j] for s in range(p)) for j in range(n)]
        RiBT = _mm([Ri], BT)[0]
        for s in range(p):
            for l in range(q):
                X[s][l] += al / ai * Af[i][s] * RiBT[l]
    Xe = np.array([[float(x) for x in row] for row in X])
    assert res.iters == len(seq)
    assert np.max(np.abs(res.X - Xe)) <= 1e-13 * max(1.0, np.max(np.abs(Xe)))


def test_maintained_residual_equals_literal_mode():
    # Alg. 3 keeps R^k with (A A^T) and (B^T B); Algs. 1/2/5 recompute C_i - A_i X B.
    inst = workloads.gaussian_consistent(30, 12, 10, 25, seed=5)
    alpha = oracle.spectral_alpha(inst.B)
    a = oracle.solve(inst.A, inst.B, inst.C, variant="grbk", alpha=alpha, max_iters=300, seed=9)
    b = oracle.solve(inst.A, inst.B, inst.C, variant="grbk", alpha=alpha, max_iters=300, seed=9,
                     forced=a.idx, literal=True)
    assert np.allclose(a.s_hist, b.s_hist, rtol=1e-9, atol=0)
    assert np.max(np.abs(a.X - b.X)) <= 1e-11 * np.max(np.abs(a.X))
    # And the maintained residual after k steps is C - A X^k B.
    Rk = oracle.residual(inst.A, a.X, inst.B, inst.C)
    assert np.isclose((Rk ** 2).sum(), a.s_hist[-1], rtol=1e-8)


def test_residual_and_gram_helpers_vs_numpy():
    rng = np.random.default_rng(0)
    A, X, B, C = (rng.standard_normal(s) for s in [(7, 5), (5, 4), (4, 9), (7, 9)])
    assert np.allclose(oracle.residual(A, X, B, C), C - A @ X @ B, rtol=1e-13, atol=1e-13)
    assert np.allclose(oracle.gram_rows(A), A @ A.T, rtol=1e-13, atol=1e-13)
    assert np.allclose(oracle.gram_cols(B), B.T @ B, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------------------
# Theory: invariant, one-step identity, limits, special case.
# ---------------------------------------------------------------------------

def _trajectory(inst, variant, K, X0=None, theta=0.5, seed=1, alpha=None):
    """X^0..X^K of one run (the oracle is deterministic given the seed)."""
    Xs = []
    for k in range(K + 1):
        r = oracle.solve(inst.A, inst.B, inst.C, X0=X0, variant=variant, theta=theta,
                         alpha=alpha, max_iters=k, seed=seed)
        Xs.append(r.X)
    return Xs, r


@pytest.mark.parametrize("variant", ["bk", "rbk", "grbk", "rgrbk", "mwrbk"])
def test_lemma_3_2_invariant(variant):
    inst = workloads.stacked_rank_deficient(10, 8, 6, 9, seed=4)
    rng = np.random.default_rng(1)
    X0 = rng.standard_normal((8, 6))
    Ap, Bp = np.linalg.pinv(inst.A), np.linalg.pinv(inst.B)
    P = lambda X: X - Ap @ inst.A @ X @ inst.B @ Bp
    Xs, _ = _trajectory(inst, variant, 25, X0=X0, theta=0.7)
    base = P(X0)
    for X in Xs:
        assert np.max(np.abs(P(X) - base)) <= 1e-11 * max(1, np.max(np.abs(X0)))


@pytest.mark.parametrize("variant", ["grbk", "mwrbk", "rbk"])
def test_one_step_identity_and_3_7(variant):
    inst = workloads.gaussian_consistent(12, 5, 4, 10, seed=8)
    Xs_star = oracle.least_norm(inst.A, inst.C, inst.B)
    alpha = oracle.spectral_alpha(inst.B) * 1.3          # any alpha in (0, 2/||B||^2)
    B2 = np.linalg.norm(inst.B, 2) ** 2
    Xs, res = _trajectory(inst, variant, 30, alpha=alpha)
    for k in range(30):
        i = res.idx[k]
        Rk = inst.C - inst.A @ Xs[k] @ inst.B
        ri, ai = (Rk[i] ** 2).sum(), (inst.A[i] ** 2).sum()
        e0 = ((Xs[k] - Xs_star) ** 2).sum()
        e1 = ((Xs[k + 1] - Xs_star) ** 2).sum()
        exact = e0 - 2 * alpha * ri / ai + alpha ** 2 / ai * ((Rk[i] @ inst.B.T) ** 2).sum()
        assert abs(e1 - exact) <= 1e-9 * max(e0, 1e-30)
        assert e1 <= e0 - (2 * alpha - alpha ** 2 * B2) * ri / ai + 1e-9 * e0


def test_theorem_3_3_bk_limit():
    # ME-BK from X0 != 0 converges to A^+ C B^+ + X0 - A^+ A X0 B B^+.
    inst = workloads.stacked_rank_deficient(8, 10, 8, 7, seed=2, a_mode="cols", b_mode="rows")
    X0 = np.random.default_rng(5).standard_normal((10, 8))
    lim = oracle.bk_limit(inst.A, inst.B, inst.C, X0)
    ln = oracle.least_norm(inst.A, inst.C, inst.B)
    assert np.linalg.norm(lim - ln) > 1e-2 * np.linalg.norm(ln)    # the shift is visible
    res = oracle.solve(inst.A, inst.B, inst.C, X0=X0, variant="bk", stop=oracle.STOP_REL_ERR,
                       tol=1e-11, Xref=lim, max_iters=2_000_000)
    assert res.status == oracle.OK


def test_theorem_3_3_wide_A_tall_B():
    # Table 1 Set 4 shape class: A wide (40 x 110), B tall (130 x 50); X0 = 1e-5 I.
    inst = workloads.gaussian_consistent(12, 30, 34, 14, seed=6)
    X0 = 1e-5 * np.eye(30, 34)
    lim = oracle.bk_limit(inst.A, inst.B, inst.C, X0)
    res = oracle.solve(inst.A, inst.B, inst.C, X0=X0, variant="bk", stop=oracle.STOP_REL_ERR,
                       tol=1e-10, Xref=lim, max_iters=2_000_000)
    assert res.status == oracle.OK


@pytest.mark.parametrize("variant,theta", [("grbk", 0.5), ("rgrbk", 0.2), ("rgrbk", 1.0),
                                           ("mwrbk", 0.5), ("rbk", 0.5)])
def test_greedy_limit_is_least_norm(variant, theta):
    # Theorems 4.2, 4.5, 4.7 (and Lemma 2.2): X^0 = 0 -> A^+ C B^+, rank deficient.
    inst = workloads.stacked_rank_deficient(14, 10, 8, 12, seed=3, a_mode="rows", b_mode="cols")
    ln = oracle.least_norm(inst.A, inst.C, inst.B)
    res = oracle.solve(inst.A, inst.B, inst.C, variant=variant, theta=theta,
                       stop=oracle.STOP_REL_ERR, tol=1e-10, Xref=ln, max_iters=2_000_000, seed=3)
    assert res.status == oracle.OK


def test_least_norm_closed_forms():
    # Sec. 2: full column rank A / full row rank B: (A^T A)^-1 A^T C B^T (B B^T)^-1;
    # full row rank A / full column rank B: A^T (A A^T)^-1 C (B^T B)^-1 B^T.
    i1 = workloads.gaussian_consistent(20, 6, 5, 15, seed=1)
    A, B, C = i1.A, i1.B, i1.C
    f1 = np.linalg.solve(A.T @ A, A.T @ C @ B.T) @ np.linalg.inv(B @ B.T)
    assert np.allclose(oracle.least_norm(A, C, B), f1, rtol=1e-10, atol=1e-10)
    i2 = workloads.gaussian_consistent(5, 12, 14, 6, seed=2)
    A, B, C = i2.A, i2.B, i2.C
    f2 = A.T @ np.linalg.solve(A @ A.T, C) @ np.linalg.inv(B.T @ B) @ B.T
    assert np.allclose(oracle.least_norm(A, C, B), f2, rtol=1e-10, atol=1e-10)


def test_classical_kaczmarz_special_case():
    # q = n = 1, B = [1], alpha = 1: ME-BK is the classical Kaczmarz method (1.2)
    # and converges to the least-norm solution of the consistent system A x = b.
    rng = np.random.default_rng(4)
    A = rng.standard_normal((15, 22))
    b = A @ rng.standard_normal(22)
    B = np.ones((1, 1))
    res = oracle.solve(A, B, b[:, None], variant="bk", alpha=1.0, max_iters=37)
    x = np.zeros(22)
    for k in range(37):
        i = k % 15
        x = x + (b[i] - A[i] @ x) / (A[i] @ A[i]) * A[i]
    assert np.allclose(res.X[:, 0], x, rtol=1e-12, atol=1e-12)
    full = oracle.solve(A, B, b[:, None], variant="bk", alpha=1.0, stop=oracle.STOP_REL_ERR,
                        tol=1e-10, Xref=np.linalg.lstsq(A, b, rcond=None)[0][:, None],
                        max_iters=10 ** 6)
    assert full.status == oracle.OK


def test_void_rows_never_selected_and_exact_status():
    inst = workloads.with_zero_rows(workloads.gaussian_consistent(20, 6, 5, 12, seed=2), [0, 7])
    for v in ["bk", "rbk", "grbk", "mwrbk"]:
        res = oracle.solve(inst.A, inst.B, inst.C, variant=v, max_iters=200, seed=4)
        assert 0 not in res.idx and 7 not in res.idx
    # X0 that already solves the system: zero updates, EXACT status.
    i2 = workloads.gaussian_consistent(8, 3, 3, 8, seed=1)
    B = np.eye(3, 8)
    A = np.eye(8, 3)
    X = i2.X_star
    res = oracle.solve(A, B, A @ X @ B, X0=X, variant="grbk", max_iters=10)
    assert res.iters == 0 and res.status == oracle.EXACT


def test_invalid_arguments_rejected():
    inst = workloads.gaussian_consistent(6, 3, 3, 6, seed=1)
    with pytest.raises(ValueError):
        oracle.solve(inst.A, inst.B, inst.C, alpha=-1.0)
    with pytest.raises(ValueError):
        oracle.solve(inst.A, inst.B, inst.C, stop=oracle.STOP_REL_ERR, tol=1e-3)


# ---------------------------------------------------------------------------
# The paper's printed statistics (Section 5), regenerated in distribution.
# ---------------------------------------------------------------------------

def test_paper_table4_set2_iteration_counts():
    g = json.load(open(GOLDEN))["table4_set2"]["IT"]
    its = {v: [] for v in ["rbk", "grbk", "mwrbk"]}
    for t in range(10):
        inst = workloads.paper_table3_set2(t)
        ref = oracle.least_norm(inst.A, inst.C, inst.B)
        for v in its:
            # squared RRN <= 1e-6 is relative error <= 1e-3.
            r = oracle.solve(inst.A, inst.B, inst.C, variant=v, stop=oracle.STOP_REL_ERR,
                             tol=1e-3, Xref=ref, max_iters=10 ** 6, seed=100 + t)
            assert r.status == oracle.OK
            its[v].append(r.iters)
    mean = {v: np.mean(x) for v, x in its.items()}
    sd = {v: np.std(x) for v, x in its.items()}
    for v in its:
        # The paper's value comes from other random matrices of the same law:
        # it must be a plausible draw of our per-matrix distribution.
        assert abs(g[v] - mean[v]) <= 3 * sd[v] + 0.05 * mean[v], (v, g[v], mean[v], sd[v])
    # The ordering every row of Table 4 shows.
    assert mean["mwrbk"] <= mean["grbk"] < mean["rbk"]


def test_paper_table2_set2_bk_iterations():
    g = json.load(open(GOLDEN))["table2_set2"]["IT"]
    its = []
    for t in range(8):
        inst = workloads.paper_table1_set2(t)
        X0 = 1e-5 * np.eye(45, 50)
        lim = oracle.bk_limit(inst.A, inst.B, inst.C, X0)
        r = oracle.solve(inst.A, inst.B, inst.C, X0=X0, variant="bk", stop=oracle.STOP_REL_ERR,
                         tol=1e-3, Xref=lim, max_iters=10 ** 6)
        assert r.status == oracle.OK
        its.append(r.iters)
    assert abs(g - np.mean(its)) <= 3 * np.std(its) + 0.05 * np.mean(its), (g, its)
