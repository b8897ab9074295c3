"""GPU parity: every stage of the HIP path against the CPU oracle on the same
seeded inputs, through the C ABI.

Tolerances (derived from FP64 rounding, unit roundoff u = 1.1e-16):
  * Philox draws, selection indices, index sets: bit-exact / identical.
  * GEMM stages: |R_gpu - R_oracle| <= 1e-12 * max|.| (K <= 600 terms of
    size O(1): accumulated rounding ~ K u).
  * Trajectories under identical index sequences: iterates agree to 1e-9
    relative after 3000 updates (each update adds O(u) relative error; the
    contraction of the method keeps it from growing geometrically).
  * Converged solutions: ||X - X*||/||X*|| <= 1e-6 on the FP64 and mixed
    paths and <= 1e-5 on the FP32 path (residual refreshed from the iterate
    on the split-BF16 engine); FP32 without refreshes stalls near 1e-4.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2408_05444_amd as mek
import workloads

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")]


def cuda(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def seq_sum(x):
    s = 0.0
    for v in x:
        s += float(v)
    return s


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ---------------------------------------------------------------------------
# Stage: Philox draws
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,inst", [(0, 0), (12345, 7), (2 ** 64 - 1, 3), (2408054440, 1)])
def test_philox_bit_exact(seed, inst):
    u = host(mek.mek_philox_uniform(seed, inst, 0, 4096))
    ref = np.array([oracle.uniform(seed, inst, k) for k in range(4096)])
    assert (u == ref).all()
    u = host(mek.mek_philox_uniform(seed, inst, 2 ** 40 + 3, 65))
    ref = np.array([oracle.uniform(seed, inst, 2 ** 40 + 3 + k) for k in range(65)])
    assert (u == ref).all()


# ---------------------------------------------------------------------------
# Stage: selection (thresholds, index-set compaction, sampling)
# ---------------------------------------------------------------------------

VARIANTS = [("bk", 0.5), ("rbk", 0.5), ("grbk", 0.5), ("rgrbk", 0.0), ("rgrbk", 0.3),
            ("rgrbk", 1.0), ("mwrbk", 0.5)]


@pytest.mark.parametrize("m", [1, 7, 100, 513, 2000, 4099])
@pytest.mark.parametrize("variant,theta", VARIANTS)
def test_select_matches_oracle(m, variant, theta):
    rng = np.random.default_rng(1000 + m)
    a = rng.uniform(0.2, 3.0, m)
    if m > 3:
        a[rng.choice(m, size=max(1, m // 50), replace=False)] = 0.0
    r = rng.exponential(1.0, m) * np.where(a > 0, a, 1.0)
    F_A = seq_sum(a)
    idx, in_set, lst, st = mek.mek_select(variant, cuda(r), cuda(a), F_A, theta, seed=99,
                                          instance=4, k0=10, count=64)
    ref = [oracle.select(variant, r, a, theta=theta, seed=99, inst=4, k=10 + j) for j in range(64)]
    assert host(idx).tolist() == [x[0] for x in ref]
    if variant in ("grbk", "rgrbk", "mwrbk"):
        assert (host(in_set) == ref[0][1]).all()
        assert host(lst).tolist() == np.flatnonzero(ref[0][1]).tolist()
        assert st["size"] == int(ref[0][1].sum())
        # t and T depend on sum orders (block reduction vs ascending loop).
        assert st["t"] == pytest.approx(ref[0][2], rel=1e-14)
        assert st["T"] == pytest.approx(ref[0][3], rel=1e-13)


def test_select_ties_and_flat_ratios():
    # All ratios equal: every row is in the set (Remark 4.1's equality case).
    m = 300
    a = np.full(m, 0.5)
    r = np.full(m, 2.0)
    idx, in_set, _, _ = mek.mek_select("grbk", cuda(r), cuda(a), seq_sum(a), 0.5, seed=3, count=200)
    ref = [oracle.select("grbk", r, a, seed=3, k=j)[0] for j in range(200)]
    assert host(in_set).all() and host(idx).tolist() == ref
    # MWRBK ties go to the lowest index.
    a = np.array([1.0, 2.0, 1.0, 4.0, 0.0])
    r = np.array([1.0, 4.0, 2.0, 8.0, 100.0])
    idx, _, _, _ = mek.mek_select("mwrbk", cuda(r), cuda(a), seq_sum(a))
    assert int(host(idx)[0]) == 1


# ---------------------------------------------------------------------------
# Stage: residual engine and Gram matrices (MFMA GEMMs)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(1, 1, 1, 1), (63, 17, 9, 65), (130, 70, 52, 261),
                                   (100, 40, 40, 100), (257, 3, 130, 66),
                                   (2050, 40, 70, 2100)])   # last: the 128 x 128 tile kernel
def test_residual_engine(shape):
    m, p, q, n = shape
    rng = np.random.default_rng(sum(shape))
    A, X, B, C = (rng.standard_normal(s) for s in [(m, p), (p, q), (q, n), (m, n)])
    R = host(mek.mek_residual(cuda(A), cuda(X), cuda(B), cuda(C)))
    ref = oracle.residual(A, X, B, C)
    assert np.max(np.abs(R - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("nb,shape", [(3, (512, 512, 512, 512)), (2, (300, 70, 45, 650)),
                                      (5, (17, 3, 40, 129)), (2, (2050, 40, 70, 2100)),
                                      (2, (1500, 60, 50, 1500))])   # batch: 128-tiles, one: 64
def test_residual_engine_batched(nb, shape):
    # One launch per product for the whole batch: each instance equals the
    # oracle residual, and is bit-identical to the single-instance call
    # (the per-element accumulation order does not depend on the tile shape).
    m, p, q, n = shape
    rng = np.random.default_rng(nb + sum(shape))
    A, B = rng.standard_normal((m, p)), rng.standard_normal((q, n))
    X, C = rng.standard_normal((nb, p, q)), rng.standard_normal((nb, m, n))
    R = host(mek.mek_residual_batched(cuda(A), cuda(X), cuda(B), cuda(C)))
    for b in range(nb):
        ref = oracle.residual(A, X[b], B, C[b])
        assert np.max(np.abs(R[b] - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
        one = host(mek.mek_residual(cuda(A), cuda(X[b]), cuda(B), cuda(C[b])))
        assert np.array_equal(one, R[b])


@pytest.mark.parametrize("shape", [(1, 5), (7, 3), (70, 130), (129, 64), (300, 17),
                                   (2050, 300), (300, 2050)])   # 128 x 128 tiles, both layouts
def test_gram(shape):
    M = np.random.default_rng(shape[0]).standard_normal(shape)
    G1 = host(mek.mek_gram(cuda(M), False))
    G2 = host(mek.mek_gram(cuda(M), True))
    assert np.max(np.abs(G1 - oracle.gram_rows(M))) <= 1e-12 * max(1, np.abs(G1).max())
    assert np.max(np.abs(G2 - oracle.gram_cols(M))) <= 1e-12 * max(1, np.abs(G2).max())


def test_plan_precompute():
    inst = workloads.ragged()
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B))
    a, GA, GB, alpha = mek.mek_plan_query(plan)
    assert np.allclose(host(a), (inst.A ** 2).sum(axis=1), rtol=1e-13)
    assert np.max(np.abs(host(GA) - oracle.gram_rows(inst.A))) <= 1e-11
    assert np.max(np.abs(host(GB) - oracle.gram_cols(inst.B))) <= 1e-11
    assert alpha == pytest.approx(oracle.spectral_alpha(inst.B), rel=1e-9)


# ---------------------------------------------------------------------------
# Whole path: trajectories against the oracle.
# ---------------------------------------------------------------------------

def _both(inst, variant, theta, K, seed, plan_kw=None, X0=None, **kw):
    alpha = oracle.spectral_alpha(inst.B)
    ref = oracle.solve(inst.A, inst.B, inst.C, X0=X0, variant=variant, theta=theta, alpha=alpha,
                       max_iters=K, seed=seed, Xref=inst.X_star, **kw)
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), alpha=alpha, **(plan_kw or {}))
    res = mek.mek_solve(plan, cuda(inst.C), X0=None if X0 is None else cuda(X0), variant=variant,
                        theta=theta, alpha=alpha, max_iters=K, seed=seed, hist_cap=K + 1,
                        X_ref=cuda(inst.X_star))
    return ref, res


@pytest.mark.parametrize("case", ["wide_B", "tall_B", "blur"])
def test_plan_alpha_is_inverse_spectral_norm(case):
    # alpha = 1/||B||_2^2 (Sec. 5) from the plan, against the SVD. The blur
    # matrix has a cluster of singular values at the top (slow for power
    # iteration); the estimate lies inside that cluster.
    rng = np.random.default_rng(77)
    if case == "wide_B":
        B = rng.standard_normal((60, 300))
    elif case == "tall_B":
        B = rng.standard_normal((300, 60))
    else:
        B = workloads.blur_toeplitz(64, 1.0).T.copy()
    A = rng.standard_normal((50, B.shape[0]))
    plan = mek.mek_plan_create(cuda(A), cuda(B))
    _, _, _, alpha = mek.mek_plan_query(plan)
    ref = oracle.spectral_alpha(B)
    assert alpha == pytest.approx(ref, rel=1e-12 if case != "blur" else 1e-5)
    assert alpha >= ref * (1 - 1e-12)       # never beyond 1/sigma_max^2 by more than rounding


@pytest.mark.parametrize("variant,theta", VARIANTS)
def test_small_trajectory_matches_oracle(variant, theta):
    inst = workloads.small()
    K = 3000
    ref, res = _both(inst, variant, theta, K, seed=17)
    assert res.status == mek.MEK_MAXITER and res.iters == K
    assert host(res.idx_hist).tolist() == ref.idx.tolist()
    assert np.allclose(host(res.resid_hist), ref.s_hist, rtol=1e-8, atol=0)
    assert np.allclose(host(res.err_hist), ref.e_hist, rtol=1e-8, atol=0)
    assert rel(host(res.X), ref.X) <= 1e-9
    if variant in ("grbk", "rgrbk"):
        assert host(res.set_hist).tolist() == ref.set_sizes.tolist()


@pytest.mark.parametrize("team,lds", [(5, 1), (16, 1), (64, 1), (200, 1), (2, 0), (33, 0), (1, 0)])
@pytest.mark.parametrize("variant,theta", [("grbk", 0.5), ("rgrbk", 0.8), ("mwrbk", 0.5),
                                           ("rbk", 0.5), ("bk", 0.5)])
def test_multi_workgroup_trajectory(team, lds, variant, theta):
    inst = workloads.ragged()
    K = 600
    ref, res = _both(inst, variant, theta, K, seed=5, plan_kw=dict(team_wgs=team, r_in_lds=lds))
    assert res.r_in_lds == bool(lds)
    m = inst.A.shape[0]
    rpw = -(-m // min(team, m))
    assert res.team_wgs == -(-m // rpw)        # no work-group is left without rows
    assert host(res.idx_hist).tolist() == ref.idx.tolist()
    assert np.allclose(host(res.resid_hist), ref.s_hist, rtol=1e-8, atol=0)
    assert rel(host(res.X), ref.X) <= 1e-9


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("variant,theta", [("grbk", 0.5), ("rgrbk", 0.8), ("mwrbk", 0.5),
                                           ("rbk", 0.5), ("bk", 0.5)])
def test_one_work_group_with_b_in_lds(variant, theta, precision):
    """A one-work-group team holding R, B and B^T in LDS (the dot products
    read no device memory) follows the oracle's trajectory."""
    inst = workloads.small(seed=7)
    K = 1500
    alpha = oracle.spectral_alpha(inst.B)
    ref = oracle.solve(inst.A, inst.B, inst.C, variant=variant, theta=theta, alpha=alpha,
                       max_iters=K, seed=19, Xref=inst.X_star)
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), alpha=alpha, team_wgs=1, r_in_lds=1,
                               precision=precision)
    res = mek.mek_solve(plan, cuda(inst.C), variant=variant, theta=theta, alpha=alpha,
                        max_iters=K, seed=19, hist_cap=K + 1, X_ref=cuda(inst.X_star),
                        refresh_period=-1)
    assert res.team_wgs == 1 and res.r_in_lds
    if precision == "fp64":
        assert host(res.idx_hist).tolist() == ref.idx.tolist()
        assert rel(host(res.X), ref.X) <= 1e-9
    else:
        assert (host(res.idx_hist)[:100] == ref.idx[:100]).all()
        assert rel(host(res.X), ref.X) <= 1e-2


def test_replay_of_oracle_indices():
    inst = workloads.ragged(seed=12)
    alpha = oracle.spectral_alpha(inst.B)
    seq = oracle.solve(inst.A, inst.B, inst.C, variant="rbk", alpha=alpha, max_iters=400, seed=8).idx
    ref = oracle.solve(inst.A, inst.B, inst.C, variant="grbk", alpha=alpha, max_iters=400,
                       forced=seq)
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), alpha=alpha, team_wgs=4)
    res = mek.mek_solve(plan, cuda(inst.C), variant="grbk", alpha=alpha, max_iters=400,
                        replay_idx=cuda(seq, torch.int32), hist_cap=401)
    assert host(res.idx_hist).tolist() == seq.tolist()
    assert rel(host(res.X), ref.X) <= 1e-10
    assert np.allclose(host(res.resid_hist), ref.s_hist, rtol=1e-9)


def test_warm_start_trajectory():
    inst = workloads.small(seed=4)
    X0 = np.random.default_rng(2).standard_normal((40, 40))
    ref, res = _both(inst, "grbk", 0.5, 500, seed=3, X0=X0)
    assert host(res.idx_hist).tolist() == ref.idx.tolist()
    assert rel(host(res.X), ref.X) <= 1e-9


# ---------------------------------------------------------------------------
# Whole path: convergence to the closed-form limits.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant,theta", [("grbk", 0.5), ("rgrbk", 1.0), ("mwrbk", 0.5),
                                           ("rbk", 0.5)])
def test_small_converges_like_oracle(variant, theta):
    inst = workloads.small()
    alpha = oracle.spectral_alpha(inst.B)
    ref = oracle.solve(inst.A, inst.B, inst.C, variant=variant, theta=theta, alpha=alpha,
                       stop=oracle.STOP_REL_ERR, tol=1e-6, Xref=inst.X_star, max_iters=10 ** 6,
                       seed=21)
    res = mek.solve(cuda(inst.A), cuda(inst.B), cuda(inst.C), variant=variant,
                    relaxation=theta, tol=1e-6, seed=21, X_ref=cuda(inst.X_star), alpha=alpha,
                    max_iters=2_000_000)
    assert res.status == mek.MEK_OK and ref.status == oracle.OK
    assert rel(host(res.X), inst.X_star) <= 1e-6
    assert abs(res.iters - ref.iters) <= max(2, 0.02 * ref.iters)


def test_large_first_updates_match_oracle():
    """The 2000 x 500 / 500 x 2000 workload in the launch the bench times
    (250 work-groups, R in LDS), over its first 2000 updates."""
    inst = workloads.large()
    K = 2000
    ref, res = _both(inst, "grbk", 0.5, K, seed=2408054440)
    assert res.r_in_lds and res.team_wgs > 100
    assert host(res.idx_hist).tolist() == ref.idx.tolist()
    assert np.allclose(host(res.resid_hist), ref.s_hist, rtol=1e-9)
    assert rel(host(res.X), ref.X) <= 1e-9


@pytest.mark.parametrize("variant,theta", [("grbk", 0.5), ("rgrbk", 1.0), ("mwrbk", 0.5)])
def test_large_converges(variant, theta):
    inst = workloads.large()
    A, B, C, Xs = cuda(inst.A), cuda(inst.B), cuda(inst.C), cuda(inst.X_star)
    res = mek.solve(A, B, C, variant=variant, relaxation=theta, tol=1e-6, seed=7, X_ref=Xs,
                    max_iters=2_000_000)
    assert res.status == mek.MEK_OK
    assert rel(host(res.X), inst.X_star) <= 1e-6


def test_large_rank_deficient_least_norm():
    inst = workloads.large_rankdef()
    Xln = oracle.least_norm(inst.A, inst.C, inst.B)
    res = mek.solve(cuda(inst.A), cuda(inst.B), cuda(inst.C), tol=1e-6, seed=9, X_ref=cuda(Xln),
                    max_iters=2_000_000)
    assert res.status == mek.MEK_OK
    assert rel(host(res.X), Xln) <= 1e-6
    assert rel(host(res.X), inst.X_star) > 1e-2     # not the generating X*


# ---------------------------------------------------------------------------
# Precision modes.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["small", "ragged", "large"])
def test_fp32_path(name):
    inst = getattr(workloads, name)()
    # FP32 keeps R, X and the Gram matrices in float; the residual is
    # recomputed from the iterate (split-BF16 engine, FP32 accuracy) every
    # max(2048, 4 m) updates, so its drift never builds up and the iteration
    # reaches 1e-5 (the error of the FP32 iterate itself is about 1e-6 here).
    res = mek.solve(cuda(inst.A), cuda(inst.B), cuda(inst.C), tol=1e-5, seed=3,
                    X_ref=cuda(inst.X_star), precision="fp32", max_iters=2_000_000)
    assert res.status == mek.MEK_OK
    assert rel(host(res.X), inst.X_star) <= 1e-5
    assert res.passes >= -(-res.iters // max(2048, 4 * inst.A.shape[0]))


def test_fp32_refresh_passes_keep_the_trajectory():
    """Passes split by refreshes continue one iteration: under the oracle's
    index sequence (replayed across passes) the FP32 iterate with refreshes
    every 500 updates follows the FP64 oracle's to FP32 accuracy, and the
    pass count is ceil(K / 500)."""
    inst = workloads.small()
    K = 1800
    alpha = oracle.spectral_alpha(inst.B)
    seq = oracle.solve(inst.A, inst.B, inst.C, variant="grbk", alpha=alpha, max_iters=K, seed=3).idx
    ref = oracle.solve(inst.A, inst.B, inst.C, variant="grbk", alpha=alpha, max_iters=K, forced=seq)
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), precision="fp32", alpha=alpha)
    res = mek.mek_solve(plan, cuda(inst.C), variant="grbk", alpha=alpha, max_iters=K,
                        replay_idx=cuda(seq, torch.int32), hist_cap=K + 1, refresh_period=500)
    assert res.iters == K and res.passes == 4
    assert host(res.idx_hist).tolist() == seq.tolist()
    assert rel(host(res.X), ref.X) <= 1e-5


def test_fp32_without_refresh_stalls_above_the_refreshed_form():
    """refresh_period < 0: the incrementally updated FP32 residual alone (its
    drift of O(1e-7) relative per sweep limits it near 1e-4)."""
    inst = workloads.ragged()
    A, B, C, Xs = cuda(inst.A), cuda(inst.B), cuda(inst.C), cuda(inst.X_star)
    res = mek.solve(A, B, C, tol=1e-4, seed=3, X_ref=Xs, precision="fp32", max_iters=2_000_000,
                    refresh_period=-1)
    assert res.status == mek.MEK_OK and res.passes == 1
    assert rel(host(res.X), inst.X_star) <= 1e-4


def test_mixed_bk_cycles_across_passes():
    """ME-BK's cyclic order (Alg. 2, i_k = k mod m) runs over the whole solve,
    not from the first row again in every refinement pass."""
    inst = workloads.small()
    alpha = oracle.spectral_alpha(inst.B)
    K = 700
    p64 = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), alpha=alpha)
    pmx = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), alpha=alpha, precision="mixed")
    r64 = mek.mek_solve(p64, cuda(inst.C), variant="bk", alpha=alpha, max_iters=K, hist_cap=K + 1)
    rmx = mek.mek_solve(pmx, cuda(inst.C), variant="bk", alpha=alpha, max_iters=K, hist_cap=K + 1,
                        inner_iters=130)
    assert rmx.passes >= 5
    assert host(rmx.idx_hist).tolist() == host(r64.idx_hist).tolist() == [k % 100 for k in range(K)]


@pytest.mark.parametrize("name", ["small", "ragged", "large"])
def test_mixed_path(name):
    inst = getattr(workloads, name)()
    res = mek.solve(cuda(inst.A), cuda(inst.B), cuda(inst.C), tol=1e-6, seed=3,
                    X_ref=cuda(inst.X_star), precision="mixed", max_iters=2_000_000)
    assert res.status == mek.MEK_OK and res.passes >= 1
    assert rel(host(res.X), inst.X_star) <= 1e-6


# ---------------------------------------------------------------------------
# Edge cases and error paths.
# ---------------------------------------------------------------------------

def test_single_row_and_classical_kaczmarz():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((15, 22))
    b = A @ rng.standard_normal(22)
    B = np.ones((1, 1))
    plan = mek.mek_plan_create(cuda(A), cuda(B), alpha=1.0)
    res = mek.mek_solve(plan, cuda(b[:, None]), variant="bk", alpha=1.0, max_iters=37)
    ref = oracle.solve(A, B, b[:, None], variant="bk", alpha=1.0, max_iters=37)
    assert rel(host(res.X), ref.X) <= 1e-12
    A1 = rng.standard_normal((1, 9))
    B1 = rng.standard_normal((4, 6))
    C1 = A1 @ rng.standard_normal((9, 4)) @ B1
    ref = oracle.solve(A1, B1, C1, variant="grbk", max_iters=50, seed=1)
    plan = mek.mek_plan_create(cuda(A1), cuda(B1), alpha=oracle.spectral_alpha(B1))
    res = mek.mek_solve(plan, cuda(C1), variant="grbk", alpha=oracle.spectral_alpha(B1),
                        max_iters=50, seed=1)
    assert rel(host(res.X), ref.X) <= 1e-12


def test_void_rows_never_selected():
    inst = workloads.with_zero_rows(workloads.ragged(), [0, 5, 332])
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), team_wgs=3)
    for v in ["bk", "rbk", "grbk", "mwrbk"]:
        res = mek.mek_solve(plan, cuda(inst.C), variant=v, max_iters=300, seed=2, hist_cap=301)
        idx = set(host(res.idx_hist).tolist())
        assert not idx & {0, 5, 332}
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve(plan, cuda(inst.C), replay_idx=cuda(np.array([1, 5]), torch.int32),
                      max_iters=2)
    assert e.value.code == mek.MEK_EINVAL


def test_status_codes():
    inst = workloads.small()
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B))
    C0 = torch.zeros(100, 100, dtype=torch.float64, device="cuda")
    res = mek.mek_solve(plan, C0, max_iters=10)
    assert res.status == mek.MEK_EXACT and res.iters == 0 and float(res.X.abs().max()) == 0.0
    X0 = cuda(np.ones((40, 40)))
    res = mek.mek_solve(plan, cuda(inst.C), X0=X0, max_iters=0)
    assert res.status == mek.MEK_MAXITER and res.iters == 0 and torch.equal(res.X, X0)
    res = mek.mek_solve(plan, cuda(inst.C), max_iters=10, diverge=0.5, raise_on_error=False)
    assert res.status == mek.MEK_EDIVERGED and res.iters == 0
    with pytest.raises(mek.MekError):
        mek.mek_solve(plan, cuda(inst.C), max_iters=10, diverge=0.5)
    # The same seed twice gives bit-identical results.
    r1 = mek.mek_solve(plan, cuda(inst.C), max_iters=2000, seed=5, hist_cap=2001)
    r2 = mek.mek_solve(plan, cuda(inst.C), max_iters=2000, seed=5, hist_cap=2001)
    assert torch.equal(r1.X, r2.X) and torch.equal(r1.idx_hist, r2.idx_hist)
    # X may alias X0.
    X = cuda(np.zeros((40, 40)))
    res = mek.mek_solve(plan, cuda(inst.C), X0=X, X_out=X, max_iters=100, seed=5)
    ref = mek.mek_solve(plan, cuda(inst.C), max_iters=100, seed=5)
    assert torch.equal(X, ref.X)
    # History shorter than the run: truncated, not overrun.
    res = mek.mek_solve(plan, cuda(inst.C), max_iters=100, hist_cap=10, seed=5)
    assert res.iters == 100 and res.idx_hist.numel() == 10


def test_error_paths():
    inst = workloads.small()
    A, B, C = cuda(inst.A), cuda(inst.B), cuda(inst.C)
    plan = mek.mek_plan_create(A, B)
    for kw in [dict(theta=1.5), dict(theta=-0.1), dict(stop="rel_err", tol=1e-6),
               dict(variant=7), dict(max_iters=-1), dict(alpha=10.0)]:
        with pytest.raises(mek.MekError) as e:
            mek.mek_solve(plan, C, **kw)
        assert e.value.code == mek.MEK_EINVAL, kw
    Cn = C.clone()
    Cn[3, 4] = float("nan")
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve(plan, Cn, max_iters=5)
    assert e.value.code == mek.MEK_ENONFINITE
    with pytest.raises(mek.MekError) as e:
        mek.mek_plan_create(torch.zeros_like(A), B)
    assert e.value.code == mek.MEK_EINVAL
    # A host address is rejected before any kernel runs.
    Ah = np.ascontiguousarray(inst.A)
    h = mek.ctypes.c_void_p()
    code = mek.lib().mek_plan_create(mek.ctypes.byref(h), 100, 40, 40, 100,
                                     mek.ctypes.c_void_p(Ah.ctypes.data),
                                     mek.ctypes.c_void_p(B.data_ptr()), None, None)
    assert code == mek.MEK_EINVAL


def test_exchange_floor_is_below_the_update_time():
    """The exchanges of the large workload's team alone take a positive time
    per round that is below the measured time of a whole update."""
    inst = workloads.large()
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B))
    res = mek.mek_solve(plan, cuda(inst.C), variant="grbk", max_iters=3000, seed=1)
    upd_us = res.kernel_ms * 1e3 / res.iters
    floor = mek.mek_exchange_floor(res.team_wgs, 2000, 2000, 500, rounds=3000)
    assert 0.5 < floor < upd_us
    small = mek.mek_exchange_floor(4, 100, 100, 40, rounds=2000)
    assert 0.0 < small < floor
    with pytest.raises(mek.MekError):
        mek.mek_exchange_floor(8, 4, 10, 10)      # fewer rows than work-groups
