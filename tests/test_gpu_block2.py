"""GPU parity of the two-sided block projection (MEK_TWOSIDED) against the
CPU oracle (mo_solve_2s), through the C ABI.

Bar: the blocks I and J of every step identical and in the same order; the
residual norms within 1e-8 relative and the iterate within 1e-9 relative
after tens of steps (each exact projection adds O(u kappa(G_I) kappa(G_J))
relative rounding; the caps keep the Gram blocks well conditioned on these
inputs); converged solutions within the tolerance of the least-norm
solution from SVD pseudoinverses.
"""
import ctypes

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


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _both(inst, s, t, theta, K, plan_kw=None, X0=None, Xref=None):
    ref = oracle.solve_2s(inst.A, inst.B, inst.C, X0=X0, theta=theta, s_max=s, t_max=t,
                          max_iters=K, Xref=Xref)
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), **(plan_kw or {}))
    res = mek.mek_solve(plan, cuda(inst.C), X0=None if X0 is None else cuda(X0),
                        variant="twosided", theta=theta, block_rows=s, block_cols=t,
                        max_iters=K, hist_cap=K + 1,
                        X_ref=None if Xref is None else cuda(Xref))
    return ref, res


def _check(ref, res, K, xtol=1e-9):
    assert res.status == mek.MEK_MAXITER and res.iters == K
    assert res.rows_hist == [I.tolist() for I in ref.I]
    assert res.cols_hist == [J.tolist() for J in ref.J]
    assert np.allclose(host(res.resid_hist), ref.s_hist, rtol=1e-8, atol=0)
    assert rel(host(res.X), ref.X) <= xtol


@pytest.mark.parametrize("s,t", [(1, 1), (4, 4), (8, 3), (32, 32)])
@pytest.mark.parametrize("theta", [0.3, 0.5, 1.0])
def test_small_steps_match_oracle(s, t, theta):
    inst = workloads.small()
    K = 40
    ref, res = _both(inst, s, t, theta, K, Xref=inst.X_star)
    _check(ref, res, K)
    assert np.allclose(host(res.err_hist), ref.e_hist, rtol=1e-8, atol=0)


@pytest.mark.parametrize("theta", [0.8, 0.95])
def test_block_sizes_that_vary_between_steps(theta):
    # With a high threshold the blocks change size from step to step, so the
    # exchange of R_IJ reuses words left from earlier, larger blocks.
    inst = workloads.ragged(seed=21)
    K = 80
    ref, res = _both(inst, 32, 32, theta, K, plan_kw=dict(team_wgs=8, r_in_lds=1),
                     Xref=inst.X_star)
    sizes = {(len(I), len(J)) for I, J in zip(res.rows_hist, res.cols_hist)}
    assert len(sizes) > 3
    _check(ref, res, K)
    assert np.all(np.diff(host(res.err_hist)) <= 1e-12)   # projections never move away


@pytest.mark.parametrize("team,lds", [(0, -1), (1, 0), (5, 1), (16, 1), (3, 0), (64, 0)])
def test_ragged_team_layouts(team, lds):
    inst = workloads.ragged()
    K = 30
    ref, res = _both(inst, 6, 5, 0.5, K, plan_kw=dict(team_wgs=team, r_in_lds=lds))
    if team:
        assert res.r_in_lds == bool(lds)
    _check(ref, res, K)


def test_dependent_rows_and_columns():
    # [A; A] and [B, B]: every selected block must skip the duplicates.
    inst = workloads.stacked_rank_deficient(24, 10, 9, 20, seed=5, a_mode="rows", b_mode="cols")
    K = 25
    ref, res = _both(inst, 8, 8, 0.2, K)
    _check(ref, res, K, xtol=1e-8)
    A, B = inst.A, inst.B
    for I, J in zip(res.rows_hist, res.cols_hist):
        assert np.linalg.matrix_rank(A[I]) == len(I)
        assert np.linalg.matrix_rank(B[:, J]) == len(J)


def test_warm_start_and_wide_shapes():
    inst = workloads.gaussian_consistent(30, 50, 45, 25, seed=8)    # m < p, n < q
    X0 = np.random.default_rng(3).standard_normal((50, 45))
    K = 30
    ref, res = _both(inst, 5, 7, 0.6, K, X0=X0)
    _check(ref, res, K)


@pytest.mark.parametrize("case", ["small", "rankdef"])
def test_converges_to_least_norm(case):
    inst = workloads.small(seed=9) if case == "small" else \
        workloads.rank_deficient_left(60, 30, 25, 50, 12, seed=10)
    Xln = oracle.least_norm(inst.A, inst.C, inst.B)
    ref = oracle.solve_2s(inst.A, inst.B, inst.C, theta=0.5, s_max=8, t_max=8,
                          stop=oracle.STOP_REL_ERR, tol=1e-10, Xref=Xln, max_iters=100000)
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B))
    res = mek.mek_solve(plan, cuda(inst.C), variant="twosided", theta=0.5, block_rows=8,
                        block_cols=8, stop="rel_err", tol=1e-10, X_ref=cuda(Xln),
                        max_iters=100000)
    assert res.status == mek.MEK_OK and ref.status == oracle.OK
    assert rel(host(res.X), Xln) <= 1e-10
    assert abs(res.iters - ref.iters) <= max(2, 0.02 * ref.iters)


def test_large_first_steps_match_oracle():
    inst = workloads.large()
    K = 4
    ref, res = _both(inst, 32, 32, 0.5, K, Xref=inst.X_star)
    assert res.r_in_lds and res.team_wgs > 100
    _check(ref, res, K, xtol=1e-11)


def test_large_converges():
    inst = workloads.large()
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B))
    res = mek.mek_solve(plan, cuda(inst.C), variant="twosided", theta=0.5, block_rows=32,
                        block_cols=32, stop="rel_err", tol=1e-6, X_ref=cuda(inst.X_star),
                        max_iters=200000)
    assert res.status == mek.MEK_OK
    assert rel(host(res.X), inst.X_star) <= 1e-6


def test_argument_checks():
    inst = workloads.small()
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B))
    C = cuda(inst.C)
    for kw in [dict(block_rows=0), dict(block_cols=33), dict(tau=1.5)]:
        with pytest.raises(mek.MekError) as e:
            mek.mek_solve(plan, C, variant="twosided", max_iters=1, **kw)
        assert e.value.code == mek.MEK_EINVAL
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve(plan, C, variant="twosided", max_iters=1,
                      replay_idx=cuda(np.array([0]), torch.int32))
    assert e.value.code == mek.MEK_EINVAL
    p32 = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), precision="fp32")
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve(p32, C, variant="twosided", max_iters=1)
    assert e.value.code == mek.MEK_EUNSUPPORTED
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve_batched(plan, cuda(np.stack([inst.C, inst.C])), variant="twosided",
                              max_iters=1)
    assert e.value.code == mek.MEK_EUNSUPPORTED
