"""GPU parity of the sparse-aware update (MEK_UPDATE_SPARSE) through the C
ABI, against the CPU oracle (which always applies the full update of
Alg. 3: the sparse form leaves out only terms that are exactly zero) and
against the dense GPU form.

Tolerances as for the dense path: index sequences identical, norms within
1e-8 relative, iterates within 1e-9 relative after a few thousand FP64
updates (O(u) relative error per update, damped by the contraction), and
1e-12 between the dense and sparse GPU forms under one forced index
sequence (the two differ only in the summation order of v and w, whose
terms outside the nonzeros are zero).
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = {
    "banded64": lambda: workloads.banded_gaussian(64, seed=3),
    "sparse_irregular": lambda: workloads.sparse_random(300, 120, 90, 257, seed=1,
                                                        empty_rows=20),
    # m above 512: several rows of the selection per thread.
    "sparse_tall": lambda: workloads.sparse_random(1100, 70, 40, 130, seed=2, empty_rows=7),
}

VARIANTS = [("grbk", 0.5), ("rgrbk", 0.8), ("rgrbk", 1.0), ("mwrbk", 0.5), ("rbk", 0.5),
            ("bk", 0.5)]


def _sparse_plan(inst, alpha, **kw):
    return mek.mek_plan_create(cuda(inst.A), cuda(inst.B), alpha=alpha, update="sparse", **kw)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("variant,theta", VARIANTS)
def test_sparse_trajectory_matches_oracle(case, variant, theta):
    inst = CASES[case]()
    K = 2000
    alpha = oracle.spectral_alpha(inst.B)
    ref = oracle.solve(inst.A, inst.B, inst.C, variant=variant, theta=theta, alpha=alpha,
                       max_iters=K, seed=31, Xref=inst.X_star)
    plan = _sparse_plan(inst, alpha)
    res = mek.mek_solve(plan, cuda(inst.C), variant=variant, theta=theta, alpha=alpha,
                        max_iters=K, seed=31, hist_cap=K + 1, X_ref=cuda(inst.X_star))
    assert res.status == mek.MEK_MAXITER and res.iters == K
    assert res.team_wgs == 1 and not res.r_in_lds
    assert host(res.idx_hist).tolist() == ref.idx.tolist()
    assert np.allclose(host(res.resid_hist), ref.s_hist, rtol=1e-8, atol=0)
    assert np.allclose(host(res.err_hist), ref.e_hist, rtol=1e-8, atol=0)
    assert rel(host(res.X), ref.X) <= 1e-9
    if variant in ("grbk", "rgrbk"):
        assert host(res.set_hist).tolist() == ref.set_sizes.tolist()


@pytest.mark.parametrize("case", sorted(CASES))
def test_sparse_widths_are_the_nonzero_counts(case):
    inst = CASES[case]()
    plan = _sparse_plan(inst, 0.0)
    G = inst.A @ inst.A.T
    want = (int((inst.A != 0).sum(1).max()), int((inst.B != 0).sum(1).max()),
            int((inst.B != 0).sum(0).max()), int((G != 0).sum(0).max()))
    assert mek.mek_plan_sparse_widths(plan) == want


def test_sparse_equals_dense_under_one_index_sequence():
    inst = CASES["sparse_irregular"]()
    alpha = oracle.spectral_alpha(inst.B)
    seq = oracle.solve(inst.A, inst.B, inst.C, variant="rbk", alpha=alpha, max_iters=3000,
                       seed=4).idx
    idx = cuda(seq, torch.int32)
    kw = dict(variant="grbk", alpha=alpha, max_iters=3000, replay_idx=idx, hist_cap=3001)
    dense = mek.mek_solve(mek.mek_plan_create(cuda(inst.A), cuda(inst.B), alpha=alpha),
                          cuda(inst.C), **kw)
    sparse = mek.mek_solve(_sparse_plan(inst, alpha), cuda(inst.C), **kw)
    assert host(sparse.idx_hist).tolist() == seq.tolist()
    assert rel(host(sparse.X), host(dense.X)) <= 1e-12
    assert np.allclose(host(sparse.resid_hist), host(dense.resid_hist), rtol=1e-11)


def test_sparse_warm_start_trajectory():
    inst = CASES["banded64"]()
    X0 = np.random.default_rng(5).standard_normal((64, 64))
    alpha = oracle.spectral_alpha(inst.B)
    ref = oracle.solve(inst.A, inst.B, inst.C, X0=X0, alpha=alpha, max_iters=1500, seed=6,
                       Xref=inst.X_star)
    res = mek.mek_solve(_sparse_plan(inst, alpha), cuda(inst.C), X0=cuda(X0), alpha=alpha,
                        max_iters=1500, seed=6, hist_cap=1501, X_ref=cuda(inst.X_star))
    assert host(res.idx_hist).tolist() == ref.idx.tolist()
    assert rel(host(res.X), ref.X) <= 1e-9


@pytest.mark.parametrize("variant,theta", [("grbk", 0.5), ("mwrbk", 0.5)])
def test_sparse_converges_like_oracle(variant, theta):
    # A blurred 64 x 64 image (sigma 0.7, 9 taps; cond(A) = 5.6), X_ref the
    # generating image.
    inst = workloads.blurred_image(64, 1, 0.7, seed=8)[0]
    alpha = oracle.spectral_alpha(inst.B)
    ref = oracle.solve(inst.A, inst.B, inst.C, variant=variant, theta=theta, alpha=alpha,
                       stop=oracle.STOP_REL_ERR, tol=1e-6, Xref=inst.X_star, max_iters=10 ** 6,
                       seed=12)
    res = mek.mek_solve(_sparse_plan(inst, alpha), cuda(inst.C), variant=variant, theta=theta,
                        alpha=alpha, stop="rel_err", tol=1e-6, X_ref=cuda(inst.X_star),
                        max_iters=10 ** 6, seed=12)
    assert ref.status == oracle.OK and res.status == mek.MEK_OK
    assert rel(host(res.X), inst.X_star) <= 1e-6
    assert abs(res.iters - ref.iters) <= max(2, 0.02 * ref.iters)


def test_sparse_empty_rows_never_selected():
    # The 64 x 64 blur (sigma 0.7) with four zero rows inserted into A: the
    # zero rows are never selected and the limit is still X* (A keeps full
    # column rank).
    base = workloads.blurred_image(64, 1, 0.7, seed=8)[0]
    A = np.ascontiguousarray(np.insert(base.A, [5, 20, 20, 63], 0.0, axis=0))
    C = A @ base.X_star @ base.B
    plan = mek.mek_plan_create(cuda(A), cuda(base.B), update="sparse")
    res = mek.mek_solve(plan, cuda(C), stop="rel_err", tol=1e-7, X_ref=cuda(base.X_star),
                        max_iters=3_000_000, seed=2, hist_cap=5000)
    assert res.status == mek.MEK_OK
    assert rel(host(res.X), base.X_star) <= 1e-7
    empty = {5, 21, 22, 66}
    assert all(np.abs(A[i]).sum() == 0 for i in empty)
    assert not empty & set(host(res.idx_hist).tolist())


def test_sparse_fp32():
    # First updates against the oracle on the banded Gaussian instance; then
    # convergence to 1e-4 (FP32's reach) on the well-conditioned blur
    # (64 x 64, sigma 0.7).
    inst = CASES["banded64"]()
    alpha = oracle.spectral_alpha(inst.B)
    ref = oracle.solve(inst.A, inst.B, inst.C, alpha=alpha, max_iters=40, seed=3)
    plan = _sparse_plan(inst, alpha, precision="fp32")
    first = mek.mek_solve(plan, cuda(inst.C), alpha=alpha, max_iters=40, seed=3, hist_cap=41)
    assert host(first.idx_hist).tolist() == ref.idx.tolist()
    img = workloads.blurred_image(64, 1, 0.7, seed=8)[0]
    plan = _sparse_plan(img, 0.0, precision="fp32")
    res = mek.mek_solve(plan, cuda(img.C), stop="rel_err", tol=1e-4, X_ref=cuda(img.X_star),
                        max_iters=3_000_000, seed=3)
    assert res.status == mek.MEK_OK
    assert rel(host(res.X), img.X_star) <= 1e-4


@pytest.mark.parametrize("nb", [3, 300])
def test_sparse_batch_equals_single_solves(nb):
    # One work-group per instance; 300 instances exceed the compute units.
    base = workloads.banded_gaussian(40, seed=9, sigma=0.7)
    rng = np.random.default_rng(10)
    Xs = rng.standard_normal((nb, 40, 40))
    C = np.stack([base.A @ X @ base.B for X in Xs])
    alpha = oracle.spectral_alpha(base.B)
    plan = _sparse_plan(base, alpha)
    kw = dict(variant="rgrbk", theta=0.6, alpha=alpha, stop="rel_err", tol=1e-5,
              max_iters=200000, seed=13, instance=100)
    st, res = mek.mek_solve_batched(plan, cuda(C), X_ref=cuda(Xs), **kw)
    assert st == mek.MEK_OK and all(r.status == mek.MEK_OK for r in res)
    for b in sorted({0, 1, nb - 1}):
        one = mek.mek_solve(plan, cuda(C[b]), X_ref=cuda(Xs[b]), **{**kw, "instance": 100 + b})
        assert res[b].iters == one.iters and one.status == mek.MEK_OK
        assert torch.equal(res[b].X, one.X)


def test_sparse_rel_resid_and_exact_stops():
    inst = workloads.blurred_image(64, 1, 0.7, seed=8)[0]
    plan = _sparse_plan(inst, 0.0)
    res = mek.mek_solve(plan, cuda(inst.C), stop="rel_resid", tol=1e-3, max_iters=10 ** 6, seed=1)
    assert res.status == mek.MEK_OK
    R = inst.C - inst.A @ host(res.X) @ inst.B
    assert np.linalg.norm(R) <= 1e-3 * np.linalg.norm(inst.C) * (1 + 1e-6)
    zero = mek.mek_solve(plan, cuda(np.zeros_like(inst.C)), max_iters=100)
    assert zero.status == mek.MEK_EXACT and zero.iters == 0


def test_sparse_refusals():
    inst = CASES["banded64"]()
    plan = _sparse_plan(inst, 0.0)
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve(plan, cuda(inst.C), variant="twosided", max_iters=5)
    assert e.value.code == mek.MEK_EUNSUPPORTED
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve_multi_async([plan], [cuda(inst.C)], variant="twosided", max_iters=5)
    assert e.value.code == mek.MEK_EUNSUPPORTED
    dense_plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B))
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve_multi([plan, dense_plan], [cuda(inst.C), cuda(inst.C)], max_iters=5)
    assert e.value.code == mek.MEK_EINVAL
    dense = mek.mek_plan_create(cuda(inst.A), cuda(inst.B))
    with pytest.raises(mek.MekError) as e:
        mek.mek_plan_sparse_widths(dense)
    assert e.value.code == mek.MEK_EUNSUPPORTED
    # A dense A: each column of A A^T has 1100 nonzeros, above the cap.
    rng = np.random.default_rng(1)
    with pytest.raises(mek.MekError) as e:
        mek.mek_plan_create(cuda(rng.standard_normal((1100, 20))),
                            cuda(rng.standard_normal((20, 30))), update="sparse")
    assert e.value.code == mek.MEK_EUNSUPPORTED
    with pytest.raises(mek.MekError) as e:
        mek.mek_plan_create(cuda(inst.A), cuda(inst.B), precision="mixed", update="sparse")
    assert e.value.code == mek.MEK_EUNSUPPORTED


# ---------------------------------------------------------------------------
# Ragged batches of sparse plans (mek_solve_multi): one work-group per
# instance, plans of different sizes, plans shared between instances.
# ---------------------------------------------------------------------------

def test_sparse_ragged_equals_single_solves():
    insts = [workloads.banded_gaussian(40, seed=1, sigma=0.7), CASES["sparse_irregular"](),
             CASES["sparse_tall"](), workloads.banded_gaussian(64, seed=2, sigma=0.7)]
    plans = [_sparse_plan(i, oracle.spectral_alpha(i.B)) for i in insts]
    # plan 0 twice (a second instance of the same A, B with its own C), plan 3 twice
    rng = np.random.default_rng(3)
    X2 = rng.standard_normal(insts[0].X_star.shape)
    X5 = rng.standard_normal(insts[3].X_star.shape)
    order = [0, 1, 2, 3, 0, 3]
    Cs = [insts[0].C, insts[1].C, insts[2].C, insts[3].C, insts[0].A @ X2 @ insts[0].B,
          insts[3].A @ X5 @ insts[3].B]
    Xr = [insts[0].X_star, insts[1].X_star, insts[2].X_star, insts[3].X_star, X2, X5]
    kw = dict(variant="grbk", max_iters=1500, seed=17, instance=40)
    st, res = mek.mek_solve_multi([plans[i] for i in order], [cuda(c) for c in Cs],
                                  X_ref=[cuda(x) for x in Xr], hist_cap=1501, **kw)
    assert st == mek.MEK_MAXITER
    for b, (i, C, x) in enumerate(zip(order, Cs, Xr)):
        one = mek.mek_solve(plans[i], cuda(C), X_ref=cuda(x), hist_cap=1501,
                            **{**kw, "instance": 40 + b})
        assert res[b].iters == one.iters == 1500 and res[b].team_wgs == 1
        assert torch.equal(res[b].X, one.X)
        assert torch.equal(res[b].idx_hist, one.idx_hist)
        assert res[b].rel_err == one.rel_err


def test_sparse_ragged_against_oracle_with_warm_start():
    insts = [CASES["sparse_irregular"](), workloads.banded_gaussian(48, seed=4, sigma=0.7)]
    alphas = [oracle.spectral_alpha(i.B) for i in insts]
    plans = [_sparse_plan(i, a) for i, a in zip(insts, alphas)]
    rng = np.random.default_rng(8)
    X0 = [rng.standard_normal(i.X_star.shape) for i in insts]
    st, res = mek.mek_solve_multi(plans, [cuda(i.C) for i in insts], X0=[cuda(x) for x in X0],
                                  X_ref=[cuda(i.X_star) for i in insts], variant="rgrbk",
                                  theta=0.7, max_iters=1000, seed=5, hist_cap=1001)
    for b, (inst, a) in enumerate(zip(insts, alphas)):
        ref = oracle.solve(inst.A, inst.B, inst.C, X0=X0[b], variant="rgrbk", theta=0.7, alpha=a,
                           max_iters=1000, seed=5, inst=b, Xref=inst.X_star)
        assert host(res[b].idx_hist).tolist() == ref.idx.tolist()
        assert rel(host(res[b].X), ref.X) <= 1e-9


def test_sparse_ragged_many_instances_on_shared_plans():
    # 300 instances (above the compute units) on 3 plans, 100 each.
    bases = [workloads.banded_gaussian(32, seed=s, sigma=0.7) for s in range(3)]
    plans = [_sparse_plan(b, 0.0) for b in bases]
    rng = np.random.default_rng(9)
    order = [b % 3 for b in range(300)]
    Xs = [rng.standard_normal((32, 32)) for _ in order]
    Cs = [bases[i].A @ x @ bases[i].B for i, x in zip(order, Xs)]
    st, res = mek.mek_solve_multi([plans[i] for i in order], [cuda(c) for c in Cs],
                                  X_ref=[cuda(x) for x in Xs], stop="rel_err", tol=1e-6,
                                  max_iters=400000, seed=2)
    assert st == mek.MEK_OK
    for b in (0, 1, 2, 150, 299):
        assert rel(host(res[b].X), Xs[b]) <= 1e-6
        one = mek.mek_solve(plans[order[b]], cuda(Cs[b]), X_ref=cuda(Xs[b]), stop="rel_err",
                            tol=1e-6, max_iters=400000, seed=2, instance=b)
        assert torch.equal(res[b].X, one.X) and res[b].iters == one.iters


# ---------------------------------------------------------------------------
# Row norms and row errors in device memory (instances whose norms do not fit
# in LDS, or m above the selection's register chunks; forced on small cases
# with the plan's r_in_lds = 0): the same selection arithmetic as the LDS
# form, so the two agree bit for bit.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("variant,theta", [("grbk", 0.5), ("rgrbk", 0.8), ("mwrbk", 0.5),
                                           ("rbk", 0.5), ("bk", 0.5)])
def test_sparse_norms_in_memory_equal_lds(case, variant, theta):
    inst = CASES[case]()
    alpha = oracle.spectral_alpha(inst.B)
    kw = dict(variant=variant, theta=theta, alpha=alpha, max_iters=1500, seed=23, hist_cap=1501,
              X_ref=cuda(inst.X_star))
    a = mek.mek_solve(_sparse_plan(inst, alpha), cuda(inst.C), **kw)
    b = mek.mek_solve(_sparse_plan(inst, alpha, r_in_lds=0), cuda(inst.C), **kw)
    assert torch.equal(a.X, b.X)
    assert torch.equal(a.idx_hist, b.idx_hist) and torch.equal(a.set_hist, b.set_hist)
    assert torch.equal(a.resid_hist, b.resid_hist) and torch.equal(a.err_hist, b.err_hist)


def test_sparse_rows_beyond_lds_match_oracle():
    # 12 000 rows: above what the selection holds in registers, so the norms
    # live in device memory. 200 columns keep A A^T sparse (about 540
    # nonzeros per column); the oracle runs its literal form (R = C - A X B
    # recomputed every update, no m x m Gram matrix), which its own pins tie
    # to the maintained-residual form.
    inst = workloads.sparse_random(12000, 200, 5, 20, seed=3, empty_rows=50)
    alpha = oracle.spectral_alpha(inst.B)
    for variant, theta in [("grbk", 0.5), ("rgrbk", 0.8), ("rbk", 0.5)]:
        ref = oracle.solve(inst.A, inst.B, inst.C, variant=variant, theta=theta, alpha=alpha,
                           max_iters=300, seed=5, Xref=inst.X_star, literal=True)
        res = mek.mek_solve(_sparse_plan(inst, alpha), cuda(inst.C), variant=variant,
                            theta=theta, alpha=alpha, max_iters=300, seed=5, hist_cap=301,
                            X_ref=cuda(inst.X_star))
        assert host(res.idx_hist).tolist() == ref.idx.tolist(), variant
        assert np.allclose(host(res.resid_hist), ref.s_hist, rtol=1e-8, atol=0)
        assert rel(host(res.X), ref.X) <= 1e-9


def test_sparse_norms_in_memory_batch_and_ragged():
    base = workloads.banded_gaussian(40, seed=9, sigma=0.7)
    rng = np.random.default_rng(12)
    Xs = rng.standard_normal((3, 40, 40))
    C = np.stack([base.A @ X @ base.B for X in Xs])
    kw = dict(variant="grbk", max_iters=800, seed=3, instance=7)
    mem = _sparse_plan(base, 0.0, r_in_lds=0)
    lds = _sparse_plan(base, 0.0)
    _, rb = mek.mek_solve_batched(mem, cuda(C), **kw)
    _, rl = mek.mek_solve_batched(lds, cuda(C), **kw)
    for b in range(3):
        assert torch.equal(rb[b].X, rl[b].X)
    # A ragged batch mixing an instance that needs memory norms with one that
    # would fit: both run the memory form and still match their own solves.
    tall = workloads.sparse_random(9000, 200, 6, 30, seed=4, empty_rows=20)
    pt = _sparse_plan(tall, 0.0)
    st, res = mek.mek_solve_multi([pt, lds], [cuda(tall.C), cuda(C[0])], variant="grbk",
                                  max_iters=800, seed=3, instance=7)
    one_t = mek.mek_solve(pt, cuda(tall.C), variant="grbk", max_iters=800, seed=3, instance=7)
    one_s = mek.mek_solve(lds, cuda(C[0]), variant="grbk", max_iters=800, seed=3, instance=8)
    assert torch.equal(res[0].X, one_t.X) and torch.equal(res[1].X, one_s.X)


# ---------------------------------------------------------------------------
# The paper's colour-image model: A (hw x hw) the 2-D Gaussian blur (5 x 5
# taps, sigma 6, zero padding), B = A_c^T (3 x 3, printed in the paper).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant,theta", [("grbk", 0.5), ("rgrbk", 0.8), ("mwrbk", 0.5),
                                           ("rbk", 0.5)])
def test_paper_image_model_matches_oracle(variant, theta):
    inst = workloads.paper_image_model(18, 15, seed=5, random_image=True)
    alpha = oracle.spectral_alpha(inst.B)
    ref = oracle.solve(inst.A, inst.B, inst.C, variant=variant, theta=theta, alpha=alpha,
                       max_iters=2000, seed=31, Xref=inst.X_star)
    plan = _sparse_plan(inst, alpha)
    assert mek.mek_plan_sparse_widths(plan) == (25, 3, 3, 81)
    for p in (plan, _sparse_plan(inst, alpha, r_in_lds=0)):
        res = mek.mek_solve(p, cuda(inst.C), variant=variant, theta=theta, alpha=alpha,
                            max_iters=2000, seed=31, hist_cap=2001, X_ref=cuda(inst.X_star))
        assert host(res.idx_hist).tolist() == ref.idx.tolist()
        assert np.allclose(host(res.resid_hist), ref.s_hist, rtol=1e-8, atol=0)
        assert rel(host(res.X), ref.X) <= 1e-9


# ---------------------------------------------------------------------------
# Stream-ordered solves of sparse plans (mek_solve_async): the same result as
# mek_solve, and capture into a graph replayed with eager work in between.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision,mem", [("fp64", False), ("fp32", False), ("fp64", True)])
def test_sparse_async_equals_sync(precision, mem):
    inst = workloads.blurred_image(64, 1, 0.7, seed=8)[0]
    kw = {"r_in_lds": 0} if mem else {}
    plan = _sparse_plan(inst, 0.0, precision=precision, **kw)
    X0 = cuda(np.full(inst.X_star.shape, 0.05))
    opts = dict(variant="rgrbk", theta=0.8, stop="rel_err", tol=1e-4, X_ref=cuda(inst.X_star),
                max_iters=200000, seed=6, instance=3)
    one = mek.mek_solve(plan, cuda(inst.C), X0=X0, hist_cap=64, **opts)
    hist = mek.make_histories(64)
    X, rep = mek.mek_solve_async(plan, cuda(inst.C), X0=X0, hist=hist, **opts)
    torch.cuda.synchronize()
    r = mek.read_device_report(rep)
    assert r["status"] == one.status == mek.MEK_OK and r["iters"] == one.iters
    assert r["resid2"] == one.resid2 and r["rel_err"] == one.rel_err
    assert torch.equal(X, one.X)
    assert torch.equal(hist["idx_hist"][:64], one.idx_hist[:64])


def test_sparse_async_graph_capture_and_replay():
    inst = workloads.blurred_image(64, 1, 0.7, seed=9)[0]
    plan = _sparse_plan(inst, 0.0)
    C, Xr = cuda(inst.C), cuda(inst.X_star)
    kw = dict(variant="grbk", stop="rel_err", tol=1e-5, X_ref=Xr, max_iters=400000, seed=12)
    X_e, rep_e = mek.mek_solve_async(plan, C, **kw)   # eager first: the workspace exists
    torch.cuda.synchronize()
    eager = mek.read_device_report(rep_e)
    assert eager["status"] == mek.MEK_OK
    Xg = torch.empty_like(X_e)
    repg = torch.zeros(mek.DEVICE_REPORT_BYTES, dtype=torch.uint8, device="cuda")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mek.mek_solve_async(plan, C, X_out=Xg, report=repg, **kw)
    for rep_i in range(3):
        Xg.fill_(float(rep_i))
        repg.zero_()
        junk = mek.mek_solve(plan, C, variant="rbk", max_iters=60, seed=rep_i)
        assert junk.iters == 60
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert mek.read_device_report(repg) == eager
        assert torch.equal(Xg, X_e)



def test_sparse_ragged_async_equals_sync_and_replays():
    bases = [workloads.blurred_image(48, 1, 0.7, seed=s)[0] for s in (1, 2)]
    plans = [_sparse_plan(b, 0.0) for b in bases]
    rng = np.random.default_rng(14)
    order = [0, 1, 0, 1, 0]   # both plans shared
    Xs = [rng.uniform(0, 1, (48, 48)) for _ in order]
    Cs = [cuda(bases[i].A @ x @ bases[i].B) for i, x in zip(order, Xs)]
    Xr = [cuda(x) for x in Xs]
    kw = dict(variant="grbk", stop="rel_err", tol=1e-5, max_iters=400000, seed=21, instance=4)
    st, sync = mek.mek_solve_multi([plans[i] for i in order], Cs, X_ref=Xr, **kw)
    assert st == mek.MEK_OK
    X, rep = mek.mek_solve_multi_async([plans[i] for i in order], Cs, X_ref=Xr, **kw)
    torch.cuda.synchronize()
    for b, r in enumerate(sync):
        d = mek.read_device_report(rep[b])
        assert d["status"] == r.status and d["iters"] == r.iters and d["rel_err"] == r.rel_err
        assert torch.equal(X[b], r.X)
    Xg = [torch.empty_like(x) for x in X]
    repg = torch.zeros_like(rep)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mek.mek_solve_multi_async([plans[i] for i in order], Cs, X_ref=Xr, X_out=Xg, reports=repg,
                                  **kw)
    for rep_i in range(3):
        for x in Xg:
            x.fill_(float(rep_i))
        repg.zero_()
        _, junk = mek.mek_solve_multi([plans[i] for i in order], Cs, variant="rbk", max_iters=30,
                                      seed=rep_i)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for b, r in enumerate(sync):
            assert mek.read_device_report(repg[b])["iters"] == r.iters
            assert torch.equal(Xg[b], r.X)
