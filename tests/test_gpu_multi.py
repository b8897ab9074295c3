"""GPU parity of the ragged batch (mek_solve_multi: instances of uneven size,
each with its own plan, in one persistent launch) through the C ABI, against
the CPU oracle run instance by instance and against single-instance calls.

Bar as in test_gpu_parity: identical index sequences, residual and error
histories within 1e-8 relative, iterates within 1e-9 relative after
hundreds of FP64 updates; FP32 instances follow the single-instance FP32
call's indices and meet the FP32 tolerance.
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


def _plans(insts, precision="fp64", **kw):
    alphas = [oracle.spectral_alpha(i.B) for i in insts]
    plans = [mek.mek_plan_create(cuda(i.A), cuda(i.B), alpha=a, precision=precision, **kw)
             for i, a in zip(insts, alphas)]
    return plans, alphas


@pytest.mark.parametrize("variant,theta", [("grbk", 0.5), ("rgrbk", 0.8), ("mwrbk", 0.5),
                                           ("rbk", 0.5), ("bk", 0.5)])
def test_multi_trajectories_match_oracle(variant, theta):
    # Uneven sizes, including m < p and n < q (underdetermined instances).
    insts = workloads.ragged_batch(5, seed=41, mn_range=(20, 90), pq_range=(5, 40))
    K = 300
    plans, alphas = _plans(insts)
    code, res = mek.mek_solve_multi(plans, [cuda(i.C) for i in insts],
                                    X_ref=[cuda(i.X_star) for i in insts], variant=variant,
                                    theta=theta, max_iters=K, seed=77, instance=5,
                                    hist_cap=K + 1)
    assert code == mek.MEK_MAXITER
    for b, inst in enumerate(insts):
        ref = oracle.solve(inst.A, inst.B, inst.C, variant=variant, theta=theta, alpha=alphas[b],
                           max_iters=K, seed=77, inst=5 + b, Xref=inst.X_star)
        r = res[b]
        assert r.status == mek.MEK_MAXITER and r.iters == K
        assert host(r.idx_hist).tolist() == ref.idx.tolist()
        assert np.allclose(host(r.resid_hist), ref.s_hist, rtol=1e-8, atol=0)
        assert np.allclose(host(r.err_hist), ref.e_hist, rtol=1e-8, atol=0)
        assert rel(host(r.X), ref.X) <= 1e-9


def test_multi_equals_single_calls_and_warm_start():
    insts = workloads.ragged_batch(6, seed=42, mn_range=(30, 200), pq_range=(8, 60))
    plans, _ = _plans(insts)
    rng = np.random.default_rng(3)
    X0 = [rng.standard_normal((i.shape[1], i.shape[2])) if b % 2 else None
          for b, i in enumerate(insts)]
    K = 1200
    code, res = mek.mek_solve_multi(plans, [cuda(i.C) for i in insts],
                                    X0=[None if x is None else cuda(x) for x in X0],
                                    variant="grbk", max_iters=K, seed=9, instance=20,
                                    hist_cap=K + 1)
    for b, inst in enumerate(insts):
        one = mek.mek_solve(plans[b], cuda(inst.C), X0=None if X0[b] is None else cuda(X0[b]),
                            variant="grbk", max_iters=K, seed=9, instance=20 + b, hist_cap=K + 1)
        assert host(one.idx_hist).tolist() == host(res[b].idx_hist).tolist()
        assert rel(host(res[b].X), host(one.X)) <= 1e-12


def test_multi_stops_each_instance_at_its_tolerance():
    # Overdetermined instances (m >= p, n >= q): X* is the unique solution.
    insts = workloads.ragged_batch(7, seed=43, mn_range=(60, 160), pq_range=(10, 30))
    plans, alphas = _plans(insts)
    code, res = mek.mek_solve_multi(plans, [cuda(i.C) for i in insts],
                                    X_ref=[cuda(i.X_star) for i in insts], variant="grbk",
                                    stop="rel_err", tol=1e-6, max_iters=2_000_000, seed=5)
    assert code == mek.MEK_OK
    iters = []
    for b, inst in enumerate(insts):
        r = res[b]
        assert r.status == mek.MEK_OK and r.rel_err <= 1e-6
        assert rel(host(r.X), inst.X_star) <= 1e-6
        ref = oracle.solve(inst.A, inst.B, inst.C, variant="grbk", alpha=alphas[b],
                           stop=oracle.STOP_REL_ERR, tol=1e-6, Xref=inst.X_star,
                           max_iters=2_000_000, seed=5, inst=b)
        assert abs(r.iters - ref.iters) <= max(2, 0.01 * ref.iters)
        iters.append(r.iters)
    assert len(set(iters)) > 1   # the instances finish at their own counts


def test_multi_fp32():
    # One team size for the ragged and the single calls, so that the FP32
    # dot products are partitioned (and rounded) alike.
    insts = workloads.ragged_batch(5, seed=44, mn_range=(60, 300), pq_range=(10, 40))
    plans, _ = _plans(insts, precision="fp32", team_wgs=4)
    K = 800
    code, res = mek.mek_solve_multi(plans, [cuda(i.C) for i in insts], variant="grbk",
                                    max_iters=K, seed=13, hist_cap=K + 1)
    assert code == mek.MEK_MAXITER
    for b, inst in enumerate(insts):
        one = mek.mek_solve(plans[b], cuda(inst.C), variant="grbk", max_iters=K, seed=13,
                            instance=b, hist_cap=K + 1)
        assert res[b].team_wgs == one.team_wgs == 4
        assert host(one.idx_hist).tolist() == host(res[b].idx_hist).tolist()
        assert rel(host(res[b].X), host(one.X)) <= 1e-6
    code, res = mek.mek_solve_multi(plans, [cuda(i.C) for i in insts],
                                    X_ref=[cuda(i.X_star) for i in insts], variant="grbk",
                                    stop="rel_err", tol=1e-4, max_iters=2_000_000, seed=13)
    assert code == mek.MEK_OK
    for b, inst in enumerate(insts):
        assert res[b].status == mek.MEK_OK
        assert rel(host(res[b].X), inst.X_star) <= 1.5e-4


def test_multi_workload_shapes_first_updates():
    # Sizes of the uneven-instance workload (m, n in 128..1024; p, q in
    # 64..512), 16 instances in one launch; the first updates of three of
    # them against the oracle.
    insts = workloads.ragged_batch(16, seed=5)
    plans, alphas = _plans(insts)
    K = 60
    code, res = mek.mek_solve_multi(plans, [cuda(i.C) for i in insts],
                                    X_ref=[cuda(i.X_star) for i in insts], variant="grbk",
                                    max_iters=K, seed=2408054440, hist_cap=K + 1)
    assert code == mek.MEK_MAXITER
    assert sum(r.team_wgs for r in res) <= torch.cuda.get_device_properties(0).multi_processor_count
    for b in (0, 7, 15):
        inst = insts[b]
        ref = oracle.solve(inst.A, inst.B, inst.C, variant="grbk", alpha=alphas[b], max_iters=K,
                           seed=2408054440, inst=b, Xref=inst.X_star)
        assert host(res[b].idx_hist).tolist() == ref.idx.tolist()
        assert np.allclose(host(res[b].resid_hist), ref.s_hist, rtol=1e-8, atol=0)
        assert rel(host(res[b].X), ref.X) <= 1e-10


def test_multi_argument_checks():
    insts = workloads.ragged_batch(2, seed=45, mn_range=(20, 40), pq_range=(5, 10))
    plans, _ = _plans(insts)
    C = [cuda(i.C) for i in insts]
    with pytest.raises(mek.MekError) as e:   # the same plan twice
        mek.mek_solve_multi([plans[0], plans[0]], [C[0], C[0]], max_iters=1)
    assert e.value.code == mek.MEK_EINVAL
    p32 = mek.mek_plan_create(cuda(insts[1].A), cuda(insts[1].B), precision="fp32")
    with pytest.raises(mek.MekError) as e:   # mixed precisions
        mek.mek_solve_multi([plans[0], p32], C, max_iters=1)
    assert e.value.code == mek.MEK_EINVAL
    pm = [mek.mek_plan_create(cuda(i.A), cuda(i.B), precision="mixed") for i in insts]
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve_multi(pm, C, max_iters=1)
    assert e.value.code == mek.MEK_EUNSUPPORTED
    with pytest.raises(mek.MekError) as e:   # REL_ERR needs a reference per instance
        mek.mek_solve_multi(plans, C, stop="rel_err", tol=1e-6, max_iters=1)
    assert e.value.code == mek.MEK_EINVAL
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve_multi(plans, C, variant="twosided", max_iters=1)
    assert e.value.code == mek.MEK_EUNSUPPORTED
    # opts->X_ref must stay NULL (references come per instance).
    L = mek.lib()
    o, _ = mek._solve_opts(2, C[0].device, "grbk", 0.5, 0.0, "none", 0.0,
                           ctypes.c_void_p(insts[0].X_star.ctypes.data), 1, 0, 0, None, 0.0, 0, 0)
    handles = (ctypes.c_void_p * 2)(*[P.handle for P in plans])
    Cp = (ctypes.c_void_p * 2)(*[c.data_ptr() for c in C])
    X = [torch.empty(i.shape[1], i.shape[2], dtype=torch.float64, device="cuda") for i in insts]
    Xp = (ctypes.c_void_p * 2)(*[x.data_ptr() for x in X])
    assert L.mek_solve_multi(2, handles, Cp, None, None, ctypes.byref(o), Xp, None,
                             None) == mek.MEK_EINVAL
