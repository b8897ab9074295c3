"""The stream-ordered solve (mek_solve_async) through the C ABI: the same
iteration and result as mek_solve, calls queued without host waits, and
capture into a graph replayed several times with the program's own eager
work between the replays (every replay checked against the eager result)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2408_05444_amd as mek
import workloads

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")]


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("team", [0, 1, 5])
@pytest.mark.parametrize("warm", [False, True])
def test_async_equals_sync(team, warm):
    inst = workloads.ragged(seed=12)
    alpha = oracle.spectral_alpha(inst.B)
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), alpha=alpha, team_wgs=team)
    X0 = cuda(np.random.default_rng(1).standard_normal((inst.shape[1], inst.shape[2]))) if warm else None
    kw = dict(variant="grbk", stop="rel_err", tol=1e-7, X_ref=cuda(inst.X_star), max_iters=200000,
              seed=3, instance=2)
    one = mek.mek_solve(plan, cuda(inst.C), X0=X0, hist_cap=0, **kw)
    hist = mek.make_histories(one.iters + 1)
    X, rep = mek.mek_solve_async(plan, cuda(inst.C), X0=X0, hist=hist, **kw)
    torch.cuda.synchronize()
    r = mek.read_device_report(rep)
    assert r["status"] == one.status and r["iters"] == one.iters
    assert r["rel_err"] == one.rel_err and r["resid2"] == one.resid2
    assert torch.equal(X, one.X)
    ref = mek.mek_solve(plan, cuda(inst.C), X0=X0, hist_cap=one.iters + 1, **kw)
    assert torch.equal(hist["idx_hist"][:one.iters], ref.idx_hist[:one.iters].to(torch.int32))


def test_async_calls_queue_without_waits():
    base = workloads.small(seed=4)
    insts = workloads.shared_ab_batch(base, 4, seed=9)
    alpha = oracle.spectral_alpha(base.B)
    plan = mek.mek_plan_create(cuda(base.A), cuda(base.B), alpha=alpha)
    kw = dict(variant="rgrbk", theta=0.7, max_iters=3000, seed=5)
    Cs = [cuda(i.C) for i in insts]
    outs = [mek.mek_solve_async(plan, C, instance=b, **kw) for b, C in enumerate(Cs)]
    torch.cuda.synchronize()
    for b, (C, (X, rep)) in enumerate(zip(Cs, outs)):
        one = mek.mek_solve(plan, C, instance=b, **kw)
        assert mek.read_device_report(rep)["iters"] == one.iters == 3000
        assert torch.equal(X, one.X)


def test_async_fp32():
    inst = workloads.small(seed=5)
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), precision="fp32")
    kw = dict(variant="grbk", stop="rel_resid", tol=1e-4, max_iters=500000, seed=8)
    # The stream-ordered call runs without residual refreshes: compare with
    # the blocking call with refreshes switched off.
    one = mek.mek_solve(plan, cuda(inst.C), refresh_period=-1, **kw)
    X, rep = mek.mek_solve_async(plan, cuda(inst.C), **kw)
    torch.cuda.synchronize()
    r = mek.read_device_report(rep)
    assert r["status"] == one.status == mek.MEK_OK and r["iters"] == one.iters
    assert torch.equal(X, one.X)


def test_async_rejects_unsupported_forms():
    inst = workloads.small()
    pm = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), precision="mixed")
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve_async(pm, cuda(inst.C), max_iters=10)
    assert e.value.code == mek.MEK_EUNSUPPORTED
    p64 = mek.mek_plan_create(cuda(inst.A), cuda(inst.B))
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve_async(p64, cuda(inst.C), variant="twosided", max_iters=10)
    assert e.value.code == mek.MEK_EUNSUPPORTED
    # Residual refreshes need host decisions between passes.
    o = mek.mek_solve_opts()
    o.max_iters = 10
    o.refresh_period = 5
    C = cuda(inst.C)
    X = torch.empty(40, 40, dtype=torch.float64, device="cuda")
    rep = torch.zeros(mek.DEVICE_REPORT_BYTES, dtype=torch.uint8, device="cuda")
    st = mek.lib().mek_solve_async(p64.handle, ctypes.c_void_p(C.data_ptr()), None, ctypes.byref(o),
                                   ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(rep.data_ptr()),
                                   None)
    assert st == mek.MEK_EUNSUPPORTED


@pytest.mark.parametrize("team", [1, 6])
def test_async_graph_capture_and_replay(team):
    # team 1: a plain launch; team 6: a cooperative launch of 6 work-groups.
    inst = workloads.small(seed=6)
    alpha = oracle.spectral_alpha(inst.B)
    plan = mek.mek_plan_create(cuda(inst.A), cuda(inst.B), alpha=alpha, team_wgs=team)
    C, Xref = cuda(inst.C), cuda(inst.X_star)
    kw = dict(variant="grbk", stop="rel_err", tol=1e-6, X_ref=Xref, max_iters=100000, seed=11)
    X_e, rep_e = mek.mek_solve_async(plan, C, **kw)    # eager: the reference for every replay
    torch.cuda.synchronize()
    eager = mek.read_device_report(rep_e)
    assert eager["status"] == mek.MEK_OK
    Xg = torch.empty_like(X_e)
    repg = torch.zeros(mek.DEVICE_REPORT_BYTES, dtype=torch.uint8, device="cuda")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mek.mek_solve_async(plan, C, X_out=Xg, report=repg, **kw)
    for rep_i in range(3):
        # eager work of the program between the replays
        Xg.fill_(float(rep_i))
        repg.zero_()
        junk = mek.mek_solve(plan, C, variant="rbk", max_iters=50, seed=rep_i)
        assert junk.iters == 50
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        r = mek.read_device_report(repg)
        assert r == eager
        assert torch.equal(Xg, X_e)
