"""The stream-ordered ragged batch (mek_solve_multi_async) through the C ABI:
the same iteration and results as mek_solve_multi, enqueued without host
waits, and captured into a graph replayed several times with the program's
own eager work between the replays (every replay checked against the eager
result, bit for bit)."""
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


def _batch(nb, seed, precision="fp64"):
    # m, n at least twice p, q: full rank and well conditioned, so X* is the limit.
    insts = workloads.ragged_batch(nb, seed, mn_range=(60, 200), pq_range=(10, 30))
    plans = [mek.mek_plan_create(cuda(i.A), cuda(i.B), alpha=oracle.spectral_alpha(i.B),
                                 precision=precision) for i in insts]
    return insts, plans


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_multi_async_equals_sync(precision):
    insts, plans = _batch(7, seed=21, precision=precision)
    C = [cuda(i.C) for i in insts]
    Xr = [cuda(i.X_star) for i in insts]
    X0 = [None if b % 2 else cuda(np.full(i.X_star.shape, 0.01)) for b, i in enumerate(insts)]
    tol = 1e-6 if precision == "fp64" else 1e-4
    kw = dict(variant="rgrbk", theta=0.7, stop="rel_err", tol=tol, max_iters=400000, seed=9,
              instance=3)
    st, sync = mek.mek_solve_multi(plans, C, X0=X0, X_ref=Xr, hist_cap=50, **kw)
    assert st == mek.MEK_OK
    hist = mek.make_histories(50, nb=len(plans))
    X, rep = mek.mek_solve_multi_async(plans, C, X0=X0, X_ref=Xr, hist=hist, **kw)
    torch.cuda.synchronize()
    for b, r in enumerate(sync):
        d = mek.read_device_report(rep[b])
        assert d["status"] == r.status == mek.MEK_OK
        assert d["iters"] == r.iters
        assert d["resid2"] == r.resid2 and d["rel_err"] == r.rel_err
        assert torch.equal(X[b], r.X)
        k = min(r.iters, 50)
        assert torch.equal(hist["idx_hist"][b, :k], r.idx_hist[:k].to(torch.int32))


def test_multi_async_graph_capture_and_replay():
    insts, plans = _batch(5, seed=22)
    C = [cuda(i.C) for i in insts]
    Xr = [cuda(i.X_star) for i in insts]
    kw = dict(variant="grbk", stop="rel_err", tol=1e-6, max_iters=400000, seed=4)
    X_e, rep_e = mek.mek_solve_multi_async(plans, C, X_ref=Xr, **kw)   # eager first
    torch.cuda.synchronize()
    eager = [mek.read_device_report(rep_e[b]) for b in range(len(plans))]
    assert all(e["status"] == mek.MEK_OK for e in eager)
    Xg = [torch.empty_like(x) for x in X_e]
    repg = torch.zeros_like(rep_e)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mek.mek_solve_multi_async(plans, C, X_ref=Xr, X_out=Xg, reports=repg, **kw)
    for rep_i in range(3):
        # eager work of the program between the replays, on the same plans
        for x in Xg:
            x.fill_(float(rep_i))
        repg.zero_()
        st, junk = mek.mek_solve_multi(plans, C, variant="rbk", max_iters=40, seed=rep_i)
        assert all(r.iters == 40 for r in junk)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for b in range(len(plans)):
            assert mek.read_device_report(repg[b]) == eager[b]
            assert torch.equal(Xg[b], X_e[b])


def test_multi_async_refusals():
    insts, plans = _batch(2, seed=23)
    C = [cuda(i.C) for i in insts]
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve_multi_async(plans, C, variant="twosided", max_iters=5)
    assert e.value.code == mek.MEK_EUNSUPPORTED
    pm = [mek.mek_plan_create(cuda(i.A), cuda(i.B), precision="mixed") for i in insts]
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve_multi_async(pm, C, max_iters=5)
    assert e.value.code == mek.MEK_EUNSUPPORTED
    with pytest.raises(mek.MekError) as e:
        mek.mek_solve_multi_async([plans[0], plans[0]], [C[0], C[0]], max_iters=5)
    assert e.value.code == mek.MEK_EINVAL
