"""GPU parity of the uniform batch (instances sharing A and B in one
persistent launch) and of the image-restoration precision form, through
the C ABI, against the CPU oracle run instance by instance.

Tolerances as in test_gpu_parity: identical index sequences, iterates within
1e-9 relative after hundreds of FP64 updates; mixed vs FP64 under the same
replayed indices within 1e-5 relative (the FP32 inner iterations carry
O(1e-7) relative rounding per refinement pass, amplified by the blur's
conditioning over the budget).
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


def stack(insts, field):
    return cuda(np.stack([getattr(i, field) for i in insts]))


@pytest.mark.parametrize("team,lds", [(0, -1), (8, 1), (3, 0)])
@pytest.mark.parametrize("variant,theta", [("grbk", 0.5), ("rgrbk", 0.8), ("mwrbk", 0.5),
                                           ("rbk", 0.5), ("bk", 0.5)])
def test_batched_trajectories_match_oracle(team, lds, variant, theta):
    base = workloads.ragged()
    insts = workloads.shared_ab_batch(base, 3, seed=31)
    alpha = oracle.spectral_alpha(base.B)
    K = 400
    plan = mek.mek_plan_create(cuda(base.A), cuda(base.B), alpha=alpha, team_wgs=team,
                               r_in_lds=lds)
    code, res = mek.mek_solve_batched(plan, stack(insts, "C"), variant=variant, theta=theta,
                                      alpha=alpha, max_iters=K, seed=77, instance=5,
                                      X_ref=stack(insts, "X_star"), hist_cap=K + 1)
    assert code == mek.MEK_MAXITER
    for b, inst in enumerate(insts):
        ref = oracle.solve(inst.A, inst.B, inst.C, variant=variant, theta=theta, alpha=alpha,
                           max_iters=K, seed=77, inst=5 + b, Xref=inst.X_star)
        r = res[b]
        assert r.status == mek.MEK_MAXITER and r.iters == K
        if team:
            assert r.team_wgs == team and r.r_in_lds == bool(lds)
        assert host(r.idx_hist).tolist() == ref.idx.tolist()
        assert np.allclose(host(r.resid_hist), ref.s_hist, rtol=1e-8, atol=0)
        assert np.allclose(host(r.err_hist), ref.e_hist, rtol=1e-8, atol=0)
        assert rel(host(r.X), ref.X) <= 1e-9


def test_batched_equals_separate_calls():
    base = workloads.small(seed=6)
    insts = workloads.shared_ab_batch(base, 5, seed=8)
    alpha = oracle.spectral_alpha(base.B)
    plan = mek.mek_plan_create(cuda(base.A), cuda(base.B), alpha=alpha)
    code, res = mek.mek_solve_batched(plan, stack(insts, "C"), variant="grbk", alpha=alpha,
                                      max_iters=1500, seed=3, instance=10, hist_cap=1501)
    for b, inst in enumerate(insts):
        one = mek.mek_solve(plan, cuda(inst.C), variant="grbk", alpha=alpha, max_iters=1500,
                            seed=3, instance=10 + b, hist_cap=1501)
        assert host(one.idx_hist).tolist() == host(res[b].idx_hist).tolist()
        assert rel(host(one.X), host(res[b].X)) <= 1e-12


def test_batched_stop_per_instance_and_warm_start():
    # Instances stop on their own: instance 1 starts at its solution (0
    # updates), the others run to the tolerance.
    base = workloads.small(seed=2)
    insts = workloads.shared_ab_batch(base, 4, seed=12)
    alpha = oracle.spectral_alpha(base.B)
    X0 = np.zeros((4, 40, 40))
    X0[1] = insts[1].X_star
    plan = mek.mek_plan_create(cuda(base.A), cuda(base.B), alpha=alpha)
    code, res = mek.mek_solve_batched(plan, stack(insts, "C"), X0=cuda(X0), variant="grbk",
                                      alpha=alpha, stop="rel_err", tol=1e-6,
                                      X_ref=stack(insts, "X_star"), max_iters=2_000_000, seed=4)
    assert code == mek.MEK_OK
    assert res[1].iters == 0
    for b, inst in enumerate(insts):
        assert res[b].status == mek.MEK_OK
        assert rel(host(res[b].X), inst.X_star) <= 1e-6
        if b != 1:
            ref = oracle.solve(inst.A, inst.B, inst.C, variant="grbk", alpha=alpha,
                               stop=oracle.STOP_REL_ERR, tol=1e-6, Xref=inst.X_star,
                               max_iters=10 ** 6, seed=4, inst=b)
            assert abs(res[b].iters - ref.iters) <= max(2, 0.02 * ref.iters)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("mixed", 1e-6)])
def test_batched_precision_forms_converge(precision, tol):
    base = workloads.ragged(seed=13)
    insts = workloads.shared_ab_batch(base, 3, seed=14)
    plan = mek.mek_plan_create(cuda(base.A), cuda(base.B), precision=precision)
    code, res = mek.mek_solve_batched(plan, stack(insts, "C"), variant="grbk", stop="rel_err",
                                      tol=tol, X_ref=stack(insts, "X_star"),
                                      max_iters=2_000_000, seed=5)
    assert code == mek.MEK_OK
    for b, inst in enumerate(insts):
        assert res[b].status == mek.MEK_OK
        assert rel(host(res[b].X), inst.X_star) <= tol


def test_blur_channels_fixed_budget_matches_oracle():
    # The image-restoration form at reduced size: 3 channels of a 64 x 64
    # synthetic image, banded Gaussian blur (sigma 2, 9 taps, rows summing
    # to 1) on both sides, N(0, 1e-3^2) noise, a fixed budget of 100 m
    # updates per channel (1e-6 is out of reach at this conditioning).
    chans = workloads.blurred_image(64, 3, 2.0, seed=4, noise_std=1e-3)
    A, B = chans[0].A, chans[0].B
    alpha = oracle.spectral_alpha(B)
    K = 6400
    plan = mek.mek_plan_create(cuda(A), cuda(B), alpha=alpha)
    code, res = mek.mek_solve_batched(plan, stack(chans, "C"), variant="rgrbk", theta=0.8,
                                      alpha=alpha, max_iters=K, seed=9,
                                      X_ref=stack(chans, "X_star"), hist_cap=K + 1)
    for b, ch in enumerate(chans):
        ref = oracle.solve(A, B, ch.C, variant="rgrbk", theta=0.8, alpha=alpha, max_iters=K,
                           seed=9, inst=b, Xref=ch.X_star)
        assert host(res[b].idx_hist).tolist() == ref.idx.tolist()
        assert rel(host(res[b].X), ref.X) <= 1e-9
        # The restoration improves on the blurred image itself.
        assert rel(host(res[b].X), ch.X_star) < rel(ch.C, ch.X_star)


def test_blur_channels_mixed_vs_fp64_under_replay():
    chans = workloads.blurred_image(64, 3, 2.0, seed=4, noise_std=1e-3)
    A, B = chans[0].A, chans[0].B
    alpha = oracle.spectral_alpha(B)
    K = 6400
    p64 = mek.mek_plan_create(cuda(A), cuda(B), alpha=alpha)
    C = stack(chans, "C")
    # One index sequence for every channel: the oracle's for channel 0.
    seq = oracle.solve(A, B, chans[0].C, variant="rgrbk", theta=0.8, alpha=alpha, max_iters=K,
                       seed=9).idx
    rp = cuda(seq, torch.int32)
    _, r64 = mek.mek_solve_batched(p64, C, variant="rgrbk", theta=0.8, alpha=alpha,
                                   max_iters=K, replay_idx=rp)
    pmx = mek.mek_plan_create(cuda(A), cuda(B), alpha=alpha, precision="mixed")
    _, rmx = mek.mek_solve_batched(pmx, C, variant="rgrbk", theta=0.8, alpha=alpha,
                                   max_iters=K, replay_idx=rp, inner_iters=K // 8, hist_cap=K + 1)
    for b, ch in enumerate(chans):
        ref = oracle.solve(A, B, ch.C, variant="rgrbk", theta=0.8, alpha=alpha, max_iters=K,
                           forced=seq)
        assert rel(host(r64[b].X), ref.X) <= 1e-9
        assert rmx[b].iters == K and rmx[b].passes >= 8
        assert rel(host(rmx[b].X), host(r64[b].X)) <= 1e-5


def test_blur_full_size_mixed_vs_fp64_under_replay():
    """The image form at full size: 3 channels of a 512 x 512 image, blur
    sigma 2 on both sides, noise std 1e-3, ME-RGRBK theta 0.8, a budget of
    100 m = 51200 updates per channel. The FP64 trajectory of channel 0 is
    the oracle's over its first 2000 updates; replaying channel 0's indices
    on every channel, the mixed form (FP64 refinement around FP32 inner
    solves with split-BF16 inner residual refreshes) stays within 1e-5 of
    the FP64 iterate."""
    chans = workloads.blurred_image(512, 3, 2.0, seed=4, noise_std=1e-3)
    A, B = chans[0].A, chans[0].B
    alpha = oracle.spectral_alpha(B)
    K, W = 100 * 512, 2000
    C = stack(chans, "C")
    p64 = mek.mek_plan_create(cuda(A), cuda(B), alpha=alpha)
    _, f64 = mek.mek_solve_batched(p64, C, variant="rgrbk", theta=0.8, alpha=alpha,
                                   max_iters=K, seed=9, hist_cap=K + 1)
    seq = host(f64[0].idx_hist)
    ref = oracle.solve(A, B, chans[0].C, variant="rgrbk", theta=0.8, alpha=alpha, max_iters=W,
                       seed=9)
    assert seq[:W].tolist() == ref.idx.tolist()
    rp = cuda(seq, torch.int32)
    _, r64 = mek.mek_solve_batched(p64, C, variant="rgrbk", theta=0.8, alpha=alpha, max_iters=K,
                                   replay_idx=rp)
    pmx = mek.mek_plan_create(cuda(A), cuda(B), alpha=alpha, precision="mixed")
    _, rmx = mek.mek_solve_batched(pmx, C, variant="rgrbk", theta=0.8, alpha=alpha, max_iters=K,
                                   replay_idx=rp, inner_iters=K // 8)
    assert rel(host(r64[0].X), host(f64[0].X)) == 0.0
    for b in range(3):
        assert rmx[b].iters == K and rmx[b].passes >= 8
        assert rel(host(rmx[b].X), host(r64[b].X)) <= 1e-5
    for P in (p64, pmx):
        mek.mek_plan_destroy(P)


def test_batched_edge_cases():
    base = workloads.small()
    alpha = oracle.spectral_alpha(base.B)
    plan = mek.mek_plan_create(cuda(base.A), cuda(base.B), alpha=alpha)
    # batch of one is mek_solve
    one = mek.mek_solve(plan, cuda(base.C), variant="mwrbk", alpha=alpha, max_iters=300)
    code, res = mek.mek_solve_batched(plan, cuda(base.C[None]), variant="mwrbk", alpha=alpha,
                                      max_iters=300)
    assert code == mek.MEK_MAXITER and rel(host(res[0].X), host(one.X)) == 0.0
    # more instances than compute units, and an empty batch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    o = mek.mek_solve_opts()
    o.max_iters = 1
    C = torch.zeros(cus + 1, 100, 100, dtype=torch.float64, device="cuda")
    X = torch.zeros(cus + 1, 40, 40, dtype=torch.float64, device="cuda")
    L = mek.lib()
    st = L.mek_solve_batched(plan.handle, cus + 1, ctypes.c_void_p(C.data_ptr()), None,
                             ctypes.byref(o), ctypes.c_void_p(X.data_ptr()), None, None)
    assert st == mek.MEK_EUNSUPPORTED
    st = L.mek_solve_batched(plan.handle, 0, ctypes.c_void_p(C.data_ptr()), None,
                             ctypes.byref(o), ctypes.c_void_p(X.data_ptr()), None, None)
    assert st == mek.MEK_EINVAL
