"""The learned warm start end to end on the GPU: labels from the solver,
training by the library's BF16 kernels, and the gain on held-out images
(not in the paper: X0 = C + f(C) replaces the paper's X^0 = 0).

Workload: 3-channel 256 x 256 blurred images (sigma uniform on [1, 3], no
noise), 48 training images, 4 held-out ones. The X0 = 0 solve and the
warm-started solve stop at the same relative residual 1e-3; the trained
network must start every held-out channel below the zero start's residual
(no fallback) and cut the mean number of updates.
"""
import numpy as np
import pytest
import torch

import paper_2408_05444_amd as mek
import workloads
from paper_2408_05444_amd import warmstart

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")]


def t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def test_labels_are_solver_iterates_at_tau():
    imgs = [workloads.warmstart_image(100000 + i) for i in range(2)]
    train = [(t(A), t(B), t(C)) for A, B, C, _, _ in imgs]
    labels = warmstart.solver_labels(mek, train, tau=1e-3, seed=7)
    for (A, B, C, _, _), L in zip(imgs, labels):
        L = L.cpu().numpy()
        for c in range(3):
            r = np.linalg.norm(C[c] - A @ L[c] @ B) / np.linalg.norm(C[c])
            assert r <= 1e-3 and r > 5e-4   # stopped at the first update below tau


def test_trained_warm_start_cuts_updates_on_held_out_images():
    train = []
    for i in range(48):
        A, B, C, _, _ = workloads.warmstart_image(100000 + i)
        train.append((t(A), t(B), t(C)))
    labels = warmstart.solver_labels(mek, train, tau=1e-3, seed=2408054440)
    Cs, Ls = torch.stack([c for _, _, c in train]), torch.stack(labels)
    net = warmstart.WarmStartNet(seed=0)
    hist = net.train(Cs, Ls, epochs=40, batch=4, lr=2e-3)
    assert hist[-1] < 0.5 * hist[0]
    held = []
    for j in range(4):
        A, B, C, _, _ = workloads.warmstart_image(200000 + j)
        held.append((t(A), t(B), t(C)))
    r = warmstart.compare_warm_start(mek, net, held, tau=1e-3, seed=2408054440)
    assert len(r["iters_zero"]) == 12 and not any(r["fallback"])
    assert all(s == mek.MEK_OK for s in r["status_zero"] + r["status_warm"])
    assert max(r["start_rel_resid_warm"]) < 0.1
    assert np.mean(r["iters_warm"]) <= 0.85 * np.mean(r["iters_zero"])


def test_comparison_zero_side_equals_single_solves_and_fallback():
    # The zero-start side is the plain solve of each channel (Philox key =
    # the channel's position in the list); an untrained network whose output
    # is far off falls back to X0 = 0, and then both sides agree.
    held = []
    for j in range(2):
        A, B, C, _, _ = workloads.warmstart_image(200000 + j)
        held.append((t(A), t(B), t(C)))
    net = warmstart.WarmStartNet(seed=0)
    with torch.no_grad():
        net.w[-1].mul_(1e4)   # a wild last layer
        for src, dst in zip(net.params, net.q):
            dst.copy_(src)
    r = warmstart.compare_warm_start(mek, net, held, tau=1e-3, seed=11)
    assert all(r["fallback"])
    assert r["iters_warm"] == r["iters_zero"]
    A, B, C = held[1]
    plan = mek.mek_plan_create(A, B, update="sparse")
    one = mek.mek_solve(plan, C[2].contiguous(), variant="grbk", stop="rel_resid", tol=1e-3,
                        max_iters=1_000_000, seed=11, instance=5)
    assert one.iters == r["iters_zero"][5]
