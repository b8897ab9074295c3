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
    zero, warm = [], []
    for j in range(4):
        A, B, C, _, _ = workloads.warmstart_image(200000 + j)
        r = warmstart.compare_warm_start(mek, net, t(A), t(B), t(C), tau=1e-3, seed=2408054440)
        assert not any(r["fallback"])
        assert all(s == mek.MEK_OK for s in r["status_zero"] + r["status_warm"])
        assert max(r["start_rel_resid_warm"]) < 0.1
        zero += r["iters_zero"]
        warm += r["iters_warm"]
    assert np.mean(warm) <= 0.85 * np.mean(zero)
