"""Learned warm start X0 = C + f(C) for the image form of A X B = C (an
extension of the paper's initial guess X^0, not in the paper).

f is four 3 x 3 convolutions 3 -> 32 -> 32 -> 32 -> 3 with ReLU after the
first three, applied to the three channels of C at once; activations and
their gradients are BF16, sums FP32, the output and the loss FP64. Every
step (layers, gradients, loss, Adam) runs in the library's kernels through
the C ABI; this module only sequences the calls and owns the buffers.
"""
from __future__ import annotations

import ctypes
import time
from typing import List, Optional

import numpy as np
import torch

from . import _check, _stream, lib

CHANNELS = (3, 32, 32, 32, 3)


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class WarmStartNet:
    """The network, its FP32 master weights, BF16-rounded working weights and
    Adam moments, all on the GPU."""

    def __init__(self, seed: int = 0, device: str = "cuda"):
        self.device = torch.device(device)
        rng = np.random.default_rng(seed)
        self.w: List[torch.Tensor] = []
        self.b: List[torch.Tensor] = []
        nl = len(CHANNELS) - 1
        for li, (ci, co) in enumerate(zip(CHANNELS[:-1], CHANNELS[1:])):
            # He initialisation; the last layer starts small so that the
            # untrained network gives X0 close to C.
            std = np.sqrt(2.0 / (ci * 9)) * (0.1 if li == nl - 1 else 1.0)
            self.w.append(self._t(rng.standard_normal((co, ci, 3, 3)) * std))
            self.b.append(self._t(np.zeros(co)))
        self.params = self.w + self.b
        self.q = [torch.empty_like(t) for t in self.params]      # BF16-rounded copies
        self.m = [torch.zeros_like(t) for t in self.params]
        self.v = [torch.zeros_like(t) for t in self.params]
        self.g = [torch.zeros_like(t) for t in self.params]
        self.t = 0
        for src, dst in zip(self.params, self.q):
            _check(lib().mek_cnn_round_bf16(src.numel(), _p(src), _p(dst), _stream()),
                   "mek_cnn_round_bf16")

    def _t(self, a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(self.device)

    @property
    def wq(self):
        return self.q[:len(self.w)]

    @property
    def bq(self):
        return self.q[len(self.w):]

    def num_params(self) -> int:
        return sum(t.numel() for t in self.params)

    def to_input(self, C: torch.Tensor) -> torch.Tensor:
        """C (N, 3, H, W) float64 -> BF16 input."""
        x = torch.empty(C.shape, dtype=torch.int16, device=self.device)
        _check(lib().mek_cnn_to_bf16(C.numel(), _p(C), 1.0, _p(x), _stream()), "mek_cnn_to_bf16")
        return x

    def forward(self, C: torch.Tensor):
        """Returns (activations [x, y1, y2, y3] in BF16, X0 = C + f(C) FP64)."""
        N, _, H, W = C.shape
        acts = [self.to_input(C)]
        nl = len(CHANNELS) - 1
        for li in range(nl):
            ci, co = CHANNELS[li], CHANNELS[li + 1]
            if li < nl - 1:
                # 32-channel activations are channels-last (NHWC).
                y = torch.empty((N, H, W, co), dtype=torch.int16, device=self.device)
                _check(lib().mek_cnn_conv3x3(N, ci, H, W, co, _p(acts[-1]), _p(self.wq[li]),
                                             _p(self.bq[li]), 1, _p(y), None, None, _stream()),
                       "mek_cnn_conv3x3")
                acts.append(y)
            else:
                out = torch.empty((N, co, H, W), dtype=torch.float64, device=self.device)
                _check(lib().mek_cnn_conv3x3(N, ci, H, W, co, _p(acts[-1]), _p(self.wq[li]),
                                             _p(self.bq[li]), 0, None, _p(out), _p(C),
                                             _stream()), "mek_cnn_conv3x3")
        return acts, out

    def predict(self, C: torch.Tensor) -> torch.Tensor:
        return self.forward(C)[1]

    def loss_and_grads(self, C: torch.Tensor, label: torch.Tensor) -> float:
        """Mean squared error of X0 against label; fills self.g (weights
        then biases) with its gradients."""
        N, _, H, W = C.shape
        acts, out = self.forward(C)
        g = torch.empty(out.shape, dtype=torch.int16, device=self.device)
        loss = ctypes.c_double()
        _check(lib().mek_cnn_mse_grad(out.numel(), _p(out), _p(label), _p(g), ctypes.byref(loss),
                                      _stream()), "mek_cnn_mse_grad")
        nl = len(CHANNELS) - 1
        for li in range(nl - 1, -1, -1):
            ci, co = CHANNELS[li], CHANNELS[li + 1]
            gate = acts[li + 1] if li < nl - 1 else None   # the layer's ReLU output
            _check(lib().mek_cnn_conv3x3_grad_weight(N, ci, H, W, co, _p(acts[li]), _p(g), _p(gate),
                                                     _p(self.g[li]), _p(self.g[nl + li]),
                                                     _stream()), "mek_cnn_conv3x3_grad_weight")
            if li > 0:
                gx = torch.empty((N, H, W, ci), dtype=torch.int16, device=self.device)
                _check(lib().mek_cnn_conv3x3_grad_input(N, co, H, W, ci, _p(g), _p(gate),
                                                        _p(self.wq[li]), _p(gx), _stream()),
                       "mek_cnn_conv3x3_grad_input")
                g = gx
        return loss.value

    def adam_step(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8):
        self.t += 1
        for k in range(len(self.params)):
            _check(lib().mek_cnn_adam(self.params[k].numel(), _p(self.params[k]), _p(self.q[k]),
                                      _p(self.g[k]), _p(self.m[k]), _p(self.v[k]), lr, beta1,
                                      beta2, eps, self.t, _stream()), "mek_cnn_adam")

    def train(self, C: torch.Tensor, labels: torch.Tensor, epochs: int, batch: int = 4,
              lr: float = 1e-3, seed: int = 0) -> List[float]:
        """Adam on (C, label) pairs (N, 3, H, W) float64; returns the mean
        loss of each epoch. The order of the pairs is shuffled per epoch
        from default_rng(seed)."""
        rng = np.random.default_rng(seed)
        n = C.shape[0]
        hist = []
        for ep in range(epochs):
            order = rng.permutation(n)
            tot = 0.0
            for s in range(0, n - batch + 1, batch):
                idx = torch.as_tensor(order[s:s + batch], device=self.device)
                cb = C.index_select(0, idx).contiguous()
                lb = labels.index_select(0, idx).contiguous()
                # Step size halves over the last third of the epochs.
                tot += self.loss_and_grads(cb, lb) * batch
                self.adam_step(lr * (0.5 if ep >= (2 * epochs) // 3 else 1.0))
            hist.append(tot / (n - n % batch))
        return hist


def _instances(images):
    return [(i, c) for i in range(len(images)) for c in range(images[i][2].shape[0])]


def solver_labels(mek, images, tau: float, max_iters: int = 1_000_000, seed: int = 0,
                  chunk: int = 768):
    """Training labels produced by the solver itself: for each image
    (A, B, C) with C (channels, H, W) on the GPU, the FP64 ME-GRBK iterate
    from X0 = 0 at relative residual ||C - A X B||_F <= tau ||C||_F (or after
    max_iters). Every image is one sparse-update plan shared by its
    channels, every channel one instance (one work-group) of ragged launches
    of up to `chunk` instances; instance k of the list of (image, channel)
    pairs draws under Philox key (seed, k). Returns a list of tensors shaped
    like the C's."""
    inst = _instances(images)
    out = [torch.empty_like(im[2]) for im in images]
    for s0 in range(0, len(inst), chunk):
        part = inst[s0:s0 + chunk]
        plans = {}
        try:
            for i, _ in part:
                if i not in plans:
                    plans[i] = mek.mek_plan_create(images[i][0], images[i][1], update="sparse")
            _, res = mek.mek_solve_multi([plans[i] for i, _ in part],
                                         [images[i][2][c].contiguous() for i, c in part],
                                         variant="grbk", stop="rel_resid", tol=tau,
                                         max_iters=max_iters, seed=seed, instance=s0)
            for (i, c), r in zip(part, res):
                out[i][c].copy_(r.X)
        finally:
            for P in plans.values():
                mek.mek_plan_destroy(P)
    return out


def compare_warm_start(mek, net: WarmStartNet, images, tau: float, max_iters: int = 1_000_000,
                       seed: int = 0, chunk: int = 768, predict_batch: int = 32):
    """Solve every channel of the held-out images [(A, B, C)] to relative
    residual tau from X0 = 0 and from X0 = C + f(C), in ragged launches of
    sparse-update plans (one per image, created before the clocks start). A
    channel falls back to X0 = 0 when ||C - A X0 B||_F >= ||C||_F. Returns
    per-channel iterations, statuses, start residuals and fallbacks, and the
    wall time of each side (the warm side includes the network's
    prediction and the residual check)."""
    inst = _instances(images)
    plans = [mek.mek_plan_create(A, B, update="sparse") for A, B, _ in images]
    try:
        kw = dict(variant="grbk", stop="rel_resid", tol=tau, max_iters=max_iters, seed=seed)

        def solve_all(X0s=None, iters=None):
            res = []
            for s0 in range(0, len(inst), chunk):
                part = inst[s0:s0 + chunk]
                k = dict(kw, instance=s0)
                if iters is not None:
                    k["max_iters"] = iters
                _, r = mek.mek_solve_multi(
                    [plans[i] for i, _ in part], [images[i][2][c].contiguous() for i, c in part],
                    X0=None if X0s is None else [X0s[i][c].contiguous() for i, c in part], **k)
                res += r
            return res

        torch.cuda.synchronize()
        ts = time.perf_counter()
        base = solve_all()
        torch.cuda.synchronize()
        t_base = time.perf_counter() - ts
        ts = time.perf_counter()
        X0s = []
        for b0 in range(0, len(images), predict_batch):
            C = torch.stack([images[i][2] for i in range(b0, min(len(images), b0 + predict_batch))])
            X0s += list(net.predict(C.contiguous()))
        # The judge of the prediction: the residual it leaves against the
        # zero start's, both from solves that make no update.
        r0 = solve_all(X0s, iters=0)
        z0 = solve_all(None, iters=0)
        fallback = []
        for (i, c), r, z in zip(inst, r0, z0):
            fb = not (r.resid2 < z.resid2)
            fallback.append(fb)
            if fb:
                X0s[i][c].zero_()
        warm = solve_all(X0s)
        torch.cuda.synchronize()
        t_warm = time.perf_counter() - ts
        return {"iters_zero": [r.iters for r in base], "iters_warm": [r.iters for r in warm],
                "status_zero": [r.status for r in base], "status_warm": [r.status for r in warm],
                "time_zero_s": t_base, "time_warm_s": t_warm,
                "start_rel_resid_warm": [float(np.sqrt(r.resid2 / z.resid2))
                                         for r, z in zip(r0, z0)],
                "fallback": fallback}
    finally:
        for P in plans:
            mek.mek_plan_destroy(P)
