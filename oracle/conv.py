"""FP64 CPU oracle of the learned warm start's network (not in the paper:
the warm-start extension X0 = f(C) of the problem's initial guess X^0).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the
smoke check and the benchmark's CPU leg may import it; the GPU library and
its binding never do. It shares no code with the GPU path.

Definitions, written out with explicit shifted sums (no library convolution):
  3x3 convolution, zero padding 1, stride 1, cross-correlation convention:
    y[n,o,h,w] = b[o] + sum_{c,i,j} W[o,c,i,j] x[n,c,h+i-1,w+j-1]
  its gradients for an upstream gradient g = dL/dy:
    dx[n,c,h,w] = sum_{o,i,j} W[o,c,i,j] g[n,o,h-i+1,w-j+1]
    dW[o,c,i,j] = sum_{n,h,w} g[n,o,h,w] x[n,c,h+i-1,w+j-1]
    db[o]       = sum_{n,h,w} g[n,o,h,w]
  ReLU(z) = max(z, 0), gradient passed where the layer's output is > 0.
  Network: four 3x3 layers 3 -> 32 -> 32 -> 32 -> 3, ReLU after the first
  three; loss = mean squared error over every output element.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (3, 32, 32, 32, 3)


def _pad(x):
    return np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))


def conv3x3(x, W, b=None):
    """y = conv(x, W) + b; x (N, C, H, W), W (O, C, 3, 3), b (O,)."""
    x = np.asarray(x, np.float64)
    W = np.asarray(W, np.float64)
    N, C, H, Wd = x.shape
    O = W.shape[0]
    xp = _pad(x)
    y = np.zeros((N, O, H, Wd))
    for i in range(3):
        for j in range(3):
            # y[n,o,h,w] += sum_c W[o,c,i,j] x[n,c,h+i-1,w+j-1]
            y += np.einsum("oc,nchw->nohw", W[:, :, i, j], xp[:, :, i:i + H, j:j + Wd])
    if b is not None:
        y += np.asarray(b, np.float64)[None, :, None, None]
    return y


def conv3x3_grad_input(g, W):
    """dx[n,c,h,w] = sum_{o,i,j} W[o,c,i,j] g[n,o,h-i+1,w-j+1]."""
    g = np.asarray(g, np.float64)
    W = np.asarray(W, np.float64)
    N, O, H, Wd = g.shape
    gp = _pad(g)
    dx = np.zeros((N, W.shape[1], H, Wd))
    for i in range(3):
        for j in range(3):
            # g[n,o,h-i+1,w-j+1] = gp[n,o,h-i+2,w-j+2]
            dx += np.einsum("oc,nohw->nchw", W[:, :, i, j],
                            gp[:, :, 2 - i:2 - i + H, 2 - j:2 - j + Wd])
    return dx


def conv3x3_grad_weight(g, x):
    """dW[o,c,i,j] = sum_{n,h,w} g[n,o,h,w] x[n,c,h+i-1,w+j-1]; db[o] = sum g."""
    g = np.asarray(g, np.float64)
    x = np.asarray(x, np.float64)
    N, C, H, Wd = x.shape
    xp = _pad(x)
    dW = np.zeros((g.shape[1], C, 3, 3))
    for i in range(3):
        for j in range(3):
            dW[:, :, i, j] = np.einsum("nohw,nchw->oc", g, xp[:, :, i:i + H, j:j + Wd])
    return dW, g.sum(axis=(0, 2, 3))


def relu(z):
    return np.maximum(z, 0.0)


def bf16(x):
    """Round to the nearest BF16 value (8-bit significand), ties to even,
    from the FP32 value of x: the storage precision of the GPU network's
    activations and gradients (finite inputs)."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, x, store=None, add=None):
    """params: list of (W, b) for the four layers. Returns the list of layer
    outputs (after ReLU for the first three) with x prepended. store, if
    given, rounds each hidden layer's output (the storage precision); add
    is added to the last layer's output."""
    acts = [np.asarray(x, np.float64)]
    for li, (W, b) in enumerate(params):
        z = conv3x3(acts[-1], W, b)
        if li < len(params) - 1:
            z = relu(z)
            if store is not None:
                z = store(z)
        elif add is not None:
            z = z + np.asarray(add, np.float64)
        acts.append(z)
    return acts


def mse(y, label):
    d = np.asarray(y, np.float64) - np.asarray(label, np.float64)
    return float(np.mean(d * d))


def backward(params, acts, label, store=None):
    """Gradients of the mean squared error of forward(params, x) against
    label. Returns (loss, [(dW, db)] per layer, dx of the input). store, if
    given, rounds the loss gradient and each propagated input gradient."""
    y = acts[-1]
    loss = mse(y, label)
    g = 2.0 * (y - np.asarray(label, np.float64)) / y.size
    if store is not None:
        g = store(g)
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        if li < len(params) - 1:
            g = g * (acts[li + 1] > 0.0)
        grads[li] = conv3x3_grad_weight(g, acts[li])
        g = conv3x3_grad_input(g, W)
        if store is not None and li > 0:
            g = store(g)
    return loss, grads, g
