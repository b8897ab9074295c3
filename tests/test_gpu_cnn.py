"""GPU parity of the warm-start network's kernels (BF16 storage, FP32 sums)
against the FP64 oracle (oracle/conv.py), through the C ABI.

Tolerances follow the arithmetic: inputs and weights are BF16 values on
both sides; a layer sums at most 288 products in FP32 (error below
288 * 2^-24 of the sum of |products|) and a BF16 output adds half a unit in
its last place (2^-8 relative). Weight gradients sum over 16 x 16 tiles and
then over the tiles, in FP32. The loss gradient and the Adam step are
compared bit for bit against the same FP32/BF16 formulas in numpy. Through
the whole network the oracle rounds the stored activations and gradients to
BF16 as the GPU does, so only FP32 summation order separates the two.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2408_05444_amd as mek
import workloads
from oracle import conv
from paper_2408_05444_amd import warmstart

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")]

U32 = 2.0 ** -24


def dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def bits_dev(vals):
    """BF16 bits of an (N, C, H, W) array on the GPU: NCHW for 3 channels,
    NHWC for 32 (the library's layout of 32-channel tensors)."""
    if vals.ndim == 4 and vals.shape[1] == 32:
        vals = np.ascontiguousarray(vals.transpose(0, 2, 3, 1))
    return torch.from_numpy(workloads.bf16_bits(vals).view(np.int16)).to("cuda")


def from_bits(t, channels=None):
    """Values of a BF16 device tensor, back in (N, C, H, W) order."""
    v = workloads.bf16_values(t.cpu().numpy().view(np.uint16))
    if v.ndim == 4 and channels == 32:
        v = np.ascontiguousarray(v.transpose(0, 3, 1, 2))
    return v


def empty_bf16(N, C, H, W):
    shape = (N, H, W, C) if C == 32 else (N, C, H, W)
    return torch.empty(shape, dtype=torch.int16, device="cuda")


def p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def absconv(x, W):
    return conv.conv3x3(np.abs(x), np.abs(W))


@pytest.mark.parametrize("cin,cout,relu,bias,out", [(3, 32, 1, True, "bf16"),
                                                    (32, 32, 1, True, "bf16"),
                                                    (32, 32, 0, False, "bf16"),
                                                    (32, 3, 0, True, "f64"),
                                                    (32, 3, 0, True, "f64+add"),
                                                    (3, 3, 1, True, "bf16"),
                                                    (3, 3, 0, False, "f64+add")])
def test_conv_forward(cin, cout, relu, bias, out):
    rng = np.random.default_rng(cin + cout + relu)
    N, H, W = 2, 20, 37   # ragged 16 x 16 tiles on both axes
    x = workloads.bf16_random(rng, (N, cin, H, W))
    w = workloads.bf16_random(rng, (cout, cin, 3, 3), 0.2)
    b = workloads.bf16_random(rng, (cout,), 0.5) if bias else None
    add = rng.standard_normal((N, cout, H, W)) if out == "f64+add" else None
    ref = conv.conv3x3(x, w, b)
    if relu:
        ref = np.maximum(ref, 0.0)
    if add is not None:
        ref = ref + add
    tol = 288 * U32 * absconv(x, w) + (288 * U32 * np.abs(b)[None, :, None, None] if bias else 0)
    L = mek.lib()
    xd, wd, bd = bits_dev(x), dev(w, torch.float32), dev(b, torch.float32) if bias else None
    if out == "bf16":
        y = empty_bf16(N, cout, H, W)
        assert L.mek_cnn_conv3x3(N, cin, H, W, cout, p(xd), p(wd), p(bd), relu, p(y), None, None,
                                 None) == 0
        got = from_bits(y, cout)
        tol = tol + 2.0 ** -8 * np.abs(ref)
    else:
        y = torch.empty((N, cout, H, W), dtype=torch.float64, device="cuda")
        ad = dev(add) if add is not None else None
        assert L.mek_cnn_conv3x3(N, cin, H, W, cout, p(xd), p(wd), p(bd), relu, None, p(y), p(ad),
                                 None) == 0
        got = y.cpu().numpy()
    assert np.all(np.abs(got - ref) <= tol + 1e-30)


@pytest.mark.parametrize("cout,cin,gated", [(32, 32, True), (32, 3, True), (3, 32, False),
                                            (3, 32, True), (3, 3, True)])
def test_conv_grad_input(cout, cin, gated):
    rng = np.random.default_rng(10 + cout + cin)
    N, H, W = 2, 19, 33
    g = workloads.bf16_random(rng, (N, cout, H, W))
    gate = workloads.bf16_random(rng, (N, cout, H, W)) if gated else None
    w = workloads.bf16_random(rng, (cout, cin, 3, 3), 0.2)
    gg = g * (gate > 0) if gated else g
    ref = conv.conv3x3_grad_input(gg, w)
    tol = 288 * U32 * conv.conv3x3_grad_input(np.abs(gg), np.abs(w)) + 2.0 ** -8 * np.abs(ref)
    # Every device tensor stays referenced until the call returns.
    gd, gated_d, wd = bits_dev(g), bits_dev(gate) if gated else None, dev(w, torch.float32)
    gx = empty_bf16(N, cin, H, W)
    assert mek.lib().mek_cnn_conv3x3_grad_input(N, cout, H, W, cin, p(gd), p(gated_d), p(wd),
                                                p(gx), None) == 0
    assert np.all(np.abs(from_bits(gx, cin) - ref) <= tol + 1e-30)


@pytest.mark.parametrize("cin,cout,gated", [(3, 32, True), (32, 32, True), (32, 3, False)])
def test_conv_grad_weight(cin, cout, gated):
    rng = np.random.default_rng(20 + cout + cin)
    N, H, W = 3, 21, 34
    x = workloads.bf16_random(rng, (N, cin, H, W))
    g = workloads.bf16_random(rng, (N, cout, H, W))
    gate = workloads.bf16_random(rng, (N, cout, H, W)) if gated else None
    gg = g * (gate > 0) if gated else g
    dW_ref, db_ref = conv.conv3x3_grad_weight(gg, x)
    aW, ab = conv.conv3x3_grad_weight(np.abs(gg), np.abs(x))
    tiles = N * ((H + 15) // 16) * ((W + 15) // 16)
    k = (256 + tiles) * U32
    xd, gd, gated_d = bits_dev(x), bits_dev(g), bits_dev(gate) if gated else None
    dw = torch.empty((cout, cin, 3, 3), dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    assert mek.lib().mek_cnn_conv3x3_grad_weight(N, cin, H, W, cout, p(xd), p(gd), p(gated_d),
                                                 p(dw), p(db), None) == 0
    assert np.all(np.abs(dw.cpu().numpy() - dW_ref) <= k * aW + 1e-30)
    assert np.all(np.abs(db.cpu().numpy() - db_ref) <= k * ab + 1e-30)


def test_mse_grad_bit_exact():
    rng = np.random.default_rng(30)
    n = 3 * 37 * 41
    y, lab = rng.standard_normal(n), rng.standard_normal(n)
    yd, ld = dev(y), dev(lab)
    g = torch.empty(n, dtype=torch.int16, device="cuda")
    loss = ctypes.c_double()
    assert mek.lib().mek_cnn_mse_grad(n, p(yd), p(ld), p(g), ctypes.byref(loss), None) == 0
    assert loss.value == pytest.approx(np.mean((y - lab) ** 2), rel=1e-13)
    ref = workloads.bf16_bits(((2.0 / n) * (y - lab)).astype(np.float32))
    assert np.array_equal(g.cpu().numpy().view(np.uint16), ref)


def test_adam_step_matches_formula():
    rng = np.random.default_rng(31)
    n = 9251
    w = rng.standard_normal(n).astype(np.float32)
    gr = rng.standard_normal(n).astype(np.float32)
    m = (0.1 * rng.standard_normal(n)).astype(np.float32)
    v = np.abs(0.1 * rng.standard_normal(n)).astype(np.float32)
    t, lr, b1, b2, eps = 7, 1e-3, 0.9, 0.999, 1e-8
    wd, gd, md, vd = (dev(a, torch.float32) for a in (w, gr, m, v))
    wq = torch.empty_like(wd)
    assert mek.lib().mek_cnn_adam(n, p(wd), p(wq), p(gd), p(md), p(vd), lr, b1, b2, eps, t,
                                  None) == 0
    # The step's constants are FP32: 1 - beta and the bias corrections
    # 1 - beta^t formed from the FP32 betas.
    f = np.float32
    b1f, b2f = f(b1), f(b2)
    m2 = b1f * m + (f(1) - b1f) * gr
    v2 = b2f * v + (f(1) - b2f) * gr * gr
    c1, c2 = f(1) - np.power(b1f, f(t)), f(1) - np.power(b2f, f(t))
    w2 = w - f(lr) * (m2 / c1) / (np.sqrt(v2 / c2) + f(eps))
    assert np.allclose(md.cpu().numpy(), m2, rtol=1e-6, atol=1e-7)
    assert np.allclose(vd.cpu().numpy(), v2, rtol=1e-6, atol=1e-9)
    assert np.allclose(wd.cpu().numpy(), w2, rtol=1e-6, atol=1e-7)
    assert np.array_equal(wq.cpu().numpy(), workloads.bf16_values(workloads.bf16_bits(wd.cpu().numpy())).astype(np.float32))


def _oracle_params(net):
    return [(net.wq[li].cpu().numpy().astype(np.float64), net.bq[li].cpu().numpy().astype(np.float64))
            for li in range(4)]


def test_network_forward_and_gradients_match_oracle():
    rng = np.random.default_rng(40)
    net = warmstart.WarmStartNet(seed=3)
    N, H, W = 2, 24, 40
    # BF16 values, so that the network's BF16 input equals C exactly.
    C = workloads.bf16_values(workloads.bf16_bits(0.5 + 0.5 * rng.standard_normal((N, 3, H, W))))
    label = rng.uniform(0, 1, (N, 3, H, W))
    loss = net.loss_and_grads(dev(C), dev(label))
    params = _oracle_params(net)
    acts = conv.forward(params, C, store=conv.bf16, add=C)
    ref_loss, grads, _ = conv.backward(params, acts, label, store=conv.bf16)
    assert loss == pytest.approx(ref_loss, rel=1e-3)
    X0 = net.predict(dev(C)).cpu().numpy()
    assert np.max(np.abs(X0 - acts[-1])) <= 2e-3 * np.max(np.abs(acts[-1] - C)) + 1e-12
    for li in range(4):
        for k, ref in enumerate(grads[li]):
            got = net.g[li if k == 0 else 4 + li].cpu().numpy()
            err = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
            assert err <= 2e-2, (li, k, err)


def test_training_lowers_the_loss():
    # Four 32 x 32 blurred images, the network trained toward the images.
    imgs = [workloads.warmstart_image(300 + s, size=32) for s in range(4)]
    C = dev(np.stack([im[2] for im in imgs]))
    X = dev(np.stack([im[3] for im in imgs]))
    net = warmstart.WarmStartNet(seed=1)
    hist = net.train(C, X, epochs=40, batch=2, lr=2e-3)
    assert hist[-1] < 0.7 * hist[0]
