"""Pins of the warm-start network's FP64 oracle (oracle/conv.py) against
things other than itself: scipy's correlate2d, closed forms of identity and
shift kernels, the adjoint identity, brute-force sums and central finite
differences through the whole network on 8 x 8 images."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import conv


def _rand(rng, *shape):
    return rng.standard_normal(shape)


def test_forward_matches_scipy_correlate2d():
    rng = np.random.default_rng(0)
    x, W, b = _rand(rng, 2, 3, 9, 7), _rand(rng, 4, 3, 3, 3), _rand(rng, 4)
    y = conv.conv3x3(x, W, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, c], W[o, c], mode="same", boundary="fill")
                             for c in range(3))
            assert np.allclose(y[n, o], ref, rtol=1e-13, atol=1e-13)


def test_identity_and_shift_kernels():
    rng = np.random.default_rng(1)
    x = _rand(rng, 1, 2, 6, 5)
    W = np.zeros((2, 2, 3, 3))
    W[0, 0, 1, 1] = W[1, 1, 1, 1] = 1.0
    assert np.array_equal(conv.conv3x3(x, W), x)
    # A single tap at (i, j) reads x[h + i - 1, w + j - 1], zero outside.
    for i in range(3):
        for j in range(3):
            W = np.zeros((1, 2, 3, 3))
            W[0, 1, i, j] = 1.0
            y = conv.conv3x3(x, W)[0, 0]
            ref = np.zeros((6, 5))
            for h in range(6):
                for w in range(5):
                    hh, ww = h + i - 1, w + j - 1
                    if 0 <= hh < 6 and 0 <= ww < 5:
                        ref[h, w] = x[0, 1, hh, ww]
            assert np.array_equal(y, ref)


def test_grad_input_is_the_adjoint():
    rng = np.random.default_rng(2)
    x, W, g = _rand(rng, 3, 4, 8, 6), _rand(rng, 5, 4, 3, 3), _rand(rng, 3, 5, 8, 6)
    lhs = np.sum(conv.conv3x3(x, W) * g)
    rhs = np.sum(x * conv.conv3x3_grad_input(g, W))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_grad_weight_brute_force():
    rng = np.random.default_rng(3)
    x, g = _rand(rng, 2, 3, 5, 4), _rand(rng, 2, 2, 5, 4)
    dW, db = conv.conv3x3_grad_weight(g, x)
    ref = np.zeros((2, 3, 3, 3))
    for o in range(2):
        for c in range(3):
            for i in range(3):
                for j in range(3):
                    s = 0.0
                    for n in range(2):
                        for h in range(5):
                            for w in range(4):
                                hh, ww = h + i - 1, w + j - 1
                                if 0 <= hh < 5 and 0 <= ww < 4:
                                    s += g[n, o, h, w] * x[n, c, hh, ww]
                    ref[o, c, i, j] = s
    assert np.allclose(dW, ref, rtol=1e-13, atol=1e-13)
    assert np.allclose(db, [g[:, o].sum() for o in range(2)], rtol=1e-13)


def _net(rng, chans=conv.CHANNELS, scale=0.3):
    return [(scale * _rand(rng, co, ci, 3, 3), 0.1 * _rand(rng, co))
            for ci, co in zip(chans[:-1], chans[1:])]


def test_network_gradients_by_central_differences():
    # 8 x 8 images, the full 3-32-32-32-3 network; central differences with
    # step 1e-6 on sampled weights, every bias of the first and last layer
    # and sampled input pixels (ReLU kinks have measure zero).
    rng = np.random.default_rng(4)
    params = _net(rng)
    x, label = rng.uniform(0, 1, (2, 3, 8, 8)), rng.uniform(0, 1, (2, 3, 8, 8))
    acts = conv.forward(params, x)
    loss, grads, dx = conv.backward(params, acts, label)
    assert loss == pytest.approx(conv.mse(acts[-1], label))

    def loss_at(p, xx):
        return conv.mse(conv.forward(p, xx)[-1], label)

    eps = 1e-6
    for li in range(4):
        W, b = params[li]
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in W.shape)
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += eps
            Wm[idx] -= eps
            pp = [(Wp, b) if k == li else params[k] for k in range(4)]
            pm = [(Wm, b) if k == li else params[k] for k in range(4)]
            fd = (loss_at(pp, x) - loss_at(pm, x)) / (2 * eps)
            assert grads[li][0][idx] == pytest.approx(fd, rel=1e-5, abs=1e-10)
        for o in (range(b.size) if li in (0, 3) else rng.integers(0, b.size, 3)):
            bp, bm = b.copy(), b.copy()
            bp[o] += eps
            bm[o] -= eps
            pp = [(W, bp) if k == li else params[k] for k in range(4)]
            pm = [(W, bm) if k == li else params[k] for k in range(4)]
            fd = (loss_at(pp, x) - loss_at(pm, x)) / (2 * eps)
            assert grads[li][1][o] == pytest.approx(fd, rel=1e-5, abs=1e-10)
    for _ in range(6):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd = (loss_at(params, xp) - loss_at(params, xm)) / (2 * eps)
        assert dx[idx] == pytest.approx(fd, rel=1e-5, abs=1e-10)


def test_relu_mask_uses_the_layer_output():
    # A layer whose pre-activations are all negative passes no gradient.
    rng = np.random.default_rng(5)
    params = _net(rng)
    W0, b0 = params[0]
    params[0] = (np.zeros_like(W0), -np.ones_like(b0))
    x, label = rng.uniform(0, 1, (1, 3, 8, 8)), rng.uniform(0, 1, (1, 3, 8, 8))
    acts = conv.forward(params, x)
    _, grads, dx = conv.backward(params, acts, label)
    assert np.all(grads[0][0] == 0.0) and np.all(grads[0][1] == 0.0)
    assert np.all(dx == 0.0)


def test_bf16_rounding_closed_forms():
    # 8-bit significand: spacing 2^-7 on [1, 2); halfway cases go to even.
    cases = {1.0: 1.0, 1.0 + 2.0 ** -8: 1.0, 1.0 + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6,
             1.0 + 2.0 ** -7: 1.0 + 2.0 ** -7, 1.0 + 1.1 * 2.0 ** -8: 1.0 + 2.0 ** -7,
             -3.0 - 2.0 ** -7: -3.0, 0.0: 0.0, 2.0 ** -130: 2.0 ** -130}
    for x, r in cases.items():
        assert conv.bf16(np.array([x]))[0] == r, x
    rng = np.random.default_rng(6)
    x = rng.standard_normal(1000)
    y = conv.bf16(x)
    # every result has at most 8 significant bits, and is within half a spacing
    m, e = np.frexp(y)
    assert np.all(m * 256 == np.round(m * 256))
    assert np.all(np.abs(y - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6) + 1e-300)


def test_forward_store_and_add():
    rng = np.random.default_rng(7)
    params = _net(rng)
    x = rng.uniform(0, 1, (1, 3, 6, 6))
    add = rng.standard_normal((1, 3, 6, 6))
    a = conv.forward(params, x)
    b = conv.forward(params, x, store=conv.bf16, add=add)
    assert np.allclose(b[-1] - add, a[-1], rtol=0.05, atol=0.05)
    for li in (1, 2, 3):
        assert np.array_equal(conv.bf16(b[li]), b[li])


def _one_pixel_net(W1c, W2c, pad_tap=7.0):
    """Two 1 -> 1 channel layers on a 1 x 1 image: only the centre tap meets
    the pixel, every other tap reads the zero padding (set to pad_tap to
    show it is never used)."""
    W1 = np.full((1, 1, 3, 3), pad_tap)
    W2 = np.full((1, 1, 3, 3), -pad_tap)
    W1[0, 0, 1, 1] = W1c
    W2[0, 0, 1, 1] = W2c
    return [(W1, np.zeros(1)), (W2, np.zeros(1))]


def test_backward_store_worked_example():
    """Hand-worked BF16 storage points of backward(store=bf16) (spacing 2^-7
    on [1, 2), ties to even): the loss gradient and each propagated input
    gradient of layers above the first are rounded; the weight and bias
    gradients and the input gradient of the first layer are not."""
    e = 2.0 ** -10
    params = _one_pixel_net(1 + e, 1 + e)
    x = np.full((1, 1, 1, 1), 1 + 2.0 ** -11)
    acts = conv.forward(params, x, store=conv.bf16)
    # z1 = (1 + 2^-10)(1 + 2^-11) rounds to 1; y = (1 + 2^-10) * 1.
    assert acts[1][0, 0, 0, 0] == 1.0 and acts[2][0, 0, 0, 0] == 1 + e
    d = 0.5 * (1 + 3 * 2.0 ** -9)
    label = acts[2] - d
    loss, grads, dx = conv.backward(params, acts, label, store=conv.bf16)
    assert loss == pytest.approx(d * d, rel=1e-15)
    g2 = 1 + 2.0 ** -7          # bf16(2 d) = bf16(1 + 3 2^-9): rounds up
    g1 = 1 + 2.0 ** -7          # bf16(W2 g2) = bf16(1 + 2^-7 + 2^-10 + 2^-17): rounds down
    (dW1, db1), (dW2, db2) = grads
    assert dW2[0, 0, 1, 1] == g2 * 1.0 and db2[0] == g2
    # Weight gradient of layer 1: stored g1 times the (unrounded) input.
    assert dW1[0, 0, 1, 1] == g1 * (1 + 2.0 ** -11) and db1[0] == g1
    assert dW1[0, 0, 1, 1] != conv.bf16(np.array([dW1[0, 0, 1, 1]]))[0]
    # Taps that only meet the padding get zero gradient.
    off = np.ones((3, 3), bool)
    off[1, 1] = False
    assert np.all(dW1[0, 0][off] == 0.0) and np.all(dW2[0, 0][off] == 0.0)
    # The first layer's input gradient is not rounded.
    assert dx[0, 0, 0, 0] == (1 + e) * g1


def test_backward_store_points_and_gate_order():
    """The values handed to `store` are, in order, the loss gradient and the
    ungated input gradients of layers 3, 2, 1 (each then gated by the layer
    below's ReLU output); rounding commutes with that 0/1 gate. Checked
    against the unrounded backward with the same rounding applied by hand."""
    rng = np.random.default_rng(8)
    params = [(rng.standard_normal((o, c, 3, 3)) * 0.3, rng.standard_normal(o) * 0.1)
              for c, o in zip(conv.CHANNELS[:-1], conv.CHANNELS[1:])]
    x, label = rng.uniform(0, 1, (1, 3, 5, 5)), rng.uniform(0, 1, (1, 3, 5, 5))
    acts = conv.forward(params, x, store=conv.bf16)
    seen = []

    def rec(v):
        seen.append(np.array(v))
        return conv.bf16(v)

    _, grads, dx = conv.backward(params, acts, label, store=rec)
    assert len(seen) == 4
    # By hand: the same chain with conv.bf16 at the documented points.
    g = conv.bf16(2.0 * (acts[-1] - label) / acts[-1].size)
    assert np.array_equal(seen[0], 2.0 * (acts[-1] - label) / acts[-1].size)
    for li, k in zip((3, 2, 1), (1, 2, 3)):
        if li < 3:
            g = g * (acts[li + 1] > 0)
        dW, db = conv.conv3x3_grad_weight(g, acts[li])
        assert np.array_equal(grads[li][0], dW) and np.array_equal(grads[li][1], db)
        raw = conv.conv3x3_grad_input(g, params[li][0])
        assert np.array_equal(seen[k], raw)
        g = conv.bf16(raw)
    g = g * (acts[1] > 0)
    dW, db = conv.conv3x3_grad_weight(g, acts[0])
    assert np.array_equal(grads[0][0], dW) and np.array_equal(grads[0][1], db)
    assert np.array_equal(dx, conv.conv3x3_grad_input(g, params[0][0]))
