"""Pins for the oracle's learned-scheduler network (MLP 25-64-64-1, tanh, MSE, Adam)."""
import math

import numpy as np
import pytest

import oracle
import synth

NP = oracle.MLP_NPARAM


def _slices():
    i = 0
    out = {}
    for name, n in [("W1", 64 * 25), ("b1", 64), ("W2", 64 * 64), ("b2", 64), ("W3", 64), ("b3", 1)]:
        out[name] = slice(i, i + n)
        i += n
    return out


def test_parameter_count():
    assert NP == 5889  # 64*25 + 64 + 64*64 + 64 + 64 + 1


def test_forward_closed_form_constant_layers():
    # W1 = W2 = 0: h1 = tanh(b1), h2 = tanh(b2), y = W3 . tanh(b2) + b3 for any input.
    s = _slices()
    p = np.zeros(NP)
    p[s["b1"]] = 0.3
    p[s["b2"]] = np.linspace(-1, 1, 64)
    p[s["W3"]] = 0.5
    p[s["b3"]] = -0.25
    x = synth.normal(3, 4 * 25).reshape(4, 25)
    y = oracle.mlp_forward(p, x)
    ref = 0.5 * sum(math.tanh(v) for v in np.linspace(-1, 1, 64)) - 0.25
    assert np.allclose(y, ref, rtol=0, atol=1e-14)


def test_forward_odd_without_biases_and_single_path():
    s = _slices()
    p = synth.normal(5, NP) * 0.2
    p[s["b1"]] = 0
    p[s["b2"]] = 0
    p[s["b3"]] = 0
    x = synth.normal(6, 3 * 25).reshape(3, 25)
    assert np.allclose(oracle.mlp_forward(p, -x), -oracle.mlp_forward(p, x), atol=1e-15)
    # one active path: y = w3 tanh(w2 tanh(w1 x_0))
    q = np.zeros(NP)
    q[s["W1"]][:1] = 0  # placeholder to keep slicing obvious
    q[s["W1"].start + 0] = 0.7      # W1[0][0]
    q[s["W2"].start + 0] = -1.3     # W2[0][0]
    q[s["W3"].start + 0] = 2.0      # W3[0]
    xx = np.zeros((1, 25)); xx[0, 0] = 0.9
    assert abs(oracle.mlp_forward(q, xx)[0] - 2.0 * math.tanh(-1.3 * math.tanh(0.7 * 0.9))) <= 1e-15


def test_gradient_central_differences():
    p = synth.normal(7, NP) * 0.3
    x = synth.normal(8, 6 * 25).reshape(6, 25)
    t = synth.normal(9, 6)
    loss, g = oracle.mlp_loss_grad(p, x, t)
    y = oracle.mlp_forward(p, x)
    assert abs(loss - np.mean((y - t) ** 2)) <= 1e-14 * max(1.0, loss)
    h = 1e-6
    idx = list(range(0, NP, 97)) + [NP - 1, NP - 2, 64 * 25 + 3]
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        num = (np.mean((oracle.mlp_forward(pp, x) - t) ** 2) - np.mean((oracle.mlp_forward(pm, x) - t) ** 2)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, num, g[i])


def test_adam_first_step_is_signed_lr():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m, v = np.zeros(3), np.zeros(3)
    oracle.adam_step(p, g, m, v, 1, lr=0.01)
    # bias-corrected m = g, v = g^2: step = lr * g / (|g| + eps)
    ref = np.array([1.0, -2.0, 0.5]) - 0.01 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p, ref, atol=1e-15)


def test_training_fits_a_smooth_target():
    # 200 Adam steps on a noiseless smooth target reduce the loss by > 10x
    x = synth.normal(11, 256 * 25).reshape(256, 25) * 0.5
    t = np.tanh(x[:, 0] - 0.5 * x[:, 3]) + 0.1 * x[:, 7]
    p = synth.normal(12, NP) * 0.1
    m, v = np.zeros(NP), np.zeros(NP)
    l0, _ = oracle.mlp_loss_grad(p, x, t)
    for step in range(1, 201):
        _, g = oracle.mlp_loss_grad(p, x, t)
        oracle.adam_step(p, g, m, v, step, lr=3e-3)
    l1, _ = oracle.mlp_loss_grad(p, x, t)
    assert l1 < 0.1 * l0


def test_adam_constant_gradient_moves_by_lr_every_step():
    # with a constant gradient the bias-corrected moments are exactly g and g^2 at every step t, so each
    # step moves p by lr * g / (|g| + eps); a wrong bias correction (power, step index or a missing
    # correction of v) breaks this from t = 2 on
    g = np.array([0.3, -4.0, 2e-3, 1.0])
    p = np.zeros(4)
    m, v = np.zeros(4), np.zeros(4)
    for t in range(1, 6):
        oracle.adam_step(p, g, m, v, t, lr=0.01)
        assert np.allclose(p, -t * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-16), t


def test_adam_second_step_with_opposing_gradient_stands_still():
    # first moment after g1 then g2 = -b1 g1: (1-b1)(b1 g1 + g2) = 0, so the second step leaves p
    # where the first put it, whatever the second moment is
    b1 = 0.9
    g1 = np.array([0.5, -2.0, 1e-3])
    p = np.array([1.0, 2.0, 3.0])
    m, v = np.zeros(3), np.zeros(3)
    oracle.adam_step(p, g1, m, v, 1, lr=0.05, b1=b1)
    after1 = p.copy()
    oracle.adam_step(p, -b1 * g1, m, v, 2, lr=0.05, b1=b1)
    assert np.allclose(p, after1, rtol=0, atol=1e-15)
    assert np.allclose(after1, [1.0, 2.0, 3.0] - 0.05 * g1 / (np.abs(g1) + 1e-8), rtol=1e-13)


def test_adam_two_steps_hand_computed():
    # one parameter from 0 with gradients 1 then 3 (lr 0.1, b1 0.9, b2 0.999, eps 1e-8), by hand:
    # t = 1: m = 0.1, v = 0.001, corrected 1 and 1, p = -0.1 / (1 + 1e-8);
    # t = 2: m = 0.09 + 0.3 = 0.39, v = 0.000999 + 0.009 = 0.009999, corrected by 1 - 0.9^2 = 0.19 and
    #        1 - 0.999^2 = 0.001999: 39/19 and 9999/1999, p -= 0.1 (39/19) / (sqrt(9999/1999) + 1e-8)
    p = np.zeros(1)
    m, v = np.zeros(1), np.zeros(1)
    oracle.adam_step(p, np.array([1.0]), m, v, 1, lr=0.1)
    assert abs(p[0] - (-0.1 / (1 + 1e-8))) <= 1e-16
    oracle.adam_step(p, np.array([3.0]), m, v, 2, lr=0.1)
    assert abs(m[0] - 0.39) <= 1e-15 and abs(v[0] - 0.009999) <= 1e-16  # (1 - b2) is not exact in binary
    assert abs(p[0] - (-0.1917781104876684)) <= 1e-14
