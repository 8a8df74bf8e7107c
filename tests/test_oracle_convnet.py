"""Pins of the FP64 reference of the learned preconditioner (oracle/convnet.py).

No paper values exist for this component (it is not in the paper), so the
reference is pinned by independent facts: the free Wilson operator of the C
reference (a separately pinned implementation) written as conv weights, a 1D
reduction to numpy's correlation, exact adjoint identities of the two
gradient formulas, central finite differences of the whole network loss, and
the closed-form first steps of Adam.
"""
import numpy as np
import pytest

import synth
from oracle import convnet, wilson


def _real_rep(A):
    """24 x 24 real matrix of a complex 12 x 12 matrix acting on (spin, colour), channel 2k + ri."""
    M = np.zeros((24, 24))
    M[0::2, 0::2] = A.real
    M[0::2, 1::2] = -A.imag
    M[1::2, 0::2] = A.imag
    M[1::2, 1::2] = A.real
    return M


def _tap(t):
    return convnet.TAPS.index(tuple(t))


def wilson_free_weights(kappa):
    """D(U=1) = 1 - kappa sum_mu [(1 - g_mu) T_{+mu} + (1 + g_mu) T_{-mu}] as one conv layer."""
    W = np.zeros((81, 24, 24))
    W[_tap((0, 0, 0, 0))] = np.eye(24)
    for mu in range(4):
        g = np.kron(wilson.gamma(mu), np.eye(3))
        e = [0, 0, 0, 0]
        e[mu] = 1
        W[_tap(e)] = _real_rep(-kappa * (np.eye(12) - g)).T
        e[mu] = -1
        W[_tap(e)] = _real_rep(-kappa * (np.eye(12) + g)).T
    return W


@pytest.mark.parametrize("extent", [(4, 3, 2, 5), (2, 2, 2, 2), (1, 4, 1, 3)])
def test_free_wilson_operator_as_conv(extent):
    L = (8, 6, 6, 8)
    origin = (2, 1, 0, 3)
    kappa = 0.137
    U = synth.unit_gauge(L)
    psi = synth.gaussian_complex((int(np.prod(extent)), 4, 3), 7)
    ref = wilson.dirac_box(L, -1, kappa, U, origin, extent, psi)
    X = convnet.spinor_to_channels(psi, extent)
    Y = convnet.conv(X, wilson_free_weights(kappa))
    assert np.max(np.abs(convnet.channels_to_spinor(Y) - ref)) <= 1e-13


def test_one_dimensional_case_is_numpy_correlation():
    rng = np.random.default_rng(3)
    n = 11
    x = rng.standard_normal(n)
    w3 = rng.standard_normal(3)
    W = np.zeros((81, 1, 1))
    for j, d in enumerate((-1, 0, 1)):
        W[_tap((0, 0, 0, d)), 0, 0] = w3[j]
    Y = convnet.conv(x.reshape(1, 1, 1, n, 1), W).reshape(n)
    ref = np.correlate(np.concatenate([[0.0], x, [0.0]]), w3, mode="valid")
    assert np.allclose(Y, ref, rtol=0, atol=1e-14)


def test_gradient_formulas_are_exact_adjoints():
    rng = np.random.default_rng(4)
    e = (3, 2, 4, 2)
    X = rng.standard_normal(e + (5,))
    W = rng.standard_normal((81, 5, 3))
    G = rng.standard_normal(e + (3,))
    lhs = np.sum(G * convnet.conv(X, W))
    assert abs(lhs - np.sum(convnet.conv_grad_input(G, W) * X)) <= 1e-11 * abs(lhs) + 1e-11
    assert abs(lhs - np.sum(convnet.conv_grad_weight(X, G) * W)) <= 1e-11 * abs(lhs) + 1e-11


def _weights(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((81, a, b)) * scale / np.sqrt(81 * a)
            for a, b in zip(convnet.CHANNELS[:-1], convnet.CHANNELS[1:])]


@pytest.mark.parametrize("act", ["linear", "relu"])
def test_network_gradient_by_central_differences(act):
    rng = np.random.default_rng(5)
    e = (2, 3, 2, 2)
    Xb = rng.standard_normal((2,) + e + (24,))
    Tb = rng.standard_normal((2,) + e + (24,))
    mask = (np.indices(e).sum(axis=0) % 2 == 0).astype(float)
    Ws = _weights(6)
    loss, dWs = convnet.loss_and_grad(Xb, Tb, Ws, mask, act)
    h = 1e-6
    for l in range(3):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in Ws[l].shape)
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            fd = (convnet.loss_and_grad(Xb, Tb, Wp, mask, act)[0] - convnet.loss_and_grad(Xb, Tb, Wm, mask, act)[0]) / (2 * h)
            assert abs(fd - dWs[l][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx, fd, dWs[l][idx])
    assert loss > 0


def test_loss_vanishes_at_the_target_and_is_relative():
    rng = np.random.default_rng(8)
    e = (2, 2, 2, 2)
    Ws = _weights(9)
    Xb = rng.standard_normal((1,) + e + (24,))
    out, _, _ = convnet.forward(Xb[0], Ws)
    loss, dWs = convnet.loss_and_grad(Xb, out[None], Ws)
    assert loss == 0.0 and all(np.all(d == 0) for d in dWs)
    # a zero prediction has relative loss exactly 1
    loss0, _ = convnet.loss_and_grad(Xb, out[None], [w * 0 for w in Ws])
    assert abs(loss0 - 1.0) <= 1e-15


def test_relu_network_is_positively_homogeneous_and_linear_one_is_linear():
    rng = np.random.default_rng(10)
    e = (2, 3, 2, 2)
    X = rng.standard_normal(e + (24,))
    Y = rng.standard_normal(e + (24,))
    Ws = _weights(11)
    a = 2.75
    for act in ("relu", "linear"):
        fx = convnet.forward(X, Ws, act)[0]
        assert np.allclose(convnet.forward(a * X, Ws, act)[0], a * fx, rtol=1e-13, atol=1e-13)
    lin = lambda z: convnet.forward(z, Ws, "linear")[0]  # noqa: E731
    assert np.allclose(lin(X + Y), lin(X) + lin(Y), rtol=1e-12, atol=1e-12)


def test_adam_closed_form_steps():
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    w, m, v = np.array([0.5]), np.zeros(1), np.zeros(1)
    # constant gradient: every step moves by lr * |g| / (|g| + eps) against the gradient
    for t in range(1, 4):
        w_new, m, v = convnet.adam_step(w, np.array([3.0]), m, v, t, lr, b1, b2, eps)
        assert abs((w - w_new)[0] - lr * 3.0 / (3.0 + eps)) <= 1e-15
        w = w_new
    # gradients +1 then -1: the second step is lr (1 - b1) / (1 + b1) / (1 + eps) backwards
    w, m, v = np.array([0.0]), np.zeros(1), np.zeros(1)
    w, m, v = convnet.adam_step(w, np.array([1.0]), m, v, 1, lr, b1, b2, eps)
    w2, m, v = convnet.adam_step(w, np.array([-1.0]), m, v, 2, lr, b1, b2, eps)
    assert abs((w2 - w)[0] - lr * (1 - b1) / (1 + b1) / (1 + eps)) <= 1e-15


def test_channel_layout_round_trip():
    psi = synth.gaussian_complex((24, 4, 3), 12)
    X = convnet.spinor_to_channels(psi, (2, 3, 2, 2))
    assert X[0, 0, 0, 1, 2 * (3 * 2 + 1) + 1] == psi[1, 2, 1].imag
    assert np.array_equal(convnet.channels_to_spinor(X), psi)
