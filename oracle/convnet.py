"""Plain FP64 reference of the learned block preconditioner (a small 4D
convolutional network), its gradients, training loss and Adam update.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no learned component (its Section 5 outlook mentions machine
learning only for flow-based sampling), so nothing here is taken from it; the
network only approximates the block inverse D_Lambda^{-1} of Section 3, whose
exact action the block solver provides.  Definitions used by both this
reference and the GPU kernels:

* A field on one block is an array X[y0, y1, y2, y3, c] over the block's box
  (box-local coordinates, y3 fastest) with c the 24 real channels of a spinor:
  c = 2 * (3 * spin + colour) + (0: real, 1: imaginary part).
* A layer is a 3^4 correlation with zero padding at the block faces (no
  periodic wrap: the block is a Dirichlet domain) and no bias:
      Y[y, o] = sum_{t in {-1,0,1}^4} sum_c W[t, c, o] X[y + t, c],
  tap index t -> (t0 + 1) * 27 + (t1 + 1) * 9 + (t2 + 1) * 3 + (t3 + 1).
* The network is layer(24 -> 32), act, layer(32 -> 32), act, layer(32 -> 24),
  with act the identity ("linear") or max(0, z) ("relu").
* Loss of a batch: mean over its pairs of |mask (N(b) - x)|^2 / |mask x|^2
  with mask selecting the sites the prediction is used on (even sites when the
  network preconditions the even-odd reduced system).
* Adam (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
  w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Parity of these definitions is pinned by the tests without the paper: central
finite differences for every gradient, the free Wilson operator (U = 1) of
the C reference written as conv weights, a 1D reduction to numpy's
correlation, and Adam's closed-form first steps.
"""
from __future__ import annotations

import itertools

import numpy as np

TAPS = list(itertools.product((-1, 0, 1), repeat=4))  # tap index order above
CHANNELS = (24, 32, 32, 24)


def conv(X: np.ndarray, W: np.ndarray) -> np.ndarray:
    """One layer: X [e0, e1, e2, e3, C_in], W [81, C_in, C_out] -> [e0, e1, e2, e3, C_out]."""
    e = X.shape[:4]
    Xp = np.pad(X, [(1, 1)] * 4 + [(0, 0)])
    Y = np.zeros(e + (W.shape[2],))
    for k, t in enumerate(TAPS):
        sl = tuple(slice(1 + t[m], 1 + t[m] + e[m]) for m in range(4))
        Y += Xp[sl] @ W[k]
    return Y


def conv_grad_input(dY: np.ndarray, W: np.ndarray) -> np.ndarray:
    """dL/dX of one layer: dX[y, c] = sum_t sum_o W[t, c, o] dY[y - t, o] (zero outside the block)."""
    e = dY.shape[:4]
    dYp = np.pad(dY, [(1, 1)] * 4 + [(0, 0)])
    dX = np.zeros(e + (W.shape[1],))
    for k, t in enumerate(TAPS):
        sl = tuple(slice(1 - t[m], 1 - t[m] + e[m]) for m in range(4))
        dX += dYp[sl] @ W[k].T
    return dX


def conv_grad_weight(X: np.ndarray, dY: np.ndarray) -> np.ndarray:
    """dL/dW of one layer: dW[t, c, o] = sum_y X[y + t, c] dY[y, o]."""
    e = X.shape[:4]
    Xp = np.pad(X, [(1, 1)] * 4 + [(0, 0)])
    cin, cout = X.shape[4], dY.shape[4]
    dW = np.zeros((81, cin, cout))
    for k, t in enumerate(TAPS):
        sl = tuple(slice(1 + t[m], 1 + t[m] + e[m]) for m in range(4))
        dW[k] = Xp[sl].reshape(-1, cin).T @ dY.reshape(-1, cout)
    return dW


def _act(z, kind):
    return np.maximum(z, 0.0) if kind == "relu" else z


def forward(X: np.ndarray, Ws, act: str = "linear"):
    """Network output and the layer inputs/pre-activations (for the backward pass)."""
    acts = [X]
    pre = []
    h = X
    for l, W in enumerate(Ws):
        z = conv(h, W)
        pre.append(z)
        h = _act(z, act) if l < len(Ws) - 1 else z
        acts.append(h)
    return h, acts, pre


def backward(dOut: np.ndarray, Ws, acts, pre, act: str = "linear"):
    """Gradients of the weights (list) and of the input, given dL/dOutput."""
    dWs = [None] * len(Ws)
    g = dOut
    for l in range(len(Ws) - 1, -1, -1):
        if l < len(Ws) - 1 and act == "relu":
            g = g * (pre[l] > 0)
        dWs[l] = conv_grad_weight(acts[l], g)
        g = conv_grad_input(g, Ws[l])
    return dWs, g


def loss_and_grad(Xb, Tb, Ws, mask=None, act: str = "linear"):
    """Mean relative squared error over a batch and its weight gradients.
    Xb, Tb: [n, e0, e1, e2, e3, 24] inputs and targets; mask: [e0, e1, e2, e3] of 0/1 (None = all)."""
    n = Xb.shape[0]
    m = np.ones(Xb.shape[1:5]) if mask is None else mask
    loss = 0.0
    dWs = [np.zeros_like(W) for W in Ws]
    for i in range(n):
        out, acts, pre = forward(Xb[i], Ws, act)
        diff = (out - Tb[i]) * m[..., None]
        den = np.sum((Tb[i] * m[..., None]) ** 2)
        loss += np.sum(diff**2) / den / n
        g = 2.0 * diff / den / n
        d, _ = backward(g, Ws, acts, pre, act)
        for l in range(len(Ws)):
            dWs[l] += d[l]
    return loss, dWs


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns the new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1**t)
    vh = v / (1 - b2**t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def spinor_to_channels(psi: np.ndarray, extent) -> np.ndarray:
    """[S, 4, 3] complex (box-local canonical order) -> [e0, e1, e2, e3, 24] real channels."""
    z = np.stack([psi.real, psi.imag], axis=-1)  # [S, 4, 3, 2]
    return z.reshape(tuple(extent) + (24,))


def channels_to_spinor(X: np.ndarray) -> np.ndarray:
    """Inverse of spinor_to_channels: [e0, e1, e2, e3, 24] -> [S, 4, 3] complex."""
    z = X.reshape(-1, 4, 3, 2)
    return z[..., 0] + 1j * z[..., 1]
